// bh_integrate.hip -- orbit integration, step (4) of the timestep listed in
// Iwasawa et al. (2019) Sec. 4.2, done by the library next to the particle
// data as Sec. 6.1 proposes, and the write-back of results in caller order.
//
// The integrator is kick-drift-kick leapfrog in FP64 (the paper only says
// "integrate"; KDK is the reading): v += (dt/2) a; x += dt v; a = F(x);
// v += (dt/2) a.  Each product and sum is rounded separately.  These are
// streaming updates bound by HBM bandwidth, like the vectorisable loops of
// Sec. 6.2.
#include "bh_internal.hpp"

namespace {

constexpr int TPB = 256;

inline unsigned grid_for(size_t n) {
    size_t b = (n + TPB - 1) / TPB;
    if (b < 1) b = 1;
    if (b > 16384) b = 16384;
    return (unsigned)b;
}

__device__ __forceinline__ int sys_of(const uint32_t *sys_off, int n_sys, uint32_t i) {
    int lo = 0, hi = n_sys - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (sys_off[mid] <= i) lo = mid; else hi = mid - 1;
    }
    return lo;
}

__global__ void k_kick_drift(double4 *pos, double4 *vel, const double4 *acc, uint32_t n, double h, double dt) {
    uint32_t stride = gridDim.x * blockDim.x;
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        double4 v = vel[i], a = acc[i], p = pos[i];
        v.x = v.x + h * a.x;
        v.y = v.y + h * a.y;
        v.z = v.z + h * a.z;
        p.x = p.x + dt * v.x;
        p.y = p.y + dt * v.y;
        p.z = p.z + dt * v.z;
        vel[i] = v;
        pos[i] = p;
    }
}

__global__ void k_kick(double4 *vel, const double4 *acc, uint32_t n, double h) {
    uint32_t stride = gridDim.x * blockDim.x;
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        double4 v = vel[i], a = acc[i];
        v.x = v.x + h * a.x;
        v.y = v.y + h * a.y;
        v.z = v.z + h * a.z;
        vel[i] = v;
    }
}

// Results back in caller order, walked in caller order: the writes to the
// caller's arrays are coalesced and the reads of the sorted state gather
// through the inverse permutation.
__global__ void k_scatter_state(DevState d) {
    uint32_t stride = gridDim.x * blockDim.x;
    for (uint32_t gi = blockIdx.x * blockDim.x + threadIdx.x; gi < d.n; gi += stride) {
        const uint32_t j = d.inv[gi];
        int s = sys_of(d.sys_off, d.n_sys, gi);
        uint32_t k = gi - d.sys_off[s];
        SysPtr p = d.sys_tab[s];
        double4 q = d.pos[j], v = d.vel[j];
        p.x[k] = q.x;
        p.y[k] = q.y;
        p.z[k] = q.z;
        if (p.vx) {
            p.vx[k] = v.x;
            p.vy[k] = v.y;
            p.vz[k] = v.z;
        }
    }
}

__global__ void k_scatter_acc(DevState d, const bhk::AccPtr *tab) {
    uint32_t stride = gridDim.x * blockDim.x;
    for (uint32_t gi = blockIdx.x * blockDim.x + threadIdx.x; gi < d.n; gi += stride) {
        const uint32_t j = d.inv[gi];
        int s = sys_of(d.sys_off, d.n_sys, gi);
        uint32_t k = gi - d.sys_off[s];
        bhk::AccPtr p = tab[s];
        double4 a = d.acc[j];
        p.ax[k] = a.x;
        p.ay[k] = a.y;
        p.az[k] = a.z;
        if (p.pot) p.pot[k] = a.w;
    }
}

// Accelerations of chosen caller-order particles of one system, read
// through the inverse permutation; an index outside the system gives NaN.
__global__ void k_sample_acc(DevState d, int sys, const int64_t *targets, int64_t nt, double *ax, double *ay,
                             double *az) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nt) return;
    const int64_t i = targets[t];
    const uint32_t b = d.sys_off[sys], n = d.sys_off[sys + 1] - b;
    if (i < 0 || i >= (int64_t)n) {
        ax[t] = ay[t] = az[t] = __builtin_nan("");
        return;
    }
    const double4 a = d.acc[d.inv[b + (uint32_t)i]];
    ax[t] = a.x;
    ay[t] = a.y;
    az[t] = a.z;
}

}  // namespace

namespace bhk {

void sample_acc(const DevState &d, int sys, const int64_t *targets, int64_t nt, double *ax, double *ay, double *az,
                hipStream_t s) {
    if (nt <= 0) return;
    k_sample_acc<<<(unsigned)((nt + TPB - 1) / TPB), TPB, 0, s>>>(d, sys, targets, nt, ax, ay, az);
}


void kick_drift(const DevState &d, double h, double dt, hipStream_t s) {
    k_kick_drift<<<grid_for(d.n), TPB, 0, s>>>(d.pos, d.vel, d.acc, d.n, h, dt);
}

void kick(const DevState &d, double h, hipStream_t s) {
    k_kick<<<grid_for(d.n), TPB, 0, s>>>(d.vel, d.acc, d.n, h);
}

void scatter_state(const DevState &d, hipStream_t s) {
    k_scatter_state<<<grid_for(d.n), TPB, 0, s>>>(d);
}

void scatter_acc(const DevState &d, const AccPtr *tab, hipStream_t s) {
    k_scatter_acc<<<grid_for(d.n), TPB, 0, s>>>(d, tab);
}

}  // namespace bhk
