// bh_direct.hip -- FP64 direct summation over all particles for a set of
// target particles: the exact sum that the tree method approximates
// (Sec. 4.2 (3d) applied with every node opened), used to judge the error
// of the Barnes-Hut forces.  With a collision radius every pair follows
// Eq. (2) with both branches (all sources are particles here).
//
// Grid: (target blocks of 64, source chunks).  Each workgroup stages 256
// sources at a time in LDS; its four waves take a quarter each against the
// same 64 targets; wave partials are added in a fixed order and written per
// source chunk, and a second kernel adds the chunks in order.  Gravity
// (scaled by G at the end) and contact terms are summed separately.
#include <mutex>

#include "bh_internal.hpp"

namespace {

constexpr int DT = 256;
constexpr int DCHUNKS = 64;
constexpr int NC = 6;   // per (chunk, target): gravity x, y, z, contact x, y, z

// Partial sums of the allocation-free direct sum (bh_direct_sum_static):
// room for DIRECT_STATIC_MAX_TARGETS targets at the largest chunk count,
// 12 MiB, one copy on every GPU the library runs on, held until the process
// ends.  Host code never passes this name to a kernel: it is a host-side
// stand-in; the device address comes from hipGetSymbolAddress, per device.
constexpr int64_t DIRECT_STATIC_MAX_TARGETS = 4096;
static __device__ __align__(256) double scratch[(size_t)DCHUNKS * DIRECT_STATIC_MAX_TARGETS * NC];

constexpr int MAX_DEVICES = 64;
std::mutex scratch_mu;
double *scratch_dev[MAX_DEVICES] = {};

template <bool COLL>
__global__ void __launch_bounds__(DT) k_direct_part(const double *x, const double *y, const double *z,
                                                   const double *m, int64_t n, const int64_t *targets,
                                                   int64_t nt, double eps2, bhk::Contact ct, double *part,
                                                   int chunks) {
    __shared__ double4 tile[DT];
    __shared__ double red[NC][4][64];
    const int lane = __lane_id(), w = threadIdx.x >> 6;
    const int64_t t = (int64_t)blockIdx.x * 64 + lane;
    const bool ton = t < nt;
    int64_t i = 0;
    double xi = 0, yi = 0, zi = 0;
    bool bad = false;             // a target index outside [0, n): NaN result, nothing read out of range
    if (ton) {
        i = targets[t];
        bad = i < 0 || i >= n;
        if (bad) i = 0;
        xi = x[i];
        yi = y[i];
        zi = z[i];
    }
    const double rc2 = ct.rc * ct.rc;
    const double rce2 = rc2 + eps2;
    const double rce = sqrt(rce2);
    const int64_t per = (n + chunks - 1) / chunks;
    const int64_t j0 = (int64_t)blockIdx.y * per, j1 = (j0 + per < n) ? j0 + per : n;
    double ax = 0, ay = 0, az = 0, cx = 0, cy = 0, cz = 0;
    for (int64_t b = j0; b < j1; b += DT) {
        const int64_t j = b + threadIdx.x;
        if (j < j1) tile[threadIdx.x] = make_double4(x[j], y[j], z[j], m[j]);
        __syncthreads();
        const int cnt = (int)((j1 - b < DT) ? j1 - b : DT);
        const int q0 = cnt * w / 4, q1 = cnt * (w + 1) / 4;
        for (int k = q0; k < q1; ++k) {
            const double4 s = tile[k];
            const double dx = s.x - xi, dy = s.y - yi, dz = s.z - zi;
            const double d2 = dx * dx + dy * dy + dz * dz;
            if (COLL && d2 <= rc2) {
                if (d2 == 0.0 || !ton) continue;
                // contact: gravity frozen on the contact sphere, spring and dashpot
                const double f = s.w / (rce2 * rce);
                ax += f * dx;
                ay += f * dy;
                az += f * dz;
                const int64_t jj = b + k;
                const double dvx = ct.vx[jj] - ct.vx[i], dvy = ct.vy[jj] - ct.vy[i], dvz = ct.vz[jj] - ct.vz[i];
                const double r = sqrt(d2);
                const double rv = dx * dvx + dy * dvy + dz * dvz;
                const double fc = s.w / (m[i] + s.w) * (ct.kappa * (r - ct.rc) / r + ct.eta * rv / d2);
                cx += fc * dx;
                cy += fc * dy;
                cz += fc * dz;
                continue;
            }
            const double r2 = d2 + eps2;
            if (r2 == 0.0) continue;
            const double r = sqrt(r2);
            const double f = s.w / (r2 * r);
            ax += f * dx;
            ay += f * dy;
            az += f * dz;
        }
        __syncthreads();
    }
    red[0][w][lane] = ax;
    red[1][w][lane] = ay;
    red[2][w][lane] = az;
    red[3][w][lane] = cx;
    red[4][w][lane] = cy;
    red[5][w][lane] = cz;
    __syncthreads();
    if (w == 0 && ton) {
        double *o = part + ((size_t)blockIdx.y * nt + t) * NC;
        for (int a = 0; a < NC; ++a)
            o[a] = bad ? NAN : ((red[a][0][lane] + red[a][1][lane]) + red[a][2][lane]) + red[a][3][lane];
    }
}

__global__ void k_direct_sum(const double *part, int64_t nt, int chunks, double G, double *ax, double *ay,
                             double *az) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nt) return;
    double s[NC] = {0, 0, 0, 0, 0, 0};
    for (int c = 0; c < chunks; ++c)
        for (int a = 0; a < NC; ++a) s[a] += part[((size_t)c * nt + t) * NC + a];
    ax[t] = G * s[0] + s[3];
    ay[t] = G * s[1] + s[4];
    az[t] = G * s[2] + s[5];
}

}  // namespace

namespace bhk {

int64_t direct_static_max_targets() { return DIRECT_STATIC_MAX_TARGETS; }

hipError_t direct_static_init(int device) {
    if (device < 0 || device >= MAX_DEVICES) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(scratch_mu);
    if (scratch_dev[device]) return hipSuccess;
    int cur = -1;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return e;
    if (cur != device) return hipErrorInvalidDevice;      // the device must be current
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    scratch_dev[device] = static_cast<double *>(p);
    return hipSuccess;
}

double *direct_static_scratch(int device) {
    if (device < 0 || device >= MAX_DEVICES) return nullptr;
    std::lock_guard<std::mutex> lock(scratch_mu);
    return scratch_dev[device];
}

size_t direct_scratch_bytes(int64_t n_targets) {
    return (size_t)DCHUNKS * (size_t)n_targets * NC * sizeof(double);
}

void direct_sum(const double *x, const double *y, const double *z, const double *m, int64_t n,
                const int64_t *targets, int64_t nt, double eps2, double G, const Contact *contact, double *ax,
                double *ay, double *az, double *scratch, hipStream_t s) {
    int chunks = (int)((n + 65535) / 65536);
    if (chunks < 1) chunks = 1;
    if (chunks > DCHUNKS) chunks = DCHUNKS;
    dim3 grid((unsigned)((nt + 63) / 64), (unsigned)chunks);
    if (contact)
        k_direct_part<true><<<grid, DT, 0, s>>>(x, y, z, m, n, targets, nt, eps2, *contact, scratch, chunks);
    else
        k_direct_part<false><<<grid, DT, 0, s>>>(x, y, z, m, n, targets, nt, eps2, Contact{0, 0, 0, nullptr,
                                                 nullptr, nullptr}, scratch, chunks);
    k_direct_sum<<<(unsigned)((nt + 255) / 256), 256, 0, s>>>(scratch, nt, chunks, G, ax, ay, az);
}

}  // namespace bhk
