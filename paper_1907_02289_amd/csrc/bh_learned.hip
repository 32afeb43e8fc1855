// bh_learned.hip -- data, labels and training kernels of the learned opening
// rule (not part of the paper; see bh_learned.hpp for the rule itself).
//
// Labels come from the method itself: for a candidate (group, node) pair the
// exact force of the node's particles on every particle of the group is
// summed directly in FP64 and compared with the node's monopole (the
// centre-of-mass approximation of Sec. 5.1); the label is the largest error
// over the group in units of G M / d^2, on the lg2p scale.
//
// Training is plain minibatch Adam on the mean squared error.  Gradients of
// a batch are summed per parameter over the batch in a fixed order, so a
// run is reproducible.
#include "bh_learned.hpp"

namespace {

constexpr int TPB = 256;

inline unsigned grid_for(size_t n, size_t cap = 8192) {
    size_t b = (n + TPB - 1) / TPB;
    if (b < 1) b = 1;
    if (b > cap) b = cap;
    return (unsigned)b;
}

__global__ void k_node_qn(DevState d) {
    const uint32_t nn = d.cnt->lvl_off[BH_NLEVELS];
    uint32_t stride = gridDim.x * blockDim.x;
    for (uint32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < nn; v += stride) {
        const uint32_t meta = d.nd_meta[v];
        const double S = (double)(1u << BH_MAXLEVEL) / d.box[meta_sys(meta)].w;   // root side, exact
        const double side = ldexp(S, -(int)meta_level(meta));
        d.nd_qn[v] = node_qn(d.nd_quad + (size_t)v * 6, d.nd_mom[v].w, side);
    }
}

// Self-gravity acceleration magnitude of each group (mean, or smallest, over
// its particles): the error budget scale of the learned rule.
__global__ void __launch_bounds__(TPB) k_group_amin(DevState d) {
    const uint32_t ng = d.cnt->n_groups;
    const uint32_t wpb = TPB / 64;
    for (uint32_t g = blockIdx.x * wpb + (threadIdx.x >> 6); g < ng; g += gridDim.x * wpb) {
        const double a = group_budget(d, d.grp[g]);
        if (__lane_id() == 0) d.g_amin[g] = a;
    }
}

// One workgroup per candidate pair: features and the exact label.
__global__ void __launch_bounds__(TPB) k_cand(DevState d, uint64_t n_cand, float4 *X, float *Y) {
    __shared__ double4 tile[TPB];
    __shared__ double red[TPB / 64];
    const uint32_t ng = d.cnt->n_groups, nn = d.cnt->lvl_off[BH_NLEVELS];
    for (uint64_t p = blockIdx.x; p < n_cand; p += gridDim.x) {
        const uint2 cv = d.cand[p];
        // every loop below is bounded by the pair's group size and node
        // count; a pair outside the tree or above the cap is not evaluated
        const bool bad = cv.x >= ng || cv.y >= nn || d.nd_count[cv.y] > d.count_cap ||
                         (uint64_t)d.grp[cv.x].begin + d.grp[cv.x].count > d.n ||
                         (uint64_t)d.nd_begin[cv.y] + d.nd_count[cv.y] > d.n;
        if (bad) {
            if (threadIdx.x == 0) {
                atomicOr(&d.cnt->flags[FLAG_CAND_BAD], 1u);
                X[p] = make_float4(0.f, 0.f, 0.f, 0.f);
                Y[p] = 0.f;
            }
            continue;
        }
        const GroupInfo gi = d.grp[cv.x];
        const uint32_t v = cv.y;
        const double4 mom = d.nd_mom[v];
        const int4 wr = d.nd_walk[v];
        const double r2 = box_ratio2(d.g_lo[cv.x], d.g_hi[cv.x], wr.x & 0xffffff, wr.y & 0xffffff, wr.z,
                                     (int)((uint32_t)wr.x >> 24));
        const double Msys = d.nd_mom[gi.sys].w;
        const PairGeom pg = pair_features(mom, r2, d.nd_qn[v], d.g_cen[cv.x], d.g_rad[cv.x], Msys);
        const uint32_t cb = d.nd_begin[v], cn = d.nd_count[v];
        double emax = 0.0;
        for (uint32_t i0 = 0; i0 < gi.count; i0 += TPB) {
            const uint32_t i = gi.begin + i0 + threadIdx.x;
            const bool on = i0 + threadIdx.x < gi.count;
            double xi = 0, yi = 0, zi = 0;
            if (on) {
                const double4 q = d.pos[i];
                xi = q.x;
                yi = q.y;
                zi = q.z;
            }
            double ex = 0, ey = 0, ez = 0;
            for (uint32_t j0 = 0; j0 < cn; j0 += TPB) {
                __syncthreads();
                if (j0 + threadIdx.x < cn) tile[threadIdx.x] = d.pos[cb + j0 + threadIdx.x];
                __syncthreads();
                const uint32_t m = min((uint32_t)TPB, cn - j0);
                for (uint32_t k = 0; k < m; ++k) {
                    const double4 s = tile[k];
                    const double dx = s.x - xi, dy = s.y - yi, dz = s.z - zi;
                    const double r2 = dx * dx + dy * dy + dz * dz + d.eps2;
                    const double f = s.w / (r2 * sqrt(r2));
                    ex += f * dx;
                    ey += f * dy;
                    ez += f * dz;
                }
            }
            if (on) {
                const double dx = mom.x - xi, dy = mom.y - yi, dz = mom.z - zi;
                const double r2 = dx * dx + dy * dy + dz * dz + d.eps2;
                const double f = mom.w / (r2 * sqrt(r2));
                const double ux = d.G * (f * dx - ex), uy = d.G * (f * dy - ey), uz = d.G * (f * dz - ez);
                emax = fmax(emax, sqrt(ux * ux + uy * uy + uz * uz));
            }
        }
        emax = wave_max(emax);
        __syncthreads();
        if (__lane_id() == 0) red[threadIdx.x >> 6] = emax;
        __syncthreads();
        if (threadIdx.x == 0) {
            double e = red[0];
            for (int k = 1; k < TPB / 64; ++k) e = fmax(e, red[k]);
            const double ratio = (e * pg.d2) / (d.G * mom.w);
            X[p] = make_float4(pg.f[0], pg.f[1], pg.f[2], pg.f[3]);
            Y[p] = (float)lg2p(ratio);
        }
    }
}

// ---------------------------------------------------------------- training
// Normalisation: mean and 1/std of each feature and of the label, summed in
// FP64 by one workgroup in a fixed order.
__global__ void __launch_bounds__(TPB) k_stats(const float4 *X, const float *Y, uint64_t n, float *w) {
    __shared__ double part[TPB][10];
    double s[5] = {0, 0, 0, 0, 0}, q[5] = {0, 0, 0, 0, 0};
    for (uint64_t i = threadIdx.x; i < n; i += TPB) {
        const float4 x = X[i];
        const double v[5] = {x.x, x.y, x.z, x.w, Y[i]};
        for (int k = 0; k < 5; ++k) {
            s[k] += v[k];
            q[k] += v[k] * v[k];
        }
    }
    for (int k = 0; k < 5; ++k) {
        part[threadIdx.x][k] = s[k];
        part[threadIdx.x][5 + k] = q[k];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double S[10] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
        for (int t = 0; t < TPB; ++t)
            for (int k = 0; k < 10; ++k) S[k] += part[t][k];
        for (int k = 0; k < 5; ++k) {
            const double mean = S[k] / (double)n;
            double var = S[5 + k] / (double)n - mean * mean;
            const double sd = var > 1e-24 ? sqrt(var) : 1.0;
            if (k < 4) {
                w[MLP_XMEAN + k] = (float)mean;
                w[MLP_XISTD + k] = (float)(1.0 / sd);
            } else {
                w[MLP_YMEAN] = (float)mean;
                w[MLP_YSTD] = (float)sd;
            }
        }
    }
}

// Activations per sample of a batch: x (4), h1 (32), h2 (32), g1 (32) and g2 (32)
// the loss gradients at the two hidden pre-activations, go (1) at the output.
#define ACT_X 0
#define ACT_H1 4
#define ACT_H2 36
#define ACT_G2 68
#define ACT_G1 100
#define ACT_GO 132
#define ACT_N 133

__global__ void __launch_bounds__(TPB) k_fwd_bwd(const float *__restrict__ w, const float4 *X, const float *Y,
                                                const uint32_t *idx, uint32_t B, float *act, float *lossv) {
    const uint32_t b = blockIdx.x * TPB + threadIdx.x;
    if (b >= B) return;
    const uint32_t i = idx[b];
    const float4 xx = X[i];
    const float f[4] = {xx.x, xx.y, xx.z, xx.w};
    float x[4];
    for (int k = 0; k < 4; ++k) {
        const float t = f[k] - w[MLP_XMEAN + k];
        x[k] = t * w[MLP_XISTD + k];
    }
    float h1[MLP_NH], h2[MLP_NH];
    for (int j = 0; j < MLP_NH; ++j) {
        float a = w[MLP_B1 + j];
        for (int k = 0; k < 4; ++k) a = fmaf(w[MLP_W1 + j * 4 + k], x[k], a);
        h1[j] = a > 0.0f ? a : 0.0f;
    }
    float out = w[MLP_B3];
    for (int j = 0; j < MLP_NH; ++j) {
        float a = w[MLP_B2 + j];
        for (int k = 0; k < MLP_NH; ++k) a = fmaf(w[MLP_W2 + j * MLP_NH + k], h1[k], a);
        h2[j] = a > 0.0f ? a : 0.0f;
        out = fmaf(w[MLP_W3 + j], h2[j], out);
    }
    // loss on the normalised label: (out - (y - mean) / sd)^2, averaged over the batch
    const float yt = (Y[i] - w[MLP_YMEAN]) / w[MLP_YSTD];
    const float r = out - yt;
    const float go = 2.0f * r / (float)B;
    float *a = act + (size_t)b * ACT_N;
    for (int k = 0; k < 4; ++k) a[ACT_X + k] = x[k];
    for (int j = 0; j < MLP_NH; ++j) {
        a[ACT_H1 + j] = h1[j];
        a[ACT_H2 + j] = h2[j];
        a[ACT_G2 + j] = h2[j] > 0.0f ? go * w[MLP_W3 + j] : 0.0f;
    }
    for (int k = 0; k < MLP_NH; ++k) {
        float g = 0.0f;
        if (h1[k] > 0.0f)
            for (int j = 0; j < MLP_NH; ++j) g = fmaf(w[MLP_W2 + j * MLP_NH + k], a[ACT_G2 + j], g);
        a[ACT_G1 + k] = g;
    }
    a[ACT_GO] = go;
    lossv[b] = r * r;
}

// One thread per trained parameter: its gradient summed over the batch in order.
__global__ void k_param_grad(const float *act, uint32_t B, float *grad, const float *lossv, float *loss) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p == MLP_NTRAIN && loss) {
        double s = 0;
        for (uint32_t b = 0; b < B; ++b) s += lossv[b];
        *loss = (float)(s / B);
    }
    if (p >= MLP_NTRAIN) return;
    int src_g, src_a;      // gradient = sum_b act[g] * act[a]   (src_a < 0: act[g] alone)
    if (p < MLP_B1) {
        src_g = ACT_G1 + p / 4;
        src_a = ACT_X + p % 4;
    } else if (p < MLP_W2) {
        src_g = ACT_G1 + (p - MLP_B1);
        src_a = -1;
    } else if (p < MLP_B2) {
        const int q = p - MLP_W2;
        src_g = ACT_G2 + q / MLP_NH;
        src_a = ACT_H1 + q % MLP_NH;
    } else if (p < MLP_W3) {
        src_g = ACT_G2 + (p - MLP_B2);
        src_a = -1;
    } else if (p < MLP_B3) {
        src_g = ACT_GO;
        src_a = ACT_H2 + (p - MLP_W3);
    } else {
        src_g = ACT_GO;
        src_a = -1;
    }
    float s = 0.0f;
    for (uint32_t b = 0; b < B; ++b) {
        const float *a = act + (size_t)b * ACT_N;
        s = (src_a < 0) ? s + a[src_g] : fmaf(a[src_g], a[src_a], s);
    }
    grad[p] = s;
}

__global__ void k_adam(float *w, const float *g, float *m, float *v, float lr, float b1, float b2, float eps,
                       float c1, float c2) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= MLP_NTRAIN) return;
    const float gp = g[p];
    const float mp = b1 * m[p] + (1.0f - b1) * gp;
    const float vp = b2 * v[p] + (1.0f - b2) * gp * gp;
    m[p] = mp;
    v[p] = vp;
    w[p] -= lr * (mp / c1) / (sqrtf(vp / c2) + eps);
}

__global__ void k_eval(const float *__restrict__ w, const float4 *X, uint64_t n, float *out) {
    uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const float4 x = X[i];
        const float f[4] = {x.x, x.y, x.z, x.w};
        out[i] = mlp_forward(w, f);
    }
}

// splitmix64 of (seed, i): shuffle keys
__global__ void k_perm_keys(uint64_t *key, uint32_t *val, uint64_t n, uint64_t seed) {
    uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        uint64_t z = seed + 0x9e3779b97f4a7c15ull * (i + 1);
        z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
        z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
        key[i] = (z ^ (z >> 31)) >> 32;
        val[i] = (uint32_t)i;
    }
}

}  // namespace

namespace bhk {

void node_qn(const DevState &d, hipStream_t s) {
    k_node_qn<<<grid_for(d.node_cap, 4096), TPB, 0, s>>>(d);
}

void group_amin(const DevState &d, hipStream_t s) {
    k_group_amin<<<grid_for((size_t)d.n * 64 / 8, 8192), TPB, 0, s>>>(d);
}

void cand_features_labels(const DevState &d, uint64_t n_cand, float4 *X, float *Y, hipStream_t s) {
    if (n_cand == 0) return;
    unsigned blocks = (unsigned)(n_cand < 65536 ? n_cand : 65536);
    k_cand<<<blocks, TPB, 0, s>>>(d, n_cand, X, Y);
}

void mlp_stats(const float4 *X, const float *Y, uint64_t n, float *w, hipStream_t s) {
    k_stats<<<1, TPB, 0, s>>>(X, Y, n, w);
}

void mlp_batch_grad(const float *w, const float4 *X, const float *Y, const uint32_t *idx, uint32_t B,
                    float *act, float *grad, float *loss, hipStream_t s) {
    k_fwd_bwd<<<(B + TPB - 1) / TPB, TPB, 0, s>>>(w, X, Y, idx, B, act, act + (size_t)B * ACT_N);
    k_param_grad<<<(MLP_NTRAIN + 1 + 63) / 64, 64, 0, s>>>(act, B, grad, act + (size_t)B * ACT_N, loss);
}

void mlp_adam(float *w, const float *grad, float *m, float *v, float lr, float b1, float b2, float eps, int step,
              hipStream_t s) {
    const float c1 = 1.0f - powf(b1, (float)step), c2 = 1.0f - powf(b2, (float)step);
    k_adam<<<(MLP_NTRAIN + 255) / 256, 256, 0, s>>>(w, grad, m, v, lr, b1, b2, eps, c1, c2);
}

void mlp_eval(const float *w, const float4 *X, uint64_t n, float *out, hipStream_t s) {
    if (n == 0) return;
    k_eval<<<grid_for(n), TPB, 0, s>>>(w, X, n, out);
}

void perm_keys(uint64_t *key, uint32_t *val, uint64_t n, uint64_t seed, hipStream_t s) {
    k_perm_keys<<<grid_for(n), TPB, 0, s>>>(key, val, n, seed);
}

size_t mlp_act_floats(uint32_t B) { return (size_t)B * (ACT_N + 1); }

}  // namespace bhk
