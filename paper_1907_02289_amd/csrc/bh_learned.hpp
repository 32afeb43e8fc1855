// bh_learned.hpp -- device functions of the learned opening rule (not part of
// the paper; the paper's walk uses a fixed geometric rule).  Shared by the
// walk (inference), the feature kernel and the training kernels so that the
// three compute identical values.
//
// Rule: for a (group, node) pair with theta_min <= side/distance < theta_max
// (the geometric test of the walk at two angles), a 4-32-32-1 ReLU network
// predicts y = lg(monopole error of the node over the group /
// (G M / d^2)); the node is accepted when y < lg(tau * A_g * d^2 / (G M)),
// i.e. when the predicted error is below tau times the mean self-gravity
// acceleration A_g of the group's particles (from the last evaluation).  A single-particle node is exact and always
// accepted; nodes above the count cap fall back to the geometric theta.
//
// Every quantity that decides an acceptance is computed with correctly
// rounded operations in a fixed order (FP64 features, FP32 network with
// explicit fmaf, comparisons in FP64), so the decision is reproducible
// bit for bit by any implementation that follows the same order.
#pragma once
#include "bh_internal.hpp"

#define MLP_NIN 4
#define MLP_NH 32
#define MLP_W1 0                                   // [32][4]
#define MLP_B1 (MLP_W1 + MLP_NH * MLP_NIN)          // 128
#define MLP_W2 (MLP_B1 + MLP_NH)                    // 160, [32][32]
#define MLP_B2 (MLP_W2 + MLP_NH * MLP_NH)           // 1184
#define MLP_W3 (MLP_B2 + MLP_NH)                    // 1216
#define MLP_B3 (MLP_W3 + MLP_NH)                    // 1248
#define MLP_NTRAIN (MLP_B3 + 1)                     // 1249 trained parameters
#define MLP_XMEAN MLP_NTRAIN                        // 1249..1252
#define MLP_XISTD (MLP_XMEAN + MLP_NIN)             // 1253..1256
#define MLP_YMEAN (MLP_XISTD + MLP_NIN)             // 1257
#define MLP_YSTD (MLP_YMEAN + 1)                    // 1258
#define MLP_NPARAM (MLP_YSTD + 1)                   // 1259

// Piecewise-linear base-2 logarithm: x = m 2^e with m in [0.5, 1) gives
// e - 1 + (2m - 1); exact at powers of two, monotone, continuous, computed
// with one rounding.  0 maps to -1100, +inf to +1100.
__host__ __device__ __forceinline__ double lg2p(double x) {
    if (!(x > 0.0)) return -1100.0;
    if (x > 1.7976931348623157e308) return 1100.0;
    int e = 0;
    double m = frexp(x, &e);
    return (double)e + ((2.0 * m) - 2.0);
}

// Second-moment feature of a node: |Q|_F / (M s^2), Q the second moment
// about the centre of mass (xx, xy, xz, yy, yz, zz).
__device__ __forceinline__ float node_qn(const double *Q, double M, double s) {
    double qq = Q[0] * Q[0] + Q[3] * Q[3] + Q[5] * Q[5] + 2.0 * (Q[1] * Q[1]) + 2.0 * (Q[2] * Q[2]) +
                2.0 * (Q[4] * Q[4]);
    return (float)(sqrt(qq) / (M * (s * s)));
}

struct PairGeom {
    double d2;        // |com - group centre|^2
    float f[MLP_NIN];
};

// (side / distance from the node's centre to the group box)^2 in doubled
// integer grid units: the quantity the geometric opening test compares with
// theta^2.  The node must lie outside the box (distance > 0).
__device__ __forceinline__ double box_ratio2(int4 glo, int4 ghi, int Lx, int Ly, int Lz, int level) {
    const int64_t s = (int64_t)1 << (BH_MAXLEVEL - level);
    const int64_t L[3] = {Lx, Ly, Lz};
    const int64_t gl[3] = {glo.x, glo.y, glo.z}, gh[3] = {ghi.x, ghi.y, ghi.z};
    int64_t d2 = 0;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const int64_t C = 2 * L[a] + s;
        int64_t da = 0;
        da = (2 * gl[a] - C > da) ? 2 * gl[a] - C : da;
        da = (C - 2 * gh[a] > da) ? C - 2 * gh[a] : da;
        d2 += da * da;
    }
    return (double)((2 * s) * (2 * s)) / (double)d2;
}

// Features of node (com, M, qn, box ratio r2 = box_ratio2) for a group
// (centre, half-diagonal rg) of a system of total mass Msys, all on the lg2p
// scale: the leading monopole error on the group's nearest particle relative
// to G M / d^2 behaves like qn r2 (d/d_box)^2, which is close to linear in
// these coordinates.
__device__ __forceinline__ PairGeom pair_features(double4 com, double r2, float qn, double4 gc, double rg,
                                                  double Msys) {
    PairGeom p;
    const double dx = com.x - gc.x, dy = com.y - gc.y, dz = com.z - gc.z;
    p.d2 = dx * dx + dy * dy + dz * dz;
    const double d = sqrt(p.d2);
    p.f[0] = (float)lg2p(r2);
    p.f[1] = (float)lg2p(rg / d);
    p.f[2] = (float)lg2p(com.w / Msys);
    p.f[3] = (float)lg2p((double)qn);
    return p;
}

// Network output in label units (lg of the relative monopole error).
__device__ __forceinline__ float mlp_forward(const float *__restrict__ w, const float f[MLP_NIN]) {
    float x[MLP_NIN];
#pragma unroll
    for (int k = 0; k < MLP_NIN; ++k) {
        const float t = f[k] - w[MLP_XMEAN + k];
        x[k] = t * w[MLP_XISTD + k];
    }
    float h1[MLP_NH];
#pragma unroll
    for (int j = 0; j < MLP_NH; ++j) {
        float a = w[MLP_B1 + j];
#pragma unroll
        for (int k = 0; k < MLP_NIN; ++k) a = fmaf(w[MLP_W1 + j * MLP_NIN + k], x[k], a);
        h1[j] = a > 0.0f ? a : 0.0f;
    }
    float out = w[MLP_B3];
#pragma unroll 4
    for (int j = 0; j < MLP_NH; ++j) {
        float a = w[MLP_B2 + j];
#pragma unroll
        for (int k = 0; k < MLP_NH; ++k) a = fmaf(w[MLP_W2 + j * MLP_NH + k], h1[k], a);
        const float h2 = a > 0.0f ? a : 0.0f;
        out = fmaf(w[MLP_W3 + j], h2, out);
    }
    return fmaf(out, w[MLP_YSTD], w[MLP_YMEAN]);
}

// The acceptance decision for a node in the band.
__device__ __forceinline__ bool learned_accept(const float *__restrict__ w, const PairGeom &p, double M,
                                               double A_g, double tau, double G) {
    const float y = mlp_forward(w, p.f);
    const double Z = ((tau * A_g) * p.d2) / (G * M);
    return (double)y < lg2p(Z);
}
