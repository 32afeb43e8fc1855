// bh_force.hip -- the interaction double loop of Iwasawa et al. (2019)
// Sec. 4.2 step (3d): for every group, every particle of the group against
// every entry of the group's lists.  The pair term is the gravity branch of
// Eq. (2) with Plummer softening,
//     a_i += G m_j (x_j - x_i) / (|x_j - x_i|^2 + eps^2)^(3/2),
// nodes acting as point masses at their centre of mass (Sec. 5.1).
//
// Precision (Sec. 4.7, shifted origin): in the FP32 variant the positions
// of the group's particles and of every source are taken relative to the
// group centre in FP64 and only then rounded to FP32; the pair terms and
// their sums are FP32, the result is scaled by G and written in FP64.  The
// FP64 variant is the same loop in double precision.  In FP32, a system
// whose particles all have one mass m0 (the paper's ring particles) enters
// the particle-pair loop with unit masses and its node masses in units of
// m0, the sums being scaled by G m0 at the end: one multiply fewer per pair.
//
// Sources are staged 512 at a time (the FP32 gravity-only kernels also come
// with tiles of 256, a choice of the autotuner) in LDS as group-relative
// float4 (x, y, z, m); particle-list leaves are read 256 at a time, a prefix sum over their
// sizes places their particles in the tiles, and the FP32 gravity-only
// kernels list the chunk's particle ids in LDS once so that staging a source
// is one LDS read (a chunk of more than 2048 particles, possible only with
// big level-21 leaves, searches the leaf offsets instead).  Inside a leapfrog
// step these kernels also apply the closing half kick to each particle.
//
// Scheduling (Sec. 4.6): a persistent grid takes groups from an atomic
// queue in order of decreasing interaction count, so the longest lists start
// first and the tail is made of short ones.  All four waves of a workgroup
// share one LDS tile of sources (the paper's cores sharing a cache on one
// list).  The waves take 64-particle chunks of the group, the waves left
// over splitting the source range.  A partial chunk -- a small group, or the
// last chunk of a larger one -- keeps most of its lanes busy: at most 8, 16 or
// 25..32 particles spread the wave over 8, 4 or 2 sub-slices of the source
// range; 17..24, 33..40 and 49..56 particles (3, 5, 7 slices of 8) run in
// eighths mode and 41..48 in tail mode, where the lanes without particles
// take the last parts of the range for the particles' slices in turn (the
// tile is padded with massless sources so that every part has one length).
// Partial sums are added in a fixed order, so results do not depend on
// timing.
//
// Collision branch of Eq. (2) (particle sources only, when rc > 0): inside
// the pair loop the squared distance is clamped from below at rc^2 + eps^2,
// which is exactly the branch's gravity part (continuous at rc, so the FP32
// clamp needs no exact decision), and each lane keeps the smallest squared
// distance it met.  A wave in which some lane came within a bound that the
// FP32 rounding of the relative coordinates cannot cross runs a second pass
// over the same tile, for the candidates only: the contact decision
// dx*dx + dy*dy + dz*dz <= rc^2 and the spring and dashpot terms are taken
// in FP64 from the absolute positions and velocities, and summed in FP64
// apart from the gravity sums.  Particle tiles thus run the 13-instruction
// body plus a max and a min; node tiles run the plain loop.  These kernels
// use the sub-slice modes only (no tail or eighths mode, no id list, no
// fused kick: their LDS and registers are at the six-workgroup limit, and the
// dashpot reads other particles' velocities).
#include "bh_internal.hpp"

namespace {

constexpr int FT = 256;      // threads per workgroup (4 waves)
constexpr int TJ_MAX = 512;  // sources per LDS tile at most (two per thread); 256 is the other tile
constexpr int LC = FT;       // particle-list leaves per chunk (one per thread)
constexpr int PIDX = 2048;   // particle ids of a leaf chunk listed in LDS (FP32 gravity-only kernels)

template <typename R> struct V4;
template <> struct V4<float> { using T = float4; };
template <> struct V4<double> { using T = double4; };

template <typename R>
__device__ __forceinline__ typename V4<R>::T mk4(R a, R b, R c, R e);
template <>
__device__ __forceinline__ float4 mk4<float>(float a, float b, float c, float e) { return make_float4(a, b, c, e); }
template <>
__device__ __forceinline__ double4 mk4<double>(double a, double b, double c, double e) {
    return make_double4(a, b, c, e);
}

template <typename R>
__device__ __forceinline__ R rsqrt_r(R x);
template <>
__device__ __forceinline__ float rsqrt_r<float>(float x) { return __builtin_amdgcn_rsqf(x); }
// FP64: the hardware estimate (relative error below 2^-24 on gfx950, measured
// over 1e-20..1e20) refined by one Newton step for y = x^(-1/2),
// y <- y + (y/2)(1 - x y^2), which squares the error (below 5e-15 measured):
// far inside the FP64 bar, at a fraction of a division and a square root.
template <>
__device__ __forceinline__ double rsqrt_r<double>(double x) {
    const double y = __builtin_amdgcn_rsq(x);
    const double e = fma(-x * y, y, 1.0);
    return fma(0.5 * y, e, y);
}

template <typename R>
__device__ __forceinline__ R fma_r(R a, R b, R c);
template <>
__device__ __forceinline__ float fma_r<float>(float a, float b, float c) { return fmaf(a, b, c); }
template <>
__device__ __forceinline__ double fma_r<double>(double a, double b, double c) { return fma(a, b, c); }

// One pass of a wave over sources [j0, j1) of the LDS tile.  The bounds are
// the same for every lane of the wave; taking them through readfirstlane
// keeps the loop control on the scalar unit, so the vector unit issues only
// the pair arithmetic (every lane reads the same LDS entry: a broadcast).
// CLAMP (particle sources with the collision branch on): r^2 + eps^2 is
// raised to at least rce2 = rc^2 + eps^2 and its smallest value kept in cmin.
// EQM (particle sources of an equal-mass system): the common mass is taken
// out of the loop and applied to the sums at the end.
template <typename R, bool POT, bool ZERO_EPS, bool CLAMP, bool EQM>
__device__ __forceinline__ void interact(const typename V4<R>::T *tile, int j0, int j1, R xi, R yi, R zi, R eps2,
                                         R rce2, R &ax, R &ay, R &az, R &pot, R &cmin) {
    j0 = __builtin_amdgcn_readfirstlane(j0);
    j1 = __builtin_amdgcn_readfirstlane(j1);
#pragma unroll 8
    for (int j = j0; j < j1; ++j) {
        const typename V4<R>::T s = tile[j];
        const R dx = s.x - xi, dy = s.y - yi, dz = s.z - zi;
        R r2 = fma_r<R>(dx, dx, fma_r<R>(dy, dy, fma_r<R>(dz, dz, eps2)));
        if (CLAMP) {
            cmin = fmin(cmin, r2);
            r2 = fmax(r2, rce2);
        }
        R ri = rsqrt_r<R>(r2);
        if (ZERO_EPS && !CLAMP) ri = (r2 > (R)0) ? ri : (R)0;
        const R mri = EQM ? ri : s.w * ri;
        const R f = mri * (ri * ri);
        ax = fma_r<R>(f, dx, ax);
        ay = fma_r<R>(f, dy, ay);
        az = fma_r<R>(f, dz, az);
        if (POT) pot -= mri;
    }
}

// The same pass when the lanes of a wave work on different source ranges
// (sub-slices of a small group): lane base jb, common length L.
template <typename R, bool POT, bool ZERO_EPS, bool CLAMP, bool EQM>
__device__ __forceinline__ void interact_lanes(const typename V4<R>::T *tile, int jb, int L, R xi, R yi, R zi,
                                               R eps2, R rce2, R &ax, R &ay, R &az, R &pot, R &cmin) {
    L = __builtin_amdgcn_readfirstlane(L);
    const typename V4<R>::T *t = tile + jb;
#pragma unroll 8
    for (int k = 0; k < L; ++k) {
        const typename V4<R>::T s = t[k];
        const R dx = s.x - xi, dy = s.y - yi, dz = s.z - zi;
        R r2 = fma_r<R>(dx, dx, fma_r<R>(dy, dy, fma_r<R>(dz, dz, eps2)));
        if (CLAMP) {
            cmin = fmin(cmin, r2);
            r2 = fmax(r2, rce2);
        }
        R ri = rsqrt_r<R>(r2);
        if (ZERO_EPS && !CLAMP) ri = (r2 > (R)0) ? ri : (R)0;
        const R mri = EQM ? ri : s.w * ri;
        const R f = mri * (ri * ri);
        ax = fma_r<R>(f, dx, ax);
        ay = fma_r<R>(f, dy, ay);
        az = fma_r<R>(f, dz, az);
        if (POT) pot -= mri;
    }
}

// One lane's pass over tile entries [jl0, jl0 + L): the whole wave on one
// range (sub == 1) or each sub-slice on its own.
template <typename R, bool POT, bool ZERO_EPS, bool CLAMP, bool EQM>
__device__ __forceinline__ void tile_pass(const typename V4<R>::T *tile, int sub, int jl0, int L, R xi, R yi, R zi,
                                          R eps2, R rce2, R &ax, R &ay, R &az, R &pot, R &cmin) {
    if (sub == 1)
        interact<R, POT, ZERO_EPS, CLAMP, EQM>(tile, jl0, jl0 + L, xi, yi, zi, eps2, rce2, ax, ay, az, pot, cmin);
    else
        interact_lanes<R, POT, ZERO_EPS, CLAMP, EQM>(tile, jl0, L, xi, yi, zi, eps2, rce2, ax, ay, az, pot, cmin);
}

// Contact terms of Eq. (2) for the pair (i, j), both sorted indices, in
// FP64 from the absolute positions and velocities: the decision
// dx*dx + dy*dy + dz*dz <= rc^2, then spring, dashpot and the potential of the
// gravity part inside the contact sphere, added to the thread's FP64 sums
// c[0], c[FT], c[2 FT], c[3 FT] (x, y, z, potential) in LDS.  Values are
// loaded only as far as the decision needs them: contacts are rare.
template <bool POT>
__device__ __forceinline__ void contact_term(uint32_t i, uint32_t j, const DevState &d, double *c) {
    const double4 p = d.pos[i];
    const double4 q = d.pos[j];
    const double ex = q.x - p.x, ey = q.y - p.y, ez = q.z - p.z;
    const double d2 = ex * ex + ey * ey + ez * ez;
    const double rc2 = d.rc * d.rc;
    if (d2 == 0.0) {
        // i itself (or a coincident particle): no term at all; take back the
        // potential the pair loop added at the clamped distance
        if (POT) c[3 * FT] += d.G * q.w / sqrt(rc2 + d.eps2);
        return;
    }
    if (!(d2 <= rc2)) return;
    const double4 vi = d.vel[i];
    const double4 vj = d.vel[j];
    const double r = sqrt(d2);
    const double rv = ex * (vj.x - vi.x) + ey * (vj.y - vi.y) + ez * (vj.z - vi.z);
    const double fc = q.w / (p.w + q.w) * (d.kappa * (r - d.rc) / r + d.eta * rv / d2);
    c[0 * FT] += fc * ex;
    c[1 * FT] += fc * ey;
    c[2 * FT] += fc * ez;
    if (POT) {
        const double rce2 = rc2 + d.eps2;
        c[3 * FT] -= d.G * q.w * ((rc2 - d2) / (2.0 * rce2 * sqrt(rce2)));
    }
}

// The contact candidates of one lane's particle i among tile entries
// [jb, jb + L): entries whose FP32 squared distance (the pair loop's own
// expression) is within rcd2, a bound that rounding of the relative
// coordinates cannot cross.  jidx holds the sorted index of each entry.
template <typename R, bool POT>
__device__ __forceinline__ void contact_pass(const typename V4<R>::T *tile, const uint32_t *jidx, int jb, int L,
                                             R xi, R yi, R zi, R eps2, R rcd2, bool on, uint32_t i,
                                             const DevState &d, double *c) {
    if (!on) return;
    for (int k = 0; k < L; ++k) {
        const typename V4<R>::T s = tile[jb + k];
        const R dx = s.x - xi, dy = s.y - yi, dz = s.z - zi;
        const R r2 = fma_r<R>(dx, dx, fma_r<R>(dy, dy, fma_r<R>(dz, dz, eps2)));
        if (r2 <= rcd2) contact_term<POT>(i, jidx[jb + k], d, c);
    }
}

// FP32: registers capped so that 6 workgroups (24 waves) fit a CU; the
// pair loop needs the occupancy to hide LDS and rsqrt latency (measured:
// 100 VGPRs / 4 waves per SIMD ran 18% slower; the collision variant, at
// 5 workgroups without spills, ran 3% slower than at 6 with a few).  FP64
// gravity-only: 5 workgroups (<= 96 VGPRs, no spills); the FP64 collision
// variant keeps the default.
template <typename R, bool COLL>
struct ForceOcc {
    static constexpr int blocks = sizeof(R) == 4 ? 6 : (COLL ? 1 : 5);
};

template <typename R, bool POT, bool ZERO_EPS, bool COLL, int TJ>
// kick_h != 0: also apply the closing half kick v += kick_h a of a
// leapfrog step to each particle, as a separate pass over v and a would (the
// collision branch reads other particles' velocities, so it never fuses).
// TJ: sources per LDS tile (512, or 256 in the FP32 gravity-only kernels).
__global__ void __launch_bounds__(FT, (ForceOcc<R, COLL>::blocks)) k_force(DevState d, uint32_t ng, double kick_h) {
    static_assert(TJ == 256 || TJ == TJ_MAX, "tile of 256 or 512 sources");
    using T4 = typename V4<R>::T;
    __shared__ T4 tile[TJ + 16];
    __shared__ uint32_t lbeg[LC];
    __shared__ uint32_t lscan[LC + 1];
    __shared__ R red[4][4][64];
    __shared__ uint32_t s_item;
    __shared__ uint32_t wsum[4];
    __shared__ uint32_t jidx[COLL ? TJ : 1];            // sorted index of each particle-tile entry
    __shared__ double cacc[COLL ? 4 : 1][COLL ? FT : 1];  // per-thread FP64 contact sums
    // the particle ids of a leaf chunk, in list order, so that staging a
    // source is one LDS read instead of a search over the leaf offsets
    constexpr bool LIST_IDS = sizeof(R) == 4 && !COLL;
    __shared__ uint32_t pid[LIST_IDS ? PIDX : 1];

    const int tid = threadIdx.x;
    const int w = tid >> 6;
    const int lane = __lane_id();
    const R eps2 = (R)d.eps2;
    const R rce2 = (R)(d.rc * d.rc + d.eps2);
    // detection margin: a bound on how far FP32 (FP64) rounding of the
    // group-relative coordinates can move a squared distance
    constexpr double U = sizeof(R) == 4 ? 0x1p-20 : 0x1p-49;
    // tail mode (below) in the FP32 kernels without the collision branch
    constexpr bool TAIL = sizeof(R) == 4 && !COLL;

    for (;;) {
        if (tid == 0) s_item = atomicAdd(&d.cnt->work_counter2, 1u);
        __syncthreads();
        // the work item is the same for the whole workgroup: keep it (and all
        // per-group values derived from it) in scalar registers
        const uint32_t item = __builtin_amdgcn_readfirstlane(s_item);
        __syncthreads();
        if (item >= ng) break;
        const uint32_t g = __builtin_amdgcn_readfirstlane(d.order[item]);
        const GroupInfo gi = d.grp[g];
        const double4 cen = d.g_cen[g];
        // FP32: an equal-mass system's particles enter the pair loop with unit
        // mass, node masses in units of that mass, the sums scaled at the end
        const double m0 = sizeof(R) == 4 ? d.sys_m0[gi.sys] : 0.0;
        const bool eqm = m0 > 0.0;
        const double gscale = eqm ? d.G * m0 : d.G;
        const double inv_m0 = eqm ? 1.0 / m0 : 1.0;
        const unsigned long long pc0 = d.g_pc_off[g], pp0 = d.g_pp_off[g];
        const uint32_t npc = d.g_pc_len[g], npp = d.g_pp_len[g];

        for (uint32_t ib = 0; ib < gi.count; ib += FT) {
            const uint32_t nb = min((uint32_t)FT, gi.count - ib);
            // Waves take 64-particle chunks of the block (n_ic of them), the
            // waves left over splitting the source range (split ways).  A chunk
            // of at most 32 (16, 8) particles -- a small group, or the last chunk
            // of a larger one -- spreads its wave over 2 (4, 8) sub-slices of its
            // source range: cw lanes per particle, sub = 64 / cw parts.
            // split, sub and cw are powers of two: their divisions are shifts
            const int n_ic = (int)((nb + 63) >> 6);
            const int split_sh = n_ic == 1 ? 2 : (n_ic == 2 ? 1 : 0);
            const int split = 1 << split_sh;                         // 4 / n_ic
            const int ichunk = w % n_ic;
            const int jslice = w / n_ic;
            const bool wave_on = jslice < split;
            const int cnt_w = min(64, (int)nb - 64 * ichunk);
            // Slices of 8 particles in the chunk.  With 3, 5 or 7 of them the
            // chunk runs in eighths mode: lanes 0..8S-1 hold the particles and
            // take the first S eighths of the wave's source range; each of the
            // 8-S other groups of 8 lanes takes one of the last eighths for the
            // S slices in turn and hands each slice's partial sums to the lanes
            // that own them.  Every lane then runs S/8 of the range.
            const int s8 = (cnt_w + 7) >> 3;
            const bool e8 = TAIL && (s8 == 3 || s8 == 5 || s8 == 7);
            const int cw_sh = e8 ? 6 : (cnt_w <= 8 ? 3 : (cnt_w <= 16 ? 4 : (cnt_w <= 32 ? 5 : 6)));
            const int cw = 1 << cw_sh;
            const int sub_sh = 6 - cw_sh;
            const int sub = 1 << sub_sh;                             // 64 / cw
            const int part = lane >> cw_sh;
            // A chunk of 41 to 48 particles runs in tail mode: lanes 0..47 hold
            // the particles and take the first three quarters of the wave's
            // source range; lanes 48..63 take the last quarter for the three
            // 16-particle slices in turn and hand each slice's partial sums to
            // the lanes that own them.  Every lane then runs 3/4 of the range
            // instead of a full wave running all of it.
            const bool tailm = TAIL && cnt_w > 40 && cnt_w <= 48;
            const int last_cnt = (int)nb - 64 * (n_ic - 1);
            // the block's last chunk is sub-sliced, tailed or in eighths
            const bool any_sub = last_cnt <= (TAIL ? 56 : 32);
            const uint32_t il = 64 * ichunk + (lane & (cw - 1));
            const bool ion = wave_on && il < nb;
            const uint32_t i = gi.begin + ib + il;
            R xi = 0, yi = 0, zi = 0;
            if (ion) {
                const double4 p = d.pos[i];
                xi = (R)(p.x - cen.x);
                yi = (R)(p.y - cen.y);
                zi = (R)(p.z - cen.z);
            }
            R ax = 0, ay = 0, az = 0, pot = 0;
            R rcd2 = 0, cmin = 0;
            if (COLL) {
                const double n1 = fabs((double)xi) + fabs((double)yi) + fabs((double)zi);
                const double rcd = d.rc * (1.0 + U) + 0.5 * U * n1;
                rcd2 = (R)((rcd * rcd) * (1.0 + U) + d.eps2 * (1.0 + U));
#pragma unroll
                for (int a = 0; a < 4; ++a) cacc[a][tid] = 0.0;
            }

            // The staged tile holds cntt sources.  With a sub-sliced chunk in the
            // block the tile is padded with massless far sources to a multiple of
            // 8 split entries and cut at multiples of 8, so that every part has
            // the same length; full chunks still stop at the last real entry.
            // particles: whether the tile holds particle sources (the only ones
            // the collision branch applies to).
            auto compute_tile = [&](uint32_t cntt, bool particles) {
                const int ct = (int)cntt;
                const int cntp = any_sub ? ((ct + (8 << split_sh) - 1) >> (3 + split_sh)) << (3 + split_sh) : ct;
                for (int t = ct + tid; t < cntp; t += FT) tile[t] = mk4<R>((R)1e18, (R)1e18, (R)1e18, (R)0);
                __syncthreads();
                if (wave_on) {
                    int jb, je;
                    if (any_sub) {
                        const int q = cntp >> 3;
                        jb = 8 * ((q * jslice) >> split_sh);
                        je = 8 * ((q * (jslice + 1)) >> split_sh);
                    } else {
                        jb = (ct * jslice) >> split_sh;
                        je = (ct * (jslice + 1)) >> split_sh;
                    }
                    // this lane's part of the range: [jl0, jl0 + L)
                    int jl0, L;
                    if (sub == 1) {
                        jl0 = jb;
                        L = max(0, min(je, ct) - jb);
                    } else {
                        L = (je - jb) >> sub_sh;
                        jl0 = jb + part * L;
                    }
                    bool clamp = false;
                    if constexpr (COLL) clamp = particles;
                    const bool eq = particles && eqm;
                    if (clamp) {
                        cmin = (R)1e30;
                        if (eq)
                            tile_pass<R, POT, ZERO_EPS, true, true>(tile, sub, jl0, L, xi, yi, zi, eps2, rce2, ax, ay,
                                                                    az, pot, cmin);
                        else
                            tile_pass<R, POT, ZERO_EPS, true, false>(tile, sub, jl0, L, xi, yi, zi, eps2, rce2, ax,
                                                                     ay, az, pot, cmin);
                        if (__ballot(ion && cmin <= rcd2) != 0)
                            contact_pass<R, POT>(tile, jidx, jl0, L, xi, yi, zi, eps2, rcd2, ion, i, d,
                                                 &cacc[0][tid]);
                    } else if (e8) {
                        const int Q = (je - jb) >> 3;
                        const int lg = lane >> 3;
                        const bool tail_lane = lg >= s8;
#pragma unroll 1
                        for (int pq = 0; pq < s8; ++pq) {
                            const int src = 8 * pq + (lane & 7);
                            const R tx = __shfl(xi, src, 64), ty = __shfl(yi, src, 64), tz = __shfl(zi, src, 64);
                            if (tail_lane) {
                                xi = tx;
                                yi = ty;
                                zi = tz;
                                ax = ay = az = pot = (R)0;
                            }
                            // owners: eighth pq of their own slice; others: their own eighth
                            const int j0 = jb + (tail_lane ? lg : pq) * Q;
                            if (eq)
                                interact_lanes<R, POT, ZERO_EPS, false, true>(tile, j0, Q, xi, yi, zi, eps2, rce2,
                                                                              ax, ay, az, pot, cmin);
                            else
                                interact_lanes<R, POT, ZERO_EPS, false, false>(tile, j0, Q, xi, yi, zi, eps2, rce2,
                                                                               ax, ay, az, pot, cmin);
                            for (int t = s8; t < 8; ++t) {
                                const int tl = 8 * t + (lane & 7);
                                const R sx = __shfl(ax, tl, 64), sy = __shfl(ay, tl, 64), sz = __shfl(az, tl, 64),
                                        sp = __shfl(pot, tl, 64);
                                if (lg == pq) {
                                    ax += sx;
                                    ay += sy;
                                    az += sz;
                                    pot += sp;
                                }
                            }
                        }
                    } else if (tailm) {
                        const int Q = (je - jb) >> 2;
                        const bool tail_lane = lane >= 48;
#pragma unroll 1
                        for (int pq = 0; pq < 3; ++pq) {
                            const int src = 16 * pq + (lane & 15);
                            const R tx = __shfl(xi, src, 64), ty = __shfl(yi, src, 64), tz = __shfl(zi, src, 64);
                            if (tail_lane) {
                                xi = tx;
                                yi = ty;
                                zi = tz;
                                ax = ay = az = pot = (R)0;
                            }
                            const int j0 = tail_lane ? jb + 3 * Q : jb + pq * Q;
                            if (eq)
                                interact_lanes<R, POT, ZERO_EPS, false, true>(tile, j0, Q, xi, yi, zi, eps2, rce2,
                                                                              ax, ay, az, pot, cmin);
                            else
                                interact_lanes<R, POT, ZERO_EPS, false, false>(tile, j0, Q, xi, yi, zi, eps2, rce2,
                                                                               ax, ay, az, pot, cmin);
                            const int tl = 48 + (lane & 15);
                            const R sx = __shfl(ax, tl, 64), sy = __shfl(ay, tl, 64), sz = __shfl(az, tl, 64),
                                    sp = __shfl(pot, tl, 64);
                            if ((lane >> 4) == pq) {
                                ax += sx;
                                ay += sy;
                                az += sz;
                                pot += sp;
                            }
                        }
                    } else if (eq) {
                        tile_pass<R, POT, ZERO_EPS, false, true>(tile, sub, jl0, L, xi, yi, zi, eps2, rce2, ax, ay,
                                                                 az, pot, cmin);
                    } else {
                        tile_pass<R, POT, ZERO_EPS, false, false>(tile, sub, jl0, L, xi, yi, zi, eps2, rce2, ax, ay,
                                                                  az, pot, cmin);
                    }
                }
                __syncthreads();
            };

            // ---- node list: centre of mass and mass of each accepted node
            for (uint32_t t0 = 0; t0 < npc; t0 += TJ) {
                const uint32_t cntt = min((uint32_t)TJ, npc - t0);
                for (uint32_t e = tid; e < cntt; e += FT) {
                    const double4 m = d.nd_mom[d.pc_pool[pc0 + t0 + e]];
                    tile[e] = mk4<R>((R)(m.x - cen.x), (R)(m.y - cen.y), (R)(m.z - cen.z), (R)(m.w * inv_m0));
                }
                compute_tile(cntt, false);
            }

            // ---- particle list: the particles of each listed leaf
            for (uint32_t l0 = 0; l0 < npp; l0 += LC) {
                const uint32_t nl = min((uint32_t)LC, npp - l0);
                uint32_t lc = 0, lb = 0;
                if ((uint32_t)tid < nl) {
                    const uint32_t leaf = d.pp_pool[pp0 + l0 + tid];
                    lb = d.nd_begin[leaf];
                    lc = d.nd_count[leaf];
                }
                // exclusive scan of leaf sizes over the workgroup
                const uint32_t inc = wave_incl_scan(lc);
                if (lane == 63) wsum[w] = inc;
                __syncthreads();
                uint32_t off = 0, tot = 0;
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    off += (k < w) ? wsum[k] : 0u;
                    tot += wsum[k];
                }
                lbeg[tid] = lb;
                lscan[tid] = off + inc - lc;
                // a chunk of at most PIDX particles lists them all (each thread its
                // leaf's); a larger one (a few big level-21 leaves) searches
                const bool ids = LIST_IDS && tot <= (uint32_t)PIDX;
                if (ids)
                    for (uint32_t k = 0; k < lc; ++k) pid[off + inc - lc + k] = lb + k;
                __syncthreads();
                for (uint32_t p0 = 0; p0 < tot; p0 += TJ) {
                    const uint32_t cntt = min((uint32_t)TJ, tot - p0);
                    for (uint32_t e = tid; e < cntt; e += FT) {
                        const uint32_t f = p0 + e;
                        uint32_t j;
                        if (ids) {
                            j = pid[f];
                        } else {
                            uint32_t lo = 0, hi = nl - 1;          // last k with lscan[k] <= f
                            while (lo < hi) {
                                const uint32_t mid = (lo + hi + 1) >> 1;
                                if (lscan[mid] <= f) lo = mid; else hi = mid - 1;
                            }
                            j = lbeg[lo] + (f - lscan[lo]);
                        }
                        const double4 q = d.pos[j];
                        tile[e] = mk4<R>((R)(q.x - cen.x), (R)(q.y - cen.y), (R)(q.z - cen.z), (R)q.w);
                        if (COLL) jidx[e] = j;
                    }
                    compute_tile(cntt, true);
                }
            }

            // ---- add the j-slices in a fixed order and write FP64 results
            if (cw < 64) {
#pragma unroll
                for (int off = 32; off >= 8; off >>= 1) {
                    if (off < cw) break;
                    ax += __shfl_xor(ax, off, 64);
                    ay += __shfl_xor(ay, off, 64);
                    az += __shfl_xor(az, off, 64);
                    pot += __shfl_xor(pot, off, 64);
                }
            }
            red[0][w][lane] = ax;
            red[1][w][lane] = ay;
            red[2][w][lane] = az;
            red[3][w][lane] = pot;
            __syncthreads();
            if (ion && jslice == 0 && lane < cw) {
                R sx = 0, sy = 0, sz = 0, sp = 0;
                for (int k = 0; k < split; ++k) {
                    const int ww = k * n_ic + ichunk;
                    sx += red[0][ww][lane];
                    sy += red[1][ww][lane];
                    sz += red[2][ww][lane];
                    sp += red[3][ww][lane];
                }
                double gx = gscale * (double)sx, gy = gscale * (double)sy, gz = gscale * (double)sz;
                if (d.amag) d.amag[i] = sqrt(gx * gx + gy * gy + gz * gz);
                if (d.central_mass != 0.0) {
                    const double4 p = d.pos[i];
                    const double r2 = p.x * p.x + p.y * p.y + p.z * p.z;
                    const double r = sqrt(r2);
                    const double f = -d.G * d.central_mass / (r2 * r);
                    gx += f * p.x;
                    gy += f * p.y;
                    gz += f * p.z;
                }
                double gp = POT ? gscale * (double)sp : 0.0;
                if (COLL) {
                    // contact sums of the threads that worked on particle i, in a fixed order
                    double cx = 0, cy = 0, cz = 0, cp = 0;
                    for (int k = 0; k < split; ++k)
                        for (int sb = 0; sb < sub; ++sb) {
                            const int th = (k * n_ic + ichunk) * 64 + sb * cw + lane;
                            cx += cacc[0][th];
                            cy += cacc[1][th];
                            cz += cacc[2][th];
                            cp += cacc[3][th];
                        }
                    gx += cx;
                    gy += cy;
                    gz += cz;
                    gp += cp;
                }
                d.acc[i] = make_double4(gx, gy, gz, POT ? gp : 0.0);
                if (!COLL && kick_h != 0.0) {
                    double4 v = d.vel[i];
                    v.x = v.x + kick_h * gx;
                    v.y = v.y + kick_h * gy;
                    v.z = v.z + kick_h * gz;
                    d.vel[i] = v;
                }
            }
            __syncthreads();
        }
    }
}

__global__ void k_force_reset(DevState d) {
    if (threadIdx.x == 0 && blockIdx.x == 0) d.cnt->work_counter2 = 0;
}

template <typename R, bool POT, bool ZERO_EPS>
void launch_gravity(const DevState &d, uint32_t ng, int blocks, double kick_h, hipStream_t s) {
    if constexpr (sizeof(R) == 4) {
        if (d.force_tile == 256) {
            k_force<R, POT, ZERO_EPS, false, 256><<<blocks, FT, 0, s>>>(d, ng, kick_h);
            return;
        }
    }
    k_force<R, POT, ZERO_EPS, false, TJ_MAX><<<blocks, FT, 0, s>>>(d, ng, kick_h);
}

template <typename R, bool POT>
void launch(const DevState &d, uint32_t ng, int blocks, double kick_h, hipStream_t s) {
    if (d.rc > 0.0) {
        if (d.eps2 == 0.0)
            k_force<R, POT, true, true, TJ_MAX><<<blocks, FT, 0, s>>>(d, ng, 0.0);
        else
            k_force<R, POT, false, true, TJ_MAX><<<blocks, FT, 0, s>>>(d, ng, 0.0);
    } else if (d.eps2 == 0.0) {
        launch_gravity<R, POT, true>(d, ng, blocks, kick_h, s);
    } else {
        launch_gravity<R, POT, false>(d, ng, blocks, kick_h, s);
    }
}

}  // namespace

namespace bhk {

void forces(const DevState &d, uint32_t n_groups, bool fp32, bool pot, int blocks, double kick_h, hipStream_t s) {
    k_force_reset<<<1, 64, 0, s>>>(d);
    if (n_groups == 0) return;
    if (fp32) {
        if (pot) launch<float, true>(d, n_groups, blocks, kick_h, s);
        else launch<float, false>(d, n_groups, blocks, kick_h, s);
    } else {
        if (pot) launch<double, true>(d, n_groups, blocks, kick_h, s);
        else launch<double, false>(d, n_groups, blocks, kick_h, s);
    }
}

}  // namespace bhk
