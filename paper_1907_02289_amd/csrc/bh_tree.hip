// bh_tree.hip -- tree construction, Iwasawa et al. (2019) Sec. 4.2 step (3a):
// root box and keys, sort and permutation, level-synchronous octree,
// monopole moments (Sec. 5.1: nodes act through their centre of mass),
// and the particle groups of step (3d) taken from the tree itself.
//
// Readings where the paper is silent:
//   root cube: lower corner at the per-axis minimum, side S the smallest
//     power of two strictly above the largest extent; grid coordinate
//     q = floor((x - lo) * 2^21 / S), at most 2^21 - 1; key = the 21 bits of
//     each axis interleaved, x the most significant bit of each triple.
//   tree: a node with more than n_leaf particles below level 21 is split
//     into its non-empty octants; nodes are numbered level by level.
//   groups: the first node on the way down from the root with at most
//     n_grp particles, or a leaf; ordered by first particle.
//
// Cylindrical tree coordinates (Sec. 4.3, Eq. (1)), when cyl_r > 0: for a
// narrow ring near radius cyl_r, cyl_r phi, r and z are locally Cartesian,
// so keys, cells and groups are built on (phi, r, z) while moments and
// forces stay Cartesian.  The root cell has side S = 2 pi cyl_r; its phi
// axis spans one turn, q = floor((phi + pi) 2^21 / (2 pi)); r and z use
// q = floor((v - min v) 2^21 / S).  phi comes from angle_of below, made of
// correctly rounded operations only, so the keys do not depend on a math
// library.
#include "bh_internal.hpp"

namespace {

constexpr int TPB = 256;

__device__ __forceinline__ int sys_of(const uint32_t *sys_off, int n_sys, uint32_t i) {
    int lo = 0, hi = n_sys - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (sys_off[mid] <= i) lo = mid; else hi = mid - 1;
    }
    return lo;
}

inline unsigned grid_for(size_t n, size_t cap_blocks = 8192) {
    size_t b = (n + TPB - 1) / TPB;
    if (b < 1) b = 1;
    if (b > cap_blocks) b = cap_blocks;
    return (unsigned)b;
}

// ---------------------------------------------------------------- cylindrical coordinates
constexpr double CYL_PI = 3.141592653589793;
constexpr double CYL_TAN_PI8 = 0.41421356237309503;   // tan(pi/8)

// arctan t for |t| <= tan(pi/8): the Maclaurin series t - t^3/3 + t^5/5 - ...
// (Abramowitz & Stegun 4.4.42) through t^29 (truncation below 2e-14),
// Horner's rule in t^2 from the top term down, coefficients (-1)^k / (2k+1).
__device__ __forceinline__ double atan_small(double t) {
    const double t2 = t * t;
    double p = 0.0;
#pragma unroll
    for (int k = 14; k >= 0; --k) {
        double c = 1.0 / (double)(2 * k + 1);
        if (k & 1) c = -c;
        p = p * t2 + c;
    }
    return t * p;
}

// Angle of (x, y) in [-pi, pi]: t = min/max(|x|, |y|) in [0, 1], reduced
// above tan(pi/8) by arctan t = pi/4 + arctan((t - 1)/(t + 1)) (A&S 4.4.34),
// then reflected into the octant and quadrant of (x, y); (0, 0) gives 0.
__device__ __forceinline__ double angle_of(double y, double x) {
    const double ax = fabs(x), ay = fabs(y);
    if (ax == 0.0 && ay == 0.0) return 0.0;
    const bool swap = ay > ax;
    const double t = swap ? ax / ay : ay / ax;
    double a = (t > CYL_TAN_PI8) ? 0.25 * CYL_PI + atan_small((t - 1.0) / (t + 1.0)) : atan_small(t);
    if (swap) a = 0.5 * CYL_PI - a;
    if (x < 0.0) a = CYL_PI - a;
    if (y < 0.0) a = -a;
    return a;
}

// The coordinates the tree is built on.
__device__ __forceinline__ void tree_coords(const DevState &d, double4 p, double c[3]) {
    if (d.cyl_r > 0.0) {
        c[0] = angle_of(p.y, p.x);
        c[1] = sqrt(p.x * p.x + p.y * p.y);
        c[2] = p.z;
    } else {
        c[0] = p.x;
        c[1] = p.y;
        c[2] = p.z;
    }
}

// ---------------------------------------------------------------- load
__global__ void k_load(DevState d) {
    uint32_t stride = gridDim.x * blockDim.x;
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < d.n; i += stride) {
        int s = sys_of(d.sys_off, d.n_sys, i);
        uint32_t j = i - d.sys_off[s];
        SysPtr p = d.sys_tab[s];
        d.pos_in[i] = make_double4(p.x[j], p.y[j], p.z[j], p.m[j]);
        d.vel_in[i] = p.vx ? make_double4(p.vx[j], p.vy[j], p.vz[j], 0.0) : make_double4(0.0, 0.0, 0.0, 0.0);
        d.idx_in[i] = i;
        if (d.amag_in) d.amag_in[i] = INFINITY;      // unknown until a force evaluation
    }
}

// ---------------------------------------------------------------- root box
__global__ void __launch_bounds__(TPB) k_box_partial(DevState d) {
    const int s = blockIdx.y;
    const uint32_t b0 = d.sys_off[s], b1 = d.sys_off[s + 1];
    // per axis 0..2 the tree coordinates, axis 3 the mass
    double lo[4] = {INFINITY, INFINITY, INFINITY, INFINITY}, hi[4] = {-INFINITY, -INFINITY, -INFINITY, -INFINITY};
    bool bad = false;
    for (uint32_t i = b0 + blockIdx.x * TPB + threadIdx.x; i < b1; i += d.box_blocks * TPB) {
        const double4 p = d.pos_in[i];
        bad |= !isfinite(p.x) || !isfinite(p.y) || !isfinite(p.z);
        double c[4];
        tree_coords(d, p, c);
        c[3] = p.w;
#pragma unroll
        for (int a = 0; a < 4; ++a) {
            lo[a] = fmin(lo[a], c[a]);
            hi[a] = fmax(hi[a], c[a]);
        }
    }
    if (bad) atomicOr(&d.cnt->flags[FLAG_NONFINITE], 1u);
    __shared__ double red[TPB / 64][8];
#pragma unroll
    for (int a = 0; a < 4; ++a) {
        lo[a] = wave_min(lo[a]);
        hi[a] = wave_max(hi[a]);
    }
    const int w = threadIdx.x >> 6;
    if (__lane_id() == 0) {
        for (int a = 0; a < 4; ++a) {
            red[w][a] = lo[a];
            red[w][4 + a] = hi[a];
        }
    }
    __syncthreads();
    if (threadIdx.x < 8) {
        int a = threadIdx.x;
        double v = red[0][a];
        for (int k = 1; k < TPB / 64; ++k) v = (a < 4) ? fmin(v, red[k][a]) : fmax(v, red[k][a]);
        d.box_part[((size_t)s * d.box_blocks + blockIdx.x) * 8 + a] = v;
    }
}

__global__ void k_box_final(DevState d) {
    // one wave per system: lanes stride over the partials, then a wave reduction
    const int s = blockIdx.x;
    double lo[4], hi[4];
    for (int a = 0; a < 4; ++a) {
        lo[a] = INFINITY;
        hi[a] = -INFINITY;
    }
    for (uint32_t b = threadIdx.x; b < d.box_blocks; b += 64) {
        const double *p = d.box_part + ((size_t)s * d.box_blocks + b) * 8;
        for (int a = 0; a < 4; ++a) {
            lo[a] = fmin(lo[a], p[a]);
            hi[a] = fmax(hi[a], p[4 + a]);
        }
    }
    for (int a = 0; a < 4; ++a) {
        lo[a] = wave_min(lo[a]);
        hi[a] = wave_max(hi[a]);
    }
    if (threadIdx.x != 0) return;
    // equal-mass systems let the force kernel take the common mass out of the pair loop
    d.sys_m0[s] = (lo[3] == hi[3] && lo[3] > 0.0) ? lo[3] : 0.0;
    if (d.cyl_r > 0.0) {
        // one turn of phi; r and z must fit the cell of side 2 pi cyl_r
        const double S = (2.0 * CYL_PI) * d.cyl_r;
        if (hi[1] - lo[1] >= S || hi[2] - lo[2] >= S) atomicOr(&d.cnt->flags[FLAG_EXTENT], 1u);
        d.box[s] = make_double4(-CYL_PI, lo[1], lo[2], 2097152.0 / S);
        return;
    }
    double w = 0.0;
    for (int a = 0; a < 3; ++a) {
        double e = hi[a] - lo[a];
        if (e > w) w = e;
    }
    int e2 = 0;
    if (w > 0.0) frexp(w, &e2);            // w < 2^e2 <= 2 w: S = 2^e2
    d.box[s] = make_double4(lo[0], lo[1], lo[2], ldexp(1.0, BH_MAXLEVEL - e2));
}

// ---------------------------------------------------------------- keys
__global__ void k_keys(DevState d) {
    uint32_t stride = gridDim.x * blockDim.x;
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < d.n; i += stride) {
        int s = sys_of(d.sys_off, d.n_sys, i);
        double4 b = d.box[s];
        double4 p = d.pos_in[i];
        double c[3], l[3] = {b.x, b.y, b.z};
        tree_coords(d, p, c);
        // the phi axis of cylindrical coordinates spans one turn
        const double k0 = d.cyl_r > 0.0 ? 2097152.0 / (2.0 * CYL_PI) : b.w;
        uint32_t q[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            double t = (c[a] - l[a]) * (a == 0 ? k0 : b.w);
            double f = floor(t);
            q[a] = (f >= 2097151.0) ? 2097151u : (uint32_t)f;
        }
        d.key[i] = (spread3(q[0]) << 2) | (spread3(q[1]) << 1) | spread3(q[2]);
        d.val[i] = i;
    }
}

__global__ void k_reset_flags(DevState d) {
    if (threadIdx.x < FLAG_COUNT) d.cnt->flags[threadIdx.x] = 0;
}

// ---------------------------------------------------------------- permute
__global__ void k_permute(DevState d) {
    uint32_t stride = gridDim.x * blockDim.x;
    for (uint32_t j = blockIdx.x * blockDim.x + threadIdx.x; j < d.n; j += stride) {
        uint32_t src = d.val[j];
        d.pos[j] = d.pos_in[src];
        d.vel[j] = d.vel_in[src];
        const uint32_t gi = d.idx_in[src];
        d.idx[j] = gi;
        d.inv[gi] = j;
        if (d.amag && d.amag_in) d.amag[j] = d.amag_in[src];
    }
}

// ---------------------------------------------------------------- octree
__global__ void k_tree_init(DevState d) {
    uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s == 0) {
        d.cnt->flags[FLAG_NODE_OVF] = 0;
        d.cnt->lvl_off[0] = 0;
        for (int l = 1; l < BH_NLEVELS + 2; ++l) d.cnt->lvl_off[l] = (uint32_t)d.n_sys;
        d.cnt->max_level = 0;
        d.cnt->n_groups = 0;
    }
    if (s < (uint32_t)d.n_sys) {
        uint32_t b = d.sys_off[s], c = d.sys_off[s + 1] - b;
        bool leaf = !(c > (uint32_t)d.n_leaf);
        bool grp = (c <= (uint32_t)d.n_grp) || leaf;
        d.nd_prefix[s] = 0;
        d.nd_begin[s] = b;
        d.nd_count[s] = c;
        d.nd_first[s] = 0;
        d.nd_meta[s] = make_meta(0, 0, grp ? 1u : 0u, s);
    }
}

// octant boundaries of node v (at level l): bnd[o] = first particle with octant >= o
__device__ __forceinline__ void octant_bounds(const uint64_t *key, uint32_t b, uint32_t e, int shift,
                                              uint32_t bnd[9]) {
    bnd[0] = b;
    bnd[8] = e;
#pragma unroll
    for (uint32_t o = 1; o < 8; ++o) {
        uint32_t lo = bnd[o - 1], hi = e;     // first i in [lo, e) with octant(i) >= o
        while (lo < hi) {
            uint32_t mid = (lo + hi) >> 1;
            if (((uint32_t)(key[mid] >> shift) & 7u) < o) lo = mid + 1; else hi = mid;
        }
        bnd[o] = lo;
    }
}

__global__ void k_tree_count(DevState d, int l) {
    const uint32_t v0 = d.cnt->lvl_off[l], v1 = d.cnt->lvl_off[l + 1];
    if (blockIdx.x == 0 && threadIdx.x == 0) d.cnt->pad[0] = v1 - v0;   // level size for the scan
    const int shift = 3 * (BH_MAXLEVEL - 1 - l);
    uint32_t stride = gridDim.x * blockDim.x;
    for (uint32_t v = v0 + blockIdx.x * blockDim.x + threadIdx.x; v < v1; v += stride) {
        uint32_t c = d.nd_count[v], nch = 0;
        if (c > (uint32_t)d.n_leaf && l < BH_MAXLEVEL) {
            uint32_t bnd[9];
            octant_bounds(d.key, d.nd_begin[v], d.nd_begin[v] + c, shift, bnd);
#pragma unroll
            for (int o = 0; o < 8; ++o) nch += (bnd[o + 1] > bnd[o]) ? 1u : 0u;
        }
        d.tmp_a[v - v0] = nch;
        d.tmp_b[v - v0] = nch;
    }
}

__global__ void k_tree_emit(DevState d, int l) {
    const uint32_t v0 = d.cnt->lvl_off[l], v1 = d.cnt->lvl_off[l + 1];
    const uint32_t total = d.cnt->pad[1];
    const uint32_t base = v1;                       // first id of level l+1
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        uint64_t end = (uint64_t)base + total;
        if (end > d.node_cap) {
            atomicOr(&d.cnt->flags[FLAG_NODE_OVF], 1u);
            end = d.node_cap;
        }
        for (int k = l + 2; k < BH_NLEVELS + 2; ++k) d.cnt->lvl_off[k] = (uint32_t)end;
        if (total > 0) d.cnt->max_level = l + 1;
    }
    const int shift = 3 * (BH_MAXLEVEL - 1 - l);
    uint32_t stride = gridDim.x * blockDim.x;
    for (uint32_t v = v0 + blockIdx.x * blockDim.x + threadIdx.x; v < v1; v += stride) {
        uint32_t nch = d.tmp_b[v - v0];
        uint32_t meta = d.nd_meta[v];
        if (nch == 0) {
            d.nd_first[v] = 0;
            continue;
        }
        uint32_t first = base + d.tmp_a[v - v0];
        d.nd_first[v] = first;
        d.nd_meta[v] = make_meta(meta_level(meta), nch, meta_group(meta), meta_sys(meta));
        uint32_t c = d.nd_count[v];
        uint32_t bnd[9];
        octant_bounds(d.key, d.nd_begin[v], d.nd_begin[v] + c, shift, bnd);
        uint64_t pfx = d.nd_prefix[v];
        bool parent_big = c > (uint32_t)d.n_grp;
        uint32_t k = 0;
        for (uint32_t o = 0; o < 8; ++o) {
            uint32_t cb = bnd[o], cc = bnd[o + 1] - bnd[o];
            if (cc == 0) continue;
            uint32_t u = first + k++;
            if (u >= d.node_cap) break;     // overflow, flagged above: ids below the cap stay valid
            bool leaf = !(cc > (uint32_t)d.n_leaf && l + 1 < BH_MAXLEVEL);
            bool grp = parent_big && (cc <= (uint32_t)d.n_grp || leaf);
            d.nd_prefix[u] = (pfx << 3) | o;
            d.nd_begin[u] = cb;
            d.nd_count[u] = cc;
            d.nd_first[u] = 0;
            d.nd_meta[u] = make_meta(l + 1, 0, grp ? 1u : 0u, meta_sys(meta));
        }
    }
}

__global__ void k_node_finalize(DevState d) {
    const uint32_t nn = d.cnt->lvl_off[BH_NLEVELS];
    uint32_t stride = gridDim.x * blockDim.x;
    for (uint32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < nn; v += stride) {
        uint32_t meta = d.nd_meta[v];
        uint32_t l = meta_level(meta);
        uint64_t p = d.nd_prefix[v];
        int sh = BH_MAXLEVEL - (int)l;
        uint32_t cx = compact3(p >> 2) << sh, cy = compact3(p >> 1) << sh, cz = compact3(p) << sh;
        d.nd_walk[v] = make_int4((int)(cx | (l << 24)), (int)(cy | (meta_nch(meta) << 24)), (int)cz,
                                 (int)d.nd_first[v]);
    }
}

// ---------------------------------------------------------------- moments
// Bottom-up, one launch per level: a leaf sums its particles, an internal
// node its children (mass and mass-weighted centre).
__global__ void k_moments_level(DevState d, int l) {
    const uint32_t v0 = d.cnt->lvl_off[l], v1 = d.cnt->lvl_off[l + 1];
    uint32_t stride = gridDim.x * blockDim.x;
    for (uint32_t v = v0 + blockIdx.x * blockDim.x + threadIdx.x; v < v1; v += stride) {
        uint32_t nch = meta_nch(d.nd_meta[v]);
        double M = 0, sx = 0, sy = 0, sz = 0;
        if (nch == 0) {
            uint32_t b = d.nd_begin[v], e = b + d.nd_count[v];
            for (uint32_t i = b; i < e; ++i) {
                double4 p = d.pos[i];
                M += p.w;
                sx += p.w * p.x;
                sy += p.w * p.y;
                sz += p.w * p.z;
            }
        } else {
            uint32_t f = d.nd_first[v];
            for (uint32_t c = 0; c < nch; ++c) {
                double4 q = d.nd_mom[f + c];
                M += q.w;
                sx += q.w * q.x;
                sy += q.w * q.y;
                sz += q.w * q.z;
            }
        }
        double4 r = make_double4(sx / M, sy / M, sz / M, M);
        d.nd_mom[v] = r;
        if (d.nd_drift) {
            // Drift since the build: the largest distance by which a particle of
            // the node has moved relative to the node's centre of mass,
            //   leaf:     max_i |(x_i - x_i^b) - (c - c^b)|,
            //   internal: max_k (drift_k + |(c_k - c_k^b) - (c - c^b)|),
            // an upper bound of the leaf form over the node's particles.
            const double4 rb = d.nd_mom_b[v];
            const double ux = r.x - rb.x, uy = r.y - rb.y, uz = r.z - rb.z;
            double dr = 0.0;
            if (nch == 0) {
                uint32_t b = d.nd_begin[v], e = b + d.nd_count[v];
                for (uint32_t i = b; i < e; ++i) {
                    const double4 p = d.pos[i], q = d.pos_b[i];
                    const double ex = (p.x - q.x) - ux, ey = (p.y - q.y) - uy, ez = (p.z - q.z) - uz;
                    dr = fmax(dr, sqrt(ex * ex + ey * ey + ez * ez));
                }
            } else {
                uint32_t f = d.nd_first[v];
                for (uint32_t c = 0; c < nch; ++c) {
                    const double4 q = d.nd_mom[f + c], qb = d.nd_mom_b[f + c];
                    const double ex = (q.x - qb.x) - ux, ey = (q.y - qb.y) - uy, ez = (q.z - qb.z) - uz;
                    dr = fmax(dr, d.nd_drift[f + c] + sqrt(ex * ex + ey * ey + ez * ez));
                }
            }
            d.nd_drift[v] = dr;
            const uint32_t meta = d.nd_meta[v];
            const double side = ldexp((double)(1u << BH_MAXLEVEL) / d.box[meta_sys(meta)].w, -l);
            if (dr > d.drift_kappa * side) atomicAdd(&d.cnt->stale[l], d.nd_count[v]);
        }
        if (d.nd_quad) {
            double Q[6] = {0, 0, 0, 0, 0, 0};
            if (nch == 0) {
                uint32_t b = d.nd_begin[v], e = b + d.nd_count[v];
                for (uint32_t i = b; i < e; ++i) {
                    double4 p = d.pos[i];
                    double dx = p.x - r.x, dy = p.y - r.y, dz = p.z - r.z;
                    Q[0] += p.w * dx * dx; Q[1] += p.w * dx * dy; Q[2] += p.w * dx * dz;
                    Q[3] += p.w * dy * dy; Q[4] += p.w * dy * dz; Q[5] += p.w * dz * dz;
                }
            } else {
                uint32_t f = d.nd_first[v];
                for (uint32_t c = 0; c < nch; ++c) {
                    double4 q = d.nd_mom[f + c];
                    const double *qc = d.nd_quad + (size_t)(f + c) * 6;
                    double dx = q.x - r.x, dy = q.y - r.y, dz = q.z - r.z;
                    Q[0] += qc[0] + q.w * dx * dx; Q[1] += qc[1] + q.w * dx * dy;
                    Q[2] += qc[2] + q.w * dx * dz; Q[3] += qc[3] + q.w * dy * dy;
                    Q[4] += qc[4] + q.w * dy * dz; Q[5] += qc[5] + q.w * dz * dz;
                }
            }
            double *o = d.nd_quad + (size_t)v * 6;
            for (int k = 0; k < 6; ++k) o[k] = Q[k];
        }
    }
}

// ---------------------------------------------------------------- groups
// Group flags for the current n_grp on an existing tree: a root is a group
// when small enough or a leaf; a child is a group when its parent is larger
// than n_grp and the child is small enough or a leaf (each node has exactly
// one parent, so the writes do not collide).  With packing, the flag marks
// the first node of each pack: the parent's thread walks its children in
// order and starts a new pack where the next small child no longer fits
// (the pack's particle count is taken later from the next group's start).
__global__ void k_regroup(DevState d) {
    const uint32_t nn = d.cnt->lvl_off[BH_NLEVELS];
    const uint32_t G = (uint32_t)d.n_grp;
    uint32_t stride = gridDim.x * blockDim.x;
    for (uint32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < nn; v += stride) {
        const uint32_t meta = d.nd_meta[v], nch = meta_nch(meta), c = d.nd_count[v];
        if (v < (uint32_t)d.n_sys) {
            const bool grp = c <= G || nch == 0;
            d.nd_meta[v] = make_meta(meta_level(meta), nch, grp ? 1u : 0u, meta_sys(meta));
        }
        const uint32_t f = d.nd_first[v];
        uint32_t run = 0;    // particles in the open pack, 0 when none is open
        for (uint32_t k = 0; k < nch; ++k) {
            const uint32_t u = f + k;
            const uint32_t mu = d.nd_meta[u], cu = d.nd_count[u];
            bool grp = c > G && (cu <= G || meta_nch(mu) == 0);
            if (d.pack_groups && grp && cu <= G) {
                if (run > 0 && run + cu <= G) {
                    grp = false;             // joins the open pack
                    run += cu;
                } else {
                    run = cu;                // opens a pack
                }
            } else {
                run = 0;                     // a split child or an over-full leaf ends the run
            }
            d.nd_meta[u] = make_meta(meta_level(mu), meta_nch(mu), grp ? 1u : 0u, meta_sys(mu));
        }
    }
}

__global__ void k_group_mark(DevState d) {
    const uint32_t nn = d.cnt->lvl_off[BH_NLEVELS];
    uint32_t stride = gridDim.x * blockDim.x;
    for (uint32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < nn; v += stride)
        if (meta_group(d.nd_meta[v])) d.gmark[d.nd_begin[v]] = 1u;
}

__global__ void k_group_emit(DevState d) {
    const uint32_t nn = d.cnt->lvl_off[BH_NLEVELS];
    uint32_t stride = gridDim.x * blockDim.x;
    for (uint32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < nn; v += stride) {
        uint32_t meta = d.nd_meta[v];
        if (!meta_group(meta)) continue;
        uint32_t b = d.nd_begin[v];
        uint32_t g = d.gmark[b];
        d.grp[g] = GroupInfo{v, b, d.nd_count[v], meta_sys(meta)};
    }
}

// Packed groups: the groups partition the sorted particles in order, so a
// group ends where the next one starts.
__global__ void k_group_count(DevState d) {
    const uint32_t ng = d.cnt->n_groups;
    uint32_t stride = gridDim.x * blockDim.x;
    for (uint32_t g = blockIdx.x * blockDim.x + threadIdx.x; g < ng; g += stride) {
        const uint32_t end = g + 1 < ng ? d.grp[g + 1].begin : (uint32_t)d.n;
        d.grp[g].count = end - d.grp[g].begin;
    }
}

// One wave per group: integer grid box from the keys, centre = midpoint of
// the FP64 bounding box of the group's particles.
__global__ void __launch_bounds__(TPB) k_group_box(DevState d) {
    const uint32_t ng = d.cnt->n_groups;
    const uint32_t wpb = TPB / 64;
    for (uint32_t g = blockIdx.x * wpb + (threadIdx.x >> 6); g < ng; g += gridDim.x * wpb) {
        GroupInfo gi = d.grp[g];
        uint32_t qlo[3] = {0xffffffffu, 0xffffffffu, 0xffffffffu}, qhi[3] = {0, 0, 0};
        double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
        for (uint32_t i = gi.begin + __lane_id(); i < gi.begin + gi.count; i += 64) {
            uint64_t k = d.key[i];
            uint32_t q[3] = {compact3(k >> 2), compact3(k >> 1), compact3(k)};
            double4 p = d.pos[i];
            double c[3] = {p.x, p.y, p.z};
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                qlo[a] = min(qlo[a], q[a]);
                qhi[a] = max(qhi[a], q[a]);
                lo[a] = fmin(lo[a], c[a]);
                hi[a] = fmax(hi[a], c[a]);
            }
        }
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            qlo[a] = wave_min(qlo[a]);
            qhi[a] = wave_max(qhi[a]);
            lo[a] = wave_min(lo[a]);
            hi[a] = wave_max(hi[a]);
        }
        if (__lane_id() == 0) {
            d.g_lo[g] = make_int4((int)qlo[0], (int)qlo[1], (int)qlo[2], 0);
            d.g_hi[g] = make_int4((int)qhi[0] + 1, (int)qhi[1] + 1, (int)qhi[2] + 1, 0);
            d.g_cen[g] = make_double4(0.5 * (lo[0] + hi[0]), 0.5 * (lo[1] + hi[1]), 0.5 * (lo[2] + hi[2]), 0.0);
            if (d.g_rad) {
                const double ex = hi[0] - lo[0], ey = hi[1] - lo[1], ez = hi[2] - lo[2];
                d.g_rad[g] = 0.5 * sqrt(ex * ex + ey * ey + ez * ez);
            }
        }
        if (d.g_amin) d.g_amin[g] = group_budget(d, gi);
    }
}

}  // namespace

namespace bhk {

void load_systems(const DevState &d, hipStream_t s) {
    k_load<<<grid_for(d.n), TPB, 0, s>>>(d);
}

void root_box_keys(const DevState &d, hipStream_t s) {
    k_box_partial<<<dim3(d.box_blocks, d.n_sys), TPB, 0, s>>>(d);
    k_box_final<<<d.n_sys, 64, 0, s>>>(d);
    k_keys<<<grid_for(d.n), TPB, 0, s>>>(d);
    radix_sort(d.key, d.val, d.key_tmp, d.val_tmp, d.n, 0, 63, d.hist, d.scan_tmp, s, d.sys_off, d.n_sys);
}

void reset_flags(const DevState &d, hipStream_t s) {
    k_reset_flags<<<1, 64, 0, s>>>(d);
}

void permute(const DevState &d, hipStream_t s) {
    k_permute<<<grid_for(d.n), TPB, 0, s>>>(d);
}

void build_octree(const DevState &d, hipStream_t s) {
    k_tree_init<<<(d.n_sys + TPB - 1) / TPB, TPB, 0, s>>>(d);
    const unsigned g = grid_for(d.node_cap, 4096);
    for (int l = 0; l < BH_MAXLEVEL; ++l) {
        k_tree_count<<<g, TPB, 0, s>>>(d, l);
        scan_u32(d.tmp_a, d.tmp_a, &d.cnt->pad[0], 0, &d.cnt->pad[1], d.scan_tmp, s);
        k_tree_emit<<<g, TPB, 0, s>>>(d, l);
    }
    k_node_finalize<<<g, TPB, 0, s>>>(d);
}

void moments(const DevState &d, hipStream_t s) {
    const unsigned g = grid_for(d.node_cap, 4096);
    for (int l = BH_MAXLEVEL; l >= 0; --l) k_moments_level<<<g, TPB, 0, s>>>(d, l);
}

__global__ void k_drift_snapshot(DevState d) {
    const uint32_t nn = d.cnt->lvl_off[BH_NLEVELS];
    const uint32_t stride = gridDim.x * blockDim.x;
    const uint32_t t0 = blockIdx.x * blockDim.x + threadIdx.x;
    for (uint32_t i = t0; i < d.n; i += stride) d.pos_b[i] = d.pos[i];
    for (uint32_t v = t0; v < nn; v += stride) d.nd_mom_b[v] = d.nd_mom[v];
    if (t0 < BH_NLEVELS) d.cnt->stale[t0] = 0;
}

__global__ void k_drift_clear(DevState d) {
    if (threadIdx.x < BH_NLEVELS) d.cnt->stale[threadIdx.x] = 0;
}

void drift_snapshot(const DevState &d, hipStream_t s) {
    k_drift_snapshot<<<grid_for(d.n, 4096), TPB, 0, s>>>(d);
}

void drift_clear(const DevState &d, hipStream_t s) {
    k_drift_clear<<<1, 64, 0, s>>>(d);
}

void regroup(const DevState &d, hipStream_t s) {
    k_regroup<<<grid_for(d.node_cap, 4096), TPB, 0, s>>>(d);
}

void make_groups(const DevState &d, hipStream_t s) {
    const unsigned g = grid_for(d.node_cap, 4096);
    if (d.pack_groups) k_regroup<<<g, TPB, 0, s>>>(d);
    fill_u32(d.gmark, 0u, d.n, s);
    k_group_mark<<<g, TPB, 0, s>>>(d);
    scan_u32(d.gmark, d.gmark, nullptr, d.n, &d.cnt->n_groups, d.scan_tmp, s);
    k_group_emit<<<g, TPB, 0, s>>>(d);
    if (d.pack_groups) k_group_count<<<grid_for(d.n, 4096), TPB, 0, s>>>(d);
    k_group_box<<<grid_for((size_t)d.n * 64 / 8, 8192), TPB, 0, s>>>(d);
}

}  // namespace bhk
