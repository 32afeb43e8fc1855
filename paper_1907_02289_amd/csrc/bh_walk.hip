// bh_walk.hip -- interaction lists, Iwasawa et al. (2019) Sec. 4.2 step (3d):
// the tree is traversed once per group of neighbouring particles (the group
// variant of the walk), producing the list of tree nodes and the list of
// particles (as leaves) that act on the group; the lists are kept and reused
// over several steps (the persistent interaction list of Sec. 4.2).
//
// One wavefront walks one group.  The traversal is breadth first: the 64
// lanes test 64 frontier nodes at a time and ballots / a wave prefix sum
// compact the three outcomes (accepted node -> node list, rejected leaf ->
// particle list, rejected internal node -> its children join the next
// frontier).  Frontier order is ascending node id at every level, so both
// lists come out in ascending node id without a sort.
//
// Opening test (the paper states none; reading): a node is accepted when it
// lies outside the group's grid box and side < theta * distance from the
// node's centre to the box, evaluated in doubled integer grid units with a
// single FP64 multiply, so every device decides exactly alike.  On
// cylindrical tree coordinates (Sec. 4.3) the phi axis is periodic with one
// turn = 2^21 grid units: its distance is that of the node's nearest image
// (a node and a group box inside one turn overlap only directly).
#include "bh_learned.hpp"

namespace {

constexpr int WALK_TPB = 256;
constexpr int WALK_LFRONT = 512;    // geometric walk: frontier entries kept in LDS per wave and buffer

// doubled distance from the doubled coordinate C to [gl, gh]
__device__ __forceinline__ int64_t gap2(int64_t C, int64_t gl, int64_t gh) {
    int64_t da = 0;
    da = (2 * gl - C > da) ? 2 * gl - C : da;
    da = (C - 2 * gh > da) ? C - 2 * gh : da;
    return da;
}

__device__ __forceinline__ bool accept_cell(int4 glo, int4 ghi, int Lx, int Ly, int Lz, int level, double th2,
                                            bool periodic = false) {
    const int64_t s = (int64_t)1 << (BH_MAXLEVEL - level);
    const int64_t L[3] = {Lx, Ly, Lz};
    const int64_t gl[3] = {glo.x, glo.y, glo.z}, gh[3] = {ghi.x, ghi.y, ghi.z};
    constexpr int64_t TURN2 = (int64_t)2 << BH_MAXLEVEL;    // one turn of phi, doubled units
    bool disjoint = false;
    int64_t d2 = 0;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        disjoint |= (L[a] + s <= gl[a]) || (L[a] >= gh[a]);
        int64_t C = 2 * L[a] + s;
        int64_t da = gap2(C, gl[a], gh[a]);
        if (a == 0 && periodic) {
            const int64_t dm = gap2(C - TURN2, gl[a], gh[a]), dp = gap2(C + TURN2, gl[a], gh[a]);
            da = dm < da ? dm : da;
            da = dp < da ? dp : da;
        }
        d2 += da * da;
    }
    const int64_t s2 = (2 * s) * (2 * s);
    return disjoint && ((double)s2 < th2 * (double)d2);
}

// The same test for the geometric walk, in 32-bit integers with the squared
// distance summed in FP64: every doubled coordinate and gap is below 2^24
// and every square below 2^47, so each step is exact and the decision is
// the one above, bit for bit, in about half the instructions.
__device__ __forceinline__ int gap2_i32(int C, int gl2, int gh2) {
    return max(0, max(gl2 - C, C - gh2));
}

__device__ __forceinline__ bool accept_cell_geo(int4 glo, int4 ghi, int Lx, int Ly, int Lz, int level, double th2,
                                                bool periodic) {
    const int s = 1 << (BH_MAXLEVEL - level);
    const int L[3] = {Lx, Ly, Lz};
    const int gl[3] = {glo.x, glo.y, glo.z}, gh[3] = {ghi.x, ghi.y, ghi.z};
    constexpr int TURN2 = 2 << BH_MAXLEVEL;
    bool disjoint = false;
    double d2 = 0.0;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        disjoint |= (L[a] + s <= gl[a]) || (L[a] >= gh[a]);
        const int C = 2 * L[a] + s;
        int da = gap2_i32(C, 2 * gl[a], 2 * gh[a]);
        if (a == 0 && periodic)
            da = min(da, min(gap2_i32(C - TURN2, 2 * gl[a], 2 * gh[a]), gap2_i32(C + TURN2, 2 * gl[a], 2 * gh[a])));
        d2 = fma((double)da, (double)da, d2);
    }
    const double s2 = (double)(4 * s) * (double)s;      // (2 s)^2
    return disjoint && (s2 < th2 * d2);
}

// Number of set bits of m in the lanes below this one.
__device__ __forceinline__ uint32_t mbcnt(uint64_t m) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

// Exclusive prefix sum over the lanes of a value in 0..15, and the wave
// total, from four ballots (no cross-lane data movement).
__device__ __forceinline__ uint32_t wave_excl_small(uint32_t v, uint32_t &tot) {
    uint32_t pre = 0;
    tot = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const uint64_t b = __ballot((v >> k) & 1u);
        pre += mbcnt(b) << k;
        tot += (uint32_t)__popcll(b) << k;
    }
    return pre;
}

// Per-group constants of the learned rule.
struct GroupCtx {
    int4 glo, ghi;
    double4 cen;
    double rad, amin, Msys, S;
};

// Acceptance of node v for a group.  GEOMETRIC: the theta test.  LEARNED:
// below theta_min accept, at or above theta_max open, in between the network
// (single-particle nodes accepted, nodes above the count cap: the theta test).
// ENUMERATE: the theta_min test; *cand reports whether (group, v) lies in the
// band and is a training candidate.
// GEO: the kernel instance that serves only the geometric rule, without the
// registers of the network inference (the other instance takes the rule from
// d.walk_mode).
template <bool GEO>
__device__ __forceinline__ bool decide(const DevState &d, const GroupCtx &gc, uint32_t v, int4 wr, bool *cand) {
    const int level = (int)((uint32_t)wr.x >> 24);
    const int Lx = wr.x & 0xffffff, Ly = wr.y & 0xffffff, Lz = wr.z;
    *cand = false;
    if (GEO) return accept_cell_geo(gc.glo, gc.ghi, Lx, Ly, Lz, level, d.th2, d.cyl_r > 0.0);
    if (d.walk_mode == WALK_GEOMETRIC) return accept_cell(gc.glo, gc.ghi, Lx, Ly, Lz, level, d.th2, d.cyl_r > 0.0);
    if (accept_cell(gc.glo, gc.ghi, Lx, Ly, Lz, level, d.th2_min)) return true;
    if (!accept_cell(gc.glo, gc.ghi, Lx, Ly, Lz, level, d.th2_max)) return false;
    const uint32_t cnt = d.nd_count[v];
    if (d.walk_mode == WALK_ENUMERATE) {
        *cand = cnt >= 2 && cnt <= d.count_cap;
        return false;
    }
    if (cnt == 1) return true;
    if (cnt > d.count_cap) return accept_cell(gc.glo, gc.ghi, Lx, Ly, Lz, level, d.th2);
    const double4 mom = d.nd_mom[v];
    const PairGeom pg =
        pair_features(mom, box_ratio2(gc.glo, gc.ghi, Lx, Ly, Lz, level), d.nd_qn[v], gc.cen, gc.rad, gc.Msys);
    return learned_accept(d.mlp, pg, mom.w, gc.amin, d.tau, d.G);
}

template <bool GEO>
__global__ void __launch_bounds__(WALK_TPB, (GEO ? 8 : 1)) k_walk(DevState d) {
    const uint32_t wave = (blockIdx.x * WALK_TPB + threadIdx.x) >> 6;
    if (wave >= d.walk_waves) return;
    const int lane = __lane_id();
    const uint64_t lt = lanemask_lt();
    const uint32_t F = d.walk_front_cap, P = d.walk_list_cap;
    uint32_t *fa = d.walk_scratch + (size_t)wave * (2 * (size_t)F + 2 * (size_t)P);
    uint32_t *fb = fa + F;
    uint32_t *pcb = fb + F;
    uint32_t *ppb = pcb + P;
    const uint32_t ng = d.cnt->n_groups;
    const uint32_t n_nodes = d.cnt->lvl_off[BH_NLEVELS];
    // geometric walk: the first WALK_LFRONT entries of each frontier live in
    // LDS, the rest at the same index in the wave's global scratch
    uint32_t *la = nullptr, *lb = nullptr;
    if constexpr (GEO) {
        __shared__ uint32_t lfront[WALK_TPB / 64][2][WALK_LFRONT];
        la = lfront[threadIdx.x >> 6][0];
        lb = lfront[threadIdx.x >> 6][1];
    }

    for (;;) {
        uint32_t g = 0;
        if (lane == 0) g = atomicAdd(&d.cnt->work_counter, 1u);
        g = __shfl(g, 0, 64);
        if (g >= ng) break;
        const GroupInfo gi = d.grp[g];
        GroupCtx gc;
        gc.glo = d.g_lo[g];
        gc.ghi = d.g_hi[g];
        if (!GEO && d.walk_mode != WALK_GEOMETRIC) {
            gc.cen = d.g_cen[g];
            gc.rad = d.g_rad[g];
            gc.amin = d.walk_mode == WALK_LEARNED ? d.g_amin[g] : 0.0;
            gc.Msys = d.nd_mom[gi.sys].w;
            gc.S = (double)(1u << BH_MAXLEVEL) / d.box[gi.sys].w;
        }
        // the enumerating walk visits only the sampled groups and stores no lists
        const bool enumerate = !GEO && d.walk_mode == WALK_ENUMERATE;
        const bool record = enumerate && (g % d.group_stride) == 0;
        if (enumerate && !record) {
            if (lane == 0) {
                d.g_pc_len[g] = 0;
                d.g_pp_len[g] = 0;
                d.g_cost[g] = 0;
            }
            continue;
        }
        uint32_t *cur = fa, *nxt = fb;
        uint32_t *lcur = la, *lnxt = lb;
        if (lane == 0) {
            if constexpr (GEO) lcur[0] = gi.sys;  // root of the group's system
            else cur[0] = gi.sys;
        }
        __threadfence_block();
        uint32_t ncur = 1, npc = 0, npp = 0;
        unsigned long long pp_particles = 0;
        unsigned long long pp_lane = 0;          // geometric walk: this lane's share, summed once per group
        bool ovf = false, bound = false;
        // A walk of a well-formed tree descends one level per frontier and
        // visits every node at most once; a frontier beyond the deepest level
        // or more visits than nodes can only come from a malformed tree, and
        // ends the walk with a flag instead of running on.
        uint32_t levels = 0;
        unsigned long long visits = 0;
        while (ncur > 0 && !ovf && !bound) {
            visits += ncur;
            if (++levels > (uint32_t)BH_NLEVELS || visits > (unsigned long long)n_nodes) {
                bound = true;
                break;
            }
            uint32_t nnext = 0;
            for (uint32_t base = 0; base < ncur; base += 64) {
                const uint32_t k = base + lane;
                const bool valid = k < ncur;
                uint32_t v;
                if constexpr (GEO) v = valid ? (k < (uint32_t)WALK_LFRONT ? lcur[k] : cur[k]) : 0u;
                else v = valid ? cur[k] : 0u;
                int4 wr = valid ? d.nd_walk[v] : make_int4(0, 0, 0, 0);
                const int nch = (int)((uint32_t)wr.y >> 24);
                bool is_cand = false;
                const bool acc = valid && decide<GEO>(d, gc, v, wr, &is_cand);
                is_cand = is_cand && valid && record;
                const uint64_t mc = __ballot(is_cand);
                if (mc) {
                    unsigned long long at = 0;
                    if (lane == 0) at = atomicAdd(&d.cnt->cand_used, (unsigned long long)__popcll(mc));
                    at = __shfl(at, 0, 64) + (unsigned long long)__popcll(mc & lt);
                    if (is_cand && at < d.cand_cap) d.cand[at] = make_uint2(g, v);
                }
                const bool is_pp = valid && !acc && nch == 0;
                const uint32_t nopen = (valid && !acc && nch > 0) ? (uint32_t)nch : 0u;

                const uint64_t mpc = __ballot(acc);
                const uint64_t mpp = __ballot(is_pp);
                uint32_t o, tot;
                if constexpr (GEO) {
                    const uint32_t opc = npc + mbcnt(mpc);
                    const uint32_t opp = npp + mbcnt(mpp);
                    if (acc && opc < P) pcb[opc] = v;
                    if (is_pp && opp < P) ppb[opp] = v;
                    if (is_pp) pp_lane += d.nd_count[v];
                    npc += (uint32_t)__popcll(mpc);
                    npp += (uint32_t)__popcll(mpp);
                    o = nnext + wave_excl_small(nopen, tot);
                } else {
                    const uint32_t opc = npc + (uint32_t)__popcll(mpc & lt);
                    const uint32_t opp = npp + (uint32_t)__popcll(mpp & lt);
                    if (acc && opc < P && !enumerate) pcb[opc] = v;
                    if (is_pp && opp < P && !enumerate) ppb[opp] = v;
                    unsigned long long cnt_pp = is_pp ? (unsigned long long)d.nd_count[v] : 0ull;
                    pp_particles += wave_sum(cnt_pp);
                    npc += (uint32_t)__popcll(mpc);
                    npp += (uint32_t)__popcll(mpp);

                    const uint32_t incl = wave_incl_scan(nopen);
                    tot = __shfl(incl, 63, 64);
                    o = nnext + incl - nopen;
                }
                for (uint32_t c = 0; c < nopen; ++c)
                    if constexpr (GEO) {
                        const uint32_t q = o + c;
                        if (q < (uint32_t)WALK_LFRONT) lnxt[q] = (uint32_t)wr.w + c;
                        else if (q < F) nxt[q] = (uint32_t)wr.w + c;
                    } else if (o + c < F) {
                        nxt[o + c] = (uint32_t)wr.w + c;
                    }
                nnext += tot;
            }
            if (nnext > F || (!enumerate && (npc > P || npp > P))) ovf = true;
            __threadfence_block();
            uint32_t *t = cur; cur = nxt; nxt = t;
            if constexpr (GEO) { t = lcur; lcur = lnxt; lnxt = t; }
            ncur = nnext;
        }
        if (bound) {
            if (lane == 0) {
                atomicOr(&d.cnt->flags[FLAG_WALK_BOUND], 1u);
                d.g_pc_len[g] = 0;
                d.g_pp_len[g] = 0;
                d.g_cost[g] = 0;
            }
            continue;
        }
        if (ovf) {
            if (lane == 0) {
                atomicOr(&d.cnt->flags[FLAG_WALK_OVF], 1u);
                atomicMax(&d.cnt->walk_need_front, ncur);
                if (!enumerate) atomicMax(&d.cnt->walk_need_list, max(npc, npp));
            }
            d.g_pc_len[g] = 0;
            d.g_pp_len[g] = 0;
            d.g_cost[g] = 0;
            continue;
        }
        if (enumerate) {
            if (lane == 0) {
                d.g_pc_len[g] = 0;
                d.g_pp_len[g] = 0;
                d.g_cost[g] = 0;
            }
            continue;
        }
        if constexpr (GEO) pp_particles = wave_sum(pp_lane);
        unsigned long long at_pc = 0, at_pp = 0;
        if (lane == 0) {
            at_pc = atomicAdd(&d.cnt->pc_used, (unsigned long long)npc);
            at_pp = atomicAdd(&d.cnt->pp_used, (unsigned long long)npp);
        }
        at_pc = __shfl(at_pc, 0, 64);
        at_pp = __shfl(at_pp, 0, 64);
        const bool fit = (at_pc + npc <= d.pc_cap) && (at_pp + npp <= d.pp_cap);
        if (fit) {
            for (uint32_t k = lane; k < npc; k += 64) d.pc_pool[at_pc + k] = pcb[k];
            for (uint32_t k = lane; k < npp; k += 64) d.pp_pool[at_pp + k] = ppb[k];
        } else if (lane == 0) {
            atomicOr(&d.cnt->flags[FLAG_POOL_OVF], 1u);
        }
        const unsigned long long cost = (unsigned long long)gi.count * (pp_particles + npc);
        if (lane == 0) {
            d.g_pc_off[g] = fit ? at_pc : 0ull;
            d.g_pc_len[g] = fit ? npc : 0u;
            d.g_pp_off[g] = fit ? at_pp : 0ull;
            d.g_pp_len[g] = fit ? npp : 0u;
            d.g_cost[g] = cost;
            atomicAdd(&d.cnt->interactions, cost);
        }
        __threadfence_block();
    }
}

__global__ void k_walk_reset(DevState d) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        d.cnt->work_counter = 0;
        d.cnt->pc_used = 0;
        d.cnt->pp_used = 0;
        d.cnt->interactions = 0;
        d.cnt->walk_need_front = 0;
        d.cnt->walk_need_list = 0;
        d.cnt->flags[FLAG_WALK_OVF] = 0;
        d.cnt->flags[FLAG_POOL_OVF] = 0;
        d.cnt->flags[FLAG_WALK_BOUND] = 0;
        d.cnt->flags[FLAG_CAND_BAD] = 0;
        d.cnt->cand_used = 0;
    }
}

// Work order for the force kernel: groups by descending interaction count
// (the list-length ordering of the paper's load balance, Sec. 4.6), in
// classes of half an octave of cost; inside a class, ascending group id,
// i.e. along the Morton curve, so that the groups in flight at one time are
// neighbours whose lists share most of their sources in L2.  Key: class
// (7 bits, largest cost first) above the group id (32 bits).
__global__ void k_order_keys(DevState d, uint64_t *key, uint32_t *val) {
    const uint32_t ng = d.cnt->n_groups;
    uint32_t stride = gridDim.x * blockDim.x;
    for (uint32_t g = blockIdx.x * blockDim.x + threadIdx.x; g < ng; g += stride) {
        const unsigned long long c = d.g_cost[g];
        uint32_t cls = c ? (uint32_t)(2.0 * log2((double)c)) : 0u;
        cls = cls < 127u ? cls : 127u;
        key[g] = ((unsigned long long)(127u - cls) << 32) | (unsigned long long)g;
        val[g] = g;
    }
}

}  // namespace

namespace bhk {

void walk(const DevState &d, hipStream_t s) {
    k_walk_reset<<<1, 64, 0, s>>>(d);
    const uint32_t waves = d.walk_mode == WALK_GEOMETRIC ? d.walk_waves : d.walk_waves_net;
    unsigned blocks = (waves * 64 + WALK_TPB - 1) / WALK_TPB;
    if (d.walk_mode == WALK_GEOMETRIC)
        k_walk<true><<<blocks, WALK_TPB, 0, s>>>(d);
    else
        k_walk<false><<<blocks, WALK_TPB, 0, s>>>(d);
}

void order_groups(const DevState &d, uint32_t n_groups, uint64_t *key_a, uint32_t *val_a, uint64_t *key_b,
                  uint32_t *val_b, hipStream_t s) {
    if (n_groups == 0) return;
    unsigned blocks = (n_groups + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    k_order_keys<<<blocks, 256, 0, s>>>(d, key_a, val_a);
    radix_sort(key_a, val_a, key_b, val_b, n_groups, 0, 40, d.hist, d.scan_tmp, s, nullptr, 0);
    (void)hipMemcpyAsync(d.order, val_a, (size_t)n_groups * sizeof(uint32_t), hipMemcpyDeviceToDevice, s);
}

}  // namespace bhk
