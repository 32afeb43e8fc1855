// bh_api.hip -- the C ABI of include/bh.h: context, device buffers with
// capacity growth, the order of the stages of a timestep (Iwasawa et al.
// 2019, Sec. 4.2: tree (3a), walk and lists (3d), interaction (3d),
// integration (4), persistent lists reused over several steps), and export
// of internal structures.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "bh.h"
#include "bh_learned.hpp"

namespace bhk {
size_t mlp_act_floats(uint32_t B);
}

namespace {

struct DevBuf {
    void *p = nullptr;
    size_t bytes = 0;
};

// per-block partial sums of the scans (at least the scan kernels' block count)
constexpr size_t SCAN_TMP_WORDS = 4096;

enum StageEv { EV_KEYS = 0, EV_TREE, EV_MOM, EV_GROUPS, EV_WALK, EV_FORCE, EV_INTEG, EV_STEP, EV_N };

}  // namespace

struct bh_ctx {
    bh_params P{};
    std::string err;
    int device = 0;
    int n_cu = 256;

    // host-side sizes of the current build
    int n_sys = 0;
    uint32_t n = 0;
    uint32_t box_blocks = 1;
    std::vector<uint32_t> sys_off;
    bool tree_valid = false, lists_valid = false;
    uint32_t n_nodes = 0, n_groups = 0, max_level = 0;
    uint64_t n_pc = 0, n_pp = 0, interactions = 0;
    int n_grp_used = 64;

    // capacities
    uint32_t n_cap = 0, node_cap = 0, sys_cap = 0;
    uint64_t pc_cap = 0, pp_cap = 0;
    uint32_t walk_waves = 0, walk_waves_net = 0, walk_front = 4096, walk_list = 8192;

    // device buffers
    DevBuf sys_off_b, sys_tab_b, acc_tab_b, box_b, box_part_b, sys_m0_b;
    DevBuf pos_in, vel_in, idx_in, pos, vel, acc, idx, inv;
    DevBuf key, key_tmp, val, val_tmp, hist, scan_tmp;
    DevBuf nd_prefix, nd_begin, nd_count, nd_first, nd_meta, nd_walk, nd_mom, nd_quad, tmp_a, tmp_b;
    DevBuf gmark, grp, g_lo, g_hi, g_cen, g_pc_off, g_pc_len, g_pp_off, g_pp_len, g_cost, order;
    DevBuf gkey_a, gkey_b, gval_a, gval_b;
    DevBuf pc_pool, pp_pool, walk_scratch, counters;
    DevBuf pos_b, nd_mom_b, nd_drift;    // drift monitor: build snapshot and per-node drift

    // pinned host staging
    DevCounters *h_cnt = nullptr;
    SysPtr *h_systab = nullptr;
    bhk::AccPtr *h_acctab = nullptr;
    hipEvent_t tab_ev = nullptr;      // last copy out of the pinned tables
    bool tab_ev_pending = false;

    hipEvent_t ev0[EV_N] = {}, ev1[EV_N] = {};
    bool ev_used[EV_N] = {};
    std::vector<std::pair<hipEvent_t, hipEvent_t>> force_ev;   // one pair per force launch
    size_t force_ev_used = 0;

    // running totals and integration state
    int64_t interactions_evaluated = 0, force_evaluations = 0, tree_builds = 0;
    int64_t drift_rebuilds = 0, host_syncs = 0;
    bool state_valid = false;     // sorted x, v, a ready for bh_step_continue
    bool have_vel = false;
    int age = 0;                  // force evaluations done with the current lists
    DevBuf direct_part;

    // HIP graphs of the launch-bound part of a list-reusing step (kick-drift +
    // the per-level moment refresh), replayed on an internal stream fenced
    // with events against the caller's stream.  Two cached instances: the
    // sorted buffers alternate between two allocations from one tree build to
    // the next.
    struct GraphEntry {
        DevState key;
        double h = 0, dt = 0;
        hipGraphExec_t exec = nullptr;
    };
    // learned opening rule
    DevBuf nd_qn, amag, amag_in, g_amin, g_rad, cand, mlp_w, mlp_m, mlp_v, mlp_g, act;
    DevBuf ds_x, ds_y, ds_pairs, pk_a, pk_b, pv_a, pv_b, phist, eval_out;
    uint64_t cand_cap = 0, ds_n = 0, ds_cap = 0;
    int walk_mode = WALK_GEOMETRIC;
    uint32_t group_stride = 1, count_cap = 65536;
    bool amag_valid = false, mlp_ready = false;
    int adam_t = 0;

    GraphEntry graphs[2];
    int graph_next = 0;
    hipStream_t gs = nullptr;
    hipEvent_t fence_a = nullptr, fence_b = nullptr;
    int64_t graph_replays = 0, graph_captures = 0;

    DevState d{};
};

namespace {

bh_status fail(bh_ctx *c, bh_status st, const std::string &msg) {
    if (c) c->err = msg;
    return st;
}

bh_status hipfail(bh_ctx *c, const char *what, hipError_t e) {
    char buf[512];
    snprintf(buf, sizeof buf, "%s: %s (%d)", what, hipGetErrorString(e), (int)e);
    return fail(c, e == hipErrorOutOfMemory ? BH_ENOMEM : BH_EHIP, buf);
}

#define HIPCHK(c, x)                                    \
    do {                                                \
        hipError_t e_ = (x);                            \
        if (e_ != hipSuccess) return hipfail(c, #x, e_); \
    } while (0)

#define STCHK(x)                      \
    do {                              \
        bh_status st_ = (x);          \
        if (st_ != BH_OK) return st_; \
    } while (0)

hipError_t grow(DevBuf &b, size_t bytes) {
    if (bytes <= b.bytes && b.p) return hipSuccess;
    if (b.p) {
        hipError_t e = hipFree(b.p);
        if (e != hipSuccess) return e;
        b.p = nullptr;
        b.bytes = 0;
    }
    if (bytes == 0) bytes = 256;
    hipError_t e = hipMalloc(&b.p, bytes);
    if (e == hipSuccess) b.bytes = bytes;
    return e;
}

void release(DevBuf &b) {
    if (b.p) (void)hipFree(b.p);
    b.p = nullptr;
    b.bytes = 0;
}

template <typename T>
T *P(DevBuf &b) {
    return reinterpret_cast<T *>(b.p);
}

void refresh_state(bh_ctx *c) {
    DevState &d = c->d;
    d.n_sys = c->n_sys;
    d.n = c->n;
    d.sys_off = P<uint32_t>(c->sys_off_b);
    d.sys_tab = P<SysPtr>(c->sys_tab_b);
    d.box = P<double4>(c->box_b);
    d.box_part = P<double>(c->box_part_b);
    d.box_blocks = c->box_blocks;
    d.sys_m0 = P<double>(c->sys_m0_b);
    d.pos_in = P<double4>(c->pos_in);
    d.vel_in = P<double4>(c->vel_in);
    d.idx_in = P<uint32_t>(c->idx_in);
    d.pos = P<double4>(c->pos);
    d.vel = P<double4>(c->vel);
    d.acc = P<double4>(c->acc);
    d.idx = P<uint32_t>(c->idx);
    d.inv = P<uint32_t>(c->inv);
    d.key = P<uint64_t>(c->key);
    d.key_tmp = P<uint64_t>(c->key_tmp);
    d.val = P<uint32_t>(c->val);
    d.val_tmp = P<uint32_t>(c->val_tmp);
    d.hist = P<uint32_t>(c->hist);
    d.scan_tmp = P<uint32_t>(c->scan_tmp);
    d.node_cap = c->node_cap;
    d.nd_prefix = P<uint64_t>(c->nd_prefix);
    d.nd_begin = P<uint32_t>(c->nd_begin);
    d.nd_count = P<uint32_t>(c->nd_count);
    d.nd_first = P<uint32_t>(c->nd_first);
    d.nd_meta = P<uint32_t>(c->nd_meta);
    d.nd_walk = P<int4>(c->nd_walk);
    d.nd_mom = P<double4>(c->nd_mom);
    d.nd_quad = (c->P.criterion == BH_OPEN_LEARNED) ? P<double>(c->nd_quad) : nullptr;
    d.tmp_a = P<uint32_t>(c->tmp_a);
    d.tmp_b = P<uint32_t>(c->tmp_b);
    d.gmark = P<uint32_t>(c->gmark);
    d.grp = P<GroupInfo>(c->grp);
    d.g_lo = P<int4>(c->g_lo);
    d.g_hi = P<int4>(c->g_hi);
    d.g_cen = P<double4>(c->g_cen);
    d.g_pc_off = P<unsigned long long>(c->g_pc_off);
    d.g_pc_len = P<uint32_t>(c->g_pc_len);
    d.g_pp_off = P<unsigned long long>(c->g_pp_off);
    d.g_pp_len = P<uint32_t>(c->g_pp_len);
    d.g_cost = P<unsigned long long>(c->g_cost);
    d.order = P<uint32_t>(c->order);
    d.pc_pool = P<uint32_t>(c->pc_pool);
    d.pp_pool = P<uint32_t>(c->pp_pool);
    d.pc_cap = c->pc_cap;
    d.pp_cap = c->pp_cap;
    d.walk_scratch = P<uint32_t>(c->walk_scratch);
    d.walk_front_cap = c->walk_front;
    d.walk_list_cap = c->walk_list;
    d.walk_waves = c->walk_waves;
    d.walk_waves_net = c->walk_waves_net;
    d.cnt = P<DevCounters>(c->counters);
    const bool learned = c->P.criterion == BH_OPEN_LEARNED;
    d.walk_mode = c->walk_mode;
    d.th2_min = c->P.theta_min * c->P.theta_min;
    d.th2_max = c->P.theta_max * c->P.theta_max;
    d.tau = c->P.tau;
    d.mlp = P<float>(c->mlp_w);
    d.nd_qn = learned ? P<float>(c->nd_qn) : nullptr;
    d.amag = learned ? P<double>(c->amag) : nullptr;
    d.amag_in = learned ? P<double>(c->amag_in) : nullptr;
    d.g_amin = learned ? P<double>(c->g_amin) : nullptr;
    d.g_rad = learned ? P<double>(c->g_rad) : nullptr;
    d.cand = P<uint2>(c->cand);
    d.cand_cap = c->cand_cap;
    d.group_stride = c->group_stride;
    d.count_cap = c->count_cap;
    d.n_leaf = c->P.n_leaf;
    d.n_grp = c->n_grp_used;
    d.th2 = c->P.theta * c->P.theta;
    d.eps2 = c->P.eps * c->P.eps;
    d.G = c->P.G;
    d.central_mass = c->P.central_mass;
    d.rc = c->P.r_coll;
    d.kappa = c->P.kappa;
    d.eta = c->P.eta;
    d.cyl_r = c->P.cyl_radius;
    const bool monitor = c->P.reuse_drift > 0.0;
    d.pos_b = monitor ? P<double4>(c->pos_b) : nullptr;
    d.nd_mom_b = monitor ? P<double4>(c->nd_mom_b) : nullptr;
    d.nd_drift = nullptr;     // set only for the monitored moment pass of a list-reusing step
    d.drift_kappa = c->P.reuse_drift;
    d.force_tile = c->P.force_tile == 256 ? 256 : 512;
    d.budget_min = (c->P.flags & BH_FLAG_BUDGET_MIN) ? 1 : 0;
    d.pack_groups = (c->P.flags & BH_FLAG_PACK_GROUPS) ? 1 : 0;
}

bh_status check_params(const bh_params *p) {
    if (!p) return BH_EINVAL;
    if (!(p->theta >= 0.0) || !std::isfinite(p->theta)) return BH_EINVAL;
    if (!(p->eps >= 0.0) || !std::isfinite(p->eps)) return BH_EINVAL;
    if (!std::isfinite(p->G) || !std::isfinite(p->central_mass)) return BH_EINVAL;
    if (p->n_leaf < 1 || p->n_leaf > 4096) return BH_EINVAL;
    if (p->n_group > 65536) return BH_EINVAL;
    if (p->precision != BH_FP64 && p->precision != BH_FP32_REL) return BH_EINVAL;
    if (p->criterion != BH_OPEN_GEOMETRIC && p->criterion != BH_OPEN_LEARNED) return BH_EINVAL;
    if (!(p->r_coll >= 0.0) || !std::isfinite(p->r_coll)) return BH_EINVAL;
    if (!(p->kappa >= 0.0) || !std::isfinite(p->kappa)) return BH_EINVAL;
    if (!(p->eta >= 0.0) || !std::isfinite(p->eta)) return BH_EINVAL;
    if (!(p->cyl_radius >= 0.0) || !std::isfinite(p->cyl_radius)) return BH_EINVAL;
    if (p->cyl_radius > 0.0 && p->criterion == BH_OPEN_LEARNED) return BH_EINVAL;
    if (p->criterion == BH_OPEN_LEARNED)
        for (double v : {p->theta_min, p->theta_max, p->tau})
            if (!(v >= 0.0) || !std::isfinite(v)) return BH_EINVAL;
    if (!(p->reuse_drift >= 0.0) || !std::isfinite(p->reuse_drift)) return BH_EINVAL;
    if (!(p->reuse_frac >= 0.0) || !(p->reuse_frac <= 1.0)) return BH_EINVAL;
    if (p->force_tile != 0 && p->force_tile != 256 && p->force_tile != 512) return BH_EINVAL;
    return BH_OK;
}

void ev_begin(bh_ctx *c, int k, hipStream_t s) {
    (void)hipEventRecord(c->ev0[k], s);
}
void ev_end(bh_ctx *c, int k, hipStream_t s) {
    (void)hipEventRecord(c->ev1[k], s);
    c->ev_used[k] = true;
}

bh_status wait_tables(bh_ctx *c) {
    if (c->tab_ev_pending) {
        HIPCHK(c, hipEventSynchronize(c->tab_ev));
        c->tab_ev_pending = false;
    }
    return BH_OK;
}

bh_status read_counters(bh_ctx *c, hipStream_t s) {
    HIPCHK(c, hipMemcpyAsync(c->h_cnt, c->counters.p, sizeof(DevCounters), hipMemcpyDeviceToHost, s));
    HIPCHK(c, hipStreamSynchronize(s));
    c->host_syncs += 1;
    return BH_OK;
}

// Build snapshot and drift buffers of the drift monitor (only when it is on).
bh_status ensure_drift(bh_ctx *c) {
    if (!(c->P.reuse_drift > 0.0)) return BH_OK;
    if (c->n_cap) HIPCHK(c, grow(c->pos_b, (size_t)c->n_cap * sizeof(double4)));
    if (c->node_cap) {
        HIPCHK(c, grow(c->nd_mom_b, (size_t)c->node_cap * sizeof(double4)));
        HIPCHK(c, grow(c->nd_drift, (size_t)c->node_cap * sizeof(double)));
    }
    return BH_OK;
}

bh_status ensure_systems(bh_ctx *c, int n_sys) {
    if ((uint32_t)n_sys <= c->sys_cap && c->h_systab) return BH_OK;
    uint32_t cap = std::max<uint32_t>(n_sys, 16);
    STCHK(wait_tables(c));
    HIPCHK(c, grow(c->sys_off_b, (cap + 1) * sizeof(uint32_t)));
    HIPCHK(c, grow(c->sys_tab_b, cap * sizeof(SysPtr)));
    HIPCHK(c, grow(c->acc_tab_b, cap * sizeof(bhk::AccPtr)));
    HIPCHK(c, grow(c->box_b, cap * sizeof(double4)));
    HIPCHK(c, grow(c->sys_m0_b, cap * sizeof(double)));
    if (c->h_systab) (void)hipHostFree(c->h_systab);
    if (c->h_acctab) (void)hipHostFree(c->h_acctab);
    c->h_systab = nullptr;
    c->h_acctab = nullptr;
    HIPCHK(c, hipHostMalloc((void **)&c->h_systab, (cap + 1) * sizeof(SysPtr) + (cap + 1) * sizeof(uint32_t)));
    HIPCHK(c, hipHostMalloc((void **)&c->h_acctab, cap * sizeof(bhk::AccPtr)));
    c->sys_cap = cap;
    return BH_OK;
}

bh_status ensure_particles(bh_ctx *c, uint32_t n) {
    if (n <= c->n_cap && c->pos.p) return BH_OK;
    uint32_t cap = std::max<uint32_t>(n, 1024);
    size_t d4 = (size_t)cap * sizeof(double4), u4 = (size_t)cap * 4, u8 = (size_t)cap * 8;
    HIPCHK(c, grow(c->pos_in, d4));
    HIPCHK(c, grow(c->vel_in, d4));
    HIPCHK(c, grow(c->idx_in, u4));
    HIPCHK(c, grow(c->pos, d4));
    HIPCHK(c, grow(c->vel, d4));
    HIPCHK(c, grow(c->acc, d4));
    HIPCHK(c, grow(c->idx, u4));
    HIPCHK(c, grow(c->inv, u4));
    HIPCHK(c, grow(c->key, u8));
    HIPCHK(c, grow(c->key_tmp, u8));
    HIPCHK(c, grow(c->val, u4));
    HIPCHK(c, grow(c->val_tmp, u4));
    HIPCHK(c, grow(c->hist, bhk::radix_hist_words(cap) * 4));
    HIPCHK(c, grow(c->scan_tmp, SCAN_TMP_WORDS * 4));
    HIPCHK(c, grow(c->gmark, u4));
    HIPCHK(c, grow(c->grp, (size_t)cap * sizeof(GroupInfo)));
    HIPCHK(c, grow(c->g_lo, (size_t)cap * sizeof(int4)));
    HIPCHK(c, grow(c->g_hi, (size_t)cap * sizeof(int4)));
    HIPCHK(c, grow(c->g_cen, d4));
    HIPCHK(c, grow(c->g_pc_off, u8));
    HIPCHK(c, grow(c->g_pc_len, u4));
    HIPCHK(c, grow(c->g_pp_off, u8));
    HIPCHK(c, grow(c->g_pp_len, u4));
    HIPCHK(c, grow(c->g_cost, u8));
    HIPCHK(c, grow(c->order, u4));
    HIPCHK(c, grow(c->gkey_a, u8));
    HIPCHK(c, grow(c->gkey_b, u8));
    HIPCHK(c, grow(c->gval_a, u4));
    HIPCHK(c, grow(c->gval_b, u4));
    c->n_cap = cap;
    STCHK(ensure_drift(c));
    if (c->P.criterion == BH_OPEN_LEARNED) {
        HIPCHK(c, grow(c->amag, u8));
        HIPCHK(c, grow(c->amag_in, u8));
        HIPCHK(c, grow(c->g_amin, u8));
        HIPCHK(c, grow(c->g_rad, u8));
    }
    return BH_OK;
}

// Per-particle and per-node arrays of the learned rule, when it is switched on later.
bh_status ensure_learned(bh_ctx *c) {
    if (c->P.criterion != BH_OPEN_LEARNED) return BH_OK;
    if (c->n_cap) {
        size_t u8 = (size_t)c->n_cap * 8;
        HIPCHK(c, grow(c->amag, u8));
        HIPCHK(c, grow(c->amag_in, u8));
        HIPCHK(c, grow(c->g_amin, u8));
        HIPCHK(c, grow(c->g_rad, u8));
    }
    if (c->node_cap) {
        HIPCHK(c, grow(c->nd_quad, (size_t)c->node_cap * 6 * sizeof(double)));
        HIPCHK(c, grow(c->nd_qn, (size_t)c->node_cap * 4));
    }
    HIPCHK(c, grow(c->mlp_w, BH_MLP_NPARAM * 4));
    return BH_OK;
}

bh_status ensure_nodes(bh_ctx *c, uint32_t cap) {
    if (cap <= c->node_cap && c->nd_prefix.p) return BH_OK;
    cap = std::max<uint32_t>(cap, 1024);
    HIPCHK(c, grow(c->nd_prefix, (size_t)cap * 8));
    HIPCHK(c, grow(c->nd_begin, (size_t)cap * 4));
    HIPCHK(c, grow(c->nd_count, (size_t)cap * 4));
    HIPCHK(c, grow(c->nd_first, (size_t)cap * 4));
    HIPCHK(c, grow(c->nd_meta, (size_t)cap * 4));
    HIPCHK(c, grow(c->nd_walk, (size_t)cap * sizeof(int4)));
    HIPCHK(c, grow(c->nd_mom, (size_t)cap * sizeof(double4)));
    if (c->P.criterion == BH_OPEN_LEARNED) {
        HIPCHK(c, grow(c->nd_quad, (size_t)cap * 6 * sizeof(double)));
        HIPCHK(c, grow(c->nd_qn, (size_t)cap * 4));
    }
    HIPCHK(c, grow(c->tmp_a, (size_t)cap * 4));
    HIPCHK(c, grow(c->tmp_b, (size_t)cap * 4));
    c->node_cap = cap;
    STCHK(ensure_drift(c));
    return BH_OK;
}

bh_status ensure_walk(bh_ctx *c) {
    // at most 4 GiB of walk scratch: fewer walking waves when each needs more.
    // The geometric walk keeps 32 waves per CU resident (8 workgroups at
    // <= 64 VGPRs), the walk with the network in it (171 VGPRs) 16.
    const size_t per_wave = 2 * (size_t)c->walk_front + 2 * (size_t)c->walk_list;
    const size_t cap = ((size_t)1 << 30) / per_wave;
    c->walk_waves = (uint32_t)(std::max<size_t>(std::min<size_t>(cap, (size_t)c->n_cu * 32), 64) & ~(size_t)3);
    c->walk_waves_net = (uint32_t)(std::max<size_t>(std::min<size_t>(cap, (size_t)c->n_cu * 16), 64) & ~(size_t)3);
    c->walk_waves_net = std::min(c->walk_waves_net, c->walk_waves);
    size_t words = (size_t)c->walk_waves * per_wave;
    HIPCHK(c, grow(c->walk_scratch, words * 4));
    return BH_OK;
}

bh_status ensure_pools(bh_ctx *c, uint64_t pc, uint64_t pp) {
    if (pc > c->pc_cap || !c->pc_pool.p) {
        HIPCHK(c, grow(c->pc_pool, std::max<uint64_t>(pc, 1024) * 4));
        c->pc_cap = std::max<uint64_t>(pc, 1024);
    }
    if (pp > c->pp_cap || !c->pp_pool.p) {
        HIPCHK(c, grow(c->pp_pool, std::max<uint64_t>(pp, 1024) * 4));
        c->pp_cap = std::max<uint64_t>(pp, 1024);
    }
    return BH_OK;
}

// Stage (3a): everything from the input particles to groups.  from_caller:
// load the caller's arrays; otherwise rebuild from the current sorted state.
bh_status rebuild(bh_ctx *c, hipStream_t s, bool from_caller) {
    if (!from_caller) {
        std::swap(c->pos_in, c->pos);
        std::swap(c->vel_in, c->vel);
        std::swap(c->idx_in, c->idx);
        std::swap(c->amag_in, c->amag);
    } else {
        c->amag_valid = false;
    }
    refresh_state(c);
    ev_begin(c, EV_KEYS, s);
    bhk::reset_flags(c->d, s);
    if (from_caller) bhk::load_systems(c->d, s);
    bhk::root_box_keys(c->d, s);
    bhk::permute(c->d, s);
    ev_end(c, EV_KEYS, s);
    for (;;) {
        ev_begin(c, EV_TREE, s);
        bhk::build_octree(c->d, s);
        ev_end(c, EV_TREE, s);
        STCHK(read_counters(c, s));
        if (c->h_cnt->flags[FLAG_NONFINITE]) {
            c->tree_valid = c->lists_valid = false;
            return fail(c, BH_EINVAL, "non-finite particle coordinate");
        }
        if (c->h_cnt->flags[FLAG_EXTENT]) {
            c->tree_valid = c->lists_valid = false;
            return fail(c, BH_EINVAL, "cylindrical tree: radial or vertical extent exceeds 2 pi cyl_radius");
        }
        if (c->h_cnt->flags[FLAG_NODE_OVF]) {
            // node ids are 32-bit: the capacity doubles at most up to 2^32 - 1
            if (c->node_cap >= 0x80000000u) return fail(c, BH_ECAPACITY, "tree node capacity cannot grow further");
            STCHK(ensure_nodes(c, c->node_cap * 2));
            refresh_state(c);
            continue;
        }
        break;
    }
    c->n_nodes = c->h_cnt->lvl_off[BH_NLEVELS];
    c->max_level = c->h_cnt->max_level;
    ev_begin(c, EV_MOM, s);
    bhk::moments(c->d, s);
    if (c->P.criterion == BH_OPEN_LEARNED) bhk::node_qn(c->d, s);
    ev_end(c, EV_MOM, s);
    ev_begin(c, EV_GROUPS, s);
    bhk::make_groups(c->d, s);
    ev_end(c, EV_GROUPS, s);
    STCHK(read_counters(c, s));
    c->n_groups = c->h_cnt->n_groups;
    // the drift monitor measures motion from here
    if (c->P.reuse_drift > 0.0) bhk::drift_snapshot(c->d, s);
    c->tree_valid = true;
    c->lists_valid = false;
    c->tree_builds += 1;
    c->age = 0;
    return BH_OK;
}

// The walk, redone with larger scratch / pools until everything fits.
bh_status walk_until_fits(bh_ctx *c, hipStream_t s) {
    for (int attempt = 0;; ++attempt) {
        refresh_state(c);
        ev_begin(c, EV_WALK, s);
        bhk::walk(c->d, s);
        ev_end(c, EV_WALK, s);
        STCHK(read_counters(c, s));
        const DevCounters &h = *c->h_cnt;
        if (h.flags[FLAG_WALK_BOUND]) {
            c->lists_valid = false;
            return fail(c, BH_ECAPACITY, "walk: a traversal went deeper than the tree's levels or visited more "
                                         "nodes than the tree holds (malformed tree)");
        }
        if (h.flags[FLAG_WALK_OVF]) {
            if (attempt > 40) return fail(c, BH_ECAPACITY, "walk scratch cannot grow further");
            // a walk cut short by its frontier may also need a longer list: that shows on the next try.
            // Neither a frontier nor a list of a well-formed tree holds more entries than the tree has nodes.
            const uint64_t most = (uint64_t)c->n_nodes + 64;
            if (h.walk_need_front > most || h.walk_need_list > most)
                return fail(c, BH_ECAPACITY, "walk: frontier or list longer than the tree's node count");
            auto grown = [most](uint32_t cur, uint32_t need) {
                return (uint32_t)std::min<uint64_t>(most, std::max<uint64_t>(2ull * cur, 2ull * need));
            };
            const uint32_t f0 = c->walk_front, l0 = c->walk_list;
            if (h.walk_need_front >= c->walk_front) c->walk_front = grown(c->walk_front, h.walk_need_front);
            if (h.walk_need_list >= c->walk_list) c->walk_list = grown(c->walk_list, h.walk_need_list);
            if (c->walk_front == f0 && c->walk_list == l0)
                return fail(c, BH_ECAPACITY, "walk scratch overflow without a larger need");
            STCHK(ensure_walk(c));
            continue;
        }
        if (h.flags[FLAG_POOL_OVF]) {
            // the pools are grown to what this walk needed, so one more pass fits
            if (attempt > 40) return fail(c, BH_ECAPACITY, "list pools cannot grow further");
            STCHK(ensure_pools(c, h.pc_used + h.pc_used / 4 + 1024, h.pp_used + h.pp_used / 4 + 1024));
            continue;
        }
        if (c->walk_mode == WALK_ENUMERATE && h.cand_used > c->cand_cap) {
            if (attempt > 40) return fail(c, BH_ECAPACITY, "candidate buffer cannot grow further");
            uint64_t cap = h.cand_used + h.cand_used / 4 + 1024;
            HIPCHK(c, grow(c->cand, cap * sizeof(uint2)));
            c->cand_cap = cap;
            continue;
        }
        c->n_pc = h.pc_used;
        c->n_pp = h.pp_used;
        c->interactions = h.interactions;
        return BH_OK;
    }
}

bh_status run_forces(bh_ctx *c, hipStream_t s, bool pot, double kick_h = 0.0);

bh_status order_lists(bh_ctx *c, hipStream_t s) {
    bhk::order_groups(c->d, c->n_groups, P<uint64_t>(c->gkey_a), P<uint32_t>(c->gval_a), P<uint64_t>(c->gkey_b),
                      P<uint32_t>(c->gval_b), s);
    c->lists_valid = true;
    return BH_OK;
}

bh_status make_lists(bh_ctx *c, hipStream_t s) {
    if (!c->tree_valid) return fail(c, BH_ESTATE, "bh_make_lists: no tree (call bh_build_tree first)");
    if (c->P.criterion == BH_OPEN_LEARNED) {
        if (!c->mlp_ready) return fail(c, BH_ESTATE, "learned criterion: no weights (bh_mlp_train or bh_mlp_weights)");
        if (!c->amag_valid) {
            // the error budget needs each group's acceleration: one geometric pass first
            c->walk_mode = WALK_GEOMETRIC;
            STCHK(walk_until_fits(c, s));
            STCHK(order_lists(c, s));
            refresh_state(c);
            STCHK(run_forces(c, s, false));
            bhk::group_amin(c->d, s);
            c->amag_valid = true;
        }
        c->walk_mode = WALK_LEARNED;
    } else {
        c->walk_mode = WALK_GEOMETRIC;
    }
    STCHK(walk_until_fits(c, s));
    c->walk_mode = WALK_GEOMETRIC;
    return order_lists(c, s);
}

// Persistent workgroups of the force kernel: as many as stay resident (FP32:
// 6 per CU by its register cap; FP64: 5 by its cap, 3 with the collision branch).
int force_blocks(const bh_ctx *c) {
    if (c->P.precision == BH_FP32_REL) return c->n_cu * 6;
    return c->n_cu * (c->P.r_coll > 0.0 ? 3 : 5);
}

// kick_h != 0: the launch also applies the closing half kick v += kick_h a.
// The kernels with the collision branch ignore it, so callers pass it only
// when the branch is off.
bh_status run_forces(bh_ctx *c, hipStream_t s, bool pot, double kick_h) {
    if (c->force_ev_used == c->force_ev.size()) {
        if (c->force_ev.size() >= 65536) {
            c->force_ev_used = 0;                    // drop the oldest window
        } else {
            hipEvent_t a, b;
            HIPCHK(c, hipEventCreate(&a));
            HIPCHK(c, hipEventCreate(&b));
            c->force_ev.emplace_back(a, b);
        }
    }
    auto &pr = c->force_ev[c->force_ev_used++];
    ev_begin(c, EV_FORCE, s);
    HIPCHK(c, hipEventRecord(pr.first, s));
    bhk::forces(c->d, c->n_groups, c->P.precision == BH_FP32_REL, pot, force_blocks(c), kick_h, s);
    HIPCHK(c, hipEventRecord(pr.second, s));
    ev_end(c, EV_FORCE, s);
    c->interactions_evaluated += (int64_t)c->interactions;
    c->force_evaluations += 1;
    c->age += 1;
    if (c->d.amag) c->amag_valid = true;
    return BH_OK;
}

bh_status set_systems(bh_ctx *c, const bh_system *sys, int32_t n_sys, hipStream_t s) {
    if (!sys || n_sys < 1) return fail(c, BH_EINVAL, "need at least one system");
    if (n_sys > 65535) return fail(c, BH_EINVAL, "too many systems (limit 65535)");
    uint64_t total = 0;
    for (int k = 0; k < n_sys; ++k) {
        if (sys[k].n < 1) return fail(c, BH_EINVAL, "empty system");
        if (!sys[k].x || !sys[k].y || !sys[k].z || !sys[k].m) return fail(c, BH_EINVAL, "null particle array");
        total += (uint64_t)sys[k].n;
    }
    if (total >= (1ull << 31)) return fail(c, BH_EINVAL, "too many particles (limit 2^31 - 1)");
    STCHK(ensure_systems(c, n_sys));
    STCHK(ensure_learned(c));
    STCHK(wait_tables(c));
    c->n_sys = n_sys;
    c->n = (uint32_t)total;
    c->sys_off.assign(n_sys + 1, 0);
    for (int k = 0; k < n_sys; ++k) {
        c->sys_off[k + 1] = c->sys_off[k] + (uint32_t)sys[k].n;
        SysPtr &t = c->h_systab[k];
        t.x = sys[k].x;
        t.y = sys[k].y;
        t.z = sys[k].z;
        t.vx = sys[k].vx;
        t.vy = sys[k].vy;
        t.vz = sys[k].vz;
        t.m = sys[k].m;
        t.n = sys[k].n;
    }
    uint32_t *h_off = reinterpret_cast<uint32_t *>(c->h_systab + c->sys_cap + 1);
    std::copy(c->sys_off.begin(), c->sys_off.end(), h_off);
    HIPCHK(c, hipMemcpyAsync(c->sys_tab_b.p, c->h_systab, n_sys * sizeof(SysPtr), hipMemcpyHostToDevice, s));
    HIPCHK(c, hipMemcpyAsync(c->sys_off_b.p, h_off, (n_sys + 1) * sizeof(uint32_t), hipMemcpyHostToDevice, s));
    HIPCHK(c, hipEventRecord(c->tab_ev, s));
    c->tab_ev_pending = true;
    // root-box partials: one system alone fills the chip, and the partials
    // stay O(n / BOX_PER_BLOCK) however the particles split into systems
    const uint64_t per = (total + (uint64_t)n_sys - 1) / (uint64_t)n_sys;
    c->box_blocks = (uint32_t)std::min<uint64_t>(BOX_BLOCKS_MAX, std::max<uint64_t>(1, per / BOX_PER_BLOCK));
    HIPCHK(c, grow(c->box_part_b, (size_t)n_sys * c->box_blocks * 8 * sizeof(double)));
    STCHK(ensure_particles(c, c->n));
    if (c->node_cap < c->n + (uint32_t)n_sys) STCHK(ensure_nodes(c, c->n + n_sys + 1024));
    if (!c->pc_pool.p) STCHK(ensure_pools(c, (uint64_t)c->n * 8 + 65536, (uint64_t)c->n * 2 + 65536));
    return BH_OK;
}

}  // namespace

// ====================================================================== ABI
extern "C" {

bh_status bh_create(bh_ctx **out, const bh_params *p) {
    if (!out) return BH_EINVAL;
    *out = nullptr;
    if (check_params(p) != BH_OK) return BH_EINVAL;
    bh_ctx *c = new (std::nothrow) bh_ctx();
    if (!c) return BH_ENOMEM;
    c->P = *p;
    c->n_grp_used = p->n_group > 0 ? p->n_group : 64;
    if (hipGetDevice(&c->device) != hipSuccess) {
        delete c;
        return BH_EHIP;
    }
    int ncu = 0;
    if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, c->device) == hipSuccess && ncu > 0)
        c->n_cu = ncu;
    c->walk_waves = (uint32_t)c->n_cu * 32;
    c->walk_waves_net = (uint32_t)c->n_cu * 16;
    bool ok = hipHostMalloc((void **)&c->h_cnt, sizeof(DevCounters)) == hipSuccess &&
              hipEventCreateWithFlags(&c->tab_ev, hipEventDisableTiming) == hipSuccess &&
              grow(c->counters, sizeof(DevCounters)) == hipSuccess;
    for (int k = 0; ok && k < EV_N; ++k)
        ok = hipEventCreate(&c->ev0[k]) == hipSuccess && hipEventCreate(&c->ev1[k]) == hipSuccess;
    ok = ok && hipStreamCreateWithFlags(&c->gs, hipStreamNonBlocking) == hipSuccess &&
         hipEventCreateWithFlags(&c->fence_a, hipEventDisableTiming) == hipSuccess &&
         hipEventCreateWithFlags(&c->fence_b, hipEventDisableTiming) == hipSuccess;
    if (!ok || ensure_walk(c) != BH_OK || ensure_learned(c) != BH_OK) {
        bh_destroy(c);
        return BH_ENOMEM;
    }
    // the device address of the allocation-free direct sum's static scratch on this GPU
    if (bhk::direct_static_init(c->device) != hipSuccess) {
        bh_destroy(c);
        return BH_EHIP;
    }
    (void)hipMemset(c->counters.p, 0, sizeof(DevCounters));
    *out = c;
    return BH_OK;
}

bh_status bh_destroy(bh_ctx *c) {
    if (!c) return BH_EINVAL;
    (void)hipDeviceSynchronize();
    DevBuf *all[] = {&c->sys_off_b, &c->sys_tab_b, &c->acc_tab_b, &c->box_b, &c->box_part_b, &c->sys_m0_b, &c->pos_in,
                     &c->vel_in, &c->idx_in, &c->pos, &c->vel, &c->acc, &c->idx, &c->inv, &c->key, &c->key_tmp,
                     &c->val, &c->val_tmp, &c->hist, &c->scan_tmp, &c->nd_prefix, &c->nd_begin, &c->nd_count,
                     &c->nd_first, &c->nd_meta, &c->nd_walk, &c->nd_mom, &c->nd_quad, &c->tmp_a, &c->tmp_b,
                     &c->gmark, &c->grp, &c->g_lo, &c->g_hi, &c->g_cen, &c->g_pc_off, &c->g_pc_len,
                     &c->g_pp_off, &c->g_pp_len, &c->g_cost, &c->order, &c->gkey_a, &c->gkey_b, &c->gval_a,
                     &c->gval_b, &c->pc_pool, &c->pp_pool, &c->walk_scratch, &c->counters, &c->direct_part,
                     &c->nd_qn, &c->amag, &c->amag_in, &c->g_amin, &c->g_rad, &c->cand, &c->mlp_w, &c->mlp_m,
                     &c->mlp_v, &c->mlp_g, &c->act, &c->ds_x, &c->ds_y, &c->ds_pairs, &c->pk_a, &c->pk_b,
                     &c->pv_a, &c->pv_b, &c->phist, &c->eval_out, &c->pos_b, &c->nd_mom_b, &c->nd_drift};
    for (DevBuf *b : all) release(*b);
    if (c->h_cnt) (void)hipHostFree(c->h_cnt);
    if (c->h_systab) (void)hipHostFree(c->h_systab);
    if (c->h_acctab) (void)hipHostFree(c->h_acctab);
    if (c->tab_ev) (void)hipEventDestroy(c->tab_ev);
    for (int k = 0; k < EV_N; ++k) {
        if (c->ev0[k]) (void)hipEventDestroy(c->ev0[k]);
        if (c->ev1[k]) (void)hipEventDestroy(c->ev1[k]);
    }
    for (auto &pr : c->force_ev) {
        (void)hipEventDestroy(pr.first);
        (void)hipEventDestroy(pr.second);
    }
    for (auto &g : c->graphs)
        if (g.exec) (void)hipGraphExecDestroy(g.exec);
    if (c->fence_a) (void)hipEventDestroy(c->fence_a);
    if (c->fence_b) (void)hipEventDestroy(c->fence_b);
    if (c->gs) (void)hipStreamDestroy(c->gs);
    delete c;
    return BH_OK;
}

bh_status bh_set_params(bh_ctx *c, const bh_params *p) {
    if (!c) return BH_EINVAL;
    if (check_params(p) != BH_OK) return fail(c, BH_EINVAL, "invalid parameters");
    int ng = p->n_group > 0 ? p->n_group : 64;
    // the tree depends on the leaf and group sizes (and group packing), on the
    // criterion (second moments) and on the coordinates it is built in
    if (ng != c->n_grp_used || p->n_leaf != c->P.n_leaf || p->criterion != c->P.criterion ||
        p->cyl_radius != c->P.cyl_radius || ((p->flags ^ c->P.flags) & BH_FLAG_PACK_GROUPS))
        c->tree_valid = false;
    // switching the drift monitor on needs a build snapshot: the tree is rebuilt first
    if (p->reuse_drift > 0.0 && !(c->P.reuse_drift > 0.0)) c->tree_valid = false;
    c->P = *p;
    c->n_grp_used = ng;
    c->lists_valid = false;
    STCHK(ensure_learned(c));
    STCHK(ensure_drift(c));
    return BH_OK;
}

bh_status bh_build_tree(bh_ctx *c, const bh_system *sys, int32_t n_sys, void *stream) {
    if (!c) return BH_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    c->tree_valid = c->lists_valid = c->state_valid = false;
    STCHK(set_systems(c, sys, n_sys, s));
    c->have_vel = true;
    for (int k = 0; k < n_sys; ++k) c->have_vel &= sys[k].vx && sys[k].vy && sys[k].vz;
    return rebuild(c, s, true);
}

bh_status bh_make_lists(bh_ctx *c, void *stream) {
    if (!c) return BH_EINVAL;
    return make_lists(c, (hipStream_t)stream);
}

bh_status bh_forces(bh_ctx *c, const bh_accel *out, void *stream) {
    if (!c) return BH_EINVAL;
    if (!c->lists_valid) return fail(c, BH_ESTATE, "bh_forces: no interaction lists (call bh_make_lists)");
    if (c->P.r_coll > 0.0 && !c->have_vel)
        return fail(c, BH_EINVAL, "bh_forces: the collision branch needs velocities in bh_build_tree");
    hipStream_t s = (hipStream_t)stream;
    bool pot = false;
    if (out)
        for (int k = 0; k < c->n_sys; ++k) {
            if (!out[k].ax || !out[k].ay || !out[k].az) return fail(c, BH_EINVAL, "null acceleration array");
            pot |= out[k].pot != nullptr;
        }
    refresh_state(c);
    STCHK(run_forces(c, s, pot || !out));
    c->state_valid = true;
    if (out) {
        STCHK(wait_tables(c));
        for (int k = 0; k < c->n_sys; ++k)
            c->h_acctab[k] = bhk::AccPtr{out[k].ax, out[k].ay, out[k].az, out[k].pot};
        HIPCHK(c, hipMemcpyAsync(c->acc_tab_b.p, c->h_acctab, c->n_sys * sizeof(bhk::AccPtr),
                                 hipMemcpyHostToDevice, s));
        HIPCHK(c, hipEventRecord(c->tab_ev, s));
        c->tab_ev_pending = true;
        bhk::scatter_acc(c->d, P<bhk::AccPtr>(c->acc_tab_b), s);
    }
    HIPCHK(c, hipGetLastError());
    return BH_OK;
}

}  // extern "C"

namespace {

// The integration loop shared by bh_step and bh_step_continue: kick-drift,
// then a new tree and lists when the current lists have served
// rebuild_every force evaluations, else moments refreshed on the same tree
// (Sec. 4.2, list-reusing steps), then forces and the closing kick.
bool same_key(const bh_ctx::GraphEntry &g, const DevState &d, double h, double dt) {
    return g.exec && g.h == h && g.dt == dt && std::memcmp(&g.key, &d, sizeof(DevState)) == 0;
}

// Kick-drift and moment refresh of a list-reusing step, from a cached graph
// (with the drift monitor on, dd carries its buffers: the counts are cleared
// by a kernel inside the graph and the moment pass measures the drift).
bh_status reuse_prefix_graph(bh_ctx *c, const DevState &dd, double h, double dt, hipStream_t s) {
    bh_ctx::GraphEntry *hit = nullptr;
    for (auto &g : c->graphs)
        if (same_key(g, dd, h, dt)) hit = &g;
    if (!hit) {
        hit = &c->graphs[c->graph_next];
        c->graph_next ^= 1;
        if (hit->exec) {
            HIPCHK(c, hipGraphExecDestroy(hit->exec));
            hit->exec = nullptr;
        }
        hipGraph_t graph = nullptr;
        HIPCHK(c, hipStreamBeginCapture(c->gs, hipStreamCaptureModeThreadLocal));
        bhk::kick_drift(dd, h, dt, c->gs);
        if (dd.nd_drift) bhk::drift_clear(dd, c->gs);
        bhk::moments(dd, c->gs);
        HIPCHK(c, hipStreamEndCapture(c->gs, &graph));
        hipError_t e = hipGraphInstantiate(&hit->exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        HIPCHK(c, e);
        std::memcpy(&hit->key, &dd, sizeof(DevState));
        hit->h = h;
        hit->dt = dt;
        c->graph_captures += 1;
    }
    HIPCHK(c, hipEventRecord(c->fence_a, s));
    HIPCHK(c, hipStreamWaitEvent(c->gs, c->fence_a, 0));
    HIPCHK(c, hipGraphLaunch(hit->exec, c->gs));
    HIPCHK(c, hipEventRecord(c->fence_b, c->gs));
    HIPCHK(c, hipStreamWaitEvent(s, c->fence_b, 0));
    c->graph_replays += 1;
    return BH_OK;
}

bh_status integrate(bh_ctx *c, double dt, int32_t n_steps, int32_t rebuild_every, hipStream_t s) {
    const double h = 0.5 * dt;
    const bool graphs = !(c->P.flags & BH_FLAG_NO_GRAPH);
    const bool monitor = c->P.reuse_drift > 0.0;
    for (int k = 0; k < n_steps; ++k) {
        if (c->age >= rebuild_every) {
            ev_begin(c, EV_INTEG, s);
            bhk::kick_drift(c->d, h, dt, s);
            ev_end(c, EV_INTEG, s);
            STCHK(rebuild(c, s, false));
            STCHK(make_lists(c, s));
        } else {
            refresh_state(c);
            DevState dd = c->d;
            if (monitor) dd.nd_drift = P<double>(c->nd_drift);
            if (graphs) {
                STCHK(reuse_prefix_graph(c, dd, h, dt, s));
            } else {
                ev_begin(c, EV_INTEG, s);
                bhk::kick_drift(dd, h, dt, s);
                ev_end(c, EV_INTEG, s);
                ev_begin(c, EV_MOM, s);
                if (monitor) bhk::drift_clear(dd, s);
                bhk::moments(dd, s);
                ev_end(c, EV_MOM, s);
            }
            if (monitor) {
                // Drift monitor: the lists are rebuilt before this force
                // evaluation when, at some tree level, the nodes whose particles
                // moved by more than reuse_drift times the node's side relative to
                // its centre of mass since the build hold more than reuse_frac of
                // the particles.
                STCHK(read_counters(c, s));
                uint32_t most = 0;
                for (int l = 0; l < BH_NLEVELS; ++l) most = std::max(most, c->h_cnt->stale[l]);
                if ((double)most > c->P.reuse_frac * (double)c->n) {
                    STCHK(rebuild(c, s, false));
                    STCHK(make_lists(c, s));
                    c->drift_rebuilds += 1;
                }
            }
        }
        refresh_state(c);
        // the closing kick rides in the force launch unless the collision
        // branch is on (its dashpot reads other particles' velocities)
        const bool fused = !(c->P.r_coll > 0.0);
        STCHK(run_forces(c, s, false, fused ? h : 0.0));
        if (!fused) bhk::kick(c->d, h, s);
    }
    bhk::scatter_state(c->d, s);
    HIPCHK(c, hipGetLastError());
    return BH_OK;
}

}  // namespace

extern "C" {

bh_status bh_step(bh_ctx *c, const bh_system *sys, int32_t n_sys, double dt, int32_t n_steps,
                  int32_t rebuild_every, void *stream) {
    if (!c) return BH_EINVAL;
    if (!std::isfinite(dt) || n_steps < 0 || rebuild_every < 1) return fail(c, BH_EINVAL, "bad step arguments");
    for (int k = 0; sys && k < n_sys; ++k)
        if (!sys[k].vx || !sys[k].vy || !sys[k].vz) return fail(c, BH_EINVAL, "bh_step needs velocities");
    hipStream_t s = (hipStream_t)stream;
    c->tree_valid = c->lists_valid = c->state_valid = false;
    // the step event pair stays balanced on every return
    auto body = [&]() -> bh_status {
        STCHK(set_systems(c, sys, n_sys, s));
        STCHK(rebuild(c, s, true));
        STCHK(make_lists(c, s));
        refresh_state(c);
        STCHK(run_forces(c, s, false));
        c->have_vel = true;
        c->state_valid = true;
        return integrate(c, dt, n_steps, rebuild_every, s);
    };
    ev_begin(c, EV_STEP, s);
    bh_status st = body();
    if (st != BH_OK) c->state_valid = false;
    ev_end(c, EV_STEP, s);
    return st;
}

bh_status bh_step_continue(bh_ctx *c, double dt, int32_t n_steps, int32_t rebuild_every, void *stream) {
    if (!c) return BH_EINVAL;
    if (!std::isfinite(dt) || n_steps < 0 || rebuild_every < 1) return fail(c, BH_EINVAL, "bad step arguments");
    if (!c->state_valid || !c->have_vel || !c->lists_valid)
        return fail(c, BH_ESTATE, "bh_step_continue: no integration state (call bh_step first)");
    hipStream_t s = (hipStream_t)stream;
    ev_begin(c, EV_STEP, s);
    refresh_state(c);
    bh_status st = integrate(c, dt, n_steps, rebuild_every, s);
    if (st != BH_OK) c->state_valid = false;
    ev_end(c, EV_STEP, s);
    return st;
}

bh_status bh_direct_sum(bh_ctx *c, const bh_system *sys, const int64_t *targets, int64_t n_targets, double *ax,
                        double *ay, double *az, void *stream) {
    if (!c || !sys) return BH_EINVAL;
    if (sys->n < 1 || !sys->x || !sys->y || !sys->z || !sys->m || n_targets < 0 || sys->n >= (1ll << 31))
        return fail(c, BH_EINVAL, "bh_direct_sum: bad system or targets");
    if (n_targets > 0 && (!targets || !ax || !ay || !az))
        return fail(c, BH_EINVAL, "bh_direct_sum: null target or output array");
    const bool coll = c->P.r_coll > 0.0;
    if (coll && (!sys->vx || !sys->vy || !sys->vz))
        return fail(c, BH_EINVAL, "bh_direct_sum: the collision branch needs velocities");
    if (n_targets == 0) return BH_OK;
    size_t need = bhk::direct_scratch_bytes(n_targets);
    HIPCHK(c, grow(c->direct_part, need));
    const bhk::Contact ct{c->P.r_coll, c->P.kappa, c->P.eta, sys->vx, sys->vy, sys->vz};
    bhk::direct_sum(sys->x, sys->y, sys->z, sys->m, sys->n, targets, n_targets, c->P.eps * c->P.eps, c->P.G,
                    coll ? &ct : nullptr, ax, ay, az, P<double>(c->direct_part), (hipStream_t)stream);
    HIPCHK(c, hipGetLastError());
    return BH_OK;
}

bh_status bh_direct_sum_static(bh_ctx *c, const bh_system *sys, const int64_t *targets, int64_t n_targets,
                               double *ax, double *ay, double *az, void *stream) {
    if (!c || !sys) return BH_EINVAL;
    if (sys->n < 1 || !sys->x || !sys->y || !sys->z || !sys->m || n_targets < 0 || sys->n >= (1ll << 31))
        return fail(c, BH_EINVAL, "bh_direct_sum_static: bad system or targets");
    if (n_targets > bhk::direct_static_max_targets())
        return fail(c, BH_EINVAL, "bh_direct_sum_static: more targets than its static scratch holds (4096)");
    if (n_targets > 0 && (!targets || !ax || !ay || !az))
        return fail(c, BH_EINVAL, "bh_direct_sum_static: null target or output array");
    const bool coll = c->P.r_coll > 0.0;
    if (coll && (!sys->vx || !sys->vy || !sys->vz))
        return fail(c, BH_EINVAL, "bh_direct_sum_static: the collision branch needs velocities");
    int dev = -1;
    HIPCHK(c, hipGetDevice(&dev));
    if (dev != c->device) return fail(c, BH_EINVAL, "bh_direct_sum_static: the context's device must be current");
    double *part = bhk::direct_static_scratch(dev);
    if (!part) return fail(c, BH_ESTATE, "bh_direct_sum_static: no static scratch on this device");
    if (n_targets == 0) return BH_OK;
    const bhk::Contact ct{c->P.r_coll, c->P.kappa, c->P.eta, sys->vx, sys->vy, sys->vz};
    bhk::direct_sum(sys->x, sys->y, sys->z, sys->m, sys->n, targets, n_targets, c->P.eps * c->P.eps, c->P.G,
                    coll ? &ct : nullptr, ax, ay, az, part, (hipStream_t)stream);
    HIPCHK(c, hipGetLastError());
    return BH_OK;
}

bh_status bh_sample_acc(bh_ctx *c, int32_t sys, const int64_t *targets, int64_t n_targets, double *ax, double *ay,
                        double *az, void *stream) {
    if (!c) return BH_EINVAL;
    if (!c->state_valid) return fail(c, BH_ESTATE, "bh_sample_acc: no force evaluation to read");
    if (sys < 0 || sys >= c->n_sys || n_targets < 0) return fail(c, BH_EINVAL, "bh_sample_acc: bad system or count");
    if (n_targets > 0 && (!targets || !ax || !ay || !az))
        return fail(c, BH_EINVAL, "bh_sample_acc: null target or output array");
    refresh_state(c);
    bhk::sample_acc(c->d, sys, targets, n_targets, ax, ay, az, (hipStream_t)stream);
    HIPCHK(c, hipGetLastError());
    return BH_OK;
}

bh_status bh_force_timing(bh_ctx *c, double *total_ms, int64_t *launches, int32_t reset) {
    if (!c) return BH_EINVAL;
    double tot = 0.0;
    for (size_t k = 0; k < c->force_ev_used; ++k) {
        HIPCHK(c, hipEventSynchronize(c->force_ev[k].second));
        float t = 0.f;
        HIPCHK(c, hipEventElapsedTime(&t, c->force_ev[k].first, c->force_ev[k].second));
        tot += t;
    }
    if (total_ms) *total_ms = tot;
    if (launches) *launches = (int64_t)c->force_ev_used;
    if (reset) c->force_ev_used = 0;
    return BH_OK;
}

bh_status bh_autotune(bh_ctx *c, const int32_t *cand, int32_t n_cand, int32_t rebuild_every, int32_t *chosen,
                      void *stream) {
    if (!c) return BH_EINVAL;
    if (!c->tree_valid) return fail(c, BH_ESTATE, "bh_autotune: no tree (call bh_build_tree first)");
    if (!cand || n_cand < 1 || rebuild_every < 1) return fail(c, BH_EINVAL, "bh_autotune: bad candidates");
    for (int k = 0; k < n_cand; ++k)
        if (cand[k] < 1 || cand[k] > 65536) return fail(c, BH_EINVAL, "bh_autotune: bad group size");
    hipStream_t s = (hipStream_t)stream;
    double best = 1e300;
    int best_g = cand[0], best_tile = c->P.force_tile;
    // the force kernel's tile (sources per LDS tile) is tried for each group
    // size where there is a choice: the FP32 gravity-only kernels
    std::vector<int> tiles{c->P.force_tile == 256 ? 256 : 512};
    if (c->P.precision == BH_FP32_REL && !(c->P.r_coll > 0.0)) tiles = {512, 256};
    for (int pass = 0; pass < 2; ++pass) {
        for (int k = 0; k < (pass == 0 ? n_cand : 1); ++k) {
            c->n_grp_used = pass == 0 ? cand[k] : best_g;
            refresh_state(c);
            bhk::regroup(c->d, s);
            bhk::make_groups(c->d, s);
            STCHK(read_counters(c, s));
            c->n_groups = c->h_cnt->n_groups;
            STCHK(make_lists(c, s));
            if (pass == 1) {
                c->P.force_tile = best_tile;
                refresh_state(c);
                STCHK(run_forces(c, s, false));
                break;
            }
            double ms[EV_N];
            STCHK(bh_stage_times(c, ms));
            const double walk_ms = ms[EV_WALK];
            for (int tile : tiles) {
                c->P.force_tile = tile;
                refresh_state(c);
                STCHK(run_forces(c, s, false));
                STCHK(bh_stage_times(c, ms));
                const double t = ms[EV_FORCE] + walk_ms / rebuild_every;
                if (t < best) {
                    best = t;
                    best_g = cand[k];
                    best_tile = tile;
                }
            }
        }
    }
    c->P.n_group = best_g;
    c->P.force_tile = best_tile;
    c->state_valid = false;
    if (chosen) *chosen = best_g;
    return BH_OK;
}

}  // extern "C"

namespace {

// Grow a device buffer keeping its first `keep` bytes.
hipError_t grow_keep(DevBuf &b, size_t bytes, size_t keep) {
    if (bytes <= b.bytes && b.p) return hipSuccess;
    void *p = nullptr;
    hipError_t e = hipMalloc(&p, bytes);
    if (e != hipSuccess) return e;
    if (b.p && keep) e = hipMemcpy(p, b.p, keep, hipMemcpyDeviceToDevice);
    if (b.p) (void)hipFree(b.p);
    b.p = p;
    b.bytes = bytes;
    return e;
}

uint64_t splitmix64(uint64_t &st) {
    uint64_t z = (st += 0x9e3779b97f4a7c15ull);
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

// He-uniform weights (bound sqrt(6 / fan_in)), zero biases, identity normalisation.
void init_weights(float *w, uint64_t seed) {
    uint64_t st = seed;
    auto uni = [&](double a) { return (float)(a * (2.0 * ((splitmix64(st) >> 11) * 0x1.0p-53) - 1.0)); };
    for (int k = 0; k < BH_MLP_NPARAM; ++k) w[k] = 0.0f;
    for (int k = 0; k < MLP_NH * MLP_NIN; ++k) w[MLP_W1 + k] = uni(std::sqrt(6.0 / MLP_NIN));
    for (int k = 0; k < MLP_NH * MLP_NH; ++k) w[MLP_W2 + k] = uni(std::sqrt(6.0 / MLP_NH));
    for (int k = 0; k < MLP_NH; ++k) w[MLP_W3 + k] = uni(std::sqrt(3.0 / MLP_NH));
    for (int k = 0; k < MLP_NIN; ++k) w[MLP_XISTD + k] = 1.0f;
    w[MLP_YSTD] = 1.0f;
}

bh_status ensure_mlp_train_buffers(bh_ctx *c, uint32_t B, uint64_t n) {
    HIPCHK(c, grow(c->mlp_m, MLP_NTRAIN * 4));
    HIPCHK(c, grow(c->mlp_v, MLP_NTRAIN * 4));
    HIPCHK(c, grow(c->mlp_g, (MLP_NTRAIN + 1) * 4));
    HIPCHK(c, grow(c->act, bhk::mlp_act_floats(B) * 4));
    HIPCHK(c, grow(c->pk_a, std::max<uint64_t>(n, B) * 8));
    HIPCHK(c, grow(c->pk_b, std::max<uint64_t>(n, B) * 8));
    HIPCHK(c, grow(c->pv_a, std::max<uint64_t>(n, B) * 4));
    HIPCHK(c, grow(c->pv_b, std::max<uint64_t>(n, B) * 4));
    HIPCHK(c, grow(c->phist, bhk::radix_hist_words((uint32_t)std::max<uint64_t>(n, B)) * 4));
    // the epoch shuffle's sort scans with it; a context that never built a
    // tree (training on a set from bh_mlp_set_dataset) has none yet
    HIPCHK(c, grow(c->scan_tmp, SCAN_TMP_WORDS * 4));
    return BH_OK;
}

}  // namespace

extern "C" {

bh_status bh_mlp_collect(bh_ctx *c, int32_t max_groups, int32_t count_cap, void *stream) {
    if (!c) return BH_EINVAL;
    if (c->P.criterion != BH_OPEN_LEARNED)
        return fail(c, BH_ESTATE, "bh_mlp_collect: context not created with the learned criterion");
    if (!c->tree_valid) return fail(c, BH_ESTATE, "bh_mlp_collect: no tree");
    if (max_groups < 1 || count_cap < 2) return fail(c, BH_EINVAL, "bh_mlp_collect: bad arguments");
    hipStream_t s = (hipStream_t)stream;
    if (!c->cand.p) {
        c->cand_cap = 1u << 22;
        HIPCHK(c, grow(c->cand, c->cand_cap * sizeof(uint2)));
    }
    c->group_stride = std::max<uint32_t>(1, (c->n_groups + max_groups - 1) / max_groups);
    c->count_cap = (uint32_t)count_cap;
    c->walk_mode = WALK_ENUMERATE;
    bh_status st = walk_until_fits(c, s);
    c->walk_mode = WALK_GEOMETRIC;
    c->lists_valid = false;
    c->state_valid = false;
    STCHK(st);
    const uint64_t nc = c->h_cnt->cand_used;
    const uint64_t need = c->ds_n + nc;
    if (need > c->ds_cap) {
        const uint64_t cap = need + need / 2 + 1024;
        HIPCHK(c, grow_keep(c->ds_x, cap * sizeof(float4), c->ds_n * sizeof(float4)));
        HIPCHK(c, grow_keep(c->ds_y, cap * 4, c->ds_n * 4));
        HIPCHK(c, grow_keep(c->ds_pairs, cap * sizeof(uint2), c->ds_n * sizeof(uint2)));
        c->ds_cap = cap;
    }
    refresh_state(c);
    bhk::cand_features_labels(c->d, nc, P<float4>(c->ds_x) + c->ds_n, P<float>(c->ds_y) + c->ds_n, s);
    HIPCHK(c, hipMemcpyAsync(P<uint2>(c->ds_pairs) + c->ds_n, c->cand.p, nc * sizeof(uint2),
                             hipMemcpyDeviceToDevice, s));
    STCHK(read_counters(c, s));
    if (c->h_cnt->flags[FLAG_CAND_BAD])
        return fail(c, BH_ECAPACITY, "bh_mlp_collect: a candidate pair named a group or node outside the tree "
                                     "or a node above the particle cap; nothing was added");
    c->ds_n = need;
    return BH_OK;
}

bh_status bh_mlp_train(bh_ctx *c, const bh_train_opts *o, double *mse, void *stream) {
    if (!c || !o) return BH_EINVAL;
    if (c->ds_n == 0) return fail(c, BH_ESTATE, "bh_mlp_train: empty training set (bh_mlp_collect)");
    if (o->iters < 0 || o->batch < 1 || o->batch > 65536 || !(o->lr > 0.f))
        return fail(c, BH_EINVAL, "bh_mlp_train: bad options");
    if (c->ds_n >= (1ull << 31)) return fail(c, BH_EINVAL, "bh_mlp_train: training set too large");
    hipStream_t s = (hipStream_t)stream;
    const uint64_t n = c->ds_n;
    const uint32_t B = (uint32_t)std::min<uint64_t>((uint64_t)o->batch, n);
    HIPCHK(c, grow(c->mlp_w, BH_MLP_NPARAM * 4));
    STCHK(ensure_mlp_train_buffers(c, B, n));
    float *w = P<float>(c->mlp_w);
    if (o->init || !c->mlp_ready) {
        std::vector<float> h(BH_MLP_NPARAM);
        init_weights(h.data(), o->seed);
        HIPCHK(c, hipMemcpyAsync(w, h.data(), BH_MLP_NPARAM * 4, hipMemcpyHostToDevice, s));
        bhk::mlp_stats(P<float4>(c->ds_x), P<float>(c->ds_y), n, w, s);
        HIPCHK(c, hipMemsetAsync(c->mlp_m.p, 0, MLP_NTRAIN * 4, s));
        HIPCHK(c, hipMemsetAsync(c->mlp_v.p, 0, MLP_NTRAIN * 4, s));
        HIPCHK(c, hipStreamSynchronize(s));
        c->adam_t = 0;
    }
    const uint64_t spe = std::max<uint64_t>(1, n / B);
    for (int it = 0; it < o->iters; ++it) {
        if ((uint64_t)it % spe == 0) {
            const uint64_t epoch = (uint64_t)it / spe;
            bhk::perm_keys(P<uint64_t>(c->pk_a), P<uint32_t>(c->pv_a), n, o->seed * 0x100000001b3ull + epoch, s);
            bhk::radix_sort(P<uint64_t>(c->pk_a), P<uint32_t>(c->pv_a), P<uint64_t>(c->pk_b), P<uint32_t>(c->pv_b),
                            (uint32_t)n, 0, 32, P<uint32_t>(c->phist), P<uint32_t>(c->scan_tmp), s, nullptr, 0);
        }
        const uint32_t *idx = P<uint32_t>(c->pv_a) + ((uint64_t)it % spe) * B;
        bhk::mlp_batch_grad(w, P<float4>(c->ds_x), P<float>(c->ds_y), idx, B, P<float>(c->act), P<float>(c->mlp_g),
                            nullptr, s);
        bhk::mlp_adam(w, P<float>(c->mlp_g), P<float>(c->mlp_m), P<float>(c->mlp_v), o->lr, o->beta1, o->beta2,
                      o->eps, ++c->adam_t, s);
    }
    HIPCHK(c, hipGetLastError());
    c->mlp_ready = true;
    c->lists_valid = false;
    if (mse) {
        HIPCHK(c, grow(c->eval_out, n * 4));
        bhk::mlp_eval(w, P<float4>(c->ds_x), n, P<float>(c->eval_out), s);
        std::vector<float> pr(n), y(n);
        HIPCHK(c, hipMemcpyAsync(pr.data(), c->eval_out.p, n * 4, hipMemcpyDeviceToHost, s));
        HIPCHK(c, hipMemcpyAsync(y.data(), c->ds_y.p, n * 4, hipMemcpyDeviceToHost, s));
        HIPCHK(c, hipStreamSynchronize(s));
        double acc = 0;
        for (uint64_t k = 0; k < n; ++k) acc += ((double)pr[k] - y[k]) * ((double)pr[k] - y[k]);
        *mse = acc / (double)n;
    }
    return BH_OK;
}

bh_status bh_mlp_weights(bh_ctx *c, float *get, const float *set) {
    if (!c) return BH_EINVAL;
    HIPCHK(c, grow(c->mlp_w, BH_MLP_NPARAM * 4));
    HIPCHK(c, hipDeviceSynchronize());
    if (get) HIPCHK(c, hipMemcpy(get, c->mlp_w.p, BH_MLP_NPARAM * 4, hipMemcpyDeviceToHost));
    if (set) {
        HIPCHK(c, hipMemcpy(c->mlp_w.p, set, BH_MLP_NPARAM * 4, hipMemcpyHostToDevice));
        // new weights start a new optimisation: Adam's moments and step count from zero
        HIPCHK(c, grow(c->mlp_m, MLP_NTRAIN * 4));
        HIPCHK(c, grow(c->mlp_v, MLP_NTRAIN * 4));
        HIPCHK(c, hipMemset(c->mlp_m.p, 0, MLP_NTRAIN * 4));
        HIPCHK(c, hipMemset(c->mlp_v.p, 0, MLP_NTRAIN * 4));
        c->adam_t = 0;
        c->mlp_ready = true;
        c->lists_valid = false;
    }
    return BH_OK;
}

bh_status bh_mlp_adam(bh_ctx *c, const float *grad, float lr, float beta1, float beta2, float eps, void *stream) {
    if (!c) return BH_EINVAL;
    if (!grad || !(lr > 0.f) || !(beta1 >= 0.f && beta1 < 1.f) || !(beta2 >= 0.f && beta2 < 1.f) || !(eps >= 0.f))
        return fail(c, BH_EINVAL, "bh_mlp_adam: bad arguments");
    if (!c->mlp_ready || !c->mlp_m.p || !c->mlp_v.p)
        return fail(c, BH_ESTATE, "bh_mlp_adam: no weights (bh_mlp_train or bh_mlp_weights)");
    bhk::mlp_adam(P<float>(c->mlp_w), grad, P<float>(c->mlp_m), P<float>(c->mlp_v), lr, beta1, beta2, eps,
                  ++c->adam_t, (hipStream_t)stream);
    c->lists_valid = false;
    HIPCHK(c, hipGetLastError());
    return BH_OK;
}

bh_status bh_mlp_dataset(bh_ctx *c, int64_t *n, uint32_t *pairs, float *x, float *y) {
    if (!c) return BH_EINVAL;
    if (n) *n = (int64_t)c->ds_n;
    if (c->ds_n == 0) return BH_OK;
    HIPCHK(c, hipDeviceSynchronize());
    if (pairs) HIPCHK(c, hipMemcpy(pairs, c->ds_pairs.p, c->ds_n * sizeof(uint2), hipMemcpyDeviceToHost));
    if (x) HIPCHK(c, hipMemcpy(x, c->ds_x.p, c->ds_n * sizeof(float4), hipMemcpyDeviceToHost));
    if (y) HIPCHK(c, hipMemcpy(y, c->ds_y.p, c->ds_n * 4, hipMemcpyDeviceToHost));
    return BH_OK;
}

bh_status bh_mlp_clear(bh_ctx *c) {
    if (!c) return BH_EINVAL;
    c->ds_n = 0;
    return BH_OK;
}

bh_status bh_mlp_set_dataset(bh_ctx *c, int64_t n, const uint32_t *pairs, const float *x, const float *y) {
    if (!c) return BH_EINVAL;
    if (n < 1 || n >= (1ll << 31) || !x || !y) return fail(c, BH_EINVAL, "bh_mlp_set_dataset: bad arguments");
    const uint64_t un = (uint64_t)n;
    HIPCHK(c, hipDeviceSynchronize());
    if (un > c->ds_cap) {
        // the set is empty until all three buffers hold the new size: a
        // failed allocation leaves no count that points past a buffer
        c->ds_n = 0;
        c->ds_cap = 0;
        HIPCHK(c, grow(c->ds_x, un * sizeof(float4)));
        HIPCHK(c, grow(c->ds_y, un * 4));
        HIPCHK(c, grow(c->ds_pairs, un * sizeof(uint2)));
        c->ds_cap = un;
    }
    HIPCHK(c, hipMemcpy(c->ds_x.p, x, un * sizeof(float4), hipMemcpyHostToDevice));
    HIPCHK(c, hipMemcpy(c->ds_y.p, y, un * 4, hipMemcpyHostToDevice));
    if (pairs)
        HIPCHK(c, hipMemcpy(c->ds_pairs.p, pairs, un * sizeof(uint2), hipMemcpyHostToDevice));
    else
        HIPCHK(c, hipMemset(c->ds_pairs.p, 0, un * sizeof(uint2)));
    c->ds_n = un;
    return BH_OK;
}

bh_status bh_mlp_predict(bh_ctx *c, const float *x, int64_t n, float *out, void *stream) {
    if (!c || (n > 0 && (!x || !out)) || n < 0) return BH_EINVAL;
    if (!c->mlp_ready) return fail(c, BH_ESTATE, "bh_mlp_predict: no weights (bh_mlp_train or bh_mlp_weights)");
    bhk::mlp_eval(P<float>(c->mlp_w), reinterpret_cast<const float4 *>(x), (uint64_t)n, out, (hipStream_t)stream);
    HIPCHK(c, hipGetLastError());
    return BH_OK;
}

bh_status bh_mlp_gradient(bh_ctx *c, const float *x, const float *y, int32_t B, float *grad, float *loss,
                          void *stream) {
    if (!c || !x || !y || !grad || B < 1 || B > 65536) return BH_EINVAL;
    if (!c->mlp_ready) return fail(c, BH_ESTATE, "bh_mlp_gradient: no weights (bh_mlp_train or bh_mlp_weights)");
    hipStream_t s = (hipStream_t)stream;
    STCHK(ensure_mlp_train_buffers(c, (uint32_t)B, (uint64_t)B));
    bhk::perm_keys(P<uint64_t>(c->pk_a), P<uint32_t>(c->pv_a), (uint64_t)B, 0, s);   // identity order
    bhk::mlp_batch_grad(P<float>(c->mlp_w), reinterpret_cast<const float4 *>(x), y, P<uint32_t>(c->pv_a),
                        (uint32_t)B, P<float>(c->act), grad, loss, s);
    HIPCHK(c, hipGetLastError());
    return BH_OK;
}

bh_status bh_query(const bh_ctx *c, bh_sizes *o) {
    if (!c || !o) return BH_EINVAL;
    o->n_particles = c->n;
    o->n_systems = c->n_sys;
    o->max_level = (int32_t)c->max_level;
    o->n_nodes = c->tree_valid ? c->n_nodes : 0;
    o->n_groups = c->tree_valid ? c->n_groups : 0;
    o->n_pc = c->lists_valid ? (int64_t)c->n_pc : 0;
    o->n_pp = c->lists_valid ? (int64_t)c->n_pp : 0;
    o->interactions = c->lists_valid ? (int64_t)c->interactions : 0;
    o->n_group_used = c->n_grp_used;
    o->lists_valid = c->lists_valid ? 1 : 0;
    o->interactions_evaluated = c->interactions_evaluated;
    o->force_evaluations = c->force_evaluations;
    o->tree_builds = c->tree_builds;
    o->drift_rebuilds = c->drift_rebuilds;
    o->host_syncs = c->host_syncs;
    o->force_tile = c->P.force_tile == 256 ? 256 : 512;
    return BH_OK;
}

bh_status bh_export(bh_ctx *c, int32_t what, void *dst, void *stream) {
    if (!c || !dst) return BH_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    HIPCHK(c, hipStreamSynchronize(s));
    const size_t n = c->n, nn = c->n_nodes, ng = c->n_groups;
    switch (what) {
    case BH_EXPORT_KEYS:
        if (!c->tree_valid) return fail(c, BH_ESTATE, "no tree");
        HIPCHK(c, hipMemcpy(dst, c->key.p, n * 8, hipMemcpyDeviceToHost));
        return BH_OK;
    case BH_EXPORT_PERM: {
        if (!c->tree_valid) return fail(c, BH_ESTATE, "no tree");
        uint32_t *o = (uint32_t *)dst;
        HIPCHK(c, hipMemcpy(o, c->idx.p, n * 4, hipMemcpyDeviceToHost));
        for (size_t j = 0; j < n; ++j) {
            auto it = std::upper_bound(c->sys_off.begin(), c->sys_off.end(), o[j]);
            o[j] -= *(it - 1);
        }
        return BH_OK;
    }
    case BH_EXPORT_NODES: {
        if (!c->tree_valid) return fail(c, BH_ESTATE, "no tree");
        std::vector<uint64_t> pf(nn);
        std::vector<uint32_t> b(nn), cn(nn), f(nn), m(nn);
        HIPCHK(c, hipMemcpy(pf.data(), c->nd_prefix.p, nn * 8, hipMemcpyDeviceToHost));
        HIPCHK(c, hipMemcpy(b.data(), c->nd_begin.p, nn * 4, hipMemcpyDeviceToHost));
        HIPCHK(c, hipMemcpy(cn.data(), c->nd_count.p, nn * 4, hipMemcpyDeviceToHost));
        HIPCHK(c, hipMemcpy(f.data(), c->nd_first.p, nn * 4, hipMemcpyDeviceToHost));
        HIPCHK(c, hipMemcpy(m.data(), c->nd_meta.p, nn * 4, hipMemcpyDeviceToHost));
        int64_t *o = (int64_t *)dst;
        for (size_t v = 0; v < nn; ++v) {
            o[8 * v + 0] = meta_level(m[v]);
            o[8 * v + 1] = meta_sys(m[v]);
            o[8 * v + 2] = (int64_t)pf[v];
            o[8 * v + 3] = b[v];
            o[8 * v + 4] = cn[v];
            o[8 * v + 5] = f[v];
            o[8 * v + 6] = meta_nch(m[v]);
            o[8 * v + 7] = meta_group(m[v]);
        }
        return BH_OK;
    }
    case BH_EXPORT_MOMENTS:
        if (!c->tree_valid) return fail(c, BH_ESTATE, "no tree");
        HIPCHK(c, hipMemcpy(dst, c->nd_mom.p, nn * sizeof(double4), hipMemcpyDeviceToHost));
        return BH_OK;
    case BH_EXPORT_GROUPS: {
        if (!c->tree_valid) return fail(c, BH_ESTATE, "no tree");
        std::vector<GroupInfo> g(ng);
        HIPCHK(c, hipMemcpy(g.data(), c->grp.p, ng * sizeof(GroupInfo), hipMemcpyDeviceToHost));
        int64_t *o = (int64_t *)dst;
        for (size_t k = 0; k < ng; ++k) {
            o[4 * k + 0] = g[k].node;
            o[4 * k + 1] = g[k].begin;
            o[4 * k + 2] = g[k].count;
            o[4 * k + 3] = g[k].sys;
        }
        return BH_OK;
    }
    case BH_EXPORT_LISTS: {
        if (!c->lists_valid) return fail(c, BH_ESTATE, "no lists");
        std::vector<uint64_t> po(ng), qo(ng);
        std::vector<uint32_t> pl(ng), ql(ng);
        std::vector<uint32_t> pcp(c->n_pc), ppp(c->n_pp);
        HIPCHK(c, hipMemcpy(po.data(), c->g_pc_off.p, ng * 8, hipMemcpyDeviceToHost));
        HIPCHK(c, hipMemcpy(pl.data(), c->g_pc_len.p, ng * 4, hipMemcpyDeviceToHost));
        HIPCHK(c, hipMemcpy(qo.data(), c->g_pp_off.p, ng * 8, hipMemcpyDeviceToHost));
        HIPCHK(c, hipMemcpy(ql.data(), c->g_pp_len.p, ng * 4, hipMemcpyDeviceToHost));
        if (c->n_pc) HIPCHK(c, hipMemcpy(pcp.data(), c->pc_pool.p, c->n_pc * 4, hipMemcpyDeviceToHost));
        if (c->n_pp) HIPCHK(c, hipMemcpy(ppp.data(), c->pp_pool.p, c->n_pp * 4, hipMemcpyDeviceToHost));
        int64_t *pc_off = (int64_t *)dst;
        int64_t *pp_off = pc_off + ng + 1;
        uint32_t *pc = (uint32_t *)(pp_off + ng + 1);
        uint32_t *pp = pc + c->n_pc;
        pc_off[0] = pp_off[0] = 0;
        for (size_t k = 0; k < ng; ++k) {
            std::copy(pcp.begin() + po[k], pcp.begin() + po[k] + pl[k], pc + pc_off[k]);
            std::copy(ppp.begin() + qo[k], ppp.begin() + qo[k] + ql[k], pp + pp_off[k]);
            pc_off[k + 1] = pc_off[k] + pl[k];
            pp_off[k + 1] = pp_off[k] + ql[k];
        }
        return BH_OK;
    }
    case BH_EXPORT_ACC_SORTED:
        if (!c->state_valid) return fail(c, BH_ESTATE, "no accelerations");
        HIPCHK(c, hipMemcpy(dst, c->acc.p, n * sizeof(double4), hipMemcpyDeviceToHost));
        return BH_OK;
    case BH_EXPORT_SORTED_POS:
        if (!c->n) return fail(c, BH_ESTATE, "no particles");
        HIPCHK(c, hipMemcpy(dst, c->pos.p, n * sizeof(double4), hipMemcpyDeviceToHost));
        return BH_OK;
    case BH_EXPORT_QUAD:
        if (!c->tree_valid || c->P.criterion != BH_OPEN_LEARNED) return fail(c, BH_ESTATE, "no second moments");
        HIPCHK(c, hipMemcpy(dst, c->nd_quad.p, nn * 6 * sizeof(double), hipMemcpyDeviceToHost));
        return BH_OK;
    case BH_EXPORT_NODE_QN:
        if (!c->tree_valid || c->P.criterion != BH_OPEN_LEARNED) return fail(c, BH_ESTATE, "no node features");
        HIPCHK(c, hipMemcpy(dst, c->nd_qn.p, nn * 4, hipMemcpyDeviceToHost));
        return BH_OK;
    case BH_EXPORT_GROUP_EXTRA: {
        if (!c->tree_valid || c->P.criterion != BH_OPEN_LEARNED) return fail(c, BH_ESTATE, "no group extras");
        std::vector<double> r(ng), a(ng);
        HIPCHK(c, hipMemcpy(r.data(), c->g_rad.p, ng * 8, hipMemcpyDeviceToHost));
        HIPCHK(c, hipMemcpy(a.data(), c->g_amin.p, ng * 8, hipMemcpyDeviceToHost));
        double *o = (double *)dst;
        for (size_t k = 0; k < ng; ++k) {
            o[2 * k] = r[k];
            o[2 * k + 1] = a[k];
        }
        return BH_OK;
    }
    case BH_EXPORT_DRIFT:
        if (!c->tree_valid || !(c->P.reuse_drift > 0.0)) return fail(c, BH_ESTATE, "no drift monitor");
        HIPCHK(c, hipMemcpy(dst, c->nd_drift.p, nn * sizeof(double), hipMemcpyDeviceToHost));
        return BH_OK;
    case BH_EXPORT_ROOT_BOX:
        if (!c->tree_valid) return fail(c, BH_ESTATE, "no tree");
        HIPCHK(c, hipMemcpy(dst, c->box_b.p, (size_t)c->n_sys * sizeof(double4), hipMemcpyDeviceToHost));
        return BH_OK;
    default:
        return fail(c, BH_EINVAL, "unknown export item");
    }
}

bh_status bh_export_groups(bh_ctx *c, int32_t *box, double *centre, void *stream) {
    if (!c) return BH_EINVAL;
    if (!c->tree_valid) return fail(c, BH_ESTATE, "no tree");
    HIPCHK(c, hipStreamSynchronize((hipStream_t)stream));
    const size_t ng = c->n_groups;
    if (box) {
        std::vector<int4> lo(ng), hi(ng);
        HIPCHK(c, hipMemcpy(lo.data(), c->g_lo.p, ng * sizeof(int4), hipMemcpyDeviceToHost));
        HIPCHK(c, hipMemcpy(hi.data(), c->g_hi.p, ng * sizeof(int4), hipMemcpyDeviceToHost));
        for (size_t k = 0; k < ng; ++k) {
            int32_t *o = box + 6 * k;
            o[0] = lo[k].x; o[1] = lo[k].y; o[2] = lo[k].z;
            o[3] = hi[k].x; o[4] = hi[k].y; o[5] = hi[k].z;
        }
    }
    if (centre) {
        std::vector<double4> cc(ng);
        HIPCHK(c, hipMemcpy(cc.data(), c->g_cen.p, ng * sizeof(double4), hipMemcpyDeviceToHost));
        for (size_t k = 0; k < ng; ++k) {
            centre[3 * k] = cc[k].x;
            centre[3 * k + 1] = cc[k].y;
            centre[3 * k + 2] = cc[k].z;
        }
    }
    return BH_OK;
}

bh_status bh_stage_times(bh_ctx *c, double *ms) {
    if (!c || !ms) return BH_EINVAL;
    for (int k = 0; k < EV_N; ++k) {
        ms[k] = 0.0;
        if (!c->ev_used[k]) continue;
        HIPCHK(c, hipEventSynchronize(c->ev1[k]));
        float t = 0.f;
        HIPCHK(c, hipEventElapsedTime(&t, c->ev0[k], c->ev1[k]));
        ms[k] = t;
    }
    return BH_OK;
}

const char *bh_last_error(const bh_ctx *c) {
    return c ? c->err.c_str() : "null context";
}

}  // extern "C"
