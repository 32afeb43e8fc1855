// bh_internal.hpp -- device helpers and host launchers shared by the HIP
// translation units of the Barnes-Hut library (not part of the public ABI).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#define BH_MAXLEVEL 21          // 21 bits per axis, 63-bit keys
#define BH_NLEVELS 22           // levels 0..21
#define BH_WAVE 64

// ---------------------------------------------------------------- errors
// Device-side flags, one word each, in a small array the host reads back.
enum {
    FLAG_NONFINITE = 0,         // a coordinate was NaN or Inf
    FLAG_NODE_OVF = 1,          // node capacity exceeded
    FLAG_WALK_OVF = 2,          // a walk frontier/list scratch overflowed
    FLAG_POOL_OVF = 3,          // list pool capacity exceeded
    FLAG_EXTENT = 4,            // cylindrical tree coordinates exceed the root cell
    FLAG_WALK_BOUND = 5,        // a walk went deeper than the tree's levels or visited more nodes than exist
    FLAG_CAND_BAD = 6,          // a training candidate named a group or node outside the tree, or too many particles
    FLAG_COUNT = 8
};

// Device counters written by kernels and read back by the host.
struct DevCounters {
    uint32_t flags[FLAG_COUNT];
    uint32_t lvl_off[BH_NLEVELS + 2];   // node-id range of each level
    uint32_t n_groups;
    uint32_t max_level;
    unsigned long long pc_used;         // list-pool fill (may exceed capacity: overflow)
    unsigned long long pp_used;
    unsigned long long interactions;
    uint32_t walk_need_front;           // largest frontier seen
    uint32_t walk_need_list;            // longest list seen
    uint32_t work_counter;              // persistent-kernel work queue head
    uint32_t work_counter2;
    uint32_t pad[4];
    unsigned long long cand_used;       // learned rule: candidate pairs recorded (may exceed capacity)
    uint32_t work_counter3;
    uint32_t pad2;
    uint32_t stale[BH_NLEVELS];         // drift monitor: particles in drifted nodes, per level
};

// ---------------------------------------------------------------- wave helpers
__device__ __forceinline__ int lane_id() { return __lane_id(); }

__device__ __forceinline__ uint64_t lanemask_lt() {
    int l = __lane_id();
    return (l == 0) ? 0ull : (~0ull >> (64 - l));
}

// inclusive prefix sum over the 64 lanes of a wave
template <typename T>
__device__ __forceinline__ T wave_incl_scan(T v) {
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        T u = __shfl_up(v, d, 64);
        if (__lane_id() >= d) v += u;
    }
    return v;
}

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
    return v;
}

template <typename T>
__device__ __forceinline__ T wave_min(T v) {
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) {
        T u = __shfl_xor(v, d, 64);
        v = u < v ? u : v;
    }
    return v;
}

template <typename T>
__device__ __forceinline__ T wave_max(T v) {
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) {
        T u = __shfl_xor(v, d, 64);
        v = u > v ? u : v;
    }
    return v;
}

// Morton helpers: 21 bits per axis, x the most significant bit of each triple.
__host__ __device__ __forceinline__ uint64_t spread3(uint32_t v) {
    uint64_t x = v & 0x1fffffull;
    x = (x | (x << 32)) & 0x1f00000000ffffull;
    x = (x | (x << 16)) & 0x1f0000ff0000ffull;
    x = (x | (x << 8)) & 0x100f00f00f00f00full;
    x = (x | (x << 4)) & 0x10c30c30c30c30c3ull;
    x = (x | (x << 2)) & 0x1249249249249249ull;
    return x;
}

__host__ __device__ __forceinline__ uint32_t compact3(uint64_t x) {
    x &= 0x1249249249249249ull;
    x = (x | (x >> 2)) & 0x10c30c30c30c30c3ull;
    x = (x | (x >> 4)) & 0x100f00f00f00f00full;
    x = (x | (x >> 8)) & 0x1f0000ff0000ffull;
    x = (x | (x >> 16)) & 0x1f00000000ffffull;
    x = (x | (x >> 32)) & 0x1fffffull;
    return (uint32_t)x;
}

// ---------------------------------------------------------------- device state
// Caller pointers of one system, as a device-side table.
struct SysPtr {
    double *x, *y, *z, *vx, *vy, *vz;
    const double *m;
    int64_t n;
};

// Node meta word: level (5 bits) | n_child (4 bits) << 5 | is_group << 9 | system << 10
__host__ __device__ __forceinline__ uint32_t meta_level(uint32_t m) { return m & 31u; }
__host__ __device__ __forceinline__ uint32_t meta_nch(uint32_t m) { return (m >> 5) & 15u; }
__host__ __device__ __forceinline__ uint32_t meta_group(uint32_t m) { return (m >> 9) & 1u; }
__host__ __device__ __forceinline__ uint32_t meta_sys(uint32_t m) { return m >> 10; }
__host__ __device__ __forceinline__ uint32_t make_meta(uint32_t lvl, uint32_t nch, uint32_t grp, uint32_t sys) {
    return lvl | (nch << 5) | (grp << 9) | (sys << 10);
}

// Per-group record: node id, first particle, particle count, system.
struct GroupInfo {
    uint32_t node, begin, count, sys;
};

// Raw device pointers of a context, passed by value to the launchers.
struct DevState {
    // systems
    int n_sys;
    uint32_t n;                    // particles over all systems
    const uint32_t *sys_off;       // [n_sys+1]
    const SysPtr *sys_tab;         // [n_sys]
    double4 *box;                  // [n_sys]: lo x, y, z, 2^21 / S
    double *box_part;              // [n_sys][box_blocks][8]: min, max of the tree coordinates and of the mass
    uint32_t box_blocks;           // root-box partial blocks per system (1..BOX_BLOCKS_MAX)
    double *sys_m0;                // [n_sys] the common particle mass of a system, 0 when masses differ
    // particles: input order of the current build and sorted order
    double4 *pos_in, *vel_in;
    uint32_t *idx_in;
    double4 *pos, *vel, *acc;      // sorted: (x,y,z,m), (vx,vy,vz,0), (ax,ay,az,pot)
    uint32_t *idx;                 // sorted slot -> global caller index
    uint32_t *inv;                 // global caller index -> sorted slot (the inverse of idx)
    uint64_t *key, *key_tmp;
    uint32_t *val, *val_tmp, *hist, *scan_tmp;
    // tree
    uint32_t node_cap;
    uint64_t *nd_prefix;
    uint32_t *nd_begin, *nd_count, *nd_first, *nd_meta;
    int4 *nd_walk;                 // corner x | level << 24, corner y | n_child << 24, corner z, first child
    double4 *nd_mom;               // com x, y, z, mass
    double *nd_quad;               // [node_cap][6] second moments (learned rule only), may be null
    uint32_t *tmp_a, *tmp_b;       // [node_cap] level scratch
    // groups
    uint32_t *gmark;               // [n] particle marks, then group index
    GroupInfo *grp;                // [n] (capacity: one per particle)
    int4 *g_lo, *g_hi;             // grid box, half-open
    double4 *g_cen;
    // lists
    unsigned long long *g_pc_off, *g_pp_off;   // list starts in the pools (64-bit: pools exceed 2^32)
    uint32_t *g_pc_len, *g_pp_len;
    unsigned long long *g_cost;    // interactions of the group
    uint32_t *order;               // groups by descending cost
    uint32_t *pc_pool, *pp_pool;
    unsigned long long pc_cap, pp_cap;
    uint32_t *walk_scratch;        // per walking wave: 2 frontiers + 2 lists
    uint32_t walk_front_cap, walk_list_cap, walk_waves;
    uint32_t walk_waves_net;       // walking waves of the learned and enumerating rules
    DevCounters *cnt;
    // learned opening rule
    int walk_mode;                 // WALK_GEOMETRIC, WALK_LEARNED, WALK_ENUMERATE
    double th2_min, th2_max, tau;  // band of the learned rule and its error budget
    const float *mlp;              // MLP_NPARAM weights
    float *nd_qn;                  // [node_cap] second-moment feature
    double *amag, *amag_in;        // [n] |self-gravity acceleration| of the last evaluation (sorted / staging)
    double *g_amin;                // [groups] mean amag of the group (error budget scale)
    double *g_rad;                 // [groups] half-diagonal of the group's FP64 bounding box
    uint2 *cand;                   // (group, node) candidate pairs recorded by the enumerating walk
    unsigned long long cand_cap;
    uint32_t group_stride;         // enumerating walk: record pairs of every group_stride-th group
    uint32_t count_cap;            // nodes with more particles use the geometric rule
    // parameters
    int n_leaf, n_grp;
    double th2;                    // theta * theta
    double eps2, G, central_mass;
    double rc, kappa, eta;         // collision branch of Eq. (2); rc = 0: off
    double cyl_r;                  // tree on cylindrical coordinates around this radius; 0: Cartesian
    // drift monitor of list-reusing steps (off when nd_drift is null)
    double4 *pos_b, *nd_mom_b;     // sorted positions and node moments at the last tree build
    double *nd_drift;              // [node_cap] drift of each node since the build
    double drift_kappa;            // a node has drifted when its drift exceeds drift_kappa * side
    int force_tile;                // sources per LDS tile of the FP32 gravity force kernel: 256 or 512
    int budget_min;                // learned rule: A_g is the smallest |a| of the group (else the mean)
    int pack_groups;               // groups are packs of consecutive small siblings (else single nodes)
};

// The learned rule's error budget scale A_g of a group, by one wave: the mean
// (default) or the smallest (budget_min) self-gravity |a| of its particles
// from the last force evaluation.
__device__ __forceinline__ double group_budget(const DevState &d, const GroupInfo &gi) {
    double a = d.budget_min ? 1.7976931348623157e308 : 0.0;
    for (uint32_t i = gi.begin + __lane_id(); i < gi.begin + gi.count; i += 64)
        a = d.budget_min ? fmin(a, d.amag[i]) : a + d.amag[i];
    return d.budget_min ? wave_min(a) : wave_sum(a) / (double)gi.count;
}

enum { WALK_GEOMETRIC = 0, WALK_LEARNED = 1, WALK_ENUMERATE = 2 };

// root-box reduction: blocks per system, at most BOX_BLOCKS_MAX, about
// BOX_PER_BLOCK particles each for the average system
constexpr uint32_t BOX_BLOCKS_MAX = 1024, BOX_PER_BLOCK = 1024;

// ---------------------------------------------------------------- host launchers
namespace bhk {

// tree build (bh_tree.hip)
void load_systems(const DevState &d, hipStream_t s);
void root_box_keys(const DevState &d, hipStream_t s);
void permute(const DevState &d, hipStream_t s);
void build_octree(const DevState &d, hipStream_t s);
void moments(const DevState &d, hipStream_t s);
void make_groups(const DevState &d, hipStream_t s);
// drift monitor: keep the build's positions and moments (after a build) and
// clear the per-level counts (before each monitored moment pass)
void drift_snapshot(const DevState &d, hipStream_t s);
void drift_clear(const DevState &d, hipStream_t s);
void reset_flags(const DevState &d, hipStream_t s);
void regroup(const DevState &d, hipStream_t s);   // group flags for d.n_grp on the current tree

// lists (bh_walk.hip)
void walk(const DevState &d, hipStream_t s);
void order_groups(const DevState &d, uint32_t n_groups, uint64_t *key_a, uint32_t *val_a, uint64_t *key_b,
                  uint32_t *val_b, hipStream_t s);

// forces (bh_force.hip): blocks = persistent workgroups
// kick_h != 0 (no collision branch): the closing half kick v += kick_h a is
// applied in the same launch; with the collision branch it is ignored.
void forces(const DevState &d, uint32_t n_groups, bool fp32, bool pot, int blocks, double kick_h, hipStream_t s);

// integration and caller-order output (bh_integrate.hip)
struct AccPtr {
    double *ax, *ay, *az, *pot;
};
void kick_drift(const DevState &d, double h, double dt, hipStream_t s);
void kick(const DevState &d, double h, hipStream_t s);
void scatter_state(const DevState &d, hipStream_t s);
void scatter_acc(const DevState &d, const AccPtr *tab, hipStream_t s);
void sample_acc(const DevState &d, int sys, const int64_t *targets, int64_t nt, double *ax, double *ay, double *az,
                hipStream_t s);

// learned opening rule (bh_learned.hip)
void node_qn(const DevState &d, hipStream_t s);
void group_amin(const DevState &d, hipStream_t s);
void cand_features_labels(const DevState &d, uint64_t n_cand, float4 *X, float *Y, hipStream_t s);
void mlp_stats(const float4 *X, const float *Y, uint64_t n, float *w, hipStream_t s);
void mlp_batch_grad(const float *w, const float4 *X, const float *Y, const uint32_t *idx, uint32_t B,
                    float *act, float *grad, float *loss, hipStream_t s);
void mlp_adam(float *w, const float *grad, float *m, float *v, float lr, float b1, float b2, float eps,
              int step, hipStream_t s);
void mlp_eval(const float *w, const float4 *X, uint64_t n, float *out, hipStream_t s);
void perm_keys(uint64_t *key, uint32_t *val, uint64_t n, uint64_t seed, hipStream_t s);

// FP64 direct summation for sampled targets (bh_direct.hip)
// Collision branch of Eq. (2) for the direct sum: radius, spring, dashpot and
// the caller-order velocities of the system.
struct Contact {
    double rc, kappa, eta;
    const double *vx, *vy, *vz;
};
size_t direct_scratch_bytes(int64_t n_targets);
// The allocation-free variant's scratch: a static device array per GPU.
// direct_static_init (with that device current) looks up its address once;
// direct_static_scratch returns it (nullptr before the lookup).
int64_t direct_static_max_targets();
hipError_t direct_static_init(int device);
double *direct_static_scratch(int device);
void direct_sum(const double *x, const double *y, const double *z, const double *m, int64_t n,
                const int64_t *targets, int64_t nt, double eps2, double G, const Contact *contact, double *ax,
                double *ay, double *az, double *scratch, hipStream_t s);

// exclusive scan of n uint32 (n from *n_dev when n_dev != nullptr, else n_host);
// out may alias in.  *total (if non-null) receives the sum.  tmp: >= 1024 words.
void scan_u32(const uint32_t *in, uint32_t *out, const uint32_t *n_dev, uint32_t n_host,
              uint32_t *total, uint32_t *tmp, hipStream_t s);

// fill n words with v (graph-safe replacement for hipMemsetAsync)
void fill_u32(uint32_t *p, uint32_t v, size_t n, hipStream_t s);

// Stable LSD radix sort of (key, val) pairs by key bits [lo_bit, hi_bit),
// then (when sys_off != nullptr and n_sys > 1) by the system owning input
// index val (sys_off: device array of n_sys+1 offsets), so the result is in
// (system, key, input order).  Result in key_a/val_a.  Scratch: key_b/val_b
// of n, hist of radix_hist_words(n).
size_t radix_hist_words(uint32_t n);
void radix_sort(uint64_t *key_a, uint32_t *val_a, uint64_t *key_b, uint32_t *val_b,
                uint32_t n, int lo_bit, int hi_bit, uint32_t *hist, uint32_t *tmp, hipStream_t s,
                const uint32_t *sys_off, int n_sys);

}  // namespace bhk
