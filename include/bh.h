/*
 * bh.h -- C ABI of the Barnes-Hut gravity library for one MI355X (gfx950).
 *
 * The calls follow the steps of one timestep of a self-gravitating particle
 * code as Iwasawa et al. (2019), Sec. 4.2, lists them for one domain:
 *   bh_build_tree   step (3a)/(3c): keys, sort, octree and node moments
 *   bh_make_lists   step (3d), first half: per-group tree walk that writes
 *                   the group's particle list and node list
 *   bh_forces       step (3d), second half: double loop over the group's
 *                   particles and its list, with the gravity branch of
 *                   Eq. (2) softened by a Plummer eps, nodes as point
 *                   masses at their centre of mass (Sec. 5.1); optionally
 *                   the collision branch of Eq. (2) for particle pairs
 *   bh_step         step (4) plus the persistent interaction list of
 *                   Sec. 4.2: lists are kept for `rebuild_every` steps while
 *                   node moments are recomputed from the moved particles
 *                   every step.  The integrator runs inside the library, next
 *                   to the particle data (Sec. 6.1).
 *
 * Memory and ownership
 *   - Particle arrays (bh_system) are DEVICE pointers owned by the caller,
 *     FP64, structure-of-arrays, one entry per particle in the caller's
 *     order.  The library reads and writes them only inside the calls
 *     that take them, with one exception: bh_step_continue writes its
 *     results to the arrays of the bh_step (or bh_build_tree) that started
 *     the integration.
 *   - The context owns every derived structure (sorted copy of the
 *     particles, keys, tree, groups, lists, scratch) in device memory it
 *     allocates itself.  bh_destroy frees it.
 *   - `stream` is a hipStream_t (passed as void*); all device work of a call
 *     is enqueued on it.  bh_build_tree, bh_make_lists and bh_step
 *     synchronise that stream once per tree build to read back sizes and
 *     error flags; bh_forces does not synchronise.
 *
 * Errors
 *   Every call returns a bh_status and never throws.  On failure the context
 *   keeps a message readable with bh_last_error.  Non-finite coordinates or
 *   an empty system give BH_EINVAL.  Calls out of order (bh_forces before
 *   bh_make_lists) give BH_ESTATE.  Internal buffers that turn out too small
 *   are grown and the stage redone; BH_ENOMEM is returned only when the
 *   device allocation itself fails.  A HIP runtime error gives BH_EHIP.
 *
 * Several independent systems may be handled by one context (one call, one
 * launch per stage); each keeps its own root cell, tree and lists.
 */
#ifndef BH_H
#define BH_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct bh_ctx bh_ctx;

typedef enum {
    BH_OK = 0,
    BH_EINVAL = -1,
    BH_ENOMEM = -2,
    BH_EHIP = -3,
    BH_ESTATE = -4,
    BH_ECAPACITY = -5
} bh_status;

/* Arithmetic of the interaction loop.  BH_FP32_REL: positions of the
 * group's particles and of its sources are taken relative to the group
 * centre in FP64, rounded to FP32, and the pair terms are evaluated and
 * summed in FP32 (the shifted-origin single-precision kernel of Sec. 4.7);
 * positions, moments and the integrator stay FP64. */
typedef enum { BH_FP64 = 0, BH_FP32_REL = 1 } bh_precision;

/* Opening rule of the walk.  GEOMETRIC: a node of side s is accepted for a
 * group when it lies outside the group's box and s < theta * d, d the
 * distance from the node's centre to the box.  LEARNED: inside the band
 * theta_min <= s/d < theta_max a small network predicts the node's monopole
 * error and the node is accepted when the prediction is below tau times the
 * mean (BH_FLAG_BUDGET_MIN: smallest) self-gravity acceleration of the
 * group's particles (from the last force evaluation); outside the band the
 * geometric rule holds. */
typedef enum { BH_OPEN_GEOMETRIC = 0, BH_OPEN_LEARNED = 1 } bh_criterion;

typedef struct {
    double theta;          /* opening angle, >= 0 */
    double eps;            /* Plummer softening length, >= 0 */
    double G;              /* gravitational constant */
    double central_mass;   /* point mass fixed at the origin, 0 = none; not part of the tree */
    int32_t n_leaf;        /* a node with more particles than this is split (>= 1) */
    int32_t n_group;       /* largest group; <= 0 lets the autotuner choose */
    int32_t precision;     /* bh_precision */
    int32_t criterion;     /* bh_criterion */
    double theta_min, theta_max, tau;   /* learned rule only: finite, >= 0 */
    int32_t flags;         /* BH_FLAG_* bits */
    /* Collision branch of Eq. (2) (Sec. 5.1), on when r_coll > 0.  For a
     * particle pair with r = |r_ij| <= r_coll (decided in FP64 on the
     * absolute positions as dx*dx + dy*dy + dz*dz <= r_coll*r_coll) the
     * acceleration of i is
     *   [G m_j / (r_coll^2 + eps^2)^(3/2)
     *    + m_j/(m_i + m_j) (kappa (r - r_coll)/r + eta (r_ij . v_ij)/r^2)] r_ij,
     * r_ij = r_j - r_i, v_ij = v_j - v_i: gravity held at its value on the
     * contact sphere (the paper's G m_j / r_coll^3 at eps = 0), a spring and
     * a radial dashpot.  Node (centre-of-mass) sources keep the gravity
     * branch.  The potential of a contact pair is that of its gravity part,
     * -G m_j [1/s + (r_coll^2 - r^2)/(2 s^3)], s = sqrt(r_coll^2 + eps^2).
     * The dashpot reads the velocities the context holds: those given to
     * bh_build_tree (bh_forces, which then needs non-NULL vx, vy, vz), the
     * half-kicked ones after each drift (bh_step).  The contact terms are
     * evaluated in FP64 in both precisions.  kappa, eta >= 0, finite. */
    double r_coll, kappa, eta;
    /* Tree coordinates (Sec. 4.3, Eq. (1)).  0: Cartesian.  > 0: for a
     * narrow ring near this radius the keys, cells, groups and opening test
     * use (phi, r, z): the root cell has side S = 2 pi cyl_radius, its phi
     * axis spans one turn ([-pi, pi) onto 2^21 grid cells, periodic in the
     * opening test), r and z start at their minimum.  Node moments, group
     * centres and forces stay Cartesian.  The radial and vertical extents
     * of every system must be below S (else BH_EINVAL from the build);
     * not combined with BH_OPEN_LEARNED (BH_EINVAL).  The angle is computed
     * with correctly rounded operations only (a series for arctan after
     * reduction to |t| <= tan(pi/8)), so keys do not depend on a math
     * library.  BH_EXPORT_ROOT_BOX then holds (-pi, min r, min z,
     * 2^21 / S). */
    double cyl_radius;
    /* Drift monitor of list-reusing steps (bh_step, bh_step_continue; the
     * persistent interaction list of Sec. 4.2 keeps lists for several steps,
     * the paper for a fixed number).  Off when reuse_drift is 0.  On, the
     * moment refresh of each reusing step also measures how far each node's
     * particles have moved since the tree was built relative to the node's
     * centre of mass (leaf: the largest |(x_i - x_i^build) - (c - c^build)|;
     * a parent: the largest child value plus the child's centre-of-mass
     * motion relative to the parent's), and the lists are rebuilt before
     * that step's force evaluation when, at some tree level, the nodes whose
     * drift exceeds reuse_drift times their side hold more than reuse_frac
     * of all particles.  rebuild_every then caps the list age.  One host
     * synchronisation per reusing step.  reuse_drift finite >= 0,
     * reuse_frac in [0, 1]. */
    double reuse_drift, reuse_frac;
    /* Sources per LDS tile of the FP32 gravity-only force kernel: 256 or 512
     * (0 = 512; other kernels use 512).  bh_autotune sets it. */
    int32_t force_tile;
} bh_params;

/* bh_params.flags: replay list-reusing steps eagerly instead of from a HIP graph. */
#define BH_FLAG_NO_GRAPH 1
/* bh_params.flags: the learned rule's budget scale A_g is the smallest self-gravity |a| of the
 * group's particles instead of their mean. */
#define BH_FLAG_BUDGET_MIN 2
/* bh_params.flags: pack small groups.  Below a node of more than n_group particles, runs of
 * consecutive children that would each be a group (at most n_group particles, or a leaf) are
 * merged, left to right, into one group while the merged count stays <= n_group; a child that is
 * split further, or a leaf of more than n_group coincident particles, ends the run.  A packed
 * group is a contiguous range of sorted particles inside its parent's cell; its box is the grid
 * box of its particles as for any group, and bh_export BH_EXPORT_GROUPS reports the run's first
 * node.  The paper forms its groups from tree nodes (Sec. 4.2, (3d)); packing keeps clumpy
 * regions, where many nodes hold a few particles each, from producing many tiny groups. */
#define BH_FLAG_PACK_GROUPS 4

/* One system: device arrays of n FP64 values each, caller order.
 * bh_step updates x,y,z,vx,vy,vz in place; m is read only. */
typedef struct {
    int64_t n;
    double *x, *y, *z;
    double *vx, *vy, *vz;
    const double *m;
} bh_system;

/* Output of bh_forces for one system: device arrays of n FP64 values,
 * caller order.  pot may be NULL. */
typedef struct {
    double *ax, *ay, *az, *pot;
} bh_accel;

typedef struct {
    int64_t n_particles;      /* over all systems */
    int32_t n_systems;
    int32_t max_level;        /* deepest tree level */
    int64_t n_nodes;
    int64_t n_groups;
    int64_t n_pc;             /* node-list entries over all groups */
    int64_t n_pp;             /* particle-list entries (leaves) over all groups */
    int64_t interactions;     /* sum over groups of n_g * (particles in pp leaves + pc nodes) */
    int32_t n_group_used;     /* group size in effect */
    int32_t lists_valid;      /* 1 once bh_make_lists has run on the current tree */
    int64_t interactions_evaluated;  /* running total over every force evaluation of the context */
    int64_t force_evaluations;       /* running count of force evaluations */
    int64_t tree_builds;             /* running count of tree builds */
    int64_t drift_rebuilds;          /* running count of builds the drift monitor asked for */
    int64_t host_syncs;              /* running count of host synchronisations on the work stream */
    int32_t force_tile;              /* sources per LDS tile of the FP32 gravity force kernel in effect */
} bh_sizes;

/* What bh_export copies out (to HOST memory; the call synchronises `stream`).
 * Sizes come from bh_query.  Node ids are global over all systems and
 * ordered by (level, system, key prefix). */
typedef enum {
    BH_EXPORT_KEYS = 0,       /* uint64[n_particles]  keys in sorted order */
    BH_EXPORT_PERM = 1,       /* uint32[n_particles]  sorted slot -> caller index within its system */
    BH_EXPORT_NODES = 2,      /* per node, int64[n_nodes][8]: level, system, prefix, begin,
                                 count, first_child, n_child, is_group (with packing: first of
                                 a packed run) */
    BH_EXPORT_MOMENTS = 3,    /* double[n_nodes][4]: com x, y, z, mass */
    BH_EXPORT_GROUPS = 4,     /* per group (ascending first particle), int64[n_groups][4]:
                                 node (the first of a packed run), begin, count, system;
                                 boxes: bh_export_groups */
    BH_EXPORT_LISTS = 5,      /* CSR: int64 pc_off[n_groups+1], int64 pp_off[n_groups+1],
                                 uint32 pc[n_pc], uint32 pp[n_pp], packed in that order,
                                 each list in ascending node id */
    BH_EXPORT_ACC_SORTED = 6, /* double[n_particles][4]: ax, ay, az, pot in sorted order, from the
                                 last force evaluation (BH_ESTATE before one) */
    BH_EXPORT_SORTED_POS = 7, /* double[n_particles][4]: x, y, z, m in sorted order */
    BH_EXPORT_QUAD = 8,       /* double[n_nodes][6]: second moment about the com (xx,xy,xz,yy,yz,zz);
                                 learned rule only */
    BH_EXPORT_NODE_QN = 9,    /* float[n_nodes]: |Q|_F / (M side^2); learned rule only */
    BH_EXPORT_GROUP_EXTRA = 10, /* double[n_groups][2]: half-diagonal of the group's FP64 box and the
                                   mean self-gravity |a| of its particles; learned rule only */
    BH_EXPORT_ROOT_BOX = 11,  /* double[n_systems][4]: root-box lower corner x, y, z and 2^21 / side */
    BH_EXPORT_DRIFT = 12      /* double[n_nodes]: drift of each node measured by the last list-reusing
                                 step's moment refresh (drift monitor only; undefined before one) */
} bh_what;

/* Create a context.  p is copied.  BH_EINVAL for out-of-range parameters. */
bh_status bh_create(bh_ctx **out, const bh_params *p);
/* Free the context and all its device memory (synchronises the device). */
bh_status bh_destroy(bh_ctx *ctx);
/* Replace the parameters; invalidates lists, so bh_make_lists is needed
 * again.  A change of n_group, n_leaf, criterion or cyl_radius also
 * invalidates the tree (bh_make_lists then returns BH_ESTATE until
 * bh_build_tree).  BH_EINVAL for out-of-range parameters (the context keeps
 * the old ones). */
bh_status bh_set_params(bh_ctx *ctx, const bh_params *p);

/* Sec. 4.2 (3a): root box, keys, sort and permutation, octree, node
 * moments, groups, for n_sys systems (sys[0..n_sys-1] host array of device
 * pointer sets).  Keeps a sorted FP64 copy of positions, velocities and
 * masses.  Invalidates lists.  The sort is stable: particles with equal
 * keys keep caller order.  Trees rebuilt inside bh_step / bh_step_continue
 * sort from the context's previous sorted order instead, so there equal
 * keys keep that order (the keys, tree, groups and lists are the same). */
bh_status bh_build_tree(bh_ctx *ctx, const bh_system *sys, int32_t n_sys, void *stream);

/* Sec. 4.2 (3d): walk the tree once per group and store its node list and
 * particle list.  Requires bh_build_tree. */
bh_status bh_make_lists(bh_ctx *ctx, void *stream);

/* Sec. 4.2 (3d) and Eq. (2): accelerations (and optionally potentials) of
 * every particle from its group's lists, written in caller order into
 * out[0..n_sys-1] (host array of device pointer sets).  out may be NULL to
 * keep the result only inside the context (bh_export ACC_SORTED).
 * Requires bh_make_lists.  Does not synchronise. */
bh_status bh_forces(bh_ctx *ctx, const bh_accel *out, void *stream);

/* Step (4) with the persistent interaction list: n_steps kick-drift-kick
 * steps of size dt.  The tree and lists are built at the start and rebuilt
 * before the force evaluation of every step whose index (1-based, counted
 * from the start of this call) is a multiple of rebuild_every; on the other
 * steps node moments are recomputed with the same tree and lists.  Reuse
 * steps are replayed from a captured HIP graph.  x, y, z, vx, vy, vz of
 * every system are updated in place. */
bh_status bh_step(bh_ctx *ctx, const bh_system *sys, int32_t n_sys, double dt,
                  int32_t n_steps, int32_t rebuild_every, void *stream);

/* Continue integrating the systems of the last bh_step (or of bh_build_tree
 * + bh_make_lists + bh_forces, with velocities) from the context's internal
 * state: n_steps more kick-drift-kick steps, the rebuild schedule carried on
 * from the previous call (a build every rebuild_every force evaluations).
 * The caller's arrays of that call are written at the end: they must stay
 * allocated and unchanged in between (use bh_step to start over).  BH_ESTATE
 * if there is no state to continue. */
bh_status bh_step_continue(bh_ctx *ctx, double dt, int32_t n_steps, int32_t rebuild_every, void *stream);

/* Direct summation (the exact sum the tree approximates) in FP64 for the
 * targets of one system: for t < n_targets, i = targets[t],
 *   a[t] = sum_j G m_j (x_j - x_i) / (|x_j - x_i|^2 + eps^2)^(3/2),
 * j over all n particles of sys (caller order; j = i adds nothing when
 * eps > 0 and is skipped when eps = 0).  targets, ax, ay, az: device arrays
 * of n_targets entries (may be NULL when n_targets is 0: nothing is done).
 * A target index outside [0, n) yields NaN in its three outputs; no memory
 * outside the arrays is read.  Uses the context's G and eps; independent of the
 * tree.  Serves as the error judge of the approximation.  With r_coll > 0
 * every pair follows Eq. (2) with both branches (see bh_params) and sys
 * must carry velocities. */
bh_status bh_direct_sum(bh_ctx *ctx, const bh_system *sys, const int64_t *targets, int64_t n_targets,
                        double *ax, double *ay, double *az, void *stream);

/* bh_direct_sum for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same kernels and the same result, bit for bit, with the partial sums
 * in a static device array of 12 MiB that the library holds on each GPU
 * until the process ends (its address is looked up once per device by
 * bh_create) instead of context memory grown on demand.  The call allocates
 * and frees nothing.  At most BH_DIRECT_STATIC_MAX_TARGETS targets
 * (BH_EINVAL above that); the context's device must be current (BH_EINVAL
 * otherwise).  Every call on one GPU shares its array, which keeps the last
 * call's partial sums (each call writes every partial it reads, so nothing
 * needs clearing): calls that overlap in time on one GPU, from any context
 * or stream, race and must be serialised by the caller. */
#define BH_DIRECT_STATIC_MAX_TARGETS 4096
bh_status bh_direct_sum_static(bh_ctx *ctx, const bh_system *sys, const int64_t *targets, int64_t n_targets,
                               double *ax, double *ay, double *az, void *stream);

/* Accelerations of the last force evaluation (bh_forces, bh_step,
 * bh_step_continue) for chosen particles of one system, without copying the
 * rest: for t < n_targets, (ax, ay, az)[t] = acceleration of caller index
 * targets[t] of system sys, as bh_forces writes it (self-gravity plus the
 * central mass term).  targets, ax, ay, az: device arrays of n_targets
 * entries.  An index outside [0, n) of the system gives NaN; nothing outside
 * the arrays is read.  BH_ESTATE before a force evaluation; does not
 * synchronise.  For judging the error of a running integration against
 * bh_direct_sum at the same positions. */
bh_status bh_sample_acc(bh_ctx *ctx, int32_t sys, const int64_t *targets, int64_t n_targets, double *ax,
                        double *ay, double *az, void *stream);

/* Force-kernel device time accumulated over the launches since the last
 * reset, from HIP events recorded around each launch on its stream
 * (synchronises those events).  reset != 0 clears the accumulator after
 * reading. */
bh_status bh_force_timing(bh_ctx *ctx, double *total_ms, int64_t *launches, int32_t reset);

/* Group-size and tile autotuner (the scheduling of Sec. 4.6 leaves the
 * group size free): for each candidate group size, regroup the current tree,
 * walk and evaluate forces, timing both with HIP events (FP32 without the
 * collision branch: once per force tile, 512 and 256 sources); keep the pair
 * with the smallest force time + walk time / rebuild_every, set n_group and
 * force_tile of the context's parameters to it and leave its lists in place.
 * Speed at the context's theta only: a larger group is also more accurate
 * at equal theta, which this call does not weigh.  Requires bh_build_tree.
 * *chosen (may be NULL) receives the group size; bh_query the tile. */
bh_status bh_autotune(bh_ctx *ctx, const int32_t *candidates, int32_t n_candidates, int32_t rebuild_every,
                      int32_t *chosen, void *stream);

/* ---- Learned opening rule (not in the paper: an addition to the walk of
 * Sec. 4.2 (3d)).  Network 4-32-32-1, ReLU, FP32, MLP_NPARAM = 1259 floats:
 * W1[32][4], b1[32], W2[32][32], b2[32], W3[32], b3, then input means[4],
 * input 1/std[4], label mean, label std.  Features of a (group, node) pair,
 * each on the lg2p scale: (side/d_box)^2 with d_box the distance from the
 * node's centre to the group box (the opening test's grid quantity), group
 * half-diagonal/d, M/M_system and |Q|_F/(M side^2) (rounded to FP32 before
 * lg2p), with d the distance from the node's centre of mass to the group
 * centre and
 * lg2p the piecewise-linear log2 (x = m 2^e, m in [0.5,1): e - 2 + 2m).
 * Label: lg2p(largest |monopole - exact| over the group's particles /
 * (G M / d^2)), the exact force summed directly in FP64. */
#define BH_MLP_NPARAM 1259

/* Record training pairs from the current tree (context created with the
 * learned criterion, after bh_build_tree): a walk that accepts below
 * theta_min and opens everything else lists every (group, node) pair in the
 * band theta_min <= side/distance < theta_max for about max_groups groups;
 * each pair with 2..count_cap particles gets its features and exact label
 * appended to the context's training set.  Invalidates lists. */
bh_status bh_mlp_collect(bh_ctx *ctx, int32_t max_groups, int32_t count_cap, void *stream);

typedef struct {
    int32_t iters;        /* Adam steps */
    int32_t batch;        /* samples per step */
    float lr, beta1, beta2, eps;
    uint64_t seed;        /* weight initialisation and shuffling */
    int32_t init;         /* 1: new weights and normalisation from the training set */
} bh_train_opts;

/* Train on the collected set with the library's forward, backward and Adam
 * kernels.  *mse (host, may be NULL) receives the mean squared error of the
 * final network over the whole set, in label units squared. */
bh_status bh_mlp_train(bh_ctx *ctx, const bh_train_opts *o, double *mse, void *stream);

/* Copy the weights out (get, host, BH_MLP_NPARAM floats) and/or install new
 * ones (set); either may be NULL.  Installing weights invalidates lists and
 * restarts the optimiser: Adam's moment estimates and step count return to
 * zero. */
bh_status bh_mlp_weights(bh_ctx *ctx, float *get, const float *set);

/* One Adam step (Kingma & Ba 2015) on the first 1249 weights with the
 * gradient grad (device float[1249]): with t the steps since the weights
 * were installed or initialised,
 *   m = beta1 m + (1 - beta1) g,  v = beta2 v + (1 - beta2) g^2,
 *   w -= lr (m / (1 - beta1^t)) / (sqrt(v / (1 - beta2^t)) + eps),
 * in FP32.  The step bh_mlp_train takes after each batch gradient; exposed
 * for callers that compute gradients themselves.  BH_EINVAL for lr <= 0 or
 * betas outside [0, 1); BH_ESTATE until weights are set or trained.
 * Invalidates lists.  Does not synchronise. */
bh_status bh_mlp_adam(bh_ctx *ctx, const float *grad, float lr, float beta1, float beta2, float eps,
                      void *stream);

/* Training-set size, and optionally its pairs (uint32[n][2] group, node of
 * the tree they were collected on), features (float[n][4]) and labels
 * (float[n]) to host memory.  bh_mlp_clear empties the set. */
bh_status bh_mlp_dataset(bh_ctx *ctx, int64_t *n, uint32_t *pairs, float *x, float *y);
bh_status bh_mlp_clear(bh_ctx *ctx);

/* Replace the training set with n pairs from host memory, in the layout
 * bh_mlp_dataset returns: pairs uint32[n][2] (group, node; may be NULL,
 * then zeros), features float[n][4] and labels float[n] on the scale the
 * network predicts.  For training on pairs gathered elsewhere, e.g. by a
 * CPU reference.  BH_EINVAL if n < 1 or n >= 2^31 or x or y is NULL; the
 * arrays are copied before the call returns. */
bh_status bh_mlp_set_dataset(bh_ctx *ctx, int64_t n, const uint32_t *pairs, const float *x, const float *y);

/* Network output for n feature rows (device float[n][4] -> device float[n]).
 * BH_ESTATE until weights are set (bh_mlp_weights) or trained. */
bh_status bh_mlp_predict(bh_ctx *ctx, const float *x, int64_t n, float *out, void *stream);

/* Gradient of the mean squared error (on the normalised label) of a batch
 * (device x float[B][4], y float[B], B <= 65536) with respect to the first
 * 1249 weights, and the loss, into device memory; the weights are not
 * changed.  BH_ESTATE until weights are set or trained. */
bh_status bh_mlp_gradient(bh_ctx *ctx, const float *x, const float *y, int32_t B, float *grad, float *loss,
                          void *stream);

bh_status bh_query(const bh_ctx *ctx, bh_sizes *out);

/* Copy one internal structure to host memory dst (layouts in bh_what). */
bh_status bh_export(bh_ctx *ctx, int32_t what, void *dst, void *stream);

/* Group boxes: int32[n_groups][6] grid box lo xyz, hi xyz (half-open) and
 * double[n_groups][3] centres; either pointer may be NULL. */
bh_status bh_export_groups(bh_ctx *ctx, int32_t *box, double *centre, void *stream);

/* Per-stage device times in milliseconds of the last call of each kind,
 * measured with HIP events on the call's stream:
 * [0] keys+sort+permute, [1] tree, [2] moments, [3] groups, [4] walk,
 * [5] forces (force kernel only), [6] integrate, [7] whole last bh_step. */
bh_status bh_stage_times(bh_ctx *ctx, double *ms8);

const char *bh_last_error(const bh_ctx *ctx);

#ifdef __cplusplus
}
#endif
#endif /* BH_H */
