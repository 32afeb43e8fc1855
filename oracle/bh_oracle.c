/*
 * bh_oracle.c -- plain, slow, FP64 CPU reference for the Barnes-Hut force
 * path (tree build, group walk, interaction lists, softened gravity).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the checker for the GPU library:
 * only the test suite, the smoke check and the CPU-baseline leg of the
 * benchmark load it.  It shares no code, header or constant table with the
 * HIP path, and the HIP path never calls it.
 *
 * Every function follows one step of the method as the paper states it
 * (Iwasawa et al. 2019, "Implementation and performance of Barnes-Hut
 * N-body algorithm on extreme-scale heterogeneous many-core
 * architectures"):
 *   - tree construction from the particles of the domain ........ Sec. 4.2, step (3a)/(3c)
 *   - groups of neighbouring particles taken from the tree itself Sec. 4.2, step (3d)
 *   - per-group traversal producing particle and node lists ...... Sec. 4.2, step (3d)
 *   - double loop over group particles and list entries ......... Sec. 4.2, step (3d)
 *   - gravity term of the particle-particle interaction ......... Sec. 5.1, Eq. (2)
 *   - centre-of-mass (monopole) approximation for tree nodes .... Sec. 5.1
 * Where the paper is silent (key layout, tree split rule, group rule,
 * opening test) the functions implement a stated reading of it; each reading
 * is written out in the comment of the function that implements it.
 *
 * Precision: FP64 throughout, built with -O2 -ffp-contract=off and no
 * fast-math so that every expression rounds exactly as written.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_MAXLEVEL 21            /* 21 bits per axis -> 63-bit keys */

/* ------------------------------------------------------------------ */
/* Root box and keys (tree construction, Sec. 4.2 (3a)).               */
/* Reading: the root cube has its lower corner at the per-axis minimum  */
/* and side S = the smallest power of two strictly greater than the     */
/* largest per-axis extent (S = 1 for a single point).  Grid coordinate */
/* q = floor((x - lo) * 2^21 / S), clamped to 2^21 - 1; the key         */
/* interleaves the 21 bits of each axis, x the most significant bit of  */
/* each triple.                                                          */
/* ------------------------------------------------------------------ */
static uint64_t interleave3(uint32_t qx, uint32_t qy, uint32_t qz)
{
    uint64_t key = 0;
    for (int k = 0; k < ORC_MAXLEVEL; ++k) {
        key |= (uint64_t)((qx >> k) & 1u) << (3 * k + 2);
        key |= (uint64_t)((qy >> k) & 1u) << (3 * k + 1);
        key |= (uint64_t)((qz >> k) & 1u) << (3 * k);
    }
    return key;
}

static void deinterleave3(uint64_t key, int nbits, uint32_t q[3])
{
    /* key holds nbits triples (the low 3*nbits bits) */
    q[0] = q[1] = q[2] = 0;
    for (int k = 0; k < nbits; ++k) {
        q[0] |= (uint32_t)((key >> (3 * k + 2)) & 1u) << k;
        q[1] |= (uint32_t)((key >> (3 * k + 1)) & 1u) << k;
        q[2] |= (uint32_t)((key >> (3 * k)) & 1u) << k;
    }
}

/* Returns 0, or -1 if a coordinate is not finite or n < 1. */
int orc_keys(int64_t n, const double *x, const double *y, const double *z,
             double *lo3, double *S_out, uint32_t *q3, uint64_t *key)
{
    if (n < 1) return -1;
    const double *c[3] = {x, y, z};
    double lo[3], hi[3];
    for (int d = 0; d < 3; ++d) {
        lo[d] = c[d][0];
        hi[d] = c[d][0];
    }
    for (int64_t i = 0; i < n; ++i) {
        for (int d = 0; d < 3; ++d) {
            double v = c[d][i];
            if (!isfinite(v)) return -1;
            if (v < lo[d]) lo[d] = v;
            if (v > hi[d]) hi[d] = v;
        }
    }
    double w = 0.0;
    for (int d = 0; d < 3; ++d) {
        double e = hi[d] - lo[d];
        if (e > w) w = e;
    }
    /* smallest power of two strictly greater than w */
    double S;
    int e2 = 0;
    if (w == 0.0) {
        S = 1.0;                  /* a single point: any cube works */
        e2 = 0;
    } else {
        frexp(w, &e2);            /* w = f * 2^e2, 0.5 <= f < 1  ->  w < 2^e2 */
        S = ldexp(1.0, e2);
    }
    double scale = ldexp(1.0, ORC_MAXLEVEL - e2);   /* 2^21 / S, exact */
    for (int d = 0; d < 3; ++d) lo3[d] = lo[d];
    *S_out = S;
    for (int64_t i = 0; i < n; ++i) {
        uint32_t q[3];
        for (int d = 0; d < 3; ++d) {
            double t = (c[d][i] - lo[d]) * scale;
            double f = floor(t);
            uint32_t qi = (f >= 2097151.0) ? 2097151u : (uint32_t)f;
            q[d] = qi;
        }
        if (q3) {
            q3[3 * i + 0] = q[0];
            q3[3 * i + 1] = q[1];
            q3[3 * i + 2] = q[2];
        }
        key[i] = interleave3(q[0], q[1], q[2]);
    }
    return 0;
}

/* ------------------------------------------------------------------ */
/* Cylindrical tree coordinates (Sec. 4.3, Eq. (1)): for a narrow ring  */
/* near radius r_ref the arc r_ref*phi, the radius r and the height z   */
/* are locally Cartesian, so the tree (keys, cells, groups, opening     */
/* test) is built on them while the forces stay Cartesian.  Reading:    */
/*   phi = the angle of (x, y) in [-pi, pi], r = sqrt(x*x + y*y);       */
/*   the root cell has side S = 2 pi r_ref, its phi axis spans exactly  */
/*   one turn, [-pi, pi) -> [0, 2^21) with q = floor((phi + pi) 2^21 /  */
/*   (2 pi)), and r, z use q = floor((v - min v) 2^21 / S); all q are   */
/*   clamped to 2^21 - 1.  The phi axis is periodic (period 2^21 grid   */
/*   units), which the opening test takes into account.                 */
/* The angle comes from orc_atan2 below, built from correctly rounded   */
/* operations only, so that any implementation of the same steps gets   */
/* the same bits.                                                        */
/* ------------------------------------------------------------------ */
#define ORC_PI 3.141592653589793
#define ORC_TAN_PI8 0.41421356237309503     /* tan(pi/8) = sqrt(2) - 1 */
#define ORC_ATAN_TERMS 15                   /* t, t^3, ..., t^29 */

/* arctan(t) for |t| <= tan(pi/8): the Maclaurin series
 *   t - t^3/3 + t^5/5 - ... (Abramowitz & Stegun 4.4.42)
 * up to t^29, by Horner's rule in t^2 from the highest term down; the
 * coefficients are (-1)^k / (2k+1), each one correctly rounded division.
 * Truncation error below |t|^31/31 < 2e-14. */
static double atan_series(double t)
{
    double t2 = t * t;
    double p = 0.0;
    for (int k = ORC_ATAN_TERMS - 1; k >= 0; --k) {
        double c = 1.0 / (double)(2 * k + 1);
        if (k & 1) c = -c;
        p = p * t2 + c;
    }
    return t * p;
}

/* The angle of (x, y) in [-pi, pi]: reduce to t = min/max(|x|,|y|) in
 * [0, 1]; above tan(pi/8) use arctan t = pi/4 + arctan((t-1)/(t+1))
 * (the addition formula, A&S 4.4.34); then reflect into the octant and
 * quadrant of (x, y).  (0, 0) gives 0. */
double orc_atan2(double y, double x)
{
    double ax = fabs(x), ay = fabs(y);
    if (ax == 0.0 && ay == 0.0) return 0.0;
    int swap = ay > ax;
    double t = swap ? ax / ay : ay / ax;
    double a;
    if (t > ORC_TAN_PI8)
        a = 0.25 * ORC_PI + atan_series((t - 1.0) / (t + 1.0));
    else
        a = atan_series(t);
    if (swap) a = 0.5 * ORC_PI - a;
    if (x < 0.0) a = ORC_PI - a;
    if (y < 0.0) a = -a;
    return a;
}

/* Returns 0; -1 for non-finite input, n < 1 or r_ref <= 0; -2 when the  */
/* radial or vertical extent does not fit the root cell.                 */
int orc_keys_cyl(int64_t n, const double *x, const double *y, const double *z, double r_ref,
                 double *lo3, double *S_out, uint32_t *q3, uint64_t *key)
{
    if (n < 1 || !(r_ref > 0.0) || !isfinite(r_ref)) return -1;
    double *phi = (double *)malloc((size_t)n * sizeof(double));
    double *rad = (double *)malloc((size_t)n * sizeof(double));
    double rlo = 0, rhi = 0, zlo = 0, zhi = 0;
    int bad = 0;
    for (int64_t i = 0; i < n; ++i) {
        if (!isfinite(x[i]) || !isfinite(y[i]) || !isfinite(z[i])) bad = 1;
        phi[i] = orc_atan2(y[i], x[i]);
        rad[i] = sqrt(x[i] * x[i] + y[i] * y[i]);
        if (i == 0 || rad[i] < rlo) rlo = rad[i];
        if (i == 0 || rad[i] > rhi) rhi = rad[i];
        if (i == 0 || z[i] < zlo) zlo = z[i];
        if (i == 0 || z[i] > zhi) zhi = z[i];
    }
    double S = (2.0 * ORC_PI) * r_ref;
    int rc = bad ? -1 : ((rhi - rlo >= S || zhi - zlo >= S) ? -2 : 0);
    if (rc == 0) {
        double kphi = 2097152.0 / (2.0 * ORC_PI), k = 2097152.0 / S;
        lo3[0] = -ORC_PI;
        lo3[1] = rlo;
        lo3[2] = zlo;
        *S_out = S;
        for (int64_t i = 0; i < n; ++i) {
            double t[3] = {(phi[i] + ORC_PI) * kphi, (rad[i] - rlo) * k, (z[i] - zlo) * k};
            uint32_t q[3];
            for (int d = 0; d < 3; ++d) {
                double f = floor(t[d]);
                q[d] = (f >= 2097151.0) ? 2097151u : (uint32_t)f;
            }
            if (q3) {
                q3[3 * i + 0] = q[0];
                q3[3 * i + 1] = q[1];
                q3[3 * i + 2] = q[2];
            }
            key[i] = interleave3(q[0], q[1], q[2]);
        }
    }
    free(phi);
    free(rad);
    return rc;
}

/* ------------------------------------------------------------------ */
/* Sort (Sec. 4.2: sorting is the dominant cost of tree construction). */
/* Ascending by (key, original index): a stable sort by key.           */
/* ------------------------------------------------------------------ */
static const uint64_t *g_sort_keys;
static int cmp_key_idx(const void *a, const void *b)
{
    uint32_t ia = *(const uint32_t *)a, ib = *(const uint32_t *)b;
    uint64_t ka = g_sort_keys[ia], kb = g_sort_keys[ib];
    if (ka < kb) return -1;
    if (ka > kb) return 1;
    return (ia < ib) ? -1 : (ia > ib);
}

void orc_sort(int64_t n, const uint64_t *key, uint32_t *perm)
{
    for (int64_t i = 0; i < n; ++i) perm[i] = (uint32_t)i;
    g_sort_keys = key;
    qsort(perm, (size_t)n, sizeof(uint32_t), cmp_key_idx);
    g_sort_keys = NULL;
}

/* ------------------------------------------------------------------ */
/* Octree (Sec. 4.2 (3a)).  Reading: the root covers all particles at   */
/* level 0; a node with more than n_leaf particles and level < 21 is    */
/* split by the next key triple into its non-empty children, in         */
/* ascending octant order.  Nodes are numbered breadth first, i.e. in   */
/* ascending (level, prefix).  Returns the node count, or -1 when cap   */
/* is too small.                                                        */
/* ------------------------------------------------------------------ */
int64_t orc_tree(int64_t n, const uint64_t *skey, int32_t n_leaf, int64_t cap,
                 uint8_t *level, uint64_t *prefix, uint32_t *begin,
                 uint32_t *count, uint32_t *first_child, uint8_t *n_child)
{
    if (cap < 1 || n < 1) return -1;
    int64_t nn = 1;
    level[0] = 0;
    prefix[0] = 0;
    begin[0] = 0;
    count[0] = (uint32_t)n;
    /* a FIFO over the node array itself gives breadth-first numbering */
    for (int64_t v = 0; v < nn; ++v) {
        first_child[v] = 0;
        n_child[v] = 0;
        int l = level[v];
        if (count[v] <= (uint32_t)n_leaf || l >= ORC_MAXLEVEL) continue;
        int shift = 3 * (ORC_MAXLEVEL - 1 - l);       /* bits of the child triple */
        uint32_t b = begin[v], e = begin[v] + count[v];
        first_child[v] = (uint32_t)nn;
        uint32_t i = b;
        while (i < e) {
            unsigned oct = (unsigned)((skey[i] >> shift) & 7u);
            uint32_t j = i;
            while (j < e && (unsigned)((skey[j] >> shift) & 7u) == oct) ++j;
            if (nn >= cap) return -1;
            level[nn] = (uint8_t)(l + 1);
            prefix[nn] = (prefix[v] << 3) | oct;
            begin[nn] = i;
            count[nn] = j - i;
            ++nn;
            n_child[v]++;
            i = j;
        }
    }
    return nn;
}

/* ------------------------------------------------------------------ */
/* Monopole moments (Sec. 5.1: particle-node forces use the centre-of-  */
/* mass approximation).  M = sum m, com = sum m x / M, summed directly  */
/* over each node's particle range in sorted order.  Q (optional, six   */
/* components xx,xy,xz,yy,yz,zz) is the second moment about the com.    */
/* ------------------------------------------------------------------ */
void orc_moments(int64_t n_nodes, const uint32_t *begin, const uint32_t *count,
                 const double *x, const double *y, const double *z, const double *m,
                 double *M, double *cx, double *cy, double *cz, double *Q)
{
    #pragma omp parallel for schedule(dynamic, 64)
    for (int64_t v = 0; v < n_nodes; ++v) {
        double sm = 0, sx = 0, sy = 0, sz = 0;
        uint32_t b = begin[v], e = begin[v] + count[v];
        for (uint32_t i = b; i < e; ++i) {
            sm += m[i];
            sx += m[i] * x[i];
            sy += m[i] * y[i];
            sz += m[i] * z[i];
        }
        M[v] = sm;
        cx[v] = sx / sm;
        cy[v] = sy / sm;
        cz[v] = sz / sm;
        if (Q) {
            double q[6] = {0, 0, 0, 0, 0, 0};
            for (uint32_t i = b; i < e; ++i) {
                double dx = x[i] - cx[v], dy = y[i] - cy[v], dz = z[i] - cz[v];
                q[0] += m[i] * dx * dx;
                q[1] += m[i] * dx * dy;
                q[2] += m[i] * dx * dz;
                q[3] += m[i] * dy * dy;
                q[4] += m[i] * dy * dz;
                q[5] += m[i] * dz * dz;
            }
            for (int k = 0; k < 6; ++k) Q[6 * v + k] = q[k];
        }
    }
}

/* ------------------------------------------------------------------ */
/* Groups (Sec. 4.2 (3d): groups of neighbouring particles constructed  */
/* from the tree itself).  Reading: walking down from the root, the     */
/* first node with at most n_grp particles becomes a group; a leaf is   */
/* always a group.  Depth-first in octant order lists the groups in     */
/* ascending begin.  Returns the group count or -1 if cap is too small. */
/* ------------------------------------------------------------------ */
static int64_t groups_rec(int64_t v, const uint32_t *count, const uint32_t *first_child,
                          const uint8_t *n_child, int32_t n_grp, int64_t cap,
                          uint32_t *gnode, int64_t ng)
{
    if (ng < 0) return ng;
    if (count[v] <= (uint32_t)n_grp || n_child[v] == 0) {
        if (ng >= cap) return -1;
        gnode[ng] = (uint32_t)v;
        return ng + 1;
    }
    for (int c = 0; c < n_child[v]; ++c)
        ng = groups_rec(first_child[v] + c, count, first_child, n_child, n_grp, cap, gnode, ng);
    return ng;
}

int64_t orc_groups(const uint32_t *count, const uint32_t *first_child, const uint8_t *n_child,
                   int32_t n_grp, int64_t cap, uint32_t *gnode)
{
    return groups_rec(0, count, first_child, n_child, n_grp, cap, gnode, 0);
}

/* ------------------------------------------------------------------ */
/* Packed groups (an option of this implementation; the paper's groups  */
/* are tree nodes).  Walking down as above, below a node of more than   */
/* n_grp particles its children are taken in octant order: a child of   */
/* at most n_grp particles joins the pack opened by the previous child  */
/* when the pack's count stays <= n_grp, else it opens a new pack; a    */
/* child of more than n_grp particles (split further, or a leaf of      */
/* coincident points, which is a group of its own) closes the open      */
/* pack.  gnode = first node of each pack, gbeg / gcnt = its particle   */
/* range.  Returns the group count or -1 if cap is too small.           */
/* ------------------------------------------------------------------ */
static int64_t packed_rec(int64_t v, const uint32_t *count, const uint32_t *begin, const uint32_t *first_child,
                          const uint8_t *n_child, int32_t n_grp, int64_t cap, uint32_t *gnode,
                          uint32_t *gbeg, uint32_t *gcnt, int64_t ng)
{
    if (ng < 0) return ng;
    if (count[v] <= (uint32_t)n_grp || n_child[v] == 0) {
        if (ng >= cap) return -1;
        gnode[ng] = (uint32_t)v;
        gbeg[ng] = begin[v];
        gcnt[ng] = count[v];
        return ng + 1;
    }
    int64_t open = -1;                        /* the pack the next small child may join */
    for (int c = 0; c < n_child[v]; ++c) {
        const int64_t u = first_child[v] + c;
        if (count[u] <= (uint32_t)n_grp) {
            if (open >= 0 && gcnt[open] + count[u] <= (uint32_t)n_grp) {
                gcnt[open] += count[u];
                continue;
            }
            if (ng >= cap) return -1;
            gnode[ng] = (uint32_t)u;
            gbeg[ng] = begin[u];
            gcnt[ng] = count[u];
            open = ng++;
        } else {
            open = -1;
            ng = packed_rec(u, count, begin, first_child, n_child, n_grp, cap, gnode, gbeg, gcnt, ng);
            if (ng < 0) return ng;
        }
    }
    return ng;
}

int64_t orc_groups_packed(const uint32_t *count, const uint32_t *begin, const uint32_t *first_child,
                          const uint8_t *n_child, int32_t n_grp, int64_t cap, uint32_t *gnode,
                          uint32_t *gbeg, uint32_t *gcnt)
{
    return packed_rec(0, count, begin, first_child, n_child, n_grp, cap, gnode, gbeg, gcnt, 0);
}

/* Group box in grid units, half-open [min q, max q + 1), taken from the */
/* particles' keys; group centre = midpoint of the FP64 bounding box.    */
void orc_group_boxes(int64_t n_groups, const uint32_t *gnode, const uint32_t *begin,
                     const uint32_t *count, const uint64_t *skey,
                     const double *x, const double *y, const double *z,
                     int32_t *gbox, double *gcen)
{
    for (int64_t g = 0; g < n_groups; ++g) {
        uint32_t v = gnode[g], b = begin[v], e = begin[v] + count[v];
        uint32_t qmin[3] = {0xffffffffu, 0xffffffffu, 0xffffffffu}, qmax[3] = {0, 0, 0};
        double lo[3] = {x[b], y[b], z[b]}, hi[3] = {x[b], y[b], z[b]};
        for (uint32_t i = b; i < e; ++i) {
            uint32_t q[3];
            deinterleave3(skey[i], ORC_MAXLEVEL, q);
            double p[3] = {x[i], y[i], z[i]};
            for (int d = 0; d < 3; ++d) {
                if (q[d] < qmin[d]) qmin[d] = q[d];
                if (q[d] > qmax[d]) qmax[d] = q[d];
                if (p[d] < lo[d]) lo[d] = p[d];
                if (p[d] > hi[d]) hi[d] = p[d];
            }
        }
        for (int d = 0; d < 3; ++d) {
            gbox[6 * g + d] = (int32_t)qmin[d];
            gbox[6 * g + 3 + d] = (int32_t)(qmax[d] + 1);
            gcen[3 * g + d] = 0.5 * (lo[d] + hi[d]);
        }
    }
}

/* ------------------------------------------------------------------ */
/* Opening test.  Reading of the group walk of Sec. 4.2 (3d): a node of */
/* side s is used as a single mass for the whole group when it lies     */
/* outside the group's box and s / d < theta, d being the distance from */
/* the node's geometric centre to the nearest point of the group box.   */
/* Computed in doubled integer grid units: the only floating-point      */
/* operation is the multiplication by th2 = theta*theta.  With a        */
/* periodic first axis (cylindrical coordinates, period P grid units)   */
/* the distance along it is that to the nearest image of the node; a    */
/* node and a group box, both inside one period, overlap only directly. */
/* ------------------------------------------------------------------ */
static int64_t axis_gap2(int64_t C, int64_t gl, int64_t gh)
{
    /* doubled distance from doubled centre C to the interval [gl, gh] */
    int64_t da = 0;
    if (2 * gl - C > da) da = 2 * gl - C;
    if (C - 2 * gh > da) da = C - 2 * gh;
    return da;
}

static int accept_cell_p(const int32_t *gb, int lvl, uint64_t pfx, double th2, int64_t period)
{
    uint32_t p[3];
    deinterleave3(pfx, lvl, p);
    int64_t s = (int64_t)1 << (ORC_MAXLEVEL - lvl);
    int disjoint = 0;
    int64_t d2 = 0;
    for (int a = 0; a < 3; ++a) {
        int64_t L = (int64_t)p[a] << (ORC_MAXLEVEL - lvl);
        int64_t gl = gb[a], gh = gb[3 + a];
        if (L + s <= gl || L >= gh) disjoint = 1;
        int64_t C = 2 * L + s;
        int64_t da = axis_gap2(C, gl, gh);
        if (a == 0 && period > 0) {
            int64_t dm = axis_gap2(C - 2 * period, gl, gh), dp = axis_gap2(C + 2 * period, gl, gh);
            if (dm < da) da = dm;
            if (dp < da) da = dp;
        }
        d2 += da * da;
    }
    int64_t s2 = (2 * s) * (2 * s);
    return disjoint && ((double)s2 < th2 * (double)d2);
}

static int accept_cell(const int32_t *gb, int lvl, uint64_t pfx, double th2)
{
    return accept_cell_p(gb, lvl, pfx, th2, 0);
}

typedef struct { uint32_t *v; int64_t n, cap; } u32vec;
static void vpush(u32vec *a, uint32_t x)
{
    if (a->n == a->cap) {
        a->cap = a->cap ? 2 * a->cap : 256;
        a->v = (uint32_t *)realloc(a->v, (size_t)a->cap * sizeof(uint32_t));
    }
    a->v[a->n++] = x;
}
static int cmp_u32(const void *a, const void *b)
{
    uint32_t x = *(const uint32_t *)a, y = *(const uint32_t *)b;
    return (x < y) ? -1 : (x > y);
}

/* The traversal: an accepted node goes to the node list, a rejected    */
/* leaf to the particle list, a rejected internal node is opened.       */
static void walk_rec(uint32_t v, const int32_t *gb, const uint8_t *level, const uint64_t *prefix,
                     const uint32_t *first_child, const uint8_t *n_child, double th2, int64_t period,
                     u32vec *pc, u32vec *pp)
{
    if (accept_cell_p(gb, level[v], prefix[v], th2, period)) {
        vpush(pc, v);
    } else if (n_child[v] == 0) {
        vpush(pp, v);
    } else {
        for (int c = 0; c < n_child[v]; ++c)
            walk_rec(first_child[v] + c, gb, level, prefix, first_child, n_child, th2, period, pc, pp);
    }
}

/* Interaction lists for every group, in canonical form (each list in  */
/* ascending node id).  pc_off/pp_off have n_groups+1 entries.  When    */
/* pc_ids/pp_ids are NULL only the offsets are produced.  period > 0:   */
/* the first grid axis is periodic with that many grid units.           */
void orc_lists_p(int64_t n_groups, const int32_t *gbox, const uint8_t *level, const uint64_t *prefix,
                 const uint32_t *first_child, const uint8_t *n_child, double theta, int64_t period,
                 int64_t *pc_off, int64_t *pp_off, uint32_t *pc_ids, uint32_t *pp_ids)
{
    double th2 = theta * theta;
    int64_t *pcn = (int64_t *)calloc((size_t)n_groups, sizeof(int64_t));
    int64_t *ppn = (int64_t *)calloc((size_t)n_groups, sizeof(int64_t));
    #pragma omp parallel for schedule(dynamic, 16)
    for (int64_t g = 0; g < n_groups; ++g) {
        u32vec pc = {0, 0, 0}, pp = {0, 0, 0};
        walk_rec(0, gbox + 6 * g, level, prefix, first_child, n_child, th2, period, &pc, &pp);
        pcn[g] = pc.n;
        ppn[g] = pp.n;
        free(pc.v);
        free(pp.v);
    }
    pc_off[0] = 0;
    pp_off[0] = 0;
    for (int64_t g = 0; g < n_groups; ++g) {
        pc_off[g + 1] = pc_off[g] + pcn[g];
        pp_off[g + 1] = pp_off[g] + ppn[g];
    }
    if (pc_ids && pp_ids) {
        #pragma omp parallel for schedule(dynamic, 16)
        for (int64_t g = 0; g < n_groups; ++g) {
            u32vec pc = {0, 0, 0}, pp = {0, 0, 0};
            walk_rec(0, gbox + 6 * g, level, prefix, first_child, n_child, th2, period, &pc, &pp);
            qsort(pc.v, (size_t)pc.n, sizeof(uint32_t), cmp_u32);
            qsort(pp.v, (size_t)pp.n, sizeof(uint32_t), cmp_u32);
            if (pc.n) memcpy(pc_ids + pc_off[g], pc.v, (size_t)pc.n * sizeof(uint32_t));
            if (pp.n) memcpy(pp_ids + pp_off[g], pp.v, (size_t)pp.n * sizeof(uint32_t));
            free(pc.v);
            free(pp.v);
        }
    }
    free(pcn);
    free(ppn);
}

void orc_lists(int64_t n_groups, const int32_t *gbox, const uint8_t *level, const uint64_t *prefix,
               const uint32_t *first_child, const uint8_t *n_child, double theta,
               int64_t *pc_off, int64_t *pp_off, uint32_t *pc_ids, uint32_t *pp_ids)
{
    orc_lists_p(n_groups, gbox, level, prefix, first_child, n_child, theta, 0, pc_off, pp_off, pc_ids, pp_ids);
}

/* ------------------------------------------------------------------ */
/* Forces (Sec. 4.2 (3d) double loop; Sec. 5.1 Eq. (2)).  The          */
/* acceleration of i from a source of mass mj at xj, r = |xj - xi|,     */
/* rij = xj - xi, is the gravity branch with Plummer softening          */
/*     G mj rij / (r^2 + eps^2)^(3/2),                                  */
/* and its potential -G mj / sqrt(r^2 + eps^2).  Sources are the        */
/* particles of the particle-list leaves and the centres of mass of the */
/* node-list cells.                                                     */
/*                                                                      */
/* Collision branch (particle sources only, when rc > 0): for a pair    */
/* with r <= rc (decided as dx*dx + dy*dy + dz*dz <= rc*rc, summed left */
/* to right) Eq. (2) replaces the term by                               */
/*     [ G mj / (rc^2 + eps^2)^(3/2)                                     */
/*       + mj/(mi + mj) (kappa (r - rc)/r + eta (rij . vij)/r^2) ] rij, */
/* vij = vj - vi: gravity frozen at its value on the contact sphere (at */
/* eps = 0 exactly the paper's G mj/rc^3) plus a linear spring and a    */
/* radial dashpot acting on the relative motion.  The potential of a    */
/* contact pair is that of the gravity part, continuous at rc:          */
/*     -G mj [1/sqrt(rc^2+eps^2) + (rc^2 - r^2)/(2 (rc^2+eps^2)^(3/2))]. */
/* A pair at r = 0 (i itself) adds nothing.                             */
/*                                                                      */
/* magsum[i] accumulates |term| (a scale for parity tolerances).  All   */
/* arrays are in sorted (tree) order.                                   */
/* ------------------------------------------------------------------ */
typedef struct {
    double rc, kappa, eta;          /* rc = 0: gravity branch only */
    const double *vx, *vy, *vz;     /* velocities, needed when rc > 0 */
} orc_contact;

static void add_term(double xi, double yi, double zi, double xj, double yj, double zj, double mj,
                     double eps2, double G, double acc[5])
{
    double dx = xj - xi, dy = yj - yi, dz = zj - zi;
    double r2 = dx * dx + dy * dy + dz * dz + eps2;
    if (r2 == 0.0) return;           /* only when eps = 0 and j = i */
    double r = sqrt(r2);
    double f = G * mj / (r2 * r);
    acc[0] += f * dx;
    acc[1] += f * dy;
    acc[2] += f * dz;
    acc[3] -= G * mj / r;
    acc[4] += fabs(f) * sqrt(dx * dx + dy * dy + dz * dz);
}

/* A particle source j acting on particle i: Eq. (2) with both branches. */
static void add_particle(int64_t i, int64_t j, const double *x, const double *y, const double *z,
                         const double *m, double eps2, double G, const orc_contact *C, double acc[5])
{
    if (C->rc > 0.0) {
        double dx = x[j] - x[i], dy = y[j] - y[i], dz = z[j] - z[i];
        double d2 = dx * dx + dy * dy + dz * dz;
        if (d2 <= C->rc * C->rc) {
            if (d2 == 0.0) return;
            double r = sqrt(d2);
            double rce2 = C->rc * C->rc + eps2;
            double rce = sqrt(rce2);
            double fg = G * m[j] / (rce2 * rce);
            double dvx = C->vx[j] - C->vx[i], dvy = C->vy[j] - C->vy[i], dvz = C->vz[j] - C->vz[i];
            double rv = dx * dvx + dy * dvy + dz * dvz;
            double fc = m[j] / (m[i] + m[j]) * (C->kappa * (r - C->rc) / r + C->eta * rv / d2);
            double f = fg + fc;
            acc[0] += f * dx;
            acc[1] += f * dy;
            acc[2] += f * dz;
            acc[3] -= G * m[j] * (1.0 / rce + (C->rc * C->rc - d2) / (2.0 * rce2 * rce));
            acc[4] += fabs(f) * r;
            return;
        }
    }
    add_term(x[i], y[i], z[i], x[j], y[j], z[j], m[j], eps2, G, acc);
}

void orc_forces(int64_t n_groups, const uint32_t *gbeg, const uint32_t *gcnt,
                const uint32_t *begin, const uint32_t *count,
                const double *x, const double *y, const double *z, const double *m,
                const double *M, const double *cx, const double *cy, const double *cz,
                const int64_t *pc_off, const uint32_t *pc_ids,
                const int64_t *pp_off, const uint32_t *pp_ids,
                double eps, double G,
                const double *vx, const double *vy, const double *vz, double rc, double kappa, double eta,
                double *ax, double *ay, double *az, double *pot, double *magsum)
{
    double eps2 = eps * eps;
    orc_contact C = {rc, kappa, eta, vx, vy, vz};
    #pragma omp parallel for schedule(dynamic, 4)
    for (int64_t g = 0; g < n_groups; ++g) {
        for (uint32_t i = gbeg[g]; i < gbeg[g] + gcnt[g]; ++i) {
            double acc[5] = {0, 0, 0, 0, 0};
            for (int64_t k = pp_off[g]; k < pp_off[g + 1]; ++k) {
                uint32_t leaf = pp_ids[k];
                for (uint32_t j = begin[leaf]; j < begin[leaf] + count[leaf]; ++j)
                    add_particle(i, j, x, y, z, m, eps2, G, &C, acc);
            }
            for (int64_t k = pc_off[g]; k < pc_off[g + 1]; ++k) {
                uint32_t c = pc_ids[k];
                add_term(x[i], y[i], z[i], cx[c], cy[c], cz[c], M[c], eps2, G, acc);
            }
            ax[i] = acc[0];
            ay[i] = acc[1];
            az[i] = acc[2];
            if (pot) pot[i] = acc[3];
            if (magsum) magsum[i] = acc[4];
        }
    }
}

/* ------------------------------------------------------------------ */
/* Direct summation: the exact force the tree approximates.  For each   */
/* target t the sum runs over every particle j (j = t included; with    */
/* eps > 0 it adds nothing to the acceleration); every pair is a        */
/* particle pair, so the collision branch applies wherever rc > 0.      */
/* ------------------------------------------------------------------ */
void orc_direct(int64_t n, const double *x, const double *y, const double *z, const double *m,
                double eps, double G, int64_t nt, const int64_t *targets,
                const double *vx, const double *vy, const double *vz, double rc, double kappa, double eta,
                double *ax, double *ay, double *az, double *pot)
{
    double eps2 = eps * eps;
    orc_contact C = {rc, kappa, eta, vx, vy, vz};
    #pragma omp parallel for schedule(dynamic, 8)
    for (int64_t t = 0; t < nt; ++t) {
        int64_t i = targets ? targets[t] : t;
        double acc[5] = {0, 0, 0, 0, 0};
        for (int64_t j = 0; j < n; ++j)
            add_particle(i, j, x, y, z, m, eps2, G, &C, acc);
        ax[t] = acc[0];
        ay[t] = acc[1];
        az[t] = acc[2];
        if (pot) pot[t] = acc[3];
    }
}

/* External point mass at the origin (the planet of the ring problem,  */
/* Sec. 2): acceleration -G Mc x / |x|^3, exact FP64.                   */
void orc_central(int64_t n, const double *x, const double *y, const double *z, double Mc, double G,
                 double *ax, double *ay, double *az)
{
    for (int64_t i = 0; i < n; ++i) {
        double r2 = x[i] * x[i] + y[i] * y[i] + z[i] * z[i];
        double r = sqrt(r2);
        double f = -G * Mc / (r2 * r);
        ax[i] += f * x[i];
        ay[i] += f * y[i];
        az[i] += f * z[i];
    }
}

/* Which OpenMP thread count the parallel loops above use. */
int orc_threads(void)
{
    int t = 1;
    #pragma omp parallel
    {
        #pragma omp single
        {
#ifdef _OPENMP
            extern int omp_get_num_threads(void);
            t = omp_get_num_threads();
#endif
        }
    }
    return t;
}

/* ================================================================== */
/* Learned opening rule (an addition to the walk of Sec. 4.2 (3d); the  */
/* paper's walk uses a fixed rule).  Written out in the order the rule  */
/* is defined, so that every acceptance decision can be reproduced:     */
/*   features of a (group, node) pair, lg2p of FP64 values, to FP32:    */
/*     (side/d_box)^2 (d_box: node centre to group box, grid units),    */
/*     group half-diagonal/d, M/M_system, node qn,                      */
/*     d = |com - group centre|, qn = |Q|_F/(M side^2);                 */
/*   network 4-32-32-1 (ReLU) in FP32, each unit a fused multiply-add   */
/*   chain over its inputs in index order starting from the bias;       */
/*   accept iff y < lg2p(tau A_g d^2 / (G M)), in FP64;                 */
/*   lg2p(x) = e - 2 + 2m for x = m 2^e, m in [0.5, 1).                 */
/* ================================================================== */
#define ORC_NH 32
#define ORC_NIN 4
#define ORC_W1 0
#define ORC_B1 128
#define ORC_W2 160
#define ORC_B2 1184
#define ORC_W3 1216
#define ORC_B3 1248
#define ORC_XMEAN 1249
#define ORC_XISTD 1253
#define ORC_YMEAN 1257
#define ORC_YSTD 1258

double orc_lg2p(double x)
{
    if (!(x > 0.0)) return -1100.0;
    if (isinf(x)) return 1100.0;
    int e;
    double m = frexp(x, &e);
    return (double)e + ((2.0 * m) - 2.0);
}

float orc_node_qn(const double *Q, double M, double side)
{
    double qq = Q[0] * Q[0] + Q[3] * Q[3] + Q[5] * Q[5] + 2.0 * (Q[1] * Q[1]) + 2.0 * (Q[2] * Q[2]) +
                2.0 * (Q[4] * Q[4]);
    return (float)(sqrt(qq) / (M * (side * side)));
}

/* (side / distance from the node's geometric centre to the group box)^2,  */
/* from the doubled integer grid units of the opening test.                */
double orc_box_ratio2(const int32_t *gb, int lvl, uint64_t pfx)
{
    uint32_t p[3];
    deinterleave3(pfx, lvl, p);
    int64_t s = (int64_t)1 << (ORC_MAXLEVEL - lvl);
    int64_t d2 = 0;
    for (int a = 0; a < 3; ++a) {
        int64_t L = (int64_t)p[a] << (ORC_MAXLEVEL - lvl);
        int64_t C = 2 * L + s, da = 0;
        if (2 * (int64_t)gb[a] - C > da) da = 2 * (int64_t)gb[a] - C;
        if (C - 2 * (int64_t)gb[3 + a] > da) da = C - 2 * (int64_t)gb[3 + a];
        d2 += da * da;
    }
    return (double)((2 * s) * (2 * s)) / (double)d2;
}

/* Features of node (com, M, box ratio r2, qn) for a group (centre,       */
/* half-diagonal).                                                         */
void orc_features(const double *com, double M, double r2, float qn, const double *gcen, double grad,
                  double Msys, float *f, double *d2_out)
{
    double dx = com[0] - gcen[0], dy = com[1] - gcen[1], dz = com[2] - gcen[2];
    double d2 = dx * dx + dy * dy + dz * dz;
    double d = sqrt(d2);
    f[0] = (float)orc_lg2p(r2);
    f[1] = (float)orc_lg2p(grad / d);
    f[2] = (float)orc_lg2p(M / Msys);
    f[3] = (float)orc_lg2p((double)qn);
    if (d2_out) *d2_out = d2;
}

float orc_mlp_forward(const float *w, const float *f)
{
    float x[ORC_NIN], h1[ORC_NH];
    for (int k = 0; k < ORC_NIN; ++k) {
        float t = f[k] - w[ORC_XMEAN + k];
        x[k] = t * w[ORC_XISTD + k];
    }
    for (int j = 0; j < ORC_NH; ++j) {
        float a = w[ORC_B1 + j];
        for (int k = 0; k < ORC_NIN; ++k) a = fmaf(w[ORC_W1 + j * ORC_NIN + k], x[k], a);
        h1[j] = a > 0.0f ? a : 0.0f;
    }
    float out = w[ORC_B3];
    for (int j = 0; j < ORC_NH; ++j) {
        float a = w[ORC_B2 + j];
        for (int k = 0; k < ORC_NH; ++k) a = fmaf(w[ORC_W2 + j * ORC_NH + k], h1[k], a);
        float h2 = a > 0.0f ? a : 0.0f;
        out = fmaf(w[ORC_W3 + j], h2, out);
    }
    return fmaf(out, w[ORC_YSTD], w[ORC_YMEAN]);
}

void orc_mlp_forward_batch(const float *w, int64_t n, const float *X, float *out)
{
    for (int64_t i = 0; i < n; ++i) out[i] = orc_mlp_forward(w, X + 4 * i);
}

typedef struct {
    const int32_t *gb;          /* group grid box */
    const double *gcen;         /* group centre */
    double grad, amin, Msys, S; /* half-diagonal, A_g, system mass, root side */
    const uint8_t *level;
    const uint64_t *prefix;
    const uint32_t *count;
    const double *com4;         /* per node: com x, y, z, M */
    const float *qn;
    const float *w;
    double th2, th2_min, th2_max, tau, G;
    uint32_t count_cap;
} learned_walk;

static int learned_decide(const learned_walk *L, uint32_t v)
{
    int lvl = L->level[v];
    if (accept_cell(L->gb, lvl, L->prefix[v], L->th2_min)) return 1;
    if (!accept_cell(L->gb, lvl, L->prefix[v], L->th2_max)) return 0;
    uint32_t cnt = L->count[v];
    if (cnt == 1) return 1;
    if (cnt > L->count_cap) return accept_cell(L->gb, lvl, L->prefix[v], L->th2);
    const double *c = L->com4 + 4 * (size_t)v;
    float f[4];
    double d2;
    orc_features(c, c[3], orc_box_ratio2(L->gb, lvl, L->prefix[v]), L->qn[v], L->gcen, L->grad, L->Msys, f, &d2);
    float y = orc_mlp_forward(L->w, f);
    double Z = ((L->tau * L->amin) * d2) / (L->G * c[3]);
    return (double)y < orc_lg2p(Z);
}

static void learned_rec(const learned_walk *L, uint32_t v, const uint32_t *first_child, const uint8_t *n_child,
                        u32vec *pc, u32vec *pp)
{
    if (learned_decide(L, v)) {
        vpush(pc, v);
    } else if (n_child[v] == 0) {
        vpush(pp, v);
    } else {
        for (int c = 0; c < n_child[v]; ++c) learned_rec(L, first_child[v] + c, first_child, n_child, pc, pp);
    }
}

/* Lists under the learned rule for every group of one system (root node 0),
 * given the node moments (com4: x, y, z, M per node), node features qn,
 * group boxes, centres, half-diagonals and A_g.  Output as orc_lists. */
void orc_lists_learned(int64_t n_groups, const int32_t *gbox, const double *gcen, const double *grad,
                       const double *gamin, const uint8_t *level, const uint64_t *prefix, const uint32_t *count,
                       const uint32_t *first_child, const uint8_t *n_child, const double *com4, const float *qn,
                       const float *w, double S, double theta, double theta_min, double theta_max, double tau,
                       double G, uint32_t count_cap, int64_t *pc_off, int64_t *pp_off, uint32_t *pc_ids,
                       uint32_t *pp_ids)
{
    int64_t *pcn = (int64_t *)calloc((size_t)n_groups, sizeof(int64_t));
    int64_t *ppn = (int64_t *)calloc((size_t)n_groups, sizeof(int64_t));
    for (int pass = 0; pass < (pc_ids && pp_ids ? 2 : 1); ++pass) {
        #pragma omp parallel for schedule(dynamic, 16)
        for (int64_t g = 0; g < n_groups; ++g) {
            learned_walk L;
            L.gb = gbox + 6 * g;
            L.gcen = gcen + 3 * g;
            L.grad = grad[g];
            L.amin = gamin[g];
            L.Msys = com4[3];
            L.S = S;
            L.level = level; L.prefix = prefix; L.count = count; L.com4 = com4; L.qn = qn; L.w = w;
            L.th2 = theta * theta; L.th2_min = theta_min * theta_min; L.th2_max = theta_max * theta_max;
            L.tau = tau; L.G = G; L.count_cap = count_cap;
            u32vec pc = {0, 0, 0}, pp = {0, 0, 0};
            learned_rec(&L, 0, first_child, n_child, &pc, &pp);
            if (pass == 0) {
                pcn[g] = pc.n;
                ppn[g] = pp.n;
            } else {
                qsort(pc.v, (size_t)pc.n, sizeof(uint32_t), cmp_u32);
                qsort(pp.v, (size_t)pp.n, sizeof(uint32_t), cmp_u32);
                if (pc.n) memcpy(pc_ids + pc_off[g], pc.v, (size_t)pc.n * sizeof(uint32_t));
                if (pp.n) memcpy(pp_ids + pp_off[g], pp.v, (size_t)pp.n * sizeof(uint32_t));
            }
            free(pc.v);
            free(pp.v);
        }
        if (pass == 0) {
            pc_off[0] = 0;
            pp_off[0] = 0;
            for (int64_t g = 0; g < n_groups; ++g) {
                pc_off[g + 1] = pc_off[g] + pcn[g];
                pp_off[g + 1] = pp_off[g] + ppn[g];
            }
        }
    }
    free(pcn);
    free(ppn);
}

/* Label of a (group, node) pair: the largest |monopole - exact| force of
 * the node on the group's particles, divided by G M / d^2, d = distance
 * of the node's centre of mass from the group centre; returned in FP64
 * before lg2p (the caller applies lg2p and the rounding to FP32). */
double orc_label_ratio(uint32_t gbeg, uint32_t gcnt, uint32_t cbeg, uint32_t ccnt, const double *x, const double *y,
                       const double *z, const double *m, const double *com4, const double *gcen, double eps,
                       double G)
{
    double eps2 = eps * eps, emax = 0.0;
    double M = com4[3];
    for (uint32_t i = gbeg; i < gbeg + gcnt; ++i) {
        double ex = 0, ey = 0, ez = 0;
        for (uint32_t j = cbeg; j < cbeg + ccnt; ++j) {
            double dx = x[j] - x[i], dy = y[j] - y[i], dz = z[j] - z[i];
            double r2 = dx * dx + dy * dy + dz * dz + eps2;
            double f = m[j] / (r2 * sqrt(r2));
            ex += f * dx;
            ey += f * dy;
            ez += f * dz;
        }
        double dx = com4[0] - x[i], dy = com4[1] - y[i], dz = com4[2] - z[i];
        double r2 = dx * dx + dy * dy + dz * dz + eps2;
        double f = M / (r2 * sqrt(r2));
        double ux = G * (f * dx - ex), uy = G * (f * dy - ey), uz = G * (f * dz - ez);
        double e = sqrt(ux * ux + uy * uy + uz * uz);
        if (e > emax) emax = e;
    }
    double dx = com4[0] - gcen[0], dy = com4[1] - gcen[1], dz = com4[2] - gcen[2];
    double d2 = dx * dx + dy * dy + dz * dz;
    return (emax * d2) / (G * M);
}
