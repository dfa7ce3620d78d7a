/*
 * oracle.c -- plain FP64 CPU oracle for the short-range TreePM gravity solver.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load this library.  It shares no code,
 * header or table with the GPU library and must never serve as its fallback.
 *
 * What it computes (the paper names the method -- a Gadget-style TreePM code
 * whose short-range half is a Barnes-Hut walk opened by an angular criterion,
 * Sec. 2 and Sec. 3.1 -- but leaves the numerics to Gadget-2 and Barnes & Hut;
 * the readings below follow those published definitions):
 *
 *   wrap + quantise      u = x/L - floor(x/L), X = floor(u 2^32)           (exact)
 *   Morton key           30 bits per axis (X >> 2), x-major digit order    (exact)
 *   sort                 by (key, input index)                             (exact)
 *   compressed octree    cells with >= 2 non-empty children, pre-order      (exact)
 *   moments              left-to-right fold over children, COM = S / M      (FP64)
 *   walk                 per target depth-first, BH or relative opening     (FP64)
 *   pair force           G M S_h(r) g(r / 2 r_s) d, d = min-image, r < r_cut (FP64)
 *   direct sum           every pair within r_cut (cell list), theta = 0 case
 *   adjoint              L = sum_i w_i . a_i with frozen decisions
 *
 * Everything is written straight from the definitions, with no blocking or
 * reordering; sums of many terms use Neumaier-compensated summation so that
 * the oracle's own rounding stays at the level of one ulp of the result.
 * Build with -ffp-contract=off and without fast-math.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define TWO32 4294967296.0
/* 2 / sqrt(pi) */
#define TWO_OVER_SQRTPI 1.12837916709551257390

/* ------------------------------------------------------------------------- */
/* tree and parameter records shared with the Python wrapper (ctypes)        */
/* ------------------------------------------------------------------------- */

typedef struct {
    int64_t n;            /* particles */
    double box;
    /* per particle, input order */
    const double* xw;     /* n x 3 wrapped positions */
    const double* mass;   /* n */
    const double* hsml;   /* n, spline support h = 2.8 eps */
    const uint32_t* X;    /* n x 3 integer coordinates */
    /* sorted order */
    const int64_t* perm;  /* sorted position -> input index */
    const int64_t* pparent; /* sorted position -> node holding it as a direct child (-1 if n == 1) */
    /* nodes, pre-order */
    int64_t n_nodes;
    const int32_t* level;
    const int64_t* first;
    const int64_t* count;
    const int64_t* parent;
    const int64_t* skip;
    const uint32_t* corner; /* n_nodes x 3 */
    const int64_t* child_start; /* n_nodes + 1 */
    const int64_t* child;       /* >= 0: node index; < 0: particle sorted position -(s+1) */
    const double* M;            /* n_nodes */
    const double* com;          /* n_nodes x 3 */
    const double* hmax;
    const double* hmin;
    const double* half;         /* NULL for a built tree; after a drift: per-node half-side
                                   of the cube the opening tests use (or_extents) */
} or_tree;

typedef struct {
    double G;
    double r_s;
    double r_cut;
    int32_t criterion;   /* 0 = Barnes-Hut angle, 1 = relative (with geometric guard theta) */
    double theta;
    double alpha;
} or_params;

enum { DEC_PRUNE = 0, DEC_ACCEPT = 1, DEC_OPEN = 2 };

/* ------------------------------------------------------------------------- */
/* compensated sums                                                          */
/* ------------------------------------------------------------------------- */

typedef struct { double s, c; } nsum;

static void nadd(nsum* a, double x)
{
    double t = a->s + x;
    if (fabs(a->s) >= fabs(x)) a->c += (a->s - t) + x;
    else a->c += (x - t) + a->s;
    a->s = t;
}

static double nval(nsum a) { return a.s + a.c; }

/* ------------------------------------------------------------------------- */
/* wrap, quantise, key, sort                                                 */
/* ------------------------------------------------------------------------- */

void or_wrap_quantize(int64_t n, const double* pos, double box, uint32_t* X, double* xw)
{
    for (int64_t i = 0; i < 3 * n; ++i) {
        double u = pos[i] / box;
        u = u - floor(u);
        if (u >= 1.0) u = 0.0;              /* a tiny negative rounded up to 1 */
        X[i] = (uint32_t)floor(u * TWO32);
        xw[i] = u * box;
    }
}

/* Digit at level l (1..30) of the 90-bit key: 4*bit(cx) + 2*bit(cy) + bit(cz),
 * bit index 30 - l of the 30-bit coordinates c = X >> 2. */
static int key_digit(const uint32_t* Xi, int l)
{
    int b = 30 - l;
    uint32_t cx = Xi[0] >> 2, cy = Xi[1] >> 2, cz = Xi[2] >> 2;
    return (int)(4 * ((cx >> b) & 1u) + 2 * ((cy >> b) & 1u) + ((cz >> b) & 1u));
}

void or_morton(int64_t n, const uint32_t* X, uint64_t* hi, uint64_t* lo)
{
    for (int64_t i = 0; i < n; ++i) {
        uint64_t h = 0, q = 0;
        for (int l = 1; l <= 15; ++l) h = (h << 3) | (uint64_t)key_digit(X + 3 * i, l);
        for (int l = 16; l <= 30; ++l) q = (q << 3) | (uint64_t)key_digit(X + 3 * i, l);
        hi[i] = h;
        lo[i] = q;
    }
}

static const uint64_t* g_hi;
static const uint64_t* g_lo;

static int cmp_key_index(const void* pa, const void* pb)
{
    int64_t a = *(const int64_t*)pa, b = *(const int64_t*)pb;
    if (g_hi[a] != g_hi[b]) return g_hi[a] < g_hi[b] ? -1 : 1;
    if (g_lo[a] != g_lo[b]) return g_lo[a] < g_lo[b] ? -1 : 1;
    return a < b ? -1 : (a > b);
}

void or_sort(int64_t n, const uint64_t* hi, const uint64_t* lo, int64_t* perm)
{
    for (int64_t i = 0; i < n; ++i) perm[i] = i;
    g_hi = hi;
    g_lo = lo;
    qsort(perm, (size_t)n, sizeof(int64_t), cmp_key_index);
}

/* ------------------------------------------------------------------------- */
/* compressed octree, built recursively in pre-order                         */
/* ------------------------------------------------------------------------- */

typedef struct {
    const uint64_t* hi;   /* sorted keys */
    const uint64_t* lo;
    const uint32_t* Xs;   /* sorted integer coordinates, 3 per particle */
    int32_t* level;
    int64_t* first;
    int64_t* count;
    int64_t* parent;
    int64_t* skip;
    uint32_t* corner;
    int64_t* child_start;
    int64_t* child;
    int64_t* pparent;
    int64_t n_nodes;
    int64_t n_child;
} builder;

/* digit of sorted key s at level l, read from the stored key words */
static int sorted_digit(const builder* B, int64_t s, int l)
{
    if (l <= 15) return (int)((B->hi[s] >> (3 * (15 - l))) & 7u);
    return (int)((B->lo[s] >> (3 * (30 - l))) & 7u);
}

/* number of leading equal digits of two sorted keys (0..30) */
static int common_digits(const builder* B, int64_t a, int64_t b)
{
    int l = 0;
    while (l < 30 && sorted_digit(B, a, l + 1) == sorted_digit(B, b, l + 1)) ++l;
    return l;
}

static int64_t build_node(builder* B, int64_t a, int64_t b, int64_t par)
{
    int64_t id = B->n_nodes++;
    int lev = common_digits(B, a, b - 1);   /* prefix shared by the whole sorted range */
    B->level[id] = lev;
    B->first[id] = a;
    B->count[id] = b - a;
    B->parent[id] = par;
    for (int k = 0; k < 3; ++k) {
        uint64_t keep = lev == 0 ? 0 : (~((1ull << (32 - lev)) - 1ull)) & 0xffffffffull;
        B->corner[3 * id + k] = (uint32_t)(B->Xs[3 * a + k] & keep);
    }
    /* children, in digit order, are written after this node's slot is reserved;
     * grandchildren are listed when their own node is built, so reserve the
     * child slots first. */
    int64_t kids[64];
    int64_t nk = 0;
    int64_t cstart = B->n_child;
    if (lev == 30) {
        /* bucket of identical keys: its particles are its children, in sorted order */
        B->child_start[id] = cstart;
        for (int64_t s = a; s < b; ++s) {
            B->child[B->n_child++] = -(s + 1);
            B->pparent[s] = id;
        }
        B->skip[id] = B->n_nodes;
        return id;
    }
    /* split the range by digit lev + 1 */
    int64_t lo_s = a;
    while (lo_s < b) {
        int d = sorted_digit(B, lo_s, lev + 1);
        int64_t hi_s = lo_s + 1;
        while (hi_s < b && sorted_digit(B, hi_s, lev + 1) == d) ++hi_s;
        kids[nk++] = lo_s;
        kids[nk++] = hi_s;
        lo_s = hi_s;
    }
    B->child_start[id] = cstart;
    B->n_child += nk / 2;
    for (int64_t c = 0; c < nk / 2; ++c) {
        int64_t s0 = kids[2 * c], s1 = kids[2 * c + 1];
        if (s1 - s0 == 1) {
            B->child[cstart + c] = -(s0 + 1);
            B->pparent[s0] = id;
        } else {
            B->child[cstart + c] = build_node(B, s0, s1, id);
        }
    }
    B->skip[id] = B->n_nodes;
    return id;
}

/* Builds the tree of n sorted keys.  Node arrays need room for n - 1 nodes,
 * child arrays for 2n - 2 entries, child_start for n entries.  Returns the
 * number of nodes (0 when n == 1). */
int64_t or_build_topology(int64_t n, const uint64_t* hi_sorted, const uint64_t* lo_sorted,
                          const uint32_t* X_sorted,
                          int32_t* level, int64_t* first, int64_t* count, int64_t* parent,
                          int64_t* skip, uint32_t* corner, int64_t* child_start,
                          int64_t* child, int64_t* pparent)
{
    builder B = {hi_sorted, lo_sorted, X_sorted, level, first, count, parent, skip, corner,
                 child_start, child, pparent, 0, 0};
    for (int64_t s = 0; s < n; ++s) pparent[s] = -1;
    if (n >= 2) build_node(&B, 0, n, -1);
    child_start[B.n_nodes] = B.n_child;
    return B.n_nodes;
}

/* ------------------------------------------------------------------------- */
/* moments                                                                   */
/* ------------------------------------------------------------------------- */

/* Fold the children of node nd left to right: M <- c1, M <- M + c2, ...
 * A particle child contributes (m_j, m_j x_j).  Children equal to `ov_child`
 * (node index, or -(s+1) for a particle) take the override values instead. */
static void fold_children(const or_tree* T, int64_t nd, const double* Mn, const double* Sn,
                          int64_t ov_child, double ovM, const double* ovS,
                          double* outM, double outS[3])
{
    double M = 0, S[3] = {0, 0, 0};
    for (int64_t c = T->child_start[nd]; c < T->child_start[nd + 1]; ++c) {
        int64_t ch = T->child[c];
        double cm, cs[3];
        if (ch == ov_child) {
            cm = ovM;
            for (int k = 0; k < 3; ++k) cs[k] = ovS[k];
        } else if (ch >= 0) {
            cm = Mn[ch];
            for (int k = 0; k < 3; ++k) cs[k] = Sn[3 * ch + k];
        } else {
            int64_t j = T->perm[-ch - 1];
            cm = T->mass[j];
            for (int k = 0; k < 3; ++k) cs[k] = T->mass[j] * T->xw[3 * j + k];
        }
        if (c == T->child_start[nd]) {
            M = cm;
            for (int k = 0; k < 3; ++k) S[k] = cs[k];
        } else {
            M = M + cm;
            for (int k = 0; k < 3; ++k) S[k] = S[k] + cs[k];
        }
    }
    *outM = M;
    for (int k = 0; k < 3; ++k) outS[k] = S[k];
}

/* Post-order moments; S (n_nodes x 3) is workspace for the first moments.
 * Also the FP32-path derivatives M32 = (float)M and the integer COM, and the
 * softening range h_max / h_min of every node. */
void or_moments(or_tree* T, double* M, double* S, double* com, float* M32, uint32_t* comX,
                double* hmax, double* hmin)
{
    T->M = M;
    for (int64_t nd = T->n_nodes - 1; nd >= 0; --nd) {
        double m, s[3];
        fold_children(T, nd, M, S, INT64_MIN, 0.0, NULL, &m, s);
        M[nd] = m;
        for (int k = 0; k < 3; ++k) {
            S[3 * nd + k] = s[k];
            com[3 * nd + k] = s[k] / m;
            /* modulo 2^32: a drifted centre of mass may lie just outside [0, L) */
            double q = rint(com[3 * nd + k] / T->box * TWO32);
            comX[3 * nd + k] = (uint32_t)(int64_t)q;
        }
        M32[nd] = (float)m;
        double hx = -INFINITY, hn = INFINITY;
        for (int64_t s2 = T->first[nd]; s2 < T->first[nd] + T->count[nd]; ++s2) {
            double h = T->hsml[T->perm[s2]];
            if (h > hx) hx = h;
            if (h < hn) hn = h;
        }
        hmax[nd] = hx;
        hmin[nd] = hn;
    }
}

/* ------------------------------------------------------------------------- */
/* pair kernel                                                               */
/* ------------------------------------------------------------------------- */

static double min_image(double d, double L)
{
    if (d > 0.5 * L) return d - L;
    if (d < -0.5 * L) return d + L;
    return d;
}

/* short-range factor of the erfc-split force: g(u) = erfc(u) + 2u/sqrt(pi) exp(-u^2) */
static double g_short(double u) { return erfc(u) + TWO_OVER_SQRTPI * u * exp(-u * u); }

/* g'(u) = -4 u^2 / sqrt(pi) exp(-u^2) */
static double dg_short(double u) { return -2.0 * TWO_OVER_SQRTPI * u * u * exp(-u * u); }

/* Cubic-spline softened 1/r^3: enclosed-mass fraction / r^3 of the
 * Monaghan-Lattanzio kernel with support h. */
static double spline_S(double r, double h)
{
    if (r >= h) return 1.0 / (r * r * r);
    double q = r / h;
    double h3 = h * h * h;
    if (q < 0.5) return (32.0 / 3.0 + q * q * (32.0 * q - 192.0 / 5.0)) / h3;
    return (64.0 / 3.0 - 48.0 * q + 192.0 / 5.0 * q * q - 32.0 / 3.0 * q * q * q
            - 1.0 / (15.0 * q * q * q)) / h3;
}

static double spline_dS(double r, double h)
{
    if (r >= h) return -3.0 / (r * r * r * r);
    double q = r / h;
    double h4 = h * h * h * h;
    if (q < 0.5) return (-384.0 / 5.0 * q + 96.0 * q * q) / h4;
    return (-48.0 + 384.0 / 5.0 * q - 32.0 * q * q + 1.0 / (5.0 * q * q * q * q)) / h4;
}

/* kernel K(r) = G S_h(r) g(r / 2 r_s): F = M K d */
static double pair_K(const or_params* P, double r, double h)
{
    return P->G * spline_S(r, h) * g_short(r / (2.0 * P->r_s));
}

static double pair_dK(const or_params* P, double r, double h)
{
    double u = r / (2.0 * P->r_s);
    return P->G * (spline_dS(r, h) * g_short(u) + spline_S(r, h) * dg_short(u) / (2.0 * P->r_s));
}

/* ------------------------------------------------------------------------- */
/* node geometry and the opening decision                                    */
/* ------------------------------------------------------------------------- */

/* The side the opening tests use: the cell's side, or after a drift twice the
 * node's half-side (or_extents). */
static double node_side(const or_tree* T, int64_t nd)
{
    return T->half ? 2.0 * T->half[nd] : ldexp(T->box, -T->level[nd]);
}

static double node_centre(const or_tree* T, int64_t nd, int k)
{
    return T->box * (ldexp((double)T->corner[3 * nd + k], -32) + ldexp(1.0, -T->level[nd] - 1));
}

/* Node drift (paper App. A: between rebuilds the tree nodes drift with their
 * particles; the node lengths are then enlarged to keep them conservative).  The
 * topology stays; T->xw holds the moved particles (the built positions plus the
 * displacement, not wrapped again) and or_moments refolds the moments from them.
 * The extent of node nd is the half-side of the cube about its cell centre c
 * that holds all its particles:
 *     half[nd] = max(l/2, max over members j and axes k of |x_jk - c_k|),
 * so a node whose particles stayed in its cell keeps its side. */
void or_extents(const or_tree* T, double* half)
{
    for (int64_t nd = 0; nd < T->n_nodes; ++nd) {
        double h = 0.5 * ldexp(T->box, -T->level[nd]);
        for (int64_t s = T->first[nd]; s < T->first[nd] + T->count[nd]; ++s) {
            int64_t j = T->perm[s];
            for (int k = 0; k < 3; ++k) {
                double e = fabs(T->xw[3 * j + k] - node_centre(T, nd, k));
                if (e > h) h = e;
            }
        }
        half[nd] = h;
    }
}

/* Prune (work only: every source of a pruned cube lies beyond r_cut), then the
 * open / accept decision of target position xi against node nd.  d and r2 are
 * the min-image offset and squared distance to the node's centre of mass. */
static int decide(const or_tree* T, const or_params* P, const double xi[3], double aold,
                  int64_t nd, const double* com, double d[3], double* r2)
{
    double L = T->box, l = node_side(T, nd);
    double rc2 = P->r_cut * P->r_cut;
    double t2 = 0.0;
    int inside = 1;
    for (int k = 0; k < 3; ++k) {
        double dc = min_image(node_centre(T, nd, k) - xi[k], L);
        double t = fabs(dc) - 0.5 * l;
        if (t > 0) t2 += t * t;
        if (!(fabs(dc) < 0.6 * l)) inside = 0;
    }
    if (t2 > rc2 * (1.0 + 1e-6)) return DEC_PRUNE;
    for (int k = 0; k < 3; ++k) d[k] = min_image(com[3 * nd + k] - xi[k], L);
    *r2 = (d[0] * d[0] + d[1] * d[1]) + d[2] * d[2];
    int open = inside;
    if (l * l > (P->theta * P->theta) * *r2) open = 1;
    if (P->criterion == 1 && (P->G * T->M[nd]) * (l * l) > (P->alpha * aold) * (*r2 * *r2)) open = 1;
    if (T->hmin[nd] != T->hmax[nd] && *r2 < T->hmax[nd] * T->hmax[nd]) open = 1;
    return open ? DEC_OPEN : DEC_ACCEPT;
}

/* ------------------------------------------------------------------------- */
/* forward walk                                                              */
/* ------------------------------------------------------------------------- */

typedef struct {
    const or_tree* T;
    const or_params* P;
    int64_t self;         /* input index of the target */
    double xi[3];
    double hi;
    double aold;
    nsum a[3];
    int64_t npp, npn;
    /* adjoint mode */
    const double* w;      /* target cotangent (3), or NULL */
    double* xbar_p;       /* n x 3 particle source adjoints (input order) */
    double* mbar_p;       /* n */
    double* xbar_n;       /* n_nodes x 3 */
    double* mbar_n;       /* n_nodes */
    nsum tgt[3];          /* target adjoint accumulator */
} walker;

static void interact(walker* W, double Msrc, const double d[3], double r2, double h,
                     double* xbar_src, double* mbar_src)
{
    double r = sqrt(r2);
    double K = pair_K(W->P, r, h);
    for (int k = 0; k < 3; ++k) nadd(&W->a[k], Msrc * K * d[k]);
    if (!W->w) return;
    /* J = K I + (K'/r) d d^T ; source gets +M J w, target -M J w, mass gets K (w . d) */
    double wd = (W->w[0] * d[0] + W->w[1] * d[1]) + W->w[2] * d[2];
    double c2 = r > 0 ? pair_dK(W->P, r, h) / r : 0.0;
    for (int k = 0; k < 3; ++k) {
        double v = Msrc * (K * W->w[k] + c2 * wd * d[k]);
        nadd(&W->tgt[k], -v);
        if (xbar_src) {
#ifdef _OPENMP
#pragma omp atomic
#endif
            xbar_src[k] += v;
        }
    }
    if (mbar_src) {
#ifdef _OPENMP
#pragma omp atomic
#endif
        *mbar_src += K * wd;
    }
}

static void walk_node(walker* W, int64_t nd)
{
    const or_tree* T = W->T;
    double d[3], r2 = 0.0, rc2 = W->P->r_cut * W->P->r_cut;
    int dec = decide(T, W->P, W->xi, W->aold, nd, T->com, d, &r2);
    if (dec == DEC_PRUNE) return;
    if (dec == DEC_ACCEPT) {
        if (r2 < rc2) {
            W->npn++;
            double h = W->hi > T->hmax[nd] ? W->hi : T->hmax[nd];
            interact(W, T->M[nd], d, r2, h, W->xbar_n ? W->xbar_n + 3 * nd : NULL,
                     W->mbar_n ? W->mbar_n + nd : NULL);
        }
        return;
    }
    for (int64_t c = T->child_start[nd]; c < T->child_start[nd + 1]; ++c) {
        int64_t ch = T->child[c];
        if (ch >= 0) {
            walk_node(W, ch);
            continue;
        }
        int64_t j = T->perm[-ch - 1];
        if (j == W->self) continue;
        double dj[3];
        for (int k = 0; k < 3; ++k) dj[k] = min_image(T->xw[3 * j + k] - W->xi[k], T->box);
        double rj2 = (dj[0] * dj[0] + dj[1] * dj[1]) + dj[2] * dj[2];
        if (rj2 < rc2) {
            W->npp++;
            double h = W->hi > T->hsml[j] ? W->hi : T->hsml[j];
            interact(W, T->mass[j], dj, rj2, h, W->xbar_p ? W->xbar_p + 3 * j : NULL,
                     W->mbar_p ? W->mbar_p + j : NULL);
        }
    }
}

static void walker_init(walker* W, const or_tree* T, const or_params* P, int64_t i,
                        const double* aold)
{
    memset(W, 0, sizeof(*W));
    W->T = T;
    W->P = P;
    W->self = i;
    for (int k = 0; k < 3; ++k) W->xi[k] = T->xw[3 * i + k];
    W->hi = T->hsml[i];
    W->aold = aold ? aold[i] : 0.0;
}

/* Accelerations (n_t x 3) and interaction counts (n_t x 2: particle-particle,
 * particle-node) of the targets `tgt` (input indices).  aold: |a_old| per
 * particle (input order), used by the relative criterion only. */
void or_walk(const or_tree* T, const or_params* P, int64_t n_t, const int64_t* tgt,
             const double* aold, double* acc, int64_t* counts)
{
#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic, 16)
#endif
    for (int64_t t = 0; t < n_t; ++t) {
        walker W;
        walker_init(&W, T, P, tgt[t], aold);
        if (T->n_nodes > 0) walk_node(&W, 0);
        for (int k = 0; k < 3; ++k) acc[3 * t + k] = nval(W.a[k]);
        counts[2 * t] = W.npp;
        counts[2 * t + 1] = W.npn;
    }
}

/* ------------------------------------------------------------------------- */
/* exact direct short-range sum (cell list), the theta = 0 reference          */
/* ------------------------------------------------------------------------- */

void or_direct(int64_t n, const double* xw, const double* mass, const double* hsml, double box,
               const or_params* P, int64_t n_t, const int64_t* tgt, double* acc, int64_t* counts)
{
    double rc2 = P->r_cut * P->r_cut;
    int64_t nc = (int64_t)floor(box / P->r_cut);
    if (nc > 256) nc = 256;
    int use_cells = nc >= 3;
    int64_t* head = NULL;
    int64_t* next = NULL;
    if (use_cells) {
        head = (int64_t*)malloc(sizeof(int64_t) * (size_t)(nc * nc * nc));
        next = (int64_t*)malloc(sizeof(int64_t) * (size_t)n);
        for (int64_t c = 0; c < nc * nc * nc; ++c) head[c] = -1;
        for (int64_t j = n - 1; j >= 0; --j) {
            int64_t ci[3];
            for (int k = 0; k < 3; ++k) {
                ci[k] = (int64_t)floor(xw[3 * j + k] / box * (double)nc);
                if (ci[k] >= nc) ci[k] = nc - 1;
                if (ci[k] < 0) ci[k] = 0;
            }
            int64_t c = (ci[0] * nc + ci[1]) * nc + ci[2];
            next[j] = head[c];
            head[c] = j;
        }
    }
#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic, 16)
#endif
    for (int64_t t = 0; t < n_t; ++t) {
        int64_t i = tgt[t];
        nsum a[3] = {{0, 0}, {0, 0}, {0, 0}};
        int64_t cnt = 0;
        const double* xi = xw + 3 * i;
        if (use_cells) {
            int64_t ci[3];
            for (int k = 0; k < 3; ++k) {
                ci[k] = (int64_t)floor(xi[k] / box * (double)nc);
                if (ci[k] >= nc) ci[k] = nc - 1;
                if (ci[k] < 0) ci[k] = 0;
            }
            for (int dx = -1; dx <= 1; ++dx)
                for (int dy = -1; dy <= 1; ++dy)
                    for (int dz = -1; dz <= 1; ++dz) {
                        int64_t cx = (ci[0] + dx + nc) % nc, cy = (ci[1] + dy + nc) % nc,
                                cz = (ci[2] + dz + nc) % nc;
                        for (int64_t j = head[(cx * nc + cy) * nc + cz]; j >= 0; j = next[j]) {
                            if (j == i) continue;
                            double d[3];
                            for (int k = 0; k < 3; ++k) d[k] = min_image(xw[3 * j + k] - xi[k], box);
                            double r2 = (d[0] * d[0] + d[1] * d[1]) + d[2] * d[2];
                            if (!(r2 < rc2)) continue;
                            double h = hsml[i] > hsml[j] ? hsml[i] : hsml[j];
                            double K = pair_K(P, sqrt(r2), h);
                            for (int k = 0; k < 3; ++k) nadd(&a[k], mass[j] * K * d[k]);
                            ++cnt;
                        }
                    }
        } else {
            for (int64_t j = 0; j < n; ++j) {
                if (j == i) continue;
                double d[3];
                for (int k = 0; k < 3; ++k) d[k] = min_image(xw[3 * j + k] - xi[k], box);
                double r2 = (d[0] * d[0] + d[1] * d[1]) + d[2] * d[2];
                if (!(r2 < rc2)) continue;
                double h = hsml[i] > hsml[j] ? hsml[i] : hsml[j];
                double K = pair_K(P, sqrt(r2), h);
                for (int k = 0; k < 3; ++k) nadd(&a[k], mass[j] * K * d[k]);
                ++cnt;
            }
        }
        for (int k = 0; k < 3; ++k) acc[3 * t + k] = nval(a[k]);
        counts[t] = cnt;
    }
    free(head);
    free(next);
}

/* ------------------------------------------------------------------------- */
/* adjoint of L = sum_t w_t . a_t with the forward pass's decisions           */
/* ------------------------------------------------------------------------- */

/* Gradients dL/dx (n x 3, input order) and dL/dm (n).  Scatter every
 * interaction's source term onto the particle or node that supplied it, then
 * push node terms down to the particles of the node:
 *   x_j-bar += (m_j / M_n) X_n-bar,  m_j-bar += M_n-bar + X_n-bar . (x_j - X_n) / M_n. */
void or_adjoint(const or_tree* T, const or_params* P, int64_t n_t, const int64_t* tgt,
                const double* aold, const double* w, double* dLdx, double* dLdm,
                double* xbar_n, double* mbar_n)
{
    int64_t n = T->n;
    for (int64_t i = 0; i < 3 * n; ++i) dLdx[i] = 0.0;
    for (int64_t i = 0; i < n; ++i) dLdm[i] = 0.0;
    for (int64_t i = 0; i < 3 * T->n_nodes; ++i) xbar_n[i] = 0.0;
    for (int64_t i = 0; i < T->n_nodes; ++i) mbar_n[i] = 0.0;
    double* tgt_bar = (double*)calloc((size_t)(3 * n_t), sizeof(double));
#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic, 16)
#endif
    for (int64_t t = 0; t < n_t; ++t) {
        walker W;
        walker_init(&W, T, P, tgt[t], aold);
        W.w = w + 3 * t;
        W.xbar_p = dLdx;
        W.mbar_p = dLdm;
        W.xbar_n = xbar_n;
        W.mbar_n = mbar_n;
        if (T->n_nodes > 0) walk_node(&W, 0);
        for (int k = 0; k < 3; ++k) tgt_bar[3 * t + k] = nval(W.tgt[k]);
    }
    for (int64_t t = 0; t < n_t; ++t)
        for (int k = 0; k < 3; ++k) dLdx[3 * tgt[t] + k] += tgt_bar[3 * t + k];
    free(tgt_bar);
    /* push-down over every ancestor of every particle */
#ifdef _OPENMP
#pragma omp parallel for schedule(static)
#endif
    for (int64_t s = 0; s < n; ++s) {
        int64_t j = T->perm[s];
        for (int64_t nd = T->pparent[s]; nd >= 0; nd = T->parent[nd]) {
            double Mn = T->M[nd];
            double dot = 0.0;
            for (int k = 0; k < 3; ++k) {
                dLdx[3 * j + k] += T->mass[j] / Mn * xbar_n[3 * nd + k];
                dot += xbar_n[3 * nd + k] * (T->xw[3 * j + k] - T->com[3 * nd + k]);
            }
            dLdm[j] += mbar_n[nd] + dot / Mn;
        }
    }
}

/* ------------------------------------------------------------------------- */
/* one-particle gradients: the interactions that involve particle j           */
/* ------------------------------------------------------------------------- */

/* One frozen interaction touching particle j, seen from target i: source is
 * either j itself (node == -1) or an ancestor node of j. */
typedef struct {
    int64_t t;      /* target slot */
    int64_t node;   /* -1: particle j */
} touch;

typedef struct {
    touch* v;
    int64_t n, cap;
} touch_list;

static void touch_push(touch_list* L, int64_t t, int64_t node)
{
    if (L->n == L->cap) {
        L->cap = L->cap ? 2 * L->cap : 256;
        L->v = (touch*)realloc(L->v, sizeof(touch) * (size_t)L->cap);
    }
    L->v[L->n].t = t;
    L->v[L->n].node = node;
    L->n++;
}

/* Ancestor chain of sorted particle s, root first.  Returns its length. */
static int chain_of(const or_tree* T, int64_t s, int64_t chain[64])
{
    int64_t tmp[64];
    int len = 0;
    for (int64_t nd = T->pparent[s]; nd >= 0; nd = T->parent[nd]) tmp[len++] = nd;
    for (int i = 0; i < len; ++i) chain[i] = tmp[len - 1 - i];
    return len;
}

/* Cell grid over the target slots.  A target interacting with particle j, or
 * with a node that contains j, lies within R = r_cut (1 + sqrt(3) theta) of
 * x_j: an accepted node has side l <= theta r and its centre of mass within
 * r < r_cut of the target, and x_j lies in the same cube. */
typedef struct {
    int64_t nc;
    int64_t* head;
    int64_t* next;
} tgrid;

static int64_t cell_coord(double x, double box, int64_t nc)
{
    int64_t c = (int64_t)floor(x / box * (double)nc);
    if (c >= nc) c = nc - 1;
    if (c < 0) c = 0;
    return c;
}

static void tgrid_build(tgrid* G, const or_tree* T, const or_params* P, int64_t n_t,
                        const int64_t* tgt)
{
    double R = P->r_cut * (1.0 + sqrt(3.0) * P->theta) * (1.0 + 1e-6);
    int64_t nc = (int64_t)floor(T->box / R);
    if (nc > 128) nc = 128;
    G->nc = nc >= 3 ? nc : 0;
    G->head = G->next = NULL;
    if (!G->nc) return;
    G->head = (int64_t*)malloc(sizeof(int64_t) * (size_t)(nc * nc * nc));
    G->next = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n_t > 0 ? n_t : 1));
    for (int64_t c = 0; c < nc * nc * nc; ++c) G->head[c] = -1;
    for (int64_t t = n_t - 1; t >= 0; --t) {
        const double* x = T->xw + 3 * tgt[t];
        int64_t c = (cell_coord(x[0], T->box, nc) * nc + cell_coord(x[1], T->box, nc)) * nc
                    + cell_coord(x[2], T->box, nc);
        G->next[t] = G->head[c];
        G->head[c] = t;
    }
}

static void tgrid_free(tgrid* G)
{
    free(G->head);
    free(G->next);
}

static void touch_one(const or_tree* T, const or_params* P, const int64_t* tgt, const double* aold,
                      int64_t j, const int64_t* chain, int clen, int64_t t, touch_list* out);

/* Targets (slots) whose frozen walk interacts with particle j or one of its
 * ancestors: follow j's chain from the root with target i's decisions. */
static void collect_touches(const or_tree* T, const or_params* P, const tgrid* G, int64_t n_t,
                            const int64_t* tgt, const double* aold, int64_t j,
                            const int64_t* chain, int clen, touch_list* out)
{
    if (!G->nc) {
        for (int64_t t = 0; t < n_t; ++t) touch_one(T, P, tgt, aold, j, chain, clen, t, out);
        return;
    }
    int64_t nc = G->nc, ci[3];
    for (int k = 0; k < 3; ++k) ci[k] = cell_coord(T->xw[3 * j + k], T->box, nc);
    for (int dx = -1; dx <= 1; ++dx)
        for (int dy = -1; dy <= 1; ++dy)
            for (int dz = -1; dz <= 1; ++dz) {
                int64_t c = (((ci[0] + dx + nc) % nc) * nc + (ci[1] + dy + nc) % nc) * nc
                            + (ci[2] + dz + nc) % nc;
                for (int64_t t = G->head[c]; t >= 0; t = G->next[t])
                    touch_one(T, P, tgt, aold, j, chain, clen, t, out);
            }
}

static void touch_one(const or_tree* T, const or_params* P, const int64_t* tgt, const double* aold,
                      int64_t j, const int64_t* chain, int clen, int64_t t, touch_list* out)
{
    double rc2 = P->r_cut * P->r_cut;
    {
        int64_t i = tgt[t];
        if (i == j) return;
        const double* xi = T->xw + 3 * i;
        double a = aold ? aold[i] : 0.0;
        int reached = 1;
        for (int c = 0; c < clen; ++c) {
            double d[3], r2 = 0.0;
            int dec = decide(T, P, xi, a, chain[c], T->com, d, &r2);
            if (dec == DEC_PRUNE) { reached = 0; break; }
            if (dec == DEC_ACCEPT) {
                if (r2 < rc2) touch_push(out, t, chain[c]);
                reached = 0;
                break;
            }
        }
        if (!reached) return;
        double d[3];
        for (int k = 0; k < 3; ++k) d[k] = min_image(T->xw[3 * j + k] - xi[k], T->box);
        double r2 = (d[0] * d[0] + d[1] * d[1]) + d[2] * d[2];
        if (r2 < rc2) touch_push(out, t, -1);
    }
}

/* Gradient of L with respect to the position and mass of the particles `js`
 * (input indices), each computed on its own from the interactions it takes
 * part in: as a target, as a particle source, and through the centre of mass
 * and mass of every ancestor node that some target accepts. */
void or_gradient_of(const or_tree* T, const or_params* P, int64_t n_t, const int64_t* tgt,
                    const double* aold, const double* w, int64_t n_j, const int64_t* js,
                    double* gx, double* gm)
{
    int64_t n = T->n;
    int64_t* slot = (int64_t*)malloc(sizeof(int64_t) * (size_t)n);
    int64_t* spos = (int64_t*)malloc(sizeof(int64_t) * (size_t)n);
    for (int64_t i = 0; i < n; ++i) slot[i] = -1;
    for (int64_t t = 0; t < n_t; ++t) slot[tgt[t]] = t;
    for (int64_t s = 0; s < n; ++s) spos[T->perm[s]] = s;
    tgrid G;
    tgrid_build(&G, T, P, n_t, tgt);
#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic, 1)
#endif
    for (int64_t q = 0; q < n_j; ++q) {
        int64_t j = js[q];
        nsum g[4] = {{0, 0}, {0, 0}, {0, 0}, {0, 0}};
        /* j as a target */
        if (slot[j] >= 0) {
            walker W;
            walker_init(&W, T, P, j, aold);
            W.w = w + 3 * slot[j];
            if (T->n_nodes > 0) walk_node(&W, 0);
            for (int k = 0; k < 3; ++k) nadd(&g[k], nval(W.tgt[k]));
        }
        int64_t chain[64];
        int clen = chain_of(T, spos[j], chain);
        touch_list L = {NULL, 0, 0};
        collect_touches(T, P, &G, n_t, tgt, aold, j, chain, clen, &L);
        for (int64_t e = 0; e < L.n; ++e) {
            int64_t t = L.v[e].t, nd = L.v[e].node, i = tgt[t];
            const double* xi = T->xw + 3 * i;
            const double* wi = w + 3 * t;
            double Ms, src[3], h;
            if (nd < 0) {
                Ms = T->mass[j];
                for (int k = 0; k < 3; ++k) src[k] = T->xw[3 * j + k];
                h = T->hsml[i] > T->hsml[j] ? T->hsml[i] : T->hsml[j];
            } else {
                Ms = T->M[nd];
                for (int k = 0; k < 3; ++k) src[k] = T->com[3 * nd + k];
                h = T->hsml[i] > T->hmax[nd] ? T->hsml[i] : T->hmax[nd];
            }
            double d[3];
            for (int k = 0; k < 3; ++k) d[k] = min_image(src[k] - xi[k], T->box);
            double r2 = (d[0] * d[0] + d[1] * d[1]) + d[2] * d[2];
            double r = sqrt(r2);
            double K = pair_K(P, r, h);
            double c2 = r > 0 ? pair_dK(P, r, h) / r : 0.0;
            double wd = (wi[0] * d[0] + wi[1] * d[1]) + wi[2] * d[2];
            double srcbar[3];
            for (int k = 0; k < 3; ++k) srcbar[k] = Ms * (K * wi[k] + c2 * wd * d[k]);
            if (nd < 0) {
                for (int k = 0; k < 3; ++k) nadd(&g[k], srcbar[k]);
                nadd(&g[3], K * wd);
            } else {
                double dot = 0.0;
                for (int k = 0; k < 3; ++k) {
                    nadd(&g[k], T->mass[j] / Ms * srcbar[k]);
                    dot += srcbar[k] * (T->xw[3 * j + k] - T->com[3 * nd + k]);
                }
                nadd(&g[3], K * wd);
                nadd(&g[3], dot / Ms);
            }
        }
        free(L.v);
        for (int k = 0; k < 3; ++k) gx[3 * q + k] = nval(g[k]);
        gm[q] = nval(g[3]);
    }
    tgrid_free(&G);
    free(slot);
    free(spos);
}

/* ------------------------------------------------------------------------- */
/* central finite differences of the frozen-decision loss                     */
/* ------------------------------------------------------------------------- */

/* Centres of mass and masses of j's ancestors after moving particle j to
 * (xj, mj), refolded bottom-up with the same child order as the forward. */
static void refold_chain(const or_tree* T, const double* S, int64_t s, const int64_t* chain,
                         int clen, const double xj[3], double mj, double* cM, double* cCom)
{
    double ovM = mj, ovS[3];
    for (int k = 0; k < 3; ++k) ovS[k] = mj * xj[k];
    int64_t ov = -(s + 1);
    for (int c = clen - 1; c >= 0; --c) {
        double m, sv[3];
        fold_children(T, chain[c], T->M, S, ov, ovM, ovS, &m, sv);
        cM[c] = m;
        for (int k = 0; k < 3; ++k) cCom[3 * c + k] = sv[k] / m;
        ov = chain[c];
        ovM = m;
        for (int k = 0; k < 3; ++k) ovS[k] = sv[k];
    }
}

/* Frozen interactions of target j itself: list of (kind, index). */
typedef struct {
    int64_t* v;
    int64_t n, cap;
} ilist;

static void ilist_push(ilist* L, int64_t x)
{
    if (L->n == L->cap) {
        L->cap = L->cap ? 2 * L->cap : 256;
        L->v = (int64_t*)realloc(L->v, sizeof(int64_t) * (size_t)L->cap);
    }
    L->v[L->n++] = x;
}

static void record_node(const or_tree* T, const or_params* P, const double* xi, double a,
                        int64_t self, double hi, int64_t nd, ilist* out)
{
    double d[3], r2 = 0.0, rc2 = P->r_cut * P->r_cut;
    int dec = decide(T, P, xi, a, nd, T->com, d, &r2);
    (void)hi;
    if (dec == DEC_PRUNE) return;
    if (dec == DEC_ACCEPT) {
        if (r2 < rc2) ilist_push(out, nd);
        return;
    }
    for (int64_t c = T->child_start[nd]; c < T->child_start[nd + 1]; ++c) {
        int64_t ch = T->child[c];
        if (ch >= 0) {
            record_node(T, P, xi, a, self, hi, ch, out);
            continue;
        }
        int64_t j = T->perm[-ch - 1];
        if (j == self) continue;
        double dj[3];
        for (int k = 0; k < 3; ++k) dj[k] = min_image(T->xw[3 * j + k] - xi[k], T->box);
        double rj2 = (dj[0] * dj[0] + dj[1] * dj[1]) + dj[2] * dj[2];
        if (rj2 < rc2) ilist_push(out, -(j + 1));
    }
}

static void force_on(const or_tree* T, const or_params* P, const double xi[3], double hi,
                     double Ms, const double src[3], double hs, double F[3])
{
    double d[3];
    for (int k = 0; k < 3; ++k) d[k] = min_image(src[k] - xi[k], T->box);
    double r2 = (d[0] * d[0] + d[1] * d[1]) + d[2] * d[2];
    double h = hi > hs ? hi : hs;
    double K = pair_K(P, sqrt(r2), h);
    for (int k = 0; k < 3; ++k) F[k] = Ms * K * d[k];
}

/* Central differences of the frozen-decision L for the particles `js`: the
 * position step is hx (absolute, per axis), the mass step hm_rel * m_j.
 * S (n_nodes x 3) holds the node first moments from or_moments. */
void or_fd_gradient_of(const or_tree* T, const or_params* P, const double* S, int64_t n_t,
                       const int64_t* tgt, const double* aold, const double* w, int64_t n_j,
                       const int64_t* js, double hx, double hm_rel, double* gx, double* gm)
{
    int64_t n = T->n;
    int64_t* slot = (int64_t*)malloc(sizeof(int64_t) * (size_t)n);
    int64_t* spos = (int64_t*)malloc(sizeof(int64_t) * (size_t)n);
    for (int64_t i = 0; i < n; ++i) slot[i] = -1;
    for (int64_t t = 0; t < n_t; ++t) slot[tgt[t]] = t;
    for (int64_t s = 0; s < n; ++s) spos[T->perm[s]] = s;
    tgrid G;
    tgrid_build(&G, T, P, n_t, tgt);
#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic, 1)
#endif
    for (int64_t q = 0; q < n_j; ++q) {
        int64_t j = js[q], s = spos[j];
        int64_t chain[64];
        int clen = chain_of(T, s, chain);
        touch_list L = {NULL, 0, 0};
        collect_touches(T, P, &G, n_t, tgt, aold, j, chain, clen, &L);
        ilist own = {NULL, 0, 0};
        if (slot[j] >= 0 && T->n_nodes > 0)
            record_node(T, P, T->xw + 3 * j, aold ? aold[j] : 0.0, j, T->hsml[j], 0, &own);
        double cM[64], cCom[192];
        /* 4 coordinates (x, y, z, m) x 2 signs */
        for (int comp = 0; comp < 4; ++comp) {
            nsum diff = {0, 0};
            for (int sg = 0; sg < 2; ++sg) {
                double sign = sg == 0 ? 1.0 : -1.0;
                double xj[3], mj = T->mass[j];
                for (int k = 0; k < 3; ++k) xj[k] = T->xw[3 * j + k];
                if (comp < 3) xj[comp] += sign * hx;
                else mj = T->mass[j] * (1.0 + sign * hm_rel);
                refold_chain(T, S, s, chain, clen, xj, mj, cM, cCom);
                /* j as a target (position only) */
                if (comp < 3 && slot[j] >= 0) {
                    const double* wj = w + 3 * slot[j];
                    for (int64_t e = 0; e < own.n; ++e) {
                        int64_t x = own.v[e];
                        double F[3];
                        if (x >= 0)
                            force_on(T, P, xj, T->hsml[j], T->M[x], T->com + 3 * x, T->hmax[x], F);
                        else {
                            int64_t p = -x - 1;
                            force_on(T, P, xj, T->hsml[j], T->mass[p], T->xw + 3 * p, T->hsml[p], F);
                        }
                        for (int k = 0; k < 3; ++k) nadd(&diff, sign * wj[k] * F[k]);
                    }
                }
                for (int64_t e = 0; e < L.n; ++e) {
                    int64_t t = L.v[e].t, nd = L.v[e].node, i = tgt[t];
                    const double* wi = w + 3 * t;
                    double F[3];
                    if (nd < 0) {
                        force_on(T, P, T->xw + 3 * i, T->hsml[i], mj, xj, T->hsml[j], F);
                    } else {
                        int c = 0;
                        while (chain[c] != nd) ++c;
                        force_on(T, P, T->xw + 3 * i, T->hsml[i], cM[c], cCom + 3 * c, T->hmax[nd], F);
                    }
                    for (int k = 0; k < 3; ++k) nadd(&diff, sign * wi[k] * F[k]);
                }
            }
            double step = comp < 3 ? hx : hm_rel * T->mass[j];
            if (comp < 3) gx[3 * q + comp] = nval(diff) / (2.0 * step);
            else gm[q] = nval(diff) / (2.0 * step);
        }
        free(L.v);
        free(own.v);
    }
    tgrid_free(&G);
    free(slot);
    free(spos);
}

/* Frozen interaction lists of every target (CSR over target slots), for
 * small-N references that re-evaluate the same interactions elsewhere.
 * Entry >= 0: node index; < 0: particle -(j+1) (input index).  Returns the
 * total entry count; if it exceeds cap nothing beyond cap is written. */
int64_t or_interaction_lists(const or_tree* T, const or_params* P, int64_t n_t, const int64_t* tgt,
                             const double* aold, int64_t cap, int64_t* start, int64_t* entries)
{
    int64_t total = 0;
    for (int64_t t = 0; t < n_t; ++t) {
        int64_t i = tgt[t];
        ilist L = {NULL, 0, 0};
        if (T->n_nodes > 0) record_node(T, P, T->xw + 3 * i, aold ? aold[i] : 0.0, i, T->hsml[i], 0, &L);
        start[t] = total;
        for (int64_t e = 0; e < L.n; ++e) {
            if (total + e < cap) entries[total + e] = L.v[e];
        }
        total += L.n;
        free(L.v);
    }
    start[n_t] = total;
    return total;
}

/* scalar pair-kernel probes for the pins */
double or_g_short(double u) { return g_short(u); }
double or_dg_short(double u) { return dg_short(u); }
double or_spline_S(double r, double h) { return spline_S(r, h); }
double or_spline_dS(double r, double h) { return spline_dS(r, h); }

int or_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
