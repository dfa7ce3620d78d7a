// SPH density with an iterated smoothing length, on the tree of tree_build.
//
// The paper's density module iterates each particle's smoothing length until
// its kernel sphere holds a fixed number of neighbours (Sec. 2), gathering the
// neighbours of a group of particles first and evaluating them after, in
// chunks (its GPU-porting subsection).  With Gadget-2's cubic spline of support
// h, W(r, h) = 8 / (pi h^3) w(r / h), the density rho_i(h) = sum_j m_j
// W(r_ij, h) (self included, minimum image) and the mass-weighted neighbour
// number N_i(h) = (4 pi / 3) h^3 rho_i(h) / m_i = (32/3) sum_j (m_j / m_i)
// w(r_ij / h), h_i is the root of N_i(h) = T.  N_i is strictly increasing in h
// once a neighbour lies inside, so the root is unique.
//
// Groups are 64 Morton-consecutive particles (lane l = sorted particle 64 g +
// l).  Three kernels per iteration:
//   gather  (only when some h left its group's gathered radius): one wave per
//           group walks the tree breadth-first, lane-parallel over the level's
//           nodes, and lists every particle within R of the box of the
//           group's active particles, R = a margin times their largest h; the
//           candidates go to chunks of 64, UCH chunks to a unit;
//   eval    one wave per unit: the unit's candidates are staged in LDS and
//           every lane sums m_j w, m_j q w' and m_j q^2 w'' over those inside
//           its own h;
//   update  one wave per group: the units' sums in order, then a safeguarded
//           Halley step in h^3 inside the bracket found so far.
// The candidates are kept across iterations while every active h stays within
// the gathered radius (and above half of it, so that the lists do not stay far
// larger than the balls).
#include <math.h>

#include "internal.h"

namespace {

constexpr int WAVE = 64;
constexpr int SPH_TPB = 256;
constexpr int SPH_MAX_ITER = 100;
constexpr double SPH_INIT_FRACTION = 0.25;   // the initial density from the smallest ancestor with T/4 particles
constexpr double SPH_GROW = 2.0;             // largest growth of h per step before an upper bound is known
#ifndef SR_SPH_HALLEY_BAND
#define SR_SPH_HALLEY_BAND 0.1
#endif
constexpr double SPH_HALLEY_BAND = SR_SPH_HALLEY_BAND;   // |N - T| / T below which the step is Halley's (else Newton's)
constexpr double SPH_ACCEPT = 1e-5;          // |N - T| / T below which a bracketed Halley step ends the iteration
constexpr int SPH_PARTS = 3;                 // per-unit sums per particle
// Gathered radius / largest active h of the group, and chunks per evaluation
// unit: 1.2 and 2 (against 1.3 and 8: 10.8 -> 9.6 ms per call on clustered 262k,
// 58.4 -> 57.8 ms on the 2M active subset; a wider margin gathers more candidates
// than the regathers it saves).
#ifndef SR_SPH_MARGIN
#define SR_SPH_MARGIN 1.2
#endif
#ifndef SR_SPH_UCH
#define SR_SPH_UCH 2
#endif
constexpr double SPH_MARGIN = SR_SPH_MARGIN;
// margin of a renewed (partial) gather: the groups that ask again, whose h is
// closer to its root than the initial estimate
#ifndef SR_SPH_MARGIN_RENEW
#define SR_SPH_MARGIN_RENEW 1.1
#endif
constexpr double SPH_MARGIN_RENEW = SR_SPH_MARGIN_RENEW;
constexpr int SPH_UCH = SR_SPH_UCH;
#ifndef SR_SPH_GATHER_WG_PER_CU
#define SR_SPH_GATHER_WG_PER_CU 4
#endif
constexpr int SPH_GATHER_WG_PER_CU = SR_SPH_GATHER_WG_PER_CU;   // persistent gather waves per compute unit

enum : int32_t { SPH_ACTIVE = 0, SPH_DONE = 1, SPH_FAILED = 2 };
// list counters: chunks taken, units taken, overflow, next group, active particles,
// regather request
enum { SC_CHUNKS = 0, SC_UNITS = 1, SC_OVERFLOW = 2, SC_GROUP = 3, SC_ACTIVE = 4, SC_REGATHER = 5, SC_WORDS = 8 };
static_assert(SC_WORDS <= 8, "the counters are read back through the handle's 8-word pinned buffer");

inline dim3 sph_grid(int64_t n) { return dim3((unsigned)((n + SPH_TPB - 1) / SPH_TPB)); }

// w(q), q w'(q) and q^2 w''(q) of the cubic spline for 0 <= q <= 1, without a
// branch: as a sum of truncated powers, w(q) = 2 a^3 - 8 b^3 with a = 1 - q and
// b = max(0, 1/2 - q) (which is 1 - 6 q^2 + 6 q^3 below q = 1/2 and 2 (1 - q)^3
// above), so w' = -6 a^2 + 24 b^2 and w'' = 12 a - 48 b.
__device__ inline void spline_w(double q, double& wq, double& qdw, double& q2ddw)
{
    const double a = 1.0 - q, b = fmax(0.5 - q, 0.0);
    const double a2 = a * a, b2 = b * b;
    wq = 2.0 * (a2 * a) - 8.0 * (b2 * b);
    qdw = q * (24.0 * b2 - 6.0 * a2);
    q2ddw = (q * q) * (12.0 * a - 48.0 * b);
}

// sqrt(x) for x >= 0 finite: v_rsq_f64 (relative error up to 2^-23) refined by a
// Goldschmidt step and a Newton correction (each squaring the relative error), and
// 0 for x = 0
__device__ inline double sqrt_refined(double x)
{
    const double y = __builtin_amdgcn_rsq(x);
    double g = x * y, hy = 0.5 * y;
    const double e = fma(-hy, g, 0.5);
    g = fma(g, e, g);
    hy = fma(hy, e, hy);
    const double d = fma(-g, g, x);
    g = fma(d, hy, g);
    return x > 0.0 ? g : 0.0;
}

// Inclusive sum over the 64 lanes of a wave by DPP moves (no LDS round trips):
// shifts by 1, 2, 4 and 8 within each row of 16 lanes (lanes without a source add
// 0), then the total of row 0 added to row 1 and that of row 2 to row 3 (row
// broadcast of lane 15), then the total of rows 0-1 added to rows 2 and 3 (row
// broadcast of lane 31).  Needs the full wave active.
__device__ inline uint32_t wave_scan_incl(uint32_t v)
{
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x111, 0xF, 0xF, true);   // row_shr:1
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x112, 0xF, 0xF, true);   // row_shr:2
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x114, 0xF, 0xF, true);   // row_shr:4
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x118, 0xF, 0xF, true);   // row_shr:8
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x142, 0xA, 0xF, false);  // row_bcast:15, rows 1 and 3
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x143, 0xC, 0xF, false);  // row_bcast:31, rows 2 and 3
    return v;
}

// Minimum image of a separation; inv_box = 1 / L (a product instead of an FP64
// division; the image can differ from d / L rounding only at an exact half-box
// tie, where both images are equally far).
__device__ inline double min_image(double d, double box, double inv_box) { return d - box * rint(d * inv_box); }

// A double moved between lanes by one DPP permutation (both halves; every source
// lane valid for the permutations used here).
template <int CTRL>
__device__ inline double dpp_d(double v)
{
    const uint64_t b = (uint64_t)__double_as_longlong(v);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)b, CTRL, 0xF, 0xF, false);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)(b >> 32), CTRL, 0xF, 0xF, false);
    return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}
__device__ inline double readlane_d(double v, int l)
{
    const uint64_t b = (uint64_t)__double_as_longlong(v);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)b, l);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(b >> 32), l);
    return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}
// Wave-wide max / min (exact, so independent of the order): within each row of 16
// lanes by DPP exchanges (lane pairs 1 and 2 apart in a quad, then the half-row and
// row mirrors), then over the four rows' values read from lanes 0, 16, 32 and 48.
// Needs the full wave active.
template <bool MAX>
__device__ inline double wave_ext_d(double v)
{
    auto f = [](double a, double b) { return MAX ? fmax(a, b) : fmin(a, b); };
    v = f(v, dpp_d<0xB1>(v));    // quad_perm [1, 0, 3, 2]
    v = f(v, dpp_d<0x4E>(v));    // quad_perm [2, 3, 0, 1]
    v = f(v, dpp_d<0x141>(v));   // row_half_mirror
    v = f(v, dpp_d<0x140>(v));   // row_mirror
    return f(f(readlane_d(v, 0), readlane_d(v, 16)), f(readlane_d(v, 32), readlane_d(v, 48)));
}
__device__ inline double wave_max_d(double v) { return wave_ext_d<true>(v); }
__device__ inline double wave_min_d(double v) { return wave_ext_d<false>(v); }

struct SphLists {
    uint64_t* ent;          // candidate range: first sorted particle | count (1..64) << 32; 64 per chunk
    int32_t* chunk_next;
    int32_t* chunk_cnt;
    int32_t* unit_group;
    int32_t* unit_chunk;
    int32_t* unit_nch;
    int32_t* unit_next;
    int32_t* group_head;    // first unit of each group, -1 for none
    double* rad;            // gathered radius of each group (0: no list)
    int32_t* need;          // 1: the group needs new candidates
    double* gbox;           // per group: centre of its active particles' box (3), and 1 if the box
                            // spans more than half the period on some axis
    int32_t* counters;      // SC_WORDS
    uint32_t* front;        // per gather wave: two levels of cap_front node ids
    double* partials;       // per unit: A[64], D[64], E[64]
    int64_t cap_chunks, cap_units, cap_front;
};

// Initial h: from the smallest ancestor of the particle's leaf that holds at
// least T/4 particles (a local density), the radius of a sphere with T
// particles at that node's mean density, l (3 T / (4 pi count))^(1/3), at most
// h_max.
__global__ void k_sph_init(int64_t n, int64_t m, const int32_t* __restrict__ pparent,
                           const int32_t* __restrict__ n_parent, const int32_t* __restrict__ n_count,
                           const WalkRec64* __restrict__ wrec, double target, double box, double h_max,
                           double* __restrict__ h, double* __restrict__ lo, double* __restrict__ hi,
                           int32_t* __restrict__ state)
{
    const int64_t s = blockIdx.x * (int64_t)SPH_TPB + threadIdx.x;
    if (s >= n) return;
    double side = box, count = (double)n;
    int32_t nd = m > 0 ? pparent[s] : -1;
    while (nd >= 0 && (double)n_count[nd] < SPH_INIT_FRACTION * target) nd = n_parent[nd];
    if (nd >= 0) {
        side = wrec[nd].l;
        count = (double)n_count[nd];
    }
    double h0 = side * cbrt(3.0 * target / (4.0 * M_PI * count));
    if (!(h0 > 0.0)) h0 = h_max;
    h[s] = fmin(h0, h_max);
    lo[s] = 0.0;
    hi[s] = -1.0;       // no upper bound yet
    state[s] = SPH_ACTIVE;
}

// Candidate gather, one wave per group that needs new candidates (persistent
// waves take groups from a counter).  Node cubes (cell centre, side l; grown
// after a drift) are tested against the box of the group's active particles
// grown by R along each axis's minimum image: a node farther than R is pruned;
// a node within R as a whole, a small node and a bucket of identical keys give
// all their particles (a contiguous range of the sorted order, no record read);
// any other node is opened, and its particle children within R are listed.
// The candidates are thus a superset of the particles within R of the box (the
// evaluation applies each lane's exact r < h).  The group's previous units are
// marked empty first.
#ifndef SR_SPH_WHOLE
#define SR_SPH_WHOLE 32
#endif
constexpr uint32_t SPH_WHOLE = SR_SPH_WHOLE;   // nodes of at most this many particles are listed whole
#ifndef SR_SPH_PIECE
#define SR_SPH_PIECE 64
#endif
constexpr uint32_t SPH_PIECE = SR_SPH_PIECE;   // largest candidate count of one list entry
static_assert(SPH_PIECE >= 1 && SPH_PIECE <= 64, "a list entry holds 1 to 64 candidates");
#ifndef SR_SPH_CHUNK_CAND
#define SR_SPH_CHUNK_CAND 256
#endif
#ifndef SR_SPH_UNIT_CAND
#define SR_SPH_UNIT_CAND 1024
#endif
constexpr uint32_t SPH_CHUNK_CAND = SR_SPH_CHUNK_CAND;   // a chunk closes at this many candidates
constexpr uint32_t SPH_UNIT_CAND = SR_SPH_UNIT_CAND;     // a unit closes at this many candidates
#ifndef SR_SPH_CHUNK_BATCH
#define SR_SPH_CHUNK_BATCH 16
#endif
constexpr int SPH_CHUNK_BATCH = SR_SPH_CHUNK_BATCH;  // chunk indices a wave reserves per atomic
constexpr int SPH_UNIT_BATCH = 2;    // unit indices a wave reserves per atomic

__global__ __launch_bounds__(WAVE) void k_sph_gather(int64_t n, int64_t m, int64_t groups, double margin,
                                                     const WalkRec64* __restrict__ wrec,
                                                     const int32_t* __restrict__ n_first,
                                                     const int32_t* __restrict__ n_count,
                                                     const Rec64* __restrict__ prec, double box,
                                                     const int32_t* __restrict__ state,
                                                     const double* __restrict__ hs, SphLists S)
{
    const int lane = threadIdx.x;
    const uint64_t below = (1ull << lane) - 1ull;
    const double inv_box = 1.0 / box;
    uint32_t* cur_ids = S.front + (int64_t)blockIdx.x * 2 * S.cap_front;
    uint32_t* nxt_ids = cur_ids + S.cap_front;
    // chunk and unit indices reserved in batches (one atomic per batch on the shared
    // counters) and handed out in order; reserved units never used stay empty
    int32_t c_next = 0, c_end = 0, u_next = 0, u_end = 0;
    auto take_chunk = [&]() __attribute__((always_inline)) -> int32_t {
        if (c_next == c_end) {
            int32_t b = 0;
            if (lane == 0) b = atomicAdd(&S.counters[SC_CHUNKS], SPH_CHUNK_BATCH);
            c_next = __builtin_amdgcn_readfirstlane(b);
            c_end = c_next + SPH_CHUNK_BATCH;
        }
        return c_next++;
    };
    auto take_unit = [&]() __attribute__((always_inline)) -> int32_t {
        if (u_next == u_end) {
            int32_t b = 0;
            if (lane == 0) b = atomicAdd(&S.counters[SC_UNITS], SPH_UNIT_BATCH);
            u_next = __builtin_amdgcn_readfirstlane(b);
            u_end = u_next + SPH_UNIT_BATCH;
            // a reserved unit is empty until it is filled
            if ((uint32_t)lane < (uint32_t)SPH_UNIT_BATCH && u_next + lane < S.cap_units) S.unit_nch[u_next + lane] = 0;
        }
        return u_next++;
    };
    for (;;) {
        int32_t gi = 0;
        if (lane == 0) gi = atomicAdd(&S.counters[SC_GROUP], 1);
        const int64_t g = __builtin_amdgcn_readfirstlane(gi);
        if (g >= groups) break;
        if (S.need[g] == 0) continue;
        // the group's previous units hold no work from now on
        if (lane == 0)
            for (int32_t u = S.group_head[g]; u >= 0; u = S.unit_next[u]) S.unit_nch[u] = 0;
        const int64_t s = g * WAVE + lane;
        const bool act = s < n && state[s] == SPH_ACTIVE;
        Rec64 me{0.0, 0.0, 0.0, 0.0};
        if (act) me = prec[s];
        const double hmax = wave_max_d(act ? hs[s] : 0.0);
        if (!(hmax > 0.0)) {
            if (lane == 0) {
                S.group_head[g] = -1;
                S.rad[g] = 0.0;
                S.need[g] = 0;
            }
            continue;
        }
        const double R = margin * hmax;
        const double R2 = R * R * (1.0 + 1e-6);
        // the box of the active particles: centre and half-width per axis (an axis
        // wider than half the box passes every test)
        double mid[3], hw[3];
        bool wide = false;
        const double xs[3] = {me.x, me.y, me.z};
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const double l = wave_min_d(act ? xs[k] : INFINITY), u = wave_max_d(act ? xs[k] : -INFINITY);
            mid[k] = 0.5 * (l + u);
            wide = wide || u - l > 0.5 * box;
            hw[k] = u - l > 0.5 * box ? box : 0.5 * (u - l);
        }
        // squared distances from the box to the nearest and to the farthest point of
        // the cube of half side e about c
        auto dist2 = [&](const WalkRec64& r, double& near2, double& far2) __attribute__((always_inline)) {
            const double c[3] = {r.cx, r.cy, r.cz}, e = 0.5 * r.l;
            near2 = 0.0;
            far2 = 0.0;
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                const double a = fabs(min_image(c[k] - mid[k], box, inv_box));
                const double t0 = fmax(a - hw[k] - e, 0.0), t1 = fmax(a - hw[k] + e, 0.0);
                near2 += t0 * t0;
                far2 += t1 * t1;
            }
        };

        // ---- the group's list, chunk by chunk ----
        bool overflow = false;
        int32_t cc = -1, prev_chunk = -1, cur_unit = -1, prev_unit = -1, first_unit = -1;
        uint32_t nl = 0, unit_nch = 0;
        // chunks close at 64 entries or SPH_CHUNK_CAND candidates, units at SPH_UCH
        // chunks or SPH_UNIT_CAND candidates, so that no unit holds much more work
        // than another
        uint32_t ncand = 0, ucand = 0;   // candidates in the current chunk / unit
        auto new_chunk = [&]() __attribute__((always_inline)) -> bool {
            const int32_t c = take_chunk();
            if (c >= S.cap_chunks) return false;
            if (unit_nch == 0 || unit_nch == SPH_UCH || ucand >= SPH_UNIT_CAND) {
                const int32_t u = take_unit();
                if (u >= S.cap_units) return false;
                if (lane == 0) {
                    if (cur_unit >= 0) S.unit_nch[cur_unit] = (int32_t)unit_nch;
                    S.unit_group[u] = (int32_t)g;
                    S.unit_chunk[u] = c;
                    S.unit_next[u] = -1;
                    S.unit_nch[u] = 0;
                    if (prev_unit >= 0) S.unit_next[prev_unit] = u;
                }
                if (first_unit < 0) first_unit = u;
                prev_unit = u;
                cur_unit = u;
                unit_nch = 0;
                ucand = 0;
            } else if (lane == 0) {
                S.chunk_next[prev_chunk] = c;
            }
            if (lane == 0) S.chunk_next[c] = -1;
            ++unit_nch;
            prev_chunk = c;
            cc = c;
            nl = 0;
            ncand = 0;
            return true;
        };
        auto close_chunk = [&]() __attribute__((always_inline)) {
            if (lane == 0 && cc >= 0) S.chunk_cnt[cc] = (int32_t)nl;
        };
        auto room = [&]() __attribute__((always_inline)) -> bool {
            if (cc < 0 || nl == (uint32_t)WAVE || ncand >= SPH_CHUNK_CAND) {
                close_chunk();
                if (!new_chunk()) {
                    overflow = true;
                    return false;
                }
            }
            return true;
        };
        // list the range entry p (k candidates) of every lane set in b, in lane order:
        // each pass takes the lanes whose entry starts within the chunk's room
        auto append = [&](uint64_t b, uint64_t p, uint32_t k) __attribute__((always_inline)) {
            while (b && room()) {
                const uint32_t mine = (b >> lane) & 1 ? k : 0u;
                const uint32_t incl = wave_scan_incl(mine);
                const uint32_t rank = (uint32_t)__popcll(b & below);
                const bool fits = (b >> lane) & 1 && rank < (uint32_t)WAVE - nl && incl - mine < SPH_CHUNK_CAND - ncand;
                const uint64_t take = __ballot(fits);
                if (fits) S.ent[64 * (int64_t)cc + nl + rank] = p;
                // the candidates taken: the prefix at the last lane taken
                const int last = 63 - __builtin_clzll(take);
                const uint32_t added = (uint32_t)__builtin_amdgcn_readlane((int)incl, last);
                nl += (uint32_t)__popcll(take);
                ncand += added;
                ucand += added;
                b &= ~take;
            }
        };
        // list the sorted particles f .. f + c - 1 of every lane with c > 0, as
        // entries of at most SPH_PIECE particles
        auto append_ranges = [&](uint32_t f, uint32_t c) __attribute__((always_inline)) {
            for (;;) {
                const uint64_t b = __ballot(c > 0);
                if (!b || overflow) break;
                const uint32_t k = c < SPH_PIECE ? c : SPH_PIECE;
                append(b, (uint64_t)f | ((uint64_t)k << 32), k);
                f += k;
                c -= k;
            }
        };

        if (m == 0) {
            append_ranges(0u, lane == 0 ? 1u : 0u);   // a single particle: its own candidate
        } else {
            uint32_t na = 1;
            if (lane == 0) cur_ids[0] = 0u;
            __syncthreads();   // (one wave: orders the frontier's global stores before its loads)
            while (na > 0 && !overflow) {
                uint32_t nb = 0;
                // a level's nodes in batches of 64, read ahead: the records of the next
                // batch and the ids of the one after it are read while a batch is
                // processed (lanes past the level's end read node 0, the root)
                auto ids_of = [&](uint32_t b) __attribute__((always_inline)) -> uint32_t {
                    return cur_ids[b + lane < na ? b + lane : 0u];
                };
                uint32_t id_next = ids_of(0);
                uint32_t nd_n = lane < na ? id_next : 0u;
                WalkRec64 r_n = wrec[nd_n];
                uint32_t cnt_n = (uint32_t)n_count[nd_n], first_n = (uint32_t)n_first[nd_n];
                id_next = ids_of(WAVE);
                for (uint32_t b0 = 0; b0 < na && !overflow; b0 += WAVE) {
                    const bool has = b0 + lane < na;
                    const WalkRec64 r = r_n;
                    const uint32_t ncount = cnt_n, nfirst = first_n;
                    if (b0 + WAVE < na) {
                        nd_n = b0 + WAVE + lane < na ? id_next : 0u;
                        r_n = wrec[nd_n];
                        cnt_n = (uint32_t)n_count[nd_n];
                        first_n = (uint32_t)n_first[nd_n];
                        id_next = ids_of(b0 + 2 * WAVE);
                    }
                    bool keep = false, whole = false;
                    if (has) {
                        double near2, far2;
                        dist2(r, near2, far2);
                        keep = near2 <= R2;
                        whole = keep && (far2 <= R2 || r.meta == META_BUCKET || ncount <= SPH_WHOLE);
                    }
                    // nodes listed whole: their particle ranges
                    append_ranges(whole ? nfirst : 0u, whole ? ncount : 0u);
                    // opened nodes: node children to the next level, particle children listed;
                    // the particle children's records are read together first (every
                    // address selected, slots without a particle child read particle 0)
                    const bool open = keep && !whole;
                    bool near8[8];
#pragma unroll
                    for (int k = 0; k < 8; ++k) {
                        const bool kid = open && (uint32_t)k < r.meta;
                        const uint32_t ch = kid ? r.kids[k] : 0u;
                        const bool isp = kid && (ch & ITEM_PARTICLE);
                        const Rec64 p = prec[isp ? ch & ~ITEM_PARTICLE : 0u];
                        const double xp[3] = {p.x, p.y, p.z};
                        double d2 = 0.0;
#pragma unroll
                        for (int a = 0; a < 3; ++a) {
                            const double t = fmax(fabs(min_image(xp[a] - mid[a], box, inv_box)) - hw[a], 0.0);
                            d2 += t * t;
                        }
                        near8[k] = isp && d2 <= R2;
                    }
#pragma unroll
                    for (int k = 0; k < 8; ++k) {
                        const bool kid = open && (uint32_t)k < r.meta;
                        const uint32_t ch = kid ? r.kids[k] : 0u;
                        const bool isnode = kid && !(ch & ITEM_PARTICLE);
                        const uint64_t bn = __ballot(isnode);
                        if (bn) {
                            const uint32_t cnt = (uint32_t)__popcll(bn);
                            if (nb + cnt > S.cap_front) {
                                overflow = true;
                            } else {
                                if (isnode) nxt_ids[nb + __popcll(bn & below)] = ch;
                                nb += cnt;
                            }
                        }
                        append(__ballot(near8[k]), (uint64_t)(ch & ~ITEM_PARTICLE) | (1ull << 32), 1u);
                    }
                }
                // the next level becomes the current one
                uint32_t* t = cur_ids;
                cur_ids = nxt_ids;
                nxt_ids = t;
                na = nb;
                __syncthreads();
            }
        }
        if (overflow) {
            if (lane == 0) atomicOr(&S.counters[SC_OVERFLOW], 1);
            break;
        }
        close_chunk();
        if (lane == 0) {
            if (cur_unit >= 0) S.unit_nch[cur_unit] = (int32_t)unit_nch;
            S.group_head[g] = first_unit;
            S.rad[g] = R;
            S.need[g] = 0;
            S.gbox[4 * g + 0] = mid[0];
            S.gbox[4 * g + 1] = mid[1];
            S.gbox[4 * g + 2] = mid[2];
            S.gbox[4 * g + 3] = wide ? 1.0 : 0.0;
        }
    }
}

// need[g] = 1 for every group with an active particle (a full gather).
__global__ void k_sph_need_all(int64_t n, int64_t groups, const int32_t* __restrict__ state, SphLists S)
{
    const int64_t g = blockIdx.x * (int64_t)(SPH_TPB / WAVE) + threadIdx.x / WAVE;
    const int lane = threadIdx.x % WAVE;
    if (g >= groups) return;
    const int64_t s = g * WAVE + lane;
    const uint64_t a = __ballot(s < n && state[s] == SPH_ACTIVE);
    if (lane == 0) {
        S.need[g] = a != 0;
        S.group_head[g] = -1;   // the pool is reset: no earlier unit is referenced
    }
}

// Sums over one unit's candidates: lane l (sorted particle 64 g + l) adds
// m_j w(r/h) and m_j q w'(q) of every candidate within its h.
__global__ __launch_bounds__(WAVE) void k_sph_eval(int64_t n, const Rec64* __restrict__ prec, double box,
                                                   const int32_t* __restrict__ state,
                                                   const double* __restrict__ hs, SphLists S)
{
    __shared__ Rec64 s_c[WAVE];
    __shared__ uint32_t s_off[WAVE], s_first[WAVE];
    const int lane = threadIdx.x;
    const int32_t u = (int32_t)blockIdx.x;
    if (u >= S.counters[SC_UNITS] || S.counters[SC_OVERFLOW] != 0) return;
    const int32_t nch = S.unit_nch[u];
    if (nch == 0) return;
    const int64_t g = S.unit_group[u];
    const int64_t s = g * WAVE + lane;
    const bool act = s < n && state[s] == SPH_ACTIVE;
    Rec64 me{0.0, 0.0, 0.0, 0.0};
    double hh = 0.0;
    if (act) {
        me = prec[s];
        hh = hs[s];
    }
    const double h2 = hh * hh, inv_h = act ? 1.0 / hh : 0.0, inv_box = 1.0 / box;
    // positions as minimum-image offsets from the centre of the group's box: for a
    // box narrower than half the period on every axis, the separations are the
    // offsets' differences; otherwise their minimum image
    const double cx = S.gbox[4 * g + 0], cy = S.gbox[4 * g + 1], cz = S.gbox[4 * g + 2];
    const bool wide = S.gbox[4 * g + 3] != 0.0;
    const double ox = min_image(me.x - cx, box, inv_box), oy = min_image(me.y - cy, box, inv_box),
                 oz = min_image(me.z - cz, box, inv_box);
    double A = 0.0, D = 0.0, E = 0.0;   // sums of m_j w(q_j), m_j q_j w'(q_j), m_j q_j^2 w''(q_j)
    // the box of the active lanes' offsets and their largest h: a candidate farther
    // from that box than the largest h is inside no lane's ball and is not staged (the
    // bound has a relative margin of 1e-9 over the rounding of the lanes' own
    // separations, so every candidate a lane would count is kept, in its order)
    const double blx = wave_min_d(act ? ox : INFINITY), bhx = wave_max_d(act ? ox : -INFINITY);
    const double bly = wave_min_d(act ? oy : INFINITY), bhy = wave_max_d(act ? oy : -INFINITY);
    const double blz = wave_min_d(act ? oz : INFINITY), bhz = wave_max_d(act ? oz : -INFINITY);
    const double hmax = wave_max_d(hh);
    const double lim2 = hmax * hmax * (1.0 + 1e-9);
    const uint64_t below = (1ull << lane) - 1ull;
    int32_t c = S.unit_chunk[u];
    for (int32_t q = 0; q < nch; ++q) {
        // the chunk's entries (ranges of sorted particles) and their offsets in the
        // chunk's particle sequence
        const int32_t ne = S.chunk_cnt[c];
        const int32_t cnext = S.chunk_next[c];
        uint32_t first = 0, count = 0;
        if (lane < ne) {
            const uint64_t v = S.ent[64 * (int64_t)c + lane];
            first = (uint32_t)v;
            count = (uint32_t)(v >> 32);
        }
        const uint32_t incl = wave_scan_incl(count);
        s_off[lane] = incl - count;
        s_first[lane] = first;
        const uint32_t total = (uint32_t)__builtin_amdgcn_readlane((int)incl, WAVE - 1);
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        // candidate b + lane: the last entry whose offset is at most its index; the
        // record of the next block is loaded while this block is evaluated
        auto fetch = [&](uint32_t b, Rec64& p) __attribute__((always_inline)) {
            const uint32_t idx = b + (uint32_t)lane;
            if (idx < total) {
                uint32_t e = 0;
#pragma unroll
                for (uint32_t step = 32; step; step >>= 1)
                    if (e + step < (uint32_t)ne && s_off[e + step] <= idx) e += step;
                p = prec[s_first[e] + (idx - s_off[e])];
            }
        };
        Rec64 nxt{0.0, 0.0, 0.0, 0.0};
        fetch(0, nxt);
        for (uint32_t base = 0; base < total; base += WAVE) {
            const Rec64 cand{min_image(nxt.x - cx, box, inv_box), min_image(nxt.y - cy, box, inv_box),
                             min_image(nxt.z - cz, box, inv_box), nxt.m};
            bool keep = base + (uint32_t)lane < total && hmax > 0.0;
            if (keep && !wide) {
                const double tx = fmax(fmax(blx - cand.x, cand.x - bhx), 0.0);
                const double ty = fmax(fmax(bly - cand.y, cand.y - bhy), 0.0);
                const double tz = fmax(fmax(blz - cand.z, cand.z - bhz), 0.0);
                keep = (tx * tx + ty * ty) + tz * tz <= lim2;
            }
            const uint64_t kept = __ballot(keep);
            if (keep) s_c[__popcll(kept & below)] = cand;
            fetch(base + WAVE, nxt);
            const int32_t cnt = (int32_t)__popcll(kept);
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            auto candidate = [&](const Rec64& p, double dx, double dy, double dz) __attribute__((always_inline)) {
                const double r2 = (dx * dx + dy * dy) + dz * dz;
                if (r2 < h2) {
                    double wq, qdw, q2ddw;
                    spline_w(sqrt_refined(r2) * inv_h, wq, qdw, q2ddw);
                    A += p.m * wq;
                    D += p.m * qdw;
                    E += p.m * q2ddw;
                }
            };
            if (!wide) {
                // unrolled so that the LDS reads of several candidates are in flight
#pragma unroll 4
                for (int32_t e = 0; e < cnt; ++e) {
                    const Rec64 p = s_c[e];
                    candidate(p, p.x - ox, p.y - oy, p.z - oz);
                }
            } else {
                for (int32_t e = 0; e < cnt; ++e) {
                    const Rec64 p = s_c[e];
                    candidate(p, min_image(p.x - ox, box, inv_box), min_image(p.y - oy, box, inv_box),
                              min_image(p.z - oz, box, inv_box));
                }
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        }
        c = cnext;
    }
    S.partials[(int64_t)u * SPH_PARTS * WAVE + lane] = A;
    S.partials[(int64_t)u * SPH_PARTS * WAVE + WAVE + lane] = D;
    S.partials[(int64_t)u * SPH_PARTS * WAVE + 2 * WAVE + lane] = E;
}

// One group per wave: its units' sums in unit order, then the Halley step.
__global__ __launch_bounds__(WAVE) void k_sph_update(int64_t n, const Rec64* __restrict__ prec, double target,
                                                     double h_max, double* __restrict__ h, double* __restrict__ lo,
                                                     double* __restrict__ hi, int32_t* __restrict__ state,
                                                     double* __restrict__ rho, SphLists S)
{
    const int lane = threadIdx.x;
    const int64_t g = blockIdx.x;
    if (S.counters[SC_OVERFLOW] != 0) return;   // the lists are incomplete: the iteration is repeated
    const int64_t s = g * WAVE + lane;
    const bool act = s < n && state[s] == SPH_ACTIVE;
    const double R = S.rad[g];
    double A = 0.0, D = 0.0, E = 0.0;
    for (int32_t u = S.group_head[g]; u >= 0; u = S.unit_next[u]) {
        A += S.partials[(int64_t)u * SPH_PARTS * WAVE + lane];
        D += S.partials[(int64_t)u * SPH_PARTS * WAVE + WAVE + lane];
        E += S.partials[(int64_t)u * SPH_PARTS * WAVE + 2 * WAVE + lane];
    }
    bool still = false;
    double hn = 0.0;
    if (act) {
        const double hh = h[s];
        const double mi = prec[s].m;
        const double inv_h = 1.0 / hh;
        rho[s] = 8.0 / M_PI * inv_h * inv_h * inv_h * A;
        const double N = 32.0 / 3.0 * A / mi;
        const double f = N - target;
        double l = lo[s], u = hi[s];
        if (!(mi > 0.0)) {
            state[s] = SPH_FAILED;
        } else if (fabs(f) <= 1e-13 * target) {
            state[s] = SPH_DONE;
        } else {
            if (f < 0.0)
                l = hh;
            else
                u = hh;
            if (u > 0.0 && u - l <= 4e-16 * u) {     // the bracket has closed
                state[s] = SPH_DONE;
            } else {
                // Halley's step in v = h^3, where N is close to linear, within
                // SPH_HALLEY_BAND of the target, Newton's farther out (just after a
                // first neighbour enters, N is strongly convex and Halley's steps
                // are short) or where Halley's denominator is not positive; from
                // dN/dh = -(32/3) D / (m h) and d2N/dh2 = (32/3) (E + 2 D) / (m h^2)
                const double Nh = -32.0 / 3.0 * D / (mi * hh);
                const double Nhh = 32.0 / 3.0 * (E + 2.0 * D) / (mi * hh * hh);
                const double h2 = hh * hh;
                const double Nv = Nh / (3.0 * h2);
                const double Nvv = (Nhh - 2.0 * Nh / hh) / (9.0 * h2 * h2);
                hn = -1.0;
                bool halley = false;
                if (Nv > 0.0) {
                    const double den = 2.0 * Nv * Nv - f * Nvv;
                    halley = den > 0.0 && fabs(f) <= SPH_HALLEY_BAND * target;
                    const double v = hh * h2 - (halley ? 2.0 * f * Nv / den : f / Nv);
                    if (v > 0.0) hn = cbrt(v);
                }
                bool failed = false;
                if (u < 0.0) {
                    if (!(hn > hh)) hn = SPH_GROW * hh;
                    hn = fmin(hn, SPH_GROW * hh);
                    if (hn > h_max) {
                        if (hh >= h_max) {              // N(h_max) < T: no root within h_max
                            state[s] = SPH_FAILED;
                            failed = true;
                        } else {
                            hn = h_max;
                        }
                    }
                } else if (!(hn > l && hn < u)) {
                    hn = 0.5 * (l + u);
                    halley = false;
                }
                if (!failed && halley && u > 0.0 && fabs(f) <= SPH_ACCEPT * target) {
                    // Halley's error after the step is of the order of the cube of the
                    // current one: the step lands within the tolerance and is taken as
                    // the root, where N = T gives rho = 3 T m / (4 pi h^3)
                    h[s] = hn;
                    rho[s] = 3.0 * target * mi / (4.0 * M_PI * hn * hn * hn);
                    state[s] = SPH_DONE;
                } else if (!failed) {
                    lo[s] = l;
                    hi[s] = u;
                    h[s] = hn;
                    still = true;
                }
            }
        }
    }
    // one count per wave; a regather when an active h left the gathered radius or
    // every active h fell below half of it
    // per group: new candidates when an active h left the gathered radius or every
    // active h fell below half of it; a group with no active particle left drops
    // its units.  One count per wave.
    const uint64_t live = __ballot(still);
    const uint64_t outside = __ballot(still && hn > R);
    const double hmax = wave_max_d(still ? hn : 0.0);
    if (lane == 0) {
        if (live) {
            atomicAdd(&S.counters[SC_ACTIVE], (int32_t)__popcll(live));
            const bool renew = outside || hmax < 0.5 * R;
            S.need[g] = renew ? 1 : 0;
            if (renew) atomicOr(&S.counters[SC_REGATHER], 1);
        } else {
            for (int32_t u = S.group_head[g]; u >= 0; u = S.unit_next[u]) S.unit_nch[u] = 0;
            S.group_head[g] = -1;
            S.need[g] = 0;
        }
    }
}

__global__ void k_sph_clear(int32_t* p, int32_t k0, int32_t k1)
{
    const int k = (int)threadIdx.x;
    if (k >= k0 && k < k1) p[k] = 0;
}

__global__ void k_sph_out(int64_t n, const int32_t* __restrict__ perm, const double* __restrict__ hs,
                          const double* __restrict__ rs, const int32_t* __restrict__ state,
                          double* __restrict__ h, double* __restrict__ rho, int32_t* __restrict__ failed)
{
    const int64_t s = blockIdx.x * (int64_t)SPH_TPB + threadIdx.x;
    if (s >= n) return;
    const int64_t i = perm[s];
    h[i] = hs[s];
    rho[i] = rs[s];
    if (state[s] != SPH_DONE) atomicAdd(failed, 1);
}

// Workspace of one call, from the stream-ordered allocator: per particle h, lo,
// hi, rho and state; per group the list heads and radii; the lists, frontier and
// partials sized by the capacities.
struct SphWork {
    double* buf = nullptr;      // 4 n doubles
    int32_t* ibuf = nullptr;    // n + SC_WORDS + 1 ints
    void* lists = nullptr;
    int64_t lists_bytes = 0;
};

int lists_alloc(SphWork& W, SphLists& S, int64_t groups, int64_t waves, int64_t chunks, int64_t units,
                int64_t front, int32_t* counters, hipStream_t st)
{
    if (W.lists) (void)hipFreeAsync(W.lists, st);
    W.lists = nullptr;
    auto up = [](int64_t b) { return (b + 255) & ~(int64_t)255; };
    const int64_t bytes = up(64 * chunks * 8) + 2 * up(chunks * 4) + 4 * up(units * 4) + 2 * up(groups * 4) +
                          up(groups * 8) + up(groups * 32) + up(waves * 2 * front * 4) + up(units * SPH_PARTS * WAVE * 8);
    if (hipMallocAsync(&W.lists, (size_t)bytes, st) != hipSuccess) {
        W.lists = nullptr;
        (void)hipGetLastError();
        return sr_fail(SR_ENOMEM, "sph_density: %lld bytes of candidate lists could not be allocated",
                       (long long)bytes);
    }
    W.lists_bytes = bytes;
    char* p = (char*)W.lists;
    auto take = [&](int64_t b) {
        char* q = p;
        p += up(b);
        return q;
    };
    S.ent = (uint64_t*)take(64 * chunks * 8);
    S.chunk_next = (int32_t*)take(chunks * 4);
    S.chunk_cnt = (int32_t*)take(chunks * 4);
    S.unit_group = (int32_t*)take(units * 4);
    S.unit_chunk = (int32_t*)take(units * 4);
    S.unit_nch = (int32_t*)take(units * 4);
    S.unit_next = (int32_t*)take(units * 4);
    S.group_head = (int32_t*)take(groups * 4);
    S.rad = (double*)take(groups * 8);
    S.need = (int32_t*)take(groups * 4);
    S.gbox = (double*)take(groups * 32);
    S.front = (uint32_t*)take(waves * 2 * front * 4);
    S.partials = (double*)take(units * SPH_PARTS * WAVE * 8);
    S.counters = counters;
    S.cap_chunks = chunks;
    S.cap_units = units;
    S.cap_front = front;
    return SR_OK;
}

}  // namespace

extern "C" {

int sph_density(sr_tree* t, double n_ngb, double* h, double* rho, int64_t* unconverged, void* stream)
{
    if (!t) return sr_fail(SR_ESTATE, "sph_density: tree is NULL");
    if (t->n <= 0) return sr_fail(SR_ESTATE, "sph_density: the tree holds no particles");
    if (!(n_ngb > 32.0 / 3.0) || !isfinite(n_ngb))
        return sr_fail(SR_EINVAL, "sph_density: n_ngb must be finite and above 32/3 (got %g)", n_ngb);
    if (!h || !rho) return sr_fail(SR_EINVAL, "sph_density: h and rho are required");
    int dev = 0, cus = 0;
    SR_HIP(hipGetDevice(&dev));
    if (dev != t->device) return sr_fail(SR_ESTATE, "sph_density: tree belongs to device %d, current is %d", t->device, dev);
    SR_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    hipStream_t st = (hipStream_t)stream;
    const int64_t n = t->n, m = t->n_nodes;
    const int64_t groups = (n + WAVE - 1) / WAVE;
    const int64_t waves = groups < (int64_t)SPH_GATHER_WG_PER_CU * cus ? groups : (int64_t)SPH_GATHER_WG_PER_CU * cus;
    const double box = t->box, h_max = 0.25 * box;
    SphWork W;
    if (hipMallocAsync((void**)&W.buf, sizeof(double) * 4 * n, st) != hipSuccess ||
        hipMallocAsync((void**)&W.ibuf, sizeof(int32_t) * (n + SC_WORDS + 1), st) != hipSuccess) {
        if (W.buf) (void)hipFreeAsync(W.buf, st);
        (void)hipGetLastError();
        return sr_fail(SR_ENOMEM, "sph_density: workspace allocation for %lld particles failed", (long long)n);
    }
    double *hs = W.buf, *lo = W.buf + n, *hi = W.buf + 2 * n, *rs = W.buf + 3 * n;
    int32_t *state = W.ibuf, *ctr = W.ibuf + n, *failed = W.ibuf + n + SC_WORDS;
    // list capacities: 32 chunks per group to start, doubled when a full gather overflows
    int64_t chunks = 32 * groups + 1024, units = chunks / 2 + 2 * groups + 2 * waves + 64, front = 4096;
    SphLists S{};
    int rc = lists_alloc(W, S, groups, waves, chunks, units, front, ctr, st);
    int32_t hc[SC_WORDS];
    hipLaunchKernelGGL(k_sph_init, sph_grid(n), dim3(SPH_TPB), 0, st, n, m, t->pparent, t->n_parent, t->n_count,
                       t->wrec64, n_ngb, box, h_max, hs, lo, hi, state);
    // The first gather is a full one (the pool reset, every group with an active
    // particle); later ones renew only the groups that asked, appending to the pool,
    // until one overflows (then a full gather; a full gather that overflows grows
    // the pool).
    // The host reads the counters once per iteration.  An overflowing gather sets a
    // flag that makes the evaluation and the update of that iteration do nothing;
    // the iteration is then repeated with a full gather, or with a grown pool if
    // the full gather overflowed.
    bool gather = true, full = true;
    for (int it = 0; rc == SR_OK && it < SPH_MAX_ITER;) {
        sr_timing_mark(SR_T_SPH_ITER, true, st);
        const bool gathered_full = gather && full;
        if (gather) {
            if (full) {
                hipLaunchKernelGGL(k_sph_clear, dim3(1), dim3(SC_WORDS), 0, st, ctr, 0, SC_WORDS);
                hipLaunchKernelGGL(k_sph_need_all, dim3((unsigned)((groups + SPH_TPB / WAVE - 1) / (SPH_TPB / WAVE))),
                                   dim3(SPH_TPB), 0, st, n, groups, state, S);
            } else {
                hipLaunchKernelGGL(k_sph_clear, dim3(1), dim3(SC_WORDS), 0, st, ctr, SC_OVERFLOW, SC_GROUP + 1);
            }
            hipLaunchKernelGGL(k_sph_gather, dim3((unsigned)waves), dim3(WAVE), 0, st, n, m, groups,
                               full ? SPH_MARGIN : SPH_MARGIN_RENEW, t->wrec64,
                               t->n_first, t->n_count, t->prec64, box, state, hs, S);
        }
        hipLaunchKernelGGL(k_sph_clear, dim3(1), dim3(SC_WORDS), 0, st, ctr, SC_ACTIVE, SC_REGATHER + 1);
        hipLaunchKernelGGL(k_sph_eval, dim3((unsigned)S.cap_units), dim3(WAVE), 0, st, n, t->prec64, box, state, hs, S);
        hipLaunchKernelGGL(k_sph_update, dim3((unsigned)groups), dim3(WAVE), 0, st, n, t->prec64, n_ngb, h_max, hs,
                           lo, hi, state, rs, S);
        sr_timing_mark(SR_T_SPH_ITER, false, st);
        // the counters go to the handle's pinned read-back buffer; the host waits for
        // the event behind that copy
        if (hipGetLastError() != hipSuccess ||
            hipMemcpyAsync(t->h_counters, ctr, sizeof(hc), hipMemcpyDeviceToHost, st) != hipSuccess ||
            hipEventRecord(t->ev_counters, st) != hipSuccess || hipEventSynchronize(t->ev_counters) != hipSuccess) {
            rc = sr_fail(SR_EHIP, "sph_density: iteration %d failed", it);
            break;
        }
        for (int k = 0; k < SC_WORDS; ++k) hc[k] = t->h_counters[k];
        if (hc[SC_OVERFLOW]) {
            if (gathered_full) {
                // the lists or a level of the walk did not fit: grow both
                chunks *= 2;
                units = chunks / 2 + 2 * groups + 2 * waves + 64;
                front *= 2;
                if ((rc = lists_alloc(W, S, groups, waves, chunks, units, front, ctr, st))) break;
            }
            gather = full = true;
            continue;
        }
        ++it;
        full = false;
        if (hc[SC_ACTIVE] == 0) break;
        gather = hc[SC_REGATHER] != 0;
    }
    if (rc == SR_OK) {
        int32_t count = 0;
        hipLaunchKernelGGL(k_sph_clear, dim3(1), dim3(1), 0, st, failed, 0, 1);
        hipLaunchKernelGGL(k_sph_out, sph_grid(n), dim3(SPH_TPB), 0, st, n, t->perm, hs, rs, state, h, rho, failed);
        if (hipGetLastError() != hipSuccess ||
            hipMemcpyAsync(&count, failed, sizeof(int32_t), hipMemcpyDeviceToHost, st) != hipSuccess ||
            hipStreamSynchronize(st) != hipSuccess)
            rc = sr_fail(SR_EHIP, "sph_density: output failed");
        else if (unconverged)
            *unconverged = count;
    }
    if (W.lists) (void)hipFreeAsync(W.lists, st);
    (void)hipFreeAsync(W.buf, st);
    (void)hipFreeAsync(W.ibuf, st);
    return rc;
}

}  // extern "C"
