// Group-wise Barnes-Hut walk (forward and adjoint) of the short-range force,
// in three phases:
//   1. traverse: a workgroup per 64 Morton-consecutive targets (one target per
//      lane) walks the tree breadth-first, every lane deciding against each
//      staged node, and writes the interaction list as (source, lane mask)
//      entries in chunks of 64, the chunks grouped into units of a few;
//   2. evaluate: one wavefront per unit sweeps the entries, evaluating the
//      pair force for the lanes in each mask;
//   3. reduce: the units' partial sums are added per group in a fixed order.
// The adjoint reuses the forward's lists (the frozen decisions) and scatters
// source terms with wave sums and FP64 atomics.
#include <stdio.h>
#include <string.h>

#include <mutex>
#include <type_traits>

#include "gpoly.h"
#include "internal.h"

// the compiler's writelane intrinsic, named directly (clang has no builtin for it)
__device__ int amdgcn_writelane_i32(int v, int l, int old) __asm("llvm.amdgcn.writelane.i32");

namespace {

constexpr int WAVE = 64;
constexpr double TWO32 = 4294967296.0;
constexpr double TWO_OVER_SQRTPI = 1.12837916709551257390;
constexpr float LOG2E_F = 1.44269504088896340736f;
constexpr float TWO_OVER_SQRTPI_F = 1.12837916709551257390f;
constexpr float TWO64_F = 18446744073709551616.0f;

enum { PR64 = 0, PR32 = 1, PR32A = 2 };

struct WalkArgs {
    int64_t n_t;
    const int32_t* tgt_sorted;
    const int32_t* tgt_slot;
    const Item* items;
    uint32_t n_items;
    int64_t n_nodes;
    const int32_t* perm;
    const Rec64* prec64;
    const double* ph64;
    const Rec32* prec32;
    const float* ph32;
    const Rec64* nrec64;
    const Geo64* ngeo64;
    const double* nhmax;
    const double* nhmin;
    const Rec32* nrec32;
    const float* nhmax32;
    const uint32_t* n_corner;
    const int32_t* n_level;
    const double* a_old;
    // parameters (FP64 path; box units)
    double G, box, rc2, theta2, alpha, inv2rs;
    int relative;
    // parameters (FP32 path; integer-coordinate units)
    float rc2t, theta2f, inv2rs_t, rct;
    double tau2;          // (L / 2^32)^2
    double out_scale;     // G / L^2
    // outputs / adjoint
    void* acc;
    int32_t* counts;
    const void* w;
    double* pbar;
    double* tbar;
    double* nbar;
};


__device__ inline double min_image(double d, double L)
{
    if (d > 0.5 * L) return d - L;
    if (d < -0.5 * L) return d + L;
    return d;
}

// ---- FP64 pair kernel ------------------------------------------------------------

// Spline-softened 1/r^3 (and its r-derivative) of the cubic-spline kernel with support h.
__device__ inline void spline64(double r, double h, double& S, double& dS)
{
    if (r >= h) {
        double ir = 1.0 / r;
        S = ir * ir * ir;
        dS = -3.0 * S * ir;
        return;
    }
    double q = r / h;
    double ih = 1.0 / h;
    double ih3 = ih * ih * ih;
    if (q < 0.5) {
        S = (32.0 / 3.0 + q * q * (32.0 * q - 192.0 / 5.0)) * ih3;
        dS = q * (96.0 * q - 384.0 / 5.0) * ih3 * ih;
    } else {
        S = (64.0 / 3.0 - 48.0 * q + 192.0 / 5.0 * q * q - 32.0 / 3.0 * q * q * q - 1.0 / (15.0 * q * q * q)) * ih3;
        dS = (-48.0 + 384.0 / 5.0 * q - 32.0 * q * q + 1.0 / (5.0 * q * q * q * q)) * ih3 * ih;
    }
}

// ---- FP32 pair kernel (integer-coordinate units) -----------------------------------

__device__ inline float r2_ticks(float dx, float dy, float dz)
{
    return __builtin_fmaf(dx, dx, __builtin_fmaf(dy, dy, dz * dz));
}

// g(u) = exp(-u^2) R(u), R a fitted polynomial; also exp(-u^2) for g'.
__device__ inline float gshort32(float u, float& e)
{
    e = __builtin_amdgcn_exp2f(-(u * u) * LOG2E_F);
    float t = u - GPOLY_CENTRE;
    float p = GPOLY_C[GPOLY_DEGREE];
#pragma unroll
    for (int k = GPOLY_DEGREE - 1; k >= 0; --k) p = __builtin_fmaf(p, t, GPOLY_C[k]);
    return e * p;
}

// Softened branch in FP32: h^3 S and h^4 dS/dr as functions of q = r / h, the
// outer part written around q = 1 so that nothing cancels; both pieces are
// computed and selected, 1/x by v_rcp_f32 (1 ulp).
__device__ inline float spline_h3S_32f(float q)
{
    const float inner = __builtin_fmaf(q * q, __builtin_fmaf(32.0f, q, -38.4f), 10.6666666667f);
    const float t = 1.0f - q;
    const float poly = __builtin_fmaf(t, __builtin_fmaf(t, __builtin_fmaf(t, 10.6666666667f, 6.4f), 3.2f), 1.06666666667f);
    const float outer = poly - __builtin_amdgcn_rcpf(15.0f * q * q * q);
    return q < 0.5f ? inner : outer;
}

__device__ inline float spline_h4dS_32f(float q)
{
    const float inner = q * __builtin_fmaf(96.0f, q, -76.8f);
    const float t = 1.0f - q;
    const float q2 = q * q;
    const float outer = __builtin_fmaf(t, __builtin_fmaf(t, -32.0f, -12.8f), -3.2f) + __builtin_amdgcn_rcpf(5.0f * q2 * q2);
    return q < 0.5f ? inner : outer;
}

// ---- DPP moves (lane permutations within rows of 16, used for row and group sums) ----

template <int CTRL, int ROWMASK, int BANKMASK>
__device__ inline float dpp_f32(float v)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, ROWMASK, BANKMASK, false));
}

template <int CTRL, int ROWMASK, int BANKMASK>
__device__ inline double dpp_f64(double v)
{
    const uint64_t b = (uint64_t)__double_as_longlong(v);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)b, CTRL, ROWMASK, BANKMASK, false);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)(b >> 32), CTRL, ROWMASK, BANKMASK, false);
    return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}


// ----------------------------------------------------------------------------------
// cross-lane helpers
// ----------------------------------------------------------------------------------
//
// v_readlane at a uniform lane index (a VGPR value as a scalar), and
// v_writelane (a scalar value into one lane of a VGPR).

__device__ inline uint32_t rl(uint32_t v, uint32_t l) { return (uint32_t)__builtin_amdgcn_readlane((int)v, (int)l); }
__device__ inline uint64_t rl64(uint64_t v, uint32_t l)
{
    return ((uint64_t)rl((uint32_t)(v >> 32), l) << 32) | rl((uint32_t)v, l);
}
__device__ inline uint64_t wl64(uint64_t v, uint32_t l, uint64_t old)
{
    const uint32_t lo = (uint32_t)amdgcn_writelane_i32((int)(uint32_t)v, (int)l, (int)(uint32_t)old);
    const uint32_t hi = (uint32_t)amdgcn_writelane_i32((int)(uint32_t)(v >> 32), (int)l, (int)(uint32_t)(old >> 32));
    return ((uint64_t)hi << 32) | lo;
}

// ----------------------------------------------------------------------------------
// phase 1: traversal -> interaction lists
// ----------------------------------------------------------------------------------
//
// A workgroup of TW waves per group of 64 Morton-consecutive targets (lane l =
// target l in every wave).  Each lane takes exactly the decisions of its own
// target's walk; the group walks breadth-first, a level being a list of
// (node, reach mask) entries, where the reach mask holds the targets whose walk
// opened every ancestor.  The waves split a level, stage its nodes' records in
// LDS, decide (per-target ballots, or the whole group at once when the group's
// bounding box settles the outcome) and expand: opened nodes' children form
// the next level with the opening lanes as their reach.  Accepted nodes and
// reached particles become list entries (source, lane mask); the target's own
// particle is removed from its mask here.  Entries go
// to global memory in chunks of 64; up to UCH consecutive chunks of a group
// form a unit, the work item of the evaluation phase.  This is the paper's
// chunked neighbour processing (neighbours gathered in chunks and evaluated
// chunk by chunk, its GPU-porting subsection) with chunks of a wavefront's
// width, decoupled from the walk so that heavy groups spread over many waves.

// Chunks per evaluation unit (both entry points: the units' partial sums set the
// order of the FP32 sums), and unit indices a traversal wave reserves per atomic:
// 4 on the handle's lists, 1 in the fixed scratch of the allocation-free forward.
// Against 8 chunks and 1 unit: traversal + forward and adjoint evaluation
// 1.58 -> 1.47 ms on clustered 262k, the smaller units spreading heavy groups
// over more waves.
#ifndef SR_UCH
#define SR_UCH 2
#endif
constexpr int UCH = SR_UCH;

struct ListArgs {
    uint32_t* ent_src;
    uint64_t* ent_mask;
    int32_t* chunk_next;
    int32_t* chunk_cnt;
    int32_t* unit_group;
    int32_t* unit_chunk;
    int32_t* unit_nch;
    int32_t* unit_next;
    int32_t* group_head;
    int32_t* counters;      // [0] chunks, [1] units, [2] overflow, [4..5] node tests (u64)
    int64_t cap_chunks;
    int64_t cap_units;
    int32_t unit_base;      // evaluation: first unit of this launch
    int32_t unit_end;       // evaluation: one past the last unit of this launch
    int32_t chunk_batch;    // traversal: chunk indices a wave reserves per atomic
    int32_t unit_batch;     // traversal: unit indices a wave reserves per atomic
};

// open and accept masks of one decision
struct Dec {
    uint64_t om, am;
};

struct FrontArgs {
    uint32_t* buf;          // per workgroup: ids[2][TW][cap], then masks[2][TW][cap]
    int64_t cap;
    int32_t* next_group;    // work counter of the persistent waves
    int32_t* overflow;      // set when a level does not fit
    const WalkRec32* w32;   // per-node walk records
    const WalkRec64* w64;
    int64_t groups;
    int contig;             // the targets are all particles in sorted order (target t = particle t)
};

// Orders the LDS accesses of one wavefront among its lanes: LDS operations of
// a wavefront complete in order, so this is a compiler barrier and waits for no
// memory operation (in particular not for pending atomics).
__device__ inline void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Node data of one frontier entry, staged in LDS for the decisions of a block
// (read back as a broadcast: every lane reads the same record).
template <bool DEC64>
struct NodeRec;
template <>
struct NodeRec<false> {
    // a Barnes-Hut decision reads the first 48 bytes only
    uint32_t cX, cY, cZ, tin;      // cube centre (ticks), 0.6 side rounded down (ticks)
    uint32_t X, Y, Z, l2;          // centre of mass (ticks), side^2 (float bits, ticks^2)
    uint32_t half, rlo, rhi, M;    // half side (float bits), reach mask, mass (float bits)
    uint32_t hx, mixed, id, meta;  // h_max (float bits), mixed softening, node id, child count or META_BUCKET
};
template <>
struct NodeRec<true> {
    double cx, cy, cz, l, X, Y, Z, M, hx, hn;
    uint32_t rlo, rhi, id, meta;
};

__device__ inline uint32_t wave_min_u32(uint32_t v)
{
#pragma unroll
    for (int o = 1; o < WAVE; o <<= 1) v = min(v, (uint32_t)__shfl_xor((int)v, o, WAVE));
    return v;
}
__device__ inline uint32_t wave_max_u32(uint32_t v)
{
#pragma unroll
    for (int o = 1; o < WAVE; o <<= 1) v = max(v, (uint32_t)__shfl_xor((int)v, o, WAVE));
    return v;
}

// Range of |c - x| (32-bit wrap-around differences) over x in [lo, hi]; false if
// some difference in the range is not representable (the range crosses the
// half-box point).
__device__ inline bool axis_range(uint32_t c, uint32_t lo, uint32_t hi, int64_t& amin, int64_t& amax)
{
    const uint32_t mid = lo + ((hi - lo) >> 1);
    const int64_t d0 = (int32_t)(c - mid);
    const int64_t e0 = d0 - (int64_t)(hi - mid), e1 = d0 + (int64_t)(mid - lo);
    if (e0 <= -((int64_t)1 << 31) || e1 >= ((int64_t)1 << 31) - 1) return false;
    amin = e0 > 0 ? e0 : (e1 < 0 ? -e1 : 0);
    amax = -e0 > e1 ? -e0 : e1;
    return true;
}

__device__ inline double wave_min_f64(double v)
{
#pragma unroll
    for (int o = 1; o < WAVE; o <<= 1) v = fmin(v, __shfl_xor(v, o, WAVE));
    return v;
}
__device__ inline double wave_max_f64(double v)
{
#pragma unroll
    for (int o = 1; o < WAVE; o <<= 1) v = fmax(v, __shfl_xor(v, o, WAVE));
    return v;
}

// FP64 counterpart of axis_range: bounds of |min_image(c - x, L)| over the targets'
// coordinates x in [lo, hi], with the same roundings as the per-target test.  The
// rounded difference c - x is monotone in x, so the two ends bound every target's;
// the minimum image is bounded only when it takes the same branch over the range.
// The image is monotone too, so |image| is bounded by its ends' magnitudes, and is
// zero somewhere when the ends straddle zero (after a drift, positions lie just
// outside [0, L) and an image range can cross zero on either branch).
__device__ inline bool axis_range64(double c, double lo, double hi, double L, double& amin, double& amax)
{
    const double dlo = c - hi, dhi = c - lo;
    double elo, ehi;
    if (dlo >= -(0.5 * L) && dhi <= 0.5 * L) {   // no wrap for any target
        elo = dlo;
        ehi = dhi;
    } else if (dlo > 0.5 * L) {                  // every target wraps down
        elo = dlo - L;
        ehi = dhi - L;
    } else if (dhi < -(0.5 * L)) {               // every target wraps up
        elo = dlo + L;
        ehi = dhi + L;
    } else {
        return false;
    }
    amin = (elo <= 0.0 && ehi >= 0.0) ? 0.0 : fmin(fabs(elo), fabs(ehi));
    amax = fmax(fabs(elo), fabs(ehi));
    return true;
}

// Sum of a uint32 over the 64 lanes (DPP, total in lane 63).
__device__ inline uint32_t wave_sum63_u32(uint32_t x)
{
    uint32_t v = x + (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x111, 0xf, 0xf, false);
    v = v + (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x112, 0xf, 0xf, false);
    v = v + (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x113, 0xf, 0xf, false);
    v = v + (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x114, 0xf, 0xe, false);
    v = v + (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x118, 0xf, 0xc, false);
    v = v + (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x142, 0xa, 0xf, false);
    v = v + (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x143, 0xc, 0xf, false);
    return v;
}

// Breadth-first per group, TW waves per group: every wave holds the same 64
// targets (lane l = target l).  A level's frontier entries (node, reach mask)
// are split into TW contiguous ranges, one per wave.  A wave takes its range 64
// entries at a time: it stages the entries' node data in LDS, takes their
// decisions one after the other (each a 64-lane test of every reached target
// against one node, the records read as LDS broadcasts), and then expands the
// block lane-parallel: accepted nodes become list entries, and the children of
// opened nodes -- eight nodes by eight children per step -- go to the list
// (particles, without the target that is the particle itself) or to the wave's
// region of the next level (nodes).  The next level is the concatenation of
// the waves' regions in wave order, and the group's units are the waves' unit
// chains linked in wave order, so the lists and their order do not depend on
// timing.
#ifndef SR_TRAV_WAVES
#define SR_TRAV_WAVES 2
#endif
#ifndef SR_TRAV_WG_PER_CU
#define SR_TRAV_WG_PER_CU 8
#endif

constexpr int TW = SR_TRAV_WAVES;
#ifndef SR_DEC_ILP
#define SR_DEC_ILP 2
#endif
constexpr int DEC_ILP = SR_DEC_ILP;   // decisions interleaved in the traversal
#ifndef SR_CHUNK_BATCH
#define SR_CHUNK_BATCH 64
#endif
#ifndef SR_UNIT_BATCH
#define SR_UNIT_BATCH 4
#endif
// chunk indices reserved per atomic: 64 on the handle's lists (16 fewer atomics than
// one per chunk: 0.47 -> 0.45 ms on clustered 262k against 16), 16 in the fixed
// scratch of the allocation-free forward, where each wave's unused reservation
// must fit
constexpr int TRAV_CHUNK_BATCH = SR_CHUNK_BATCH;
constexpr int TRAV_CHUNK_BATCH_NOALLOC = 16;
constexpr int TRAV_UNIT_BATCH = SR_UNIT_BATCH;
constexpr int TRAV_UNIT_BATCH_NOALLOC = 1;

template <bool DEC64, bool REL, bool MIXED>
__global__ __launch_bounds__(TW * WAVE) __attribute__((amdgpu_waves_per_eu(4, 8))) void k_traverse(WalkArgs a, ListArgs L, FrontArgs F)
{
    const int lane = threadIdx.x & (WAVE - 1);
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x / WAVE);
    const uint64_t below = (1ull << lane) - 1ull;
    // frontier regions of this workgroup: [parity][wave] x cap ids, then the same for masks
    uint32_t* fids = F.buf + (int64_t)blockIdx.x * F.cap * (6 * TW);
    uint64_t* fmasks = (uint64_t*)(fids + 2 * TW * F.cap);
    auto rid = [&](int par, int w) -> uint32_t* { return fids + (int64_t)(par * TW + w) * F.cap; };
    auto rmask = [&](int par, int w) -> uint64_t* { return fmasks + (int64_t)(par * TW + w) * F.cap; };
    __shared__ NodeRec<DEC64> s_rec[TW][WAVE];
    __shared__ uint32_t s_kids[TW][WAVE][8];
    __shared__ uint64_t s_om[TW][WAVE];
    __shared__ uint32_t s_open[TW][WAVE];     // block positions of the opened nodes
    __shared__ uint32_t s_tgt[WAVE + 1];      // sorted particle index of each target (ascending)
    __shared__ int32_t sh_g;
    __shared__ int32_t sh_cnt[2][TW];     // entries of each wave's region, by level parity
    __shared__ int32_t sh_ovf[2][TW];     // overflow of each wave, by level parity
    __shared__ int32_t sh_first[TW], sh_last[TW], sh_wovf[TW];
    NodeRec<DEC64>* rec = s_rec[wv];

    // Chunk and unit indices: each wave reserves them in batches (one atomic per
    // TRAV_CHUNK_BATCH chunks / TRAV_UNIT_BATCH units on the shared counters) and
    // hands them out in order.  `cc` is the chunk being filled and `cn` the one
    // after it; both carry over to the next group.  Reserved units a wave never
    // uses are written as empty when it exits; unused chunks are never read.
    uint32_t c_next = 0, c_end = 0, u_next = 0, u_end = 0;
    uint64_t tests_all = 0;
    auto take_chunk = [&]() __attribute__((always_inline)) -> int64_t {
        if (c_next == c_end) {
            uint32_t b = 0;
            if (lane == 0) b = atomicAdd((uint32_t*)&L.counters[0], (uint32_t)L.chunk_batch);
            c_next = rl(b, 0);
            c_end = c_next + (uint32_t)L.chunk_batch;
        }
        return c_next++;
    };
    auto take_unit = [&]() __attribute__((always_inline)) -> int32_t {
        if (u_next == u_end) {
            uint32_t b = 0;
            if (lane == 0) b = atomicAdd((uint32_t*)&L.counters[1], (uint32_t)L.unit_batch);
            u_next = rl(b, 0);
            u_end = u_next + (uint32_t)L.unit_batch;
        }
        return (int32_t)u_next++;
    };
    int64_t cc = take_chunk();
    int64_t cn = take_chunk();

    for (;;) {
        if (threadIdx.x == 0) sh_g = atomicAdd(F.next_group, 1);
        __syncthreads();
        const int64_t g = __builtin_amdgcn_readfirstlane(sh_g);
        if (g >= F.groups) break;

        // ---- targets of group g ----
        const int64_t t = g * WAVE + lane;
        const bool valid = t < a.n_t;
        const int32_t s_i = valid ? a.tgt_sorted[t] : -1;
        double x64 = 0, y64 = 0, z64 = 0, aold = 0, atau = 0;
        uint32_t X = 0, Y = 0, Z = 0;
        if (valid) {
            if constexpr (DEC64) {
                const Rec64 r = a.prec64[s_i];
                x64 = r.x;
                y64 = r.y;
                z64 = r.z;
            } else {
                const Rec32 r = a.prec32[s_i];
                X = r.X;
                Y = r.Y;
                Z = r.Z;
            }
            if (a.relative) {
                aold = a.a_old[a.perm[s_i]];
                atau = (a.alpha * aold) * a.tau2;
            }
        }
        const uint64_t active = __ballot(valid);
        // bounding box of the group's targets (integer coordinates for FP32 decisions, a
        // group wider than a quarter box on some axis is never classified as a whole;
        // FP64 coordinates for FP64 decisions)
        uint32_t bxlo = 0, bxhi = 0, bylo = 0, byhi = 0, bzlo = 0, bzhi = 0;
        double gxlo = 0, gxhi = 0, gylo = 0, gyhi = 0, gzlo = 0, gzhi = 0;   // FP64 decisions
        bool box_ok = false;
        if constexpr (DEC64) {
            gxlo = wave_min_f64(valid ? x64 : INFINITY);
            gxhi = wave_max_f64(valid ? x64 : -INFINITY);
            gylo = wave_min_f64(valid ? y64 : INFINITY);
            gyhi = wave_max_f64(valid ? y64 : -INFINITY);
            gzlo = wave_min_f64(valid ? z64 : INFINITY);
            gzhi = wave_max_f64(valid ? z64 : -INFINITY);
            box_ok = gxlo <= gxhi;
        } else {
            bxlo = wave_min_u32(valid ? X : 0xffffffffu);
            bxhi = wave_max_u32(valid ? X : 0u);
            bylo = wave_min_u32(valid ? Y : 0xffffffffu);
            byhi = wave_max_u32(valid ? Y : 0u);
            bzlo = wave_min_u32(valid ? Z : 0xffffffffu);
            bzhi = wave_max_u32(valid ? Z : 0u);
            box_ok = bxhi - bxlo < (1u << 30) && byhi - bylo < (1u << 30) && bzhi - bzlo < (1u << 30);
        }
        if (wv == 0) {
            s_tgt[lane] = valid ? (uint32_t)s_i : 0xffffffffu;
            if (lane == 0) s_tgt[WAVE] = 0xffffffffu;
        }

        // ---- list entries of this group, written straight into chunks ----
        uint32_t nl = 0;                       // entries in chunk cc
        int32_t prev_chunk = -1, cur_unit = -1, prev_unit = -1, first_unit = -1;
        uint32_t nch = 0, unit_nch = 0;
        bool overflow = false;
        // close chunk cc with `count` entries, link it into the unit chain, move on to cn
        auto finish_chunk = [&](uint32_t count) __attribute__((always_inline)) {
            const bool new_unit = (nch % UCH) == 0;
            const int32_t c = (int32_t)cc;
            const int32_t u = new_unit ? take_unit() : -1;
            if (new_unit && u >= L.cap_units) {
                if (lane == 0) atomicOr(&L.counters[2], 1);
                overflow = true;
                return;
            }
            if (lane == 0) {
                L.chunk_cnt[c] = (int32_t)count;
                L.chunk_next[c] = -1;
                if (new_unit) {
                    if (cur_unit >= 0) L.unit_nch[cur_unit] = (int32_t)unit_nch;
                    L.unit_group[u] = (int32_t)g;
                    L.unit_chunk[u] = c;
                    L.unit_next[u] = -1;
                    if (prev_unit >= 0) L.unit_next[prev_unit] = u;
                } else {
                    L.chunk_next[prev_chunk] = c;
                }
            }
            if (new_unit) {
                if (prev_unit < 0) first_unit = u;
                prev_unit = u;
                cur_unit = u;
                unit_nch = 0;
            }
            ++unit_nch;
            prev_chunk = c;
            ++nch;
            cc = cn;
            cn = take_chunk();
        };
        // append one entry per lane set in `b` (in lane order): source `src`, mask `m`
        auto append = [&](uint64_t b, uint32_t src, uint64_t m) __attribute__((always_inline)) {
            if (!b || overflow) return;
            if (cc >= L.cap_chunks || cn >= L.cap_chunks) {
                if (lane == 0) atomicOr(&L.counters[2], 1);
                overflow = true;
                return;
            }
            if ((b >> lane) & 1) {
                const uint32_t slot = nl + (uint32_t)__popcll(b & below);
                const int64_t ch = slot < (uint32_t)WAVE ? cc : cn;
                const int64_t at = 64 * ch + (slot & (WAVE - 1));
                L.ent_src[at] = src;
                L.ent_mask[at] = m;
            }
            nl += (uint32_t)__popcll(b);
            if (nl >= (uint32_t)WAVE) {
                finish_chunk((uint32_t)WAVE);
                nl -= (uint32_t)WAVE;
            }
        };
        // the lane of the target whose own particle is sorted particle s, or none:
        // with all particles as targets it is s - 64 g, else a search of the group's
        // (ascending) target particles
        auto own_bit = [&](uint32_t s) __attribute__((always_inline)) -> uint64_t {
            if (F.contig) {
                const uint32_t o = s - (uint32_t)(g * WAVE);
                return o < (uint32_t)WAVE ? (1ull << o) : 0ull;
            }
            uint32_t pos = 0;
#pragma unroll
            for (uint32_t st = 32; st; st >>= 1)
                if (s_tgt[pos + st - 1] < s) pos += st;
            return s_tgt[pos] == s ? (1ull << pos) : 0ull;
        };

        // ---- breadth-first levels ----
        uint32_t tests = 0;    // this lane's share of the node-target tests (work statistics)
        int cur = 0;

        if (threadIdx.x == 0) {
            rid(0, 0)[0] = 0u;
            rmask(0, 0)[0] = active;
            for (int w = 0; w < TW; ++w) {
                sh_cnt[0][w] = w == 0 ? 1 : 0;
                sh_ovf[0][w] = 0;
            }
        }
        __syncthreads();
        for (;;) {
            // the level's size and overflow state, the same for every wave of the group
            int32_t c[TW];
            int64_t na = 0;
            bool lvl_ovf = false;
#pragma unroll
            for (int w = 0; w < TW; ++w) {
                c[w] = __builtin_amdgcn_readfirstlane(sh_cnt[cur][w]);
                na += c[w];
                lvl_ovf = lvl_ovf || __builtin_amdgcn_readfirstlane(sh_ovf[cur][w]) != 0;
            }
            if (na == 0 || lvl_ovf) break;
            // this wave's range of the level
            const int64_t per = (na + TW - 1) / TW;
            const int64_t e0 = wv * per < na ? wv * per : na;
            const int64_t e1 = e0 + per < na ? e0 + per : na;
            uint32_t* nid = rid(cur ^ 1, wv);
            uint64_t* nmask = rmask(cur ^ 1, wv);
            int64_t nb = 0;          // entries of the next level written so far
            auto push = [&](uint64_t b, uint32_t id, uint64_t m) __attribute__((always_inline)) {
                if (!b || overflow) return;
                const uint32_t k = (uint32_t)__popcll(b);
                if (nb + k > F.cap) {
                    if (lane == 0) atomicOr(F.overflow, 1);
                    overflow = true;
                    return;
                }
                if ((b >> lane) & 1) {
                    const int64_t at = nb + __popcll(b & below);
                    nid[at] = id;
                    nmask[at] = m;
                }
                nb += k;
            };
            // the level's entry b0 + lane: it lies in the region of the first wave whose
            // cumulative count exceeds it.  Entries are read one block ahead, so that a
            // block's staging waits for its node records only.
            auto load_entry = [&](int64_t b, uint32_t& id, uint64_t& m) __attribute__((always_inline)) {
                id = 0;
                m = 0;
                if (b + lane < e1) {
                    int64_t off = b + lane;
                    int r = 0;
#pragma unroll
                    for (int w = 0; w < TW - 1; ++w) {
                        const bool past = r == w && off >= c[w];
                        off -= past ? c[w] : 0;
                        r += past ? 1 : 0;
                    }
                    id = rid(cur, r)[off];
                    m = rmask(cur, r)[off];
                }
            };
            uint32_t nxt_id;
            uint64_t nxt_mask;
            load_entry(e0, nxt_id, nxt_mask);
            for (int64_t b0 = e0; b0 < e1 && !overflow; b0 += WAVE) {
                const uint32_t cnt = (uint32_t)(e1 - b0 < WAVE ? e1 - b0 : WAVE);
                // ---- stage the block's nodes ----
                uint32_t fid = nxt_id, fmeta = 0;
                uint64_t fmask = nxt_mask;
                load_entry(b0 + WAVE, nxt_id, nxt_mask);
                int cls = 0;   // 0: decide per target, 1: pruned for all, 2: opened by all, 3: accepted by all
                if ((uint32_t)lane < cnt) {
                    tests += (uint32_t)__popcll(fmask);
                    const uint32_t nd = fid;
                    NodeRec<DEC64> nr;
                    uint4* kd = (uint4*)s_kids[wv][lane];
                    if constexpr (DEC64) {
                        const WalkRec64* wr = F.w64 + nd;
                        nr.cx = wr->cx;
                        nr.cy = wr->cy;
                        nr.cz = wr->cz;
                        nr.l = wr->l;
                        nr.X = wr->X;
                        nr.Y = wr->Y;
                        nr.Z = wr->Z;
                        nr.M = wr->M;
                        nr.hx = wr->hx;
                        nr.hn = wr->hn;
                        fmeta = wr->meta;
                        kd[0] = ((const uint4*)wr->kids)[0];
                        kd[1] = ((const uint4*)wr->kids)[1];
                    } else {
                        const WalkRec32* wr = F.w32 + nd;
                        const uint4 q0 = ((const uint4*)wr)[0], q1 = ((const uint4*)wr)[1], q2 = ((const uint4*)wr)[2];
                        nr.cX = q0.x;
                        nr.cY = q0.y;
                        nr.cZ = q0.z;
                        nr.tin = q0.w;
                        nr.X = q1.x;
                        nr.Y = q1.y;
                        nr.Z = q1.z;
                        nr.l2 = q1.w;
                        nr.half = q2.x;
                        nr.M = q2.y;
                        nr.hx = q2.z;
                        nr.mixed = MIXED ? q2.w : 0u;
                        fmeta = wr->meta;
                        kd[0] = ((const uint4*)wr->kids)[0];
                        kd[1] = ((const uint4*)wr->kids)[1];
                    }
                    nr.rlo = (uint32_t)fmask;
                    nr.rhi = (uint32_t)(fmask >> 32);
                    nr.id = nd;
                    nr.meta = fmeta;
                    rec[lane] = nr;
                    // The node against the whole group: the per-target tests below are
                    // monotone in the per-axis distances and rounding is monotone, so the
                    // same operations on the extreme distances bound every target's
                    // result.  A node whose outcome is the same for every target needs
                    // no per-target decision.
                    if constexpr (!DEC64) {
                        int64_t c0, c1, c2, c3, c4, c5, p0, p1, p2, p3, p4, p5;
                        if (box_ok && axis_range(nr.cX, bxlo, bxhi, c0, c1) && axis_range(nr.cY, bylo, byhi, c2, c3) &&
                            axis_range(nr.cZ, bzlo, bzhi, c4, c5) && axis_range(nr.X, bxlo, bxhi, p0, p1) &&
                            axis_range(nr.Y, bylo, byhi, p2, p3) && axis_range(nr.Z, bzlo, bzhi, p4, p5)) {
                            const uint32_t bm_lo = (uint32_t)max(c0, max(c2, c4));
                            const uint32_t bm_hi = (uint32_t)max(c1, max(c3, c5));
                            const float half = __uint_as_float(nr.half), l2 = __uint_as_float(nr.l2);
                            const bool prune_all = (float)bm_lo - half > a.rct;
                            const bool keep_all = !((float)bm_hi - half > a.rct);
                            const float r2_lo = r2_ticks((float)p0, (float)p2, (float)p4);
                            const float r2_hi = r2_ticks((float)p1, (float)p3, (float)p5);
                            const bool open_all = bm_hi <= nr.tin || l2 > a.theta2f * r2_hi;
                            bool open_none = bm_lo > nr.tin && !(l2 > a.theta2f * r2_lo) && !REL;
                            if constexpr (MIXED)
                                open_none = open_none && !(nr.mixed && r2_lo < __uint_as_float(nr.hx) * __uint_as_float(nr.hx));
                            const bool near_all = r2_hi < a.rc2t, far_all = !(r2_lo < a.rc2t);
                            if (prune_all) {
                                cls = 1;
                            } else if (keep_all && open_all) {
                                cls = 2;
                            } else if (keep_all && open_none && near_all) {
                                cls = 3;
                            } else if (keep_all && open_none && far_all) {
                                cls = 1;   // accepted by every target, beyond r_cut for all
                            }
                        }
                    } else {
                        double c0, c1, c2, c3, c4, c5, p0, p1, p2, p3, p4, p5;
                        const double L = a.box;
                        if (box_ok && axis_range64(nr.cx, gxlo, gxhi, L, c0, c1) &&
                            axis_range64(nr.cy, gylo, gyhi, L, c2, c3) && axis_range64(nr.cz, gzlo, gzhi, L, c4, c5) &&
                            axis_range64(nr.X, gxlo, gxhi, L, p0, p1) && axis_range64(nr.Y, gylo, gyhi, L, p2, p3) &&
                            axis_range64(nr.Z, gzlo, gzhi, L, p4, p5)) {
                            const double l = nr.l, thr = a.rc2 * (1.0 + 1e-6);
                            const double txl = fmax(c0 - 0.5 * l, 0.0), tyl = fmax(c2 - 0.5 * l, 0.0), tzl = fmax(c4 - 0.5 * l, 0.0);
                            const double txh = fmax(c1 - 0.5 * l, 0.0), tyh = fmax(c3 - 0.5 * l, 0.0), tzh = fmax(c5 - 0.5 * l, 0.0);
                            const bool prune_all = (txl * txl + tyl * tyl) + tzl * tzl > thr;
                            const bool keep_all = !((txh * txh + tyh * tyh) + tzh * tzh > thr);
                            const double am_lo = fmax(c0, fmax(c2, c4)), am_hi = fmax(c1, fmax(c3, c5));
                            const double r2_lo = (p0 * p0 + p2 * p2) + p4 * p4, r2_hi = (p1 * p1 + p3 * p3) + p5 * p5;
                            const bool open_all = am_hi < 0.6 * l || l * l > a.theta2 * r2_hi;
                            bool open_none = !(am_lo < 0.6 * l) && !(l * l > a.theta2 * r2_lo) && !REL;
                            if constexpr (MIXED) open_none = open_none && !(nr.hn != nr.hx && r2_lo < nr.hx * nr.hx);
                            const bool near_all = r2_hi < a.rc2, far_all = !(r2_lo < a.rc2);
                            if (prune_all) {
                                cls = 1;
                            } else if (keep_all && open_all) {
                                cls = 2;
                            } else if (keep_all && open_none && near_all) {
                                cls = 3;
                            } else if (keep_all && open_none && far_all) {
                                cls = 1;
                            }
                        }
                    }
                }
                wave_sync();

                // ---- decisions: all lanes against node j ----
                // The masks come from one ballot per elementary test (each a single
                // compare into a lane mask) and are combined on the scalar unit.
                auto decide = [&](uint32_t j) __attribute__((always_inline)) -> Dec {
                    const NodeRec<DEC64> nr = rec[j];
                    const uint64_t reach = ((uint64_t)__builtin_amdgcn_readfirstlane(nr.rhi) << 32) |
                                           (uint32_t)__builtin_amdgcn_readfirstlane(nr.rlo);
                    uint64_t keep_m, open_m, near_m;
                    if constexpr (DEC64) {
                        const double l = nr.l;
                        const double dcx = min_image(nr.cx - x64, a.box);
                        const double dcy = min_image(nr.cy - y64, a.box);
                        const double dcz = min_image(nr.cz - z64, a.box);
                        const double tx = fmax(fabs(dcx) - 0.5 * l, 0.0);
                        const double ty = fmax(fabs(dcy) - 0.5 * l, 0.0);
                        const double tz = fmax(fabs(dcz) - 0.5 * l, 0.0);
                        keep_m = __ballot(!((tx * tx + ty * ty) + tz * tz > a.rc2 * (1.0 + 1e-6)));
                        const double am = fmax(fabs(dcx), fmax(fabs(dcy), fabs(dcz)));
                        const uint64_t inside_m = __ballot(am < 0.6 * l);
                        const double dx = min_image(nr.X - x64, a.box);
                        const double dy = min_image(nr.Y - y64, a.box);
                        const double dz = min_image(nr.Z - z64, a.box);
                        const double r2 = (dx * dx + dy * dy) + dz * dz;
                        open_m = inside_m | __ballot(l * l > a.theta2 * r2);
                        if constexpr (REL) open_m |= __ballot((a.G * nr.M) * (l * l) > (a.alpha * aold) * (r2 * r2));
                        if constexpr (MIXED)
                            if (__builtin_amdgcn_readfirstlane(nr.hn != nr.hx ? 1 : 0))
                                open_m |= __ballot(r2 < nr.hx * nr.hx);
                        near_m = __ballot(r2 < a.rc2);
                    } else {
                        const uint32_t bx = (uint32_t)abs((int32_t)(nr.cX - X));
                        const uint32_t by = (uint32_t)abs((int32_t)(nr.cY - Y));
                        const uint32_t bz = (uint32_t)abs((int32_t)(nr.cZ - Z));
                        const uint32_t bm = max(bx, max(by, bz));
                        // prune (work only): the cube lies beyond r_cut along some axis
                        keep_m = __ballot(!((float)bm - __uint_as_float(nr.half) > a.rct));
                        const uint64_t inside_m = __ballot(bm <= nr.tin);
                        const float dx = (float)(int32_t)(nr.X - X);
                        const float dy = (float)(int32_t)(nr.Y - Y);
                        const float dz = (float)(int32_t)(nr.Z - Z);
                        const float r2 = r2_ticks(dx, dy, dz);
                        const float l2 = __uint_as_float(nr.l2);
                        open_m = inside_m | __ballot(l2 > a.theta2f * r2);
                        if constexpr (REL) {
                            const double r2d = (double)r2;
                            open_m |= __ballot((a.G * (double)__uint_as_float(nr.M)) * (double)l2 > atau * (r2d * r2d));
                        }
                        if constexpr (MIXED) {
                            const float hx = __uint_as_float(nr.hx);
                            if (__builtin_amdgcn_readfirstlane(nr.mixed)) open_m |= __ballot(r2 < hx * hx);
                        }
                        near_m = __ballot(r2 < a.rc2t);
                    }
                    const uint64_t live = reach & keep_m;
                    return Dec{live & open_m, live & ~open_m & near_m};
                };
                // lane j keeps the masks of node j: set at once for a node classified
                // as a whole, else from the per-target decision; DEC_ILP independent
                // decisions interleave (a missing one repeats the first and is not kept)
                uint64_t my_om = cls == 2 ? fmask : 0ull, my_am = cls == 3 ? fmask : 0ull;
                uint64_t todo = __ballot((uint32_t)lane < cnt && cls == 0);
                while (todo) {
                    uint32_t jj[DEC_ILP];
                    bool use[DEC_ILP];
#pragma unroll
                    for (int k = 0; k < DEC_ILP; ++k) {
                        use[k] = todo != 0;
                        jj[k] = use[k] ? (uint32_t)__builtin_ctzll(todo) : jj[0];
                        todo &= todo - 1;
                    }
                    Dec d[DEC_ILP];
#pragma unroll
                    for (int k = 0; k < DEC_ILP; ++k) d[k] = decide(jj[k]);
                    // (a repeated node wrote the same masks to the same lane already)
#pragma unroll
                    for (int k = 0; k < DEC_ILP; ++k) {
                        my_om = wl64(d[k].om, jj[k], my_om);
                        my_am = wl64(d[k].am, jj[k], my_am);
                    }
                }

                // ---- accepted nodes: one list entry each, in block order ----
                append(__ballot(my_am != 0), fid, my_am);

                // ---- opened nodes: children, eight nodes by eight children per step ----
                const bool opened = my_om != 0 && fmeta != META_BUCKET;
                const uint64_t bo = __ballot(opened);
                s_om[wv][lane] = my_om;
                if (opened) s_open[wv][__popcll(bo & below)] = (uint32_t)lane;
                wave_sync();
                const uint32_t n_open = (uint32_t)__popcll(bo);
                for (uint32_t q0 = 0; q0 < n_open && !overflow; q0 += 8) {
                    const uint32_t q = q0 + ((uint32_t)lane >> 3);
                    const uint32_t k = (uint32_t)lane & 7u;
                    uint32_t ch = 0;
                    uint64_t om = 0;
                    bool has = false;
                    if (q < n_open) {
                        const uint32_t jn = s_open[wv][q];
                        om = s_om[wv][jn];
                        has = k < rec[jn].meta;
                        ch = s_kids[wv][jn][k];
                    }
                    const bool isp = (ch & ITEM_PARTICLE) != 0;
                    const uint64_t pm = has && isp ? om & ~own_bit(ch & ~ITEM_PARTICLE) : 0ull;
                    append(__ballot(pm != 0), ch, pm);
                    push(__ballot(has && !isp), ch, om);
                }
                // ---- opened buckets (identical keys): their particles, 64 at a time ----
                uint64_t bb = __ballot(my_om != 0 && fmeta == META_BUCKET);
                while (bb && !overflow) {
                    const uint32_t jn = (uint32_t)__builtin_ctzll(bb);
                    bb &= bb - 1;
                    const uint64_t om = rl64(my_om, jn);
                    const uint32_t s0 = __builtin_amdgcn_readfirstlane(s_kids[wv][jn][0]);
                    const uint32_t sc = __builtin_amdgcn_readfirstlane(s_kids[wv][jn][1]);
                    for (uint32_t p0 = 0; p0 < sc && !overflow; p0 += WAVE) {
                        const uint32_t sidx = s0 + p0 + (uint32_t)lane;
                        const bool in = p0 + (uint32_t)lane < sc;
                        const uint64_t pm = in ? om & ~own_bit(sidx) : 0ull;
                        append(__ballot(pm != 0), sidx | ITEM_PARTICLE, pm);
                    }
                }
                wave_sync();
            }
            if (lane == 0) {
                sh_cnt[cur ^ 1][wv] = overflow ? 0 : (int32_t)nb;
                sh_ovf[cur ^ 1][wv] = overflow ? 1 : 0;
            }
            __syncthreads();
            cur ^= 1;
        }
        if (nl && !overflow) {
            finish_chunk(nl);
            nl = 0;
        }
        if (lane == 0 && cur_unit >= 0 && !overflow) L.unit_nch[cur_unit] = (int32_t)unit_nch;
        tests_all += rl(wave_sum63_u32(tests), 63);
        if (lane == 0) {
            sh_first[wv] = first_unit;
            sh_last[wv] = cur_unit;
            sh_wovf[wv] = overflow ? 1 : 0;
        }
        __syncthreads();
        bool any_ovf = false;
#pragma unroll
        for (int w = 0; w < TW; ++w) any_ovf = any_ovf || __builtin_amdgcn_readfirstlane(sh_wovf[w]) != 0;
        if (threadIdx.x == 0 && !any_ovf) {
            // link the waves' unit chains in wave order
            int32_t head = -1, tail = -1;
            for (int w = 0; w < TW; ++w) {
                if (sh_first[w] < 0) continue;
                if (tail >= 0) L.unit_next[tail] = sh_first[w];
                else head = sh_first[w];
                tail = sh_last[w];
            }
            L.group_head[g] = head;
        }
        if (any_ovf) break;
        __syncthreads();
    }
    if (lane == 0) atomicAdd((unsigned long long*)(L.counters + 4), (unsigned long long)tests_all);
    // units reserved and never used: empty units
    if ((uint32_t)lane < u_end - u_next) {
        const int64_t u = (int64_t)u_next + lane;
        if (u < L.cap_units) {
            L.unit_nch[u] = 0;
            L.unit_group[u] = 0;
            L.unit_chunk[u] = -1;
            L.unit_next[u] = -1;
        }
    }
}

// ----------------------------------------------------------------------------------
// phase 2: evaluation of one unit (a few chunks of one group)
// ----------------------------------------------------------------------------------

// per-unit partial results: acc_t[3][64] then int32[2][64] (forward) or acc_t[3][64] (adjoint)
constexpr int PARTIAL_BYTES = 64 * (3 * 8 + 2 * 4);

// Waves per workgroup of the FP32 evaluation, one unit per wave (2 and 4 were
// measured no faster than 1 on the clustered 262,144-particle step).
#ifndef SR_EVAL_WAVES
#define SR_EVAL_WAVES 1
#endif
constexpr int EVAL_WAVES = SR_EVAL_WAVES;

// Lanes (targets) per stream of the FP32 evaluation, forward and adjoint.
#ifndef SR_QL_ADJ
#define SR_QL_ADJ 16
#endif
#ifndef SR_QL_FWD
#define SR_QL_FWD 8
#endif
constexpr int QL_FWD = SR_QL_FWD;
constexpr int QL_ADJ = SR_QL_ADJ;
static_assert(QL_ADJ == 8 || QL_ADJ == 16, "stream width");

// Sums four quantities over each stream of QL lanes at once by a transposing
// butterfly: at each exchange a lane keeps half of what it holds and sends the
// other half to its partner, so the four totals cost 11 adds and selects for 16
// lanes (10 for 8) instead of 16 (12) adds.  Afterwards lane l holds the stream
// total of quantity (l mod QL) / (QL/4) (0 x, 1 y, 2 z, 3 m).  Partners: for
// 16-lane rows the row mirror (l^15), then the half-row mirror (l^7), then the
// quad swaps (l^1, l^2); for 8-lane groups the half-row mirror and the quad
// swaps.  Needs the full wave active.
template <int QL>
__device__ inline float stream_sum4(float x, float y, float z, float m, int lane)
{
    if constexpr (QL == 16) {
        const bool b3 = lane & 8, b2 = lane & 4;
        float k0 = b3 ? z : x, k1 = b3 ? m : y;
        const float s0 = b3 ? x : z, s1 = b3 ? y : m;
        k0 += dpp_f32<0x140, 0xf, 0xf>(s0);
        k1 += dpp_f32<0x140, 0xf, 0xf>(s1);
        float k = b2 ? k1 : k0;
        const float s = b2 ? k0 : k1;
        k += dpp_f32<0x141, 0xf, 0xf>(s);
        k += dpp_f32<0xb1, 0xf, 0xf>(k);
        k += dpp_f32<0x4e, 0xf, 0xf>(k);
        return k;
    } else {
        const bool b2 = lane & 4, b1 = lane & 2;
        float k0 = b2 ? z : x, k1 = b2 ? m : y;
        const float s0 = b2 ? x : z, s1 = b2 ? y : m;
        k0 += dpp_f32<0x141, 0xf, 0xf>(s0);
        k1 += dpp_f32<0x141, 0xf, 0xf>(s1);
        float k = b1 ? k1 : k0;
        const float s = b1 ? k0 : k1;
        k += dpp_f32<0x4e, 0xf, 0xf>(s);
        k += dpp_f32<0xb1, 0xf, 0xf>(k);
        return k;
    }
}

// FP64 form of stream_sum4 for 16-lane streams (each exchange moves both 32-bit
// halves): lane l ends with the row total of quantity (l mod 16) / 4.
__device__ inline double stream_sum4_f64(double x, double y, double z, double m, int lane)
{
    const bool b3 = lane & 8, b2 = lane & 4;
    double k0 = b3 ? z : x, k1 = b3 ? m : y;
    const double s0 = b3 ? x : z, s1 = b3 ? y : m;
    k0 += dpp_f64<0x140, 0xf, 0xf>(s0);
    k1 += dpp_f64<0x140, 0xf, 0xf>(s1);
    double k = b2 ? k1 : k0;
    const double s = b2 ? k0 : k1;
    k += dpp_f64<0x141, 0xf, 0xf>(s);
    k += dpp_f64<0xb1, 0xf, 0xf>(k);
    k += dpp_f64<0x4e, 0xf, 0xf>(k);
    return k;
}

// FP32 evaluation of one unit, packed into streams.  A stream is a group of QL
// lanes (QL Morton-consecutive targets).  For each chunk the entries whose mask
// touches group k form stream k; step s evaluates entry stream_k[s] on the lanes
// of group k, for all groups at once, so a chunk takes max_k |stream_k| steps
// instead of one step per entry.  Source records are staged in LDS, 32 bytes
// per entry; each group reads its own entry (a broadcast within the group).
// Slots past the end of a stream name entry 64, whose mask is empty.  The
// adjoint's source terms are summed per stream with DPP (stream_sum4),
// collected per entry in LDS, and added to the source with one FP64 atomic per
// (entry, component) after the chunk.
struct SrcLds {
    uint32_t X, Y, Z, m;        // integer position, mass bits (mass scaled by 2^64)
    uint32_t h, inc, mlo, mhi;  // support h bits, count increment, mask of lanes 0-31 / 32-63
};

template <int PREC, bool ADJ>
__global__ __launch_bounds__(EVAL_WAVES * WAVE) void k_eval32(WalkArgs a, ListArgs L, char* __restrict__ partials)
{
    using acc_t = typename std::conditional<PREC == PR32, float, double>::type;
    static_assert(PREC != PR64, "FP32 kernel");
    constexpr int QL = ADJ ? QL_ADJ : QL_FWD;
    constexpr int NQ = WAVE / QL;
    // every wave of the workgroup evaluates a unit of its own with LDS of its own
    __shared__ SrcLds s_ent_w[EVAL_WAVES][WAVE + 1];
    __shared__ uint32_t s_src_w[EVAL_WAVES][WAVE];
    __shared__ uint8_t s_stream_w[EVAL_WAVES][NQ][WAVE];
    // adjoint: the four source terms of each (stream, entry) pair of the chunk; a stream
    // visits an entry at most once per chunk, so every slot is written at most once
    // (in FP64 when the accumulation is FP64: the pair terms are FP32, their sums are not)
    constexpr bool PART64 = ADJ && PREC == PR32A;
    static_assert(!PART64 || QL == 16, "FP64 stream sums take 16-lane streams");
    __shared__ float4 s_part_w[EVAL_WAVES][ADJ && !PART64 ? NQ : 1][ADJ && !PART64 ? WAVE + 1 : 1];
    __shared__ double s_part64_w[EVAL_WAVES][PART64 ? NQ : 1][PART64 ? WAVE + 1 : 1][4];
    const int wv = threadIdx.x / WAVE;
    auto& s_ent = s_ent_w[wv];
    auto& s_src = s_src_w[wv];
    auto& s_stream = s_stream_w[wv];
    auto& s_part = s_part_w[wv];
    auto& s_part64 = s_part64_w[wv];
    const int lane = threadIdx.x % WAVE;
    const int quarter = lane / QL;
    const uint32_t bit = 1u << (lane & 31);
    const bool hi_half = lane >= 32;
    // units past the traversal's count, or the lists of a traversal that overflowed, are
    // not read (the launch may be sized before the count is known on the host)
    const int32_t u = L.unit_base + (int32_t)(blockIdx.x * EVAL_WAVES + wv);
    if (u >= L.unit_end || u >= L.counters[1] || L.counters[2] != 0) return;
    if (L.unit_nch[u] == 0) return;   // a unit reserved but not used (its partials are never read)
    const int64_t g = L.unit_group[u];
    const int64_t t = g * WAVE + lane;
    const bool valid = t < a.n_t;
    const int32_t s_i = valid ? a.tgt_sorted[t] : 0;
    const Rec32 tr = a.prec32[s_i];
    const uint32_t X = tr.X, Y = tr.Y, Z = tr.Z;
    const uint32_t h32b = __float_as_uint(a.ph32[s_i]);   // supports are >= 0: integer order is float order
    acc_t ax = 0, ay = 0, az = 0;
    uint32_t cnt2 = 0;       // interactions: particles in the low half, nodes in the high half
    float wx = 0, wy = 0, wz = 0;
    acc_t tbx = 0, tby = 0, tbz = 0;
    if constexpr (ADJ) {
        if (valid) {
            const int32_t slot = a.tgt_slot[t];
            const acc_t* w = (const acc_t*)a.w;
            wx = (float)w[3 * (int64_t)slot];
            wy = (float)w[3 * (int64_t)slot + 1];
            wz = (float)w[3 * (int64_t)slot + 2];
        }
    }
    if (lane == 0) s_ent[WAVE] = SrcLds{0u, 0u, 0u, 0u, 0u, 0u, 0u, 0u};

    int32_t c = L.unit_chunk[u];
    const int32_t nch = L.unit_nch[u];
    for (int32_t q = 0; q < nch; ++q) {
        const uint32_t cnt = (uint32_t)L.chunk_cnt[c];
        const bool has = (uint32_t)lane < cnt;
        uint64_t lmask = 0;
        if (has) {
            const uint32_t lsrc = L.ent_src[64 * (int64_t)c + lane];
            lmask = L.ent_mask[64 * (int64_t)c + lane];
            const bool isp = lsrc & ITEM_PARTICLE;
            const uint32_t idx = lsrc & ~ITEM_PARTICLE;
            const Rec32 r = isp ? a.prec32[idx] : a.nrec32[idx];
            const float hs = isp ? a.ph32[idx] : a.nhmax32[idx];
            s_ent[lane] = SrcLds{r.X, r.Y, r.Z, __float_as_uint(r.m * TWO64_F), __float_as_uint(hs),
                                 isp ? 1u : 0x10000u, (uint32_t)lmask, (uint32_t)(lmask >> 32)};
            s_src[lane] = lsrc;
        }
        // the streams (one per group of QL lanes), each in entry order, padded with entry 64
        const uint64_t below = (1ull << lane) - 1ull;
        constexpr uint64_t QMASK = (1ull << QL) - 1ull;
        uint32_t steps = 0;
#pragma unroll
        for (int k = 0; k < NQ; ++k) {
            const uint64_t b = __ballot(has && ((lmask >> (QL * k)) & QMASK) != 0);
            const uint32_t nk = __popcll(b);
            if ((b >> lane) & 1) s_stream[k][__popcll(b & below)] = (uint8_t)lane;
            if ((uint32_t)lane >= nk) s_stream[k][lane] = (uint8_t)WAVE;   // slots past the stream
            steps = max(steps, nk);
        }
        const int32_t cnext = L.chunk_next[c];
        wave_sync();
        // one step: entry stream_k[st] on each group's lanes
        auto step = [&](uint32_t st) __attribute__((always_inline)) {
            const uint32_t e = s_stream[quarter][st];
            const SrcLds src = s_ent[e];
            const uint32_t mw = hi_half ? src.mhi : src.mlo;
            const bool on = (mw & bit) != 0;
            const float hp = __uint_as_float(max(h32b, src.h));
            const float qm = __uint_as_float(src.m);
            const float dx = (float)(int32_t)(src.X - X);
            const float dy = (float)(int32_t)(src.Y - Y);
            const float dz = (float)(int32_t)(src.Z - Z);
            const float r2 = r2_ticks(dx, dy, dz);
            const bool in = on && r2 < a.rc2t;
            // r2 = 0 (coincident particles) gives r = 0 and a finite rinv; such a pair is
            // always inside the softening support
            const float rinv = __builtin_amdgcn_rsqf(__uint_as_float(max(__float_as_uint(r2), 0x0da24260u)));   // max(r2, 1e-30)
            const float r = r2 * rinv;
            const float uu = r * a.inv2rs_t;
            float ex;
            const float gg = gshort32(uu, ex);
            float S = rinv * rinv * rinv;
            float Srd = -3.0f * S;
            if (in && r < hp) {
                const float ih = __builtin_amdgcn_rcpf(hp);
                const float qq = r * ih;
                const float ih3 = ih * ih * ih;
                S = spline_h3S_32f(qq) * ih3;
                if constexpr (ADJ) Srd = spline_h4dS_32f(qq) * qq * ih3;
            }
            if constexpr (!ADJ) cnt2 += in ? src.inc : 0u;
            const float K = in ? S * gg : 0.0f;
            if constexpr (!ADJ) {
                const float f = qm * K;
                ax += (acc_t)(f * dx);
                ay += (acc_t)(f * dy);
                az += (acc_t)(f * dz);
            } else {
                // J w = K w + (K' r)(w . n) n,  K' r = r S' g + S g'(u) u; with n = d / r:
                // m J w = (m K) w + (m K' r (w . d) / r^2) d
                const float dg = -2.0f * TWO_OVER_SQRTPI_F * uu * uu * ex;
                const float Kr = in ? Srd * gg + S * dg * uu : 0.0f;
                const float wd = __builtin_fmaf(wx, dx, __builtin_fmaf(wy, dy, wz * dz));
                const float cA = qm * K;
                const float cB = qm * (Kr * wd) * (rinv * rinv);
                const float px = __builtin_fmaf(cA, wx, cB * dx);
                const float py = __builtin_fmaf(cA, wy, cB * dy);
                const float pz = __builtin_fmaf(cA, wz, cB * dz);
                tbx -= (acc_t)px;
                tby -= (acc_t)py;
                tbz -= (acc_t)pz;
                // source terms: the stream's totals, one quantity per lane, stored in the
                // (stream, entry) slot (the padding entry 64 has a slot that is never read);
                // the QL/4 lanes that hold one quantity store the same value
                if constexpr (PART64) {
                    const double ssum = stream_sum4_f64((double)px, (double)py, (double)pz, (double)(K * wd), lane);
                    s_part64[quarter][e][(lane % QL) / (QL / 4)] = ssum;
                } else {
                    const float ssum = stream_sum4<QL>(px, py, pz, K * wd, lane);
                    reinterpret_cast<float*>(&s_part[quarter][e])[(lane % QL) / (QL / 4)] = ssum;
                }
            }
        };
        // the forward takes two steps interleaved (their entries are independent):
        // 8% faster; the adjoint gains nothing from it
        if constexpr (!ADJ) {
#pragma unroll 2
            for (uint32_t st = 0; st < steps; ++st) step(st);
        } else {
            for (uint32_t st = 0; st < steps; ++st) step(st);
        }
        wave_sync();
        if constexpr (ADJ) {
            if (has) {
                const uint32_t sid = s_src[lane];
                double* dst = (sid & ITEM_PARTICLE) ? a.pbar + 4 * (int64_t)(sid & ~ITEM_PARTICLE)
                                                    : a.nbar + 4 * (int64_t)sid;
                // the streams that visited this entry, in stream order
                double v[4] = {0.0, 0.0, 0.0, 0.0};
                if constexpr (PART64) {
#pragma unroll
                    for (int k = 0; k < NQ; ++k) {
                        if (((lmask >> (QL * k)) & QMASK) != 0) {
#pragma unroll
                            for (int c = 0; c < 4; ++c) v[c] += s_part64[k][lane][c];
                        }
                    }
                } else {
                    float4 f = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
#pragma unroll
                    for (int k = 0; k < NQ; ++k) {
                        if (((lmask >> (QL * k)) & QMASK) != 0) {
                            const float4 pk = s_part[k][lane];
                            f.x += pk.x;
                            f.y += pk.y;
                            f.z += pk.z;
                            f.w += pk.w;
                        }
                    }
                    v[0] = f.x;
                    v[1] = f.y;
                    v[2] = f.z;
                    v[3] = f.w;
                }
#pragma unroll
                for (int c = 0; c < 4; ++c)
                    if (v[c] != 0.0) unsafeAtomicAdd(dst + c, v[c]);
            }
            wave_sync();
        }
        c = cnext;
    }
    acc_t* pa = (acc_t*)(partials + (int64_t)u * PARTIAL_BYTES);
    if constexpr (!ADJ) {
        pa[lane] = ax;
        pa[64 + lane] = ay;
        pa[128 + lane] = az;
        int32_t* pc = (int32_t*)(pa + 192);
        pc[lane] = (int32_t)(cnt2 & 0xffffu);
        pc[64 + lane] = (int32_t)(cnt2 >> 16);
    } else {
        pa[lane] = tbx;
        pa[64 + lane] = tby;
        pa[128 + lane] = tbz;
    }
}

// FP64 evaluation of one unit, packed into streams like the FP32 kernel (QL
// lanes per stream); the pair arithmetic is the plain FP64 form (library erfc,
// exp and square root, division) and each lane sums its entries in entry order.
struct alignas(16) SrcLds64 {
    double x, y, z, m, h;          // position, mass, support h
    uint32_t sid, inc, mlo, mhi;   // source id, count increment, mask of lanes 0-31 / 32-63
    uint32_t pad[2];
};


template <bool ADJ>
__global__ __launch_bounds__(WAVE) void k_eval64(WalkArgs a, ListArgs L, char* __restrict__ partials)
{
    constexpr int QL = 16;
    constexpr int NQ = WAVE / QL;
    __shared__ SrcLds64 s_ent[WAVE + 1];
    __shared__ uint8_t s_stream[NQ][WAVE];
    // adjoint: the four source terms of each (stream, entry) pair of the chunk, each
    // slot written at most once per chunk
    __shared__ double4 s_part[ADJ ? NQ : 1][ADJ ? WAVE + 1 : 1];
    const int lane = threadIdx.x;
    const int quarter = lane / QL;
    const uint32_t bit = 1u << (lane & 31);
    const bool hi_half = lane >= 32;
    // units past the traversal's count, or the lists of a traversal that overflowed, are
    // not read (the launch may be sized before the count is known on the host)
    const int32_t u = L.unit_base + (int32_t)blockIdx.x;
    if (u >= L.unit_end || u >= L.counters[1] || L.counters[2] != 0) return;
    if (L.unit_nch[u] == 0) return;   // a unit reserved but not used (its partials are never read)
    const int64_t g = L.unit_group[u];
    const int64_t t = g * WAVE + lane;
    const bool valid = t < a.n_t;
    const int32_t s_i = valid ? a.tgt_sorted[t] : 0;
    const Rec64 tr = a.prec64[s_i];
    const double x64 = tr.x, y64 = tr.y, z64 = tr.z, h64 = a.ph64[s_i];
    double ax = 0, ay = 0, az = 0;
    uint32_t cnt2 = 0;       // interactions: particles in the low half, nodes in the high half
    double wx = 0, wy = 0, wz = 0, tbx = 0, tby = 0, tbz = 0;
    if constexpr (ADJ) {
        if (valid) {
            const int32_t slot = a.tgt_slot[t];
            const double* w = (const double*)a.w;
            wx = w[3 * (int64_t)slot];
            wy = w[3 * (int64_t)slot + 1];
            wz = w[3 * (int64_t)slot + 2];
        }
    }
    if (lane == 0) s_ent[WAVE] = SrcLds64{0.0, 0.0, 0.0, 0.0, 0.0, 0u, 0u, 0u, 0u, {0u, 0u}};

    int32_t c = L.unit_chunk[u];
    const int32_t nch = L.unit_nch[u];
    for (int32_t q = 0; q < nch; ++q) {
        const uint32_t cnt = (uint32_t)L.chunk_cnt[c];
        const bool has = (uint32_t)lane < cnt;
        uint64_t lmask = 0;
        if (has) {
            const uint32_t lsrc = L.ent_src[64 * (int64_t)c + lane];
            lmask = L.ent_mask[64 * (int64_t)c + lane];
            const bool isp = lsrc & ITEM_PARTICLE;
            const uint32_t idx = lsrc & ~ITEM_PARTICLE;
            const Rec64 r = isp ? a.prec64[idx] : a.nrec64[idx];
            const double hs = isp ? a.ph64[idx] : a.nhmax[idx];
            s_ent[lane] = SrcLds64{r.x, r.y, r.z, r.m, hs, lsrc, isp ? 1u : 0x10000u, (uint32_t)lmask,
                                   (uint32_t)(lmask >> 32), {0u, 0u}};
        }
        const uint64_t below = (1ull << lane) - 1ull;
        constexpr uint64_t QMASK = (1ull << QL) - 1ull;
        uint32_t steps = 0;
#pragma unroll
        for (int k = 0; k < NQ; ++k) {
            const uint64_t b = __ballot(has && ((lmask >> (QL * k)) & QMASK) != 0);
            const uint32_t nk = __popcll(b);
            if ((b >> lane) & 1) s_stream[k][__popcll(b & below)] = (uint8_t)lane;
            if ((uint32_t)lane >= nk) s_stream[k][lane] = (uint8_t)WAVE;   // slots past the stream
            steps = max(steps, nk);
        }
        const int32_t cnext = L.chunk_next[c];
        wave_sync();
        for (uint32_t st = 0; st < steps; ++st) {
            const uint32_t e = s_stream[quarter][st];
            const SrcLds64 src = s_ent[e];
            const uint32_t mw = hi_half ? src.mhi : src.mlo;
            const bool on = (mw & bit) != 0;
            double vx = 0, vy = 0, vz = 0, vm = 0;
            const double dx = min_image(src.x - x64, a.box);
            const double dy = min_image(src.y - y64, a.box);
            const double dz = min_image(src.z - z64, a.box);
            const double r2 = (dx * dx + dy * dy) + dz * dz;
            if (on && r2 < a.rc2) {
                if constexpr (!ADJ) cnt2 += src.inc;
                const double r = sqrt(r2);
                const double uu = r * a.inv2rs;
                const double ex = exp(-uu * uu);
                const double gg = erfc(uu) + TWO_OVER_SQRTPI * uu * ex;
                const double hp = h64 > src.h ? h64 : src.h;
                double S, dS;
                spline64(r, hp, S, dS);
                const double K = a.G * S * gg;
                if constexpr (!ADJ) {
                    const double f = src.m * K;
                    ax += f * dx;
                    ay += f * dy;
                    az += f * dz;
                } else {
                    const double dg = -2.0 * TWO_OVER_SQRTPI * uu * uu * ex;
                    const double dK = a.G * (dS * gg + S * dg * a.inv2rs);
                    const double c2 = r > 0.0 ? dK / r : 0.0;
                    const double wd = (wx * dx + wy * dy) + wz * dz;
                    vx = src.m * (K * wx + c2 * wd * dx);
                    vy = src.m * (K * wy + c2 * wd * dy);
                    vz = src.m * (K * wz + c2 * wd * dz);
                    vm = K * wd;
                    tbx -= vx;
                    tby -= vy;
                    tbz -= vz;
                }
            }
            if constexpr (ADJ) {
                // source terms: the stream's totals, one quantity per lane, stored in the
                // (stream, entry) slot (the padding entry 64 has a slot that is never read)
                static_assert(QL == 16, "16-lane streams");
                const double ssum = stream_sum4_f64(vx, vy, vz, vm, lane);
                reinterpret_cast<double*>(&s_part[quarter][e])[(lane % QL) / 4] = ssum;
            }
        }
        wave_sync();
        if constexpr (ADJ) {
            if (has) {
                const uint32_t sid = s_ent[lane].sid;
                double* dst = (sid & ITEM_PARTICLE) ? a.pbar + 4 * (int64_t)(sid & ~ITEM_PARTICLE)
                                                    : a.nbar + 4 * (int64_t)sid;
                // the streams that visited this entry, in stream order
                double v[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
                for (int k = 0; k < NQ; ++k) {
                    if (((lmask >> (QL * k)) & QMASK) != 0) {
                        const double4 pk = s_part[k][lane];
                        v[0] += pk.x;
                        v[1] += pk.y;
                        v[2] += pk.z;
                        v[3] += pk.w;
                    }
                }
#pragma unroll
                for (int k = 0; k < 4; ++k)
                    if (v[k] != 0.0) unsafeAtomicAdd(dst + k, v[k]);
            }
            wave_sync();
        }
        c = cnext;
    }
    double* pa = (double*)(partials + (int64_t)u * PARTIAL_BYTES);
    if constexpr (!ADJ) {
        pa[lane] = ax;
        pa[64 + lane] = ay;
        pa[128 + lane] = az;
        int32_t* pc = (int32_t*)(pa + 192);
        pc[lane] = (int32_t)(cnt2 & 0xffffu);
        pc[64 + lane] = (int32_t)(cnt2 >> 16);
    } else {
        pa[lane] = tbx;
        pa[64 + lane] = tby;
        pa[128 + lane] = tbz;
    }
}

// ----------------------------------------------------------------------------------
// phase 3: per group, sum the units' partials in their order and write the outputs
// ----------------------------------------------------------------------------------

template <int PREC, bool ADJ>
__global__ __launch_bounds__(WAVE) void k_reduce(WalkArgs a, ListArgs L, const char* __restrict__ partials)
{
    using acc_t = typename std::conditional<PREC == PR32, float, double>::type;
    const int lane = threadIdx.x;
    const int64_t g = blockIdx.x;
    const int64_t t = g * WAVE + lane;
    if (t >= a.n_t) return;
    acc_t ax = 0, ay = 0, az = 0;
    int npp = 0, npn = 0;
    // A group's chain mostly runs through consecutive unit indices (a traversal wave
    // reserves several at a time): the next pointers and partials of units u .. u + 3
    // are loaded together and used as far as the chain does run consecutively, in
    // chain order.
    constexpr int RUN = 4;
    for (int32_t u = L.group_head[g]; u >= 0;) {
        int32_t nx[RUN];
        acc_t px[RUN], py[RUN], pz[RUN];
        int32_t cp[RUN], cn[RUN];
#pragma unroll
        for (int k = 0; k < RUN; ++k) {
            const int32_t v = u + k < L.cap_units ? u + k : u;
            nx[k] = L.unit_next[v];
            const acc_t* pa = (const acc_t*)(partials + (int64_t)v * PARTIAL_BYTES);
            px[k] = pa[lane];
            py[k] = pa[64 + lane];
            pz[k] = pa[128 + lane];
            if constexpr (!ADJ) {
                const int32_t* pc = (const int32_t*)(pa + 192);
                cp[k] = pc[lane];
                cn[k] = pc[64 + lane];
            }
        }
        int32_t next = nx[0];
#pragma unroll
        for (int k = 0; k < RUN; ++k) {
            ax += px[k];
            ay += py[k];
            az += pz[k];
            if constexpr (!ADJ) {
                npp += cp[k];
                npn += cn[k];
            }
            next = nx[k];
            if (k == RUN - 1 || nx[k] != u + k + 1) break;
        }
        u = next;
    }
    if constexpr (ADJ) {
        const int32_t s_i = a.tgt_sorted[t];
        a.tbar[3 * (int64_t)s_i + 0] = (double)ax;
        a.tbar[3 * (int64_t)s_i + 1] = (double)ay;
        a.tbar[3 * (int64_t)s_i + 2] = (double)az;
    } else {
        const int64_t slot = a.tgt_slot[t];
        if constexpr (PREC == PR64) {
            double* o = (double*)a.acc;
            o[3 * slot + 0] = ax;
            o[3 * slot + 1] = ay;
            o[3 * slot + 2] = az;
        } else if constexpr (PREC == PR32) {
            float* o = (float*)a.acc;
            const float sc = (float)a.out_scale;
            o[3 * slot + 0] = ax * sc;
            o[3 * slot + 1] = ay * sc;
            o[3 * slot + 2] = az * sc;
        } else {
            double* o = (double*)a.acc;
            o[3 * slot + 0] = ax * a.out_scale;
            o[3 * slot + 1] = ay * a.out_scale;
            o[3 * slot + 2] = az * a.out_scale;
        }
        if (a.counts) {
            a.counts[2 * slot] = npp;
            a.counts[2 * slot + 1] = npn;
        }
    }
}

// Push the node terms of the adjoint down to the particles and return to input
// order: for every ancestor n of particle j,
//   dL/dx_j += (m_j / M_n) Xbar_n,   dL/dm_j += Mbar_n + Xbar_n . (x_j - X_n) / M_n.
// sx / sm rescale position / mass adjoints of the FP32 path to box units.
__global__ void k_pushdown(int64_t n, const int32_t* __restrict__ perm, const int32_t* __restrict__ pparent,
                           const int32_t* __restrict__ n_parent, const Rec64* __restrict__ prec64,
                           const Rec64* __restrict__ nrec64, const double* __restrict__ pbar,
                           const double* __restrict__ tbar, const double* __restrict__ nbar, double sx, double sm,
                           double* __restrict__ dLdx, double* __restrict__ dLdm)
{
    int64_t s = blockIdx.x * (int64_t)256 + threadIdx.x;
    if (s >= n) return;
    const Rec64 p = prec64[s];
    double gx = (tbar[3 * s + 0] + pbar[4 * s + 0]) * sx;
    double gy = (tbar[3 * s + 1] + pbar[4 * s + 1]) * sx;
    double gz = (tbar[3 * s + 2] + pbar[4 * s + 2]) * sx;
    double gm = pbar[4 * s + 3] * sm;
    for (int32_t nd = pparent[s]; nd >= 0; nd = n_parent[nd]) {
        const Rec64 c = nrec64[nd];
        const double bx = nbar[4 * nd + 0] * sx, by = nbar[4 * nd + 1] * sx, bz = nbar[4 * nd + 2] * sx;
        gx += p.m / c.m * bx;
        gy += p.m / c.m * by;
        gz += p.m / c.m * bz;
        double dot = 0.0;
        dot += bx * (p.x - c.x);
        dot += by * (p.y - c.y);
        dot += bz * (p.z - c.z);
        gm += nbar[4 * nd + 3] * sm + dot / c.m;
    }
    const int32_t j = perm[s];
    dLdx[3 * (int64_t)j + 0] = gx;
    dLdx[3 * (int64_t)j + 1] = gy;
    dLdx[3 * (int64_t)j + 2] = gz;
    dLdm[j] = gm;
}

template <class Y, class X>
__global__ void k_axpy(Y* __restrict__ y, const X* __restrict__ x, double a, int64_t n)
{
    const int64_t i = blockIdx.x * (int64_t)256 + threadIdx.x;
    if (i < n) y[i] = (Y)((double)y[i] + a * (double)x[i]);
}

// Clears three FP64 arrays in one launch (the adjoint's accumulators).
__global__ void k_zero3_f64(double* a, int64_t na, double* b, int64_t nb, double* c, int64_t nc)
{
    int64_t i = blockIdx.x * (int64_t)256 + threadIdx.x;
    if (i < na) {
        a[i] = 0.0;
        return;
    }
    i -= na;
    if (i < nb) {
        b[i] = 0.0;
        return;
    }
    i -= nb;
    if (i < nc) c[i] = 0.0;
}

__global__ void k_targets_all(int64_t n, const int32_t* __restrict__ perm, int32_t* __restrict__ tgt_sorted,
                              int32_t* __restrict__ tgt_slot)
{
    int64_t s = blockIdx.x * (int64_t)256 + threadIdx.x;
    if (s >= n) return;
    tgt_sorted[s] = (int32_t)s;
    tgt_slot[s] = perm[s];
}

// mark[s] = slot + 1 of the active entry that names sorted particle s
__global__ void k_mark_active(const int32_t* __restrict__ active, int64_t n_active, int64_t n,
                              const int32_t* __restrict__ invperm, int32_t* __restrict__ mark,
                              int32_t* __restrict__ status)
{
    int64_t j = blockIdx.x * (int64_t)256 + threadIdx.x;
    if (j >= n_active) return;
    int32_t i = active[j];
    if (i < 0 || i >= n) {
        atomicOr(&status[ST_FLAGS], 2);
        return;
    }
    int32_t prev = atomicExch(&mark[invperm[i]], (int32_t)(j + 1));
    if (prev != 0) atomicOr(&status[ST_FLAGS], 4);
}

__global__ void k_flag_marked(int64_t n, const int32_t* __restrict__ mark, uint32_t* __restrict__ flag)
{
    int64_t s = blockIdx.x * (int64_t)256 + threadIdx.x;
    if (s < n) flag[s] = mark[s] != 0;
}

__global__ void k_compact_targets(int64_t n, const int32_t* __restrict__ mark, const int32_t* __restrict__ pos,
                                  int32_t* __restrict__ tgt_sorted, int32_t* __restrict__ tgt_slot)
{
    int64_t s = blockIdx.x * (int64_t)256 + threadIdx.x;
    if (s >= n || !mark[s]) return;
    int32_t k = pos[s];
    tgt_sorted[k] = (int32_t)s;
    tgt_slot[k] = mark[s] - 1;
}

__global__ void k_fill_i32w(int32_t* p, int64_t n, int32_t v)
{
    int64_t i = blockIdx.x * (int64_t)256 + threadIdx.x;
    if (i < n) p[i] = v;
}

inline dim3 g256(int64_t n) { return dim3((unsigned)((n > 0 ? n : 1) + 255) / 256); }

WalkArgs make_args(const sr_tree* t, const sr_params* p, int64_t n_t, const double* a_old)
{
    WalkArgs a{};
    a.n_t = n_t;
    a.tgt_sorted = t->tgt_sorted;
    a.tgt_slot = t->tgt_slot;
    a.items = t->items;
    a.n_items = (uint32_t)(t->n + t->n_nodes);
    a.n_nodes = t->n_nodes;
    a.perm = t->perm;
    a.prec64 = t->prec64;
    a.ph64 = t->ph64;
    a.prec32 = t->prec32;
    a.ph32 = t->ph32;
    a.nrec64 = t->nrec64;
    a.ngeo64 = t->ngeo64;
    a.nhmax = t->nhmax;
    a.nhmin = t->nhmin;
    a.nrec32 = t->nrec32;
    a.nhmax32 = t->nhmax32;
    a.n_corner = t->n_corner;
    a.n_level = t->n_level;
    a.a_old = a_old;
    a.G = p->G;
    a.box = t->box;
    a.rc2 = p->r_cut * p->r_cut;
    a.theta2 = p->theta * p->theta;
    a.alpha = p->alpha;
    a.inv2rs = 1.0 / (2.0 * p->r_s);
    a.relative = p->criterion == SR_OPEN_RELATIVE;
    const double tick = t->box / TWO32;
    a.rc2t = (float)((p->r_cut / tick) * (p->r_cut / tick));
    a.rct = (float)(p->r_cut / tick * 1.0001);
    a.theta2f = (float)(p->theta * p->theta);
    a.inv2rs_t = (float)(tick / (2.0 * p->r_s));
    a.tau2 = tick * tick;
    a.out_scale = p->G / (t->box * t->box);
    return a;
}

// Where one traversal writes its lists, frontier and partial sums: the handle's
// buffers (grown on demand) or the fixed buffer of the allocation-free forward.
struct ListStore {
    uint32_t* ent_src;
    uint64_t* ent_mask;
    int32_t *chunk_next, *chunk_cnt;
    int32_t *unit_group, *unit_chunk, *unit_nch, *unit_next;
    int32_t* group_head;
    int32_t* counters;
    char* partials;
    uint32_t* frontier;
    int64_t cap_chunks, cap_units, cap_front;
    int chunk_batch;   // chunk indices a traversal wave reserves per atomic
    int unit_batch;    // unit indices a traversal wave reserves per atomic
};

ListStore handle_store(const sr_tree* t)
{
    ListStore S{};
    S.ent_src = t->ent_src;
    S.ent_mask = t->ent_mask;
    S.chunk_next = t->chunk_next;
    S.chunk_cnt = t->chunk_cnt;
    S.unit_group = t->unit_group;
    S.unit_chunk = t->unit_chunk;
    S.unit_nch = t->unit_nch;
    S.unit_next = t->unit_next;
    S.group_head = t->group_head;
    S.counters = t->list_counters;
    S.partials = t->partials;
    S.frontier = t->frontier;
    S.cap_chunks = t->cap_chunks;
    S.cap_units = t->cap_units;
    S.cap_front = t->cap_front;
    S.chunk_batch = TRAV_CHUNK_BATCH;
    S.unit_batch = TRAV_UNIT_BATCH;
    return S;
}

ListArgs list_args(const ListStore& S)
{
    ListArgs L{};
    L.ent_src = S.ent_src;
    L.ent_mask = S.ent_mask;
    L.chunk_next = S.chunk_next;
    L.chunk_cnt = S.chunk_cnt;
    L.unit_group = S.unit_group;
    L.unit_chunk = S.unit_chunk;
    L.unit_nch = S.unit_nch;
    L.unit_next = S.unit_next;
    L.group_head = S.group_head;
    L.counters = S.counters;
    L.cap_chunks = S.cap_chunks;
    L.cap_units = S.cap_units;
    L.unit_base = 0;
    L.unit_end = 0;
    L.chunk_batch = S.chunk_batch;
    L.unit_batch = S.unit_batch;
    return L;
}

bool same_decisions(const ListKey& k, const sr_params* p)
{
    const int dec64 = p->precision == SR_FP64;
    return k.dec64 == dec64 && k.G == p->G && k.r_s == p->r_s && k.r_cut == p->r_cut && k.theta == p->theta &&
           k.alpha == p->alpha && k.criterion == p->criterion;
}

// Persistent traversal workgroups of TW waves for `groups` target groups: at
// most `per_cu` per compute unit and one per group.
int traversal_workgroups(int64_t groups, int64_t per_cu, int64_t& wgs)
{
    int dev = 0, cus = 0;
    SR_HIP(hipGetDevice(&dev));
    SR_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    wgs = groups < per_cu * (int64_t)cus ? groups : per_cu * (int64_t)cus;
    if (wgs < 1) wgs = 1;
    return SR_OK;
}

// The traversal into store S with `wgs` persistent workgroups (S holds a
// frontier for that many), then the copy of its counters to pinned host memory.
// No host synchronisation.
int launch_traversal(sr_tree* t, const sr_params* p, int64_t n_t, const int32_t* active, const double* a_old,
                     const ListStore& S, int64_t wgs, hipStream_t st)
{
    const int64_t groups = (n_t + WAVE - 1) / WAVE;
    hipLaunchKernelGGL(k_fill_i32w, g256(groups), dim3(256), 0, st, S.group_head, groups, -1);
    hipLaunchKernelGGL(k_fill_i32w, g256(8), dim3(256), 0, st, S.counters, (int64_t)8, 0);
    const WalkArgs a = make_args(t, p, n_t, a_old);
    const ListArgs L = list_args(S);
    FrontArgs F{};
    F.buf = S.frontier;
    F.cap = S.cap_front;
    F.next_group = S.counters + 3;
    F.overflow = S.counters + 2;
    F.w32 = t->wrec32;
    F.w64 = t->wrec64;
    F.contig = active == nullptr;
    F.groups = groups;
    sr_timing_mark(SR_T_TRAVERSE, true, st);
    const dim3 gw((unsigned)wgs), bw(TW * WAVE);
    const bool rel = p->criterion == SR_OPEN_RELATIVE, mix = t->mixed_soft;
    const int variant = (p->precision == SR_FP64 ? 4 : 0) + (rel ? 2 : 0) + (mix ? 1 : 0);
    switch (variant) {
    case 0: hipLaunchKernelGGL((k_traverse<false, false, false>), gw, bw, 0, st, a, L, F); break;
    case 1: hipLaunchKernelGGL((k_traverse<false, false, true>), gw, bw, 0, st, a, L, F); break;
    case 2: hipLaunchKernelGGL((k_traverse<false, true, false>), gw, bw, 0, st, a, L, F); break;
    case 3: hipLaunchKernelGGL((k_traverse<false, true, true>), gw, bw, 0, st, a, L, F); break;
    case 4: hipLaunchKernelGGL((k_traverse<true, false, false>), gw, bw, 0, st, a, L, F); break;
    case 5: hipLaunchKernelGGL((k_traverse<true, false, true>), gw, bw, 0, st, a, L, F); break;
    case 6: hipLaunchKernelGGL((k_traverse<true, true, false>), gw, bw, 0, st, a, L, F); break;
    default: hipLaunchKernelGGL((k_traverse<true, true, true>), gw, bw, 0, st, a, L, F); break;
    }
    sr_timing_mark(SR_T_TRAVERSE, false, st);
    SR_HIP(hipGetLastError());
    // the counters go to pinned host memory right behind the traversal, so that the
    // check waits for the traversal only and not for the work queued after it
    SR_HIP(hipMemcpyAsync(t->h_counters, S.counters, 8 * sizeof(int32_t), hipMemcpyDeviceToHost, st));
    SR_HIP(hipEventRecord(t->ev_counters, st));
    return SR_OK;
}

// Phase 1 launch on the handle's lists: reserve lists and frontier for `want`
// entries / `fcap` frontier entries per wave, then the traversal.  No host
// synchronisation.
int traverse_launch(sr_tree* t, const sr_params* p, int64_t n_t, const int32_t* active, const double* a_old,
                    int64_t want, int64_t fcap, hipStream_t st)
{
    t->lkey.valid = false;
    const int64_t groups = (n_t + WAVE - 1) / WAVE;
    int64_t wgs = 1;
    int rc = traversal_workgroups(groups, SR_TRAV_WG_PER_CU, wgs);
    if (rc) return rc;
    // every wave of a group may start a unit chain; each wave may leave a
    // reserved batch of chunks and units unused
    const int64_t chunks = (want + 63) / 64 + TW * wgs * (TRAV_CHUNK_BATCH + 2);
    rc = sr_list_reserve(t, groups, chunks, TW * groups + chunks / UCH + TW * wgs * TRAV_UNIT_BATCH + 1, st);
    if (rc) return rc;
    if ((rc = sr_front_reserve(t, wgs * TW, fcap, st))) return rc;
    return launch_traversal(t, p, n_t, active, a_old, handle_store(t), wgs, st);
}

// After a traversal: read its counters (the host waits until they have been
// copied, which is right after the traversal kernel).  On success record
// the list sizes and the key that identifies these lists; `overflow` tells the
// caller to grow and traverse again.
int traverse_finish(sr_tree* t, const sr_params* p, int64_t n_t, const int32_t* active, const double* a_old,
                    hipStream_t st, bool& overflow)
{
    int32_t cnt[8];
    SR_HIP(hipEventSynchronize(t->ev_counters));
    memcpy(cnt, t->h_counters, sizeof(cnt));
    overflow = cnt[2] != 0;
    if (overflow) return SR_OK;
    t->n_units = cnt[1];
    t->n_chunks = cnt[0];
    int64_t tests;
    memcpy(&tests, cnt + 4, sizeof(tests));
    t->n_tests = tests;
    ListKey& k = t->lkey;
    k.valid = true;
    k.token = ++t->list_serial;
    k.gen = t->build_gen;
    k.dec64 = p->precision == SR_FP64;
    k.G = p->G;
    k.r_s = p->r_s;
    k.r_cut = p->r_cut;
    k.theta = p->theta;
    k.alpha = p->alpha;
    k.criterion = p->criterion;
    k.n_t = n_t;
    return SR_OK;
}

int64_t initial_want(int64_t n_t)
{
    const int64_t want = 32 * n_t;
    return want < ((int64_t)1 << 16) ? ((int64_t)1 << 16) : want;
}

// Phase 1 with its check: traverse, growing the lists (and the per-wave frontier)
// until everything fits.
int traverse(sr_tree* t, const sr_params* p, int64_t n_t, const int32_t* active, const double* a_old,
             hipStream_t st)
{
    int64_t want = initial_want(n_t);
    int64_t fcap = t->cap_front > 4096 ? t->cap_front : 4096;
    for (int attempt = 0; attempt < 8; ++attempt) {
        int rc = traverse_launch(t, p, n_t, active, a_old, want, fcap, st);
        if (rc) return rc;
        bool overflow = false;
        if ((rc = traverse_finish(t, p, n_t, active, a_old, st, overflow))) return rc;
        if (!overflow) return SR_OK;
        // something did not fit: grow both (a chunk overflow and a frontier overflow share the flag)
        want = 2 * t->cap_chunks * 64;
        fcap = 2 * t->cap_front;
    }
    return sr_fail(SR_ENOMEM, "interaction lists did not fit after repeated growth");
}

// Phases 2 and 3: evaluate units [u0, u0 + nu) (units past the traversal's
// count exit at once), then reduce every group.
template <bool ADJ>
int eval_and_reduce(const sr_params* p, const WalkArgs& a, const ListStore& S, int64_t u0, int64_t nu, hipStream_t st)
{
    const int64_t groups = (a.n_t + WAVE - 1) / WAVE;
    ListArgs L = list_args(S);
    L.unit_base = (int32_t)u0;
    L.unit_end = (int32_t)(u0 + nu);
    const dim3 gu((unsigned)(nu > 0 ? nu : 1)), gu32((unsigned)(nu > 0 ? (nu + EVAL_WAVES - 1) / EVAL_WAVES : 1)),
        gg((unsigned)groups);
    const int ph_eval = ADJ ? SR_T_ADJ_EVAL : SR_T_EVAL, ph_red = ADJ ? SR_T_ADJ_REDUCE : SR_T_REDUCE;
    if (nu > 0) {
        sr_timing_mark(ph_eval, true, st);
        switch (p->precision) {
        case SR_FP64: hipLaunchKernelGGL((k_eval64<ADJ>), gu, dim3(WAVE), 0, st, a, L, S.partials); break;
        case SR_FP32:
            hipLaunchKernelGGL((k_eval32<PR32, ADJ>), gu32, dim3(EVAL_WAVES * WAVE), 0, st, a, L, S.partials);
            break;
        default:
            hipLaunchKernelGGL((k_eval32<PR32A, ADJ>), gu32, dim3(EVAL_WAVES * WAVE), 0, st, a, L, S.partials);
            break;
        }
        sr_timing_mark(ph_eval, false, st);
    }
    sr_timing_mark(ph_red, true, st);
    switch (p->precision) {
    case SR_FP64: hipLaunchKernelGGL((k_reduce<PR64, ADJ>), gg, dim3(WAVE), 0, st, a, L, S.partials); break;
    case SR_FP32: hipLaunchKernelGGL((k_reduce<PR32, ADJ>), gg, dim3(WAVE), 0, st, a, L, S.partials); break;
    default: hipLaunchKernelGGL((k_reduce<PR32A, ADJ>), gg, dim3(WAVE), 0, st, a, L, S.partials); break;
    }
    sr_timing_mark(ph_red, false, st);
    SR_HIP(hipGetLastError());
    return SR_OK;
}

}  // namespace

int sr_check_list_token(const sr_tree* t, const sr_params* p, int64_t n_t, int64_t token)
{
    const ListKey& k = t->lkey;
    if (!(k.valid && k.token == token && k.gen == t->build_gen))
        return sr_fail(SR_ESTATE, "list token %lld does not name this handle's current interaction lists "
                       "(another walk or a rebuild replaced them)", (long long)token);
    if (k.n_t != n_t)
        return sr_fail(SR_EINVAL, "n_active (%lld) differs from the forward call of this token (%lld)",
                       (long long)n_t, (long long)k.n_t);
    if (!same_decisions(k, p))
        return sr_fail(SR_EINVAL, "parameters differ from the forward call of this token");
    return SR_OK;
}

int sr_prepare_targets(sr_tree* t, const int32_t* active, int64_t n_active, hipStream_t st)
{
    const int64_t n = t->n;
    t->lkey.valid = false;   // the lists belong to the previous targets
    if (!active) {
        hipLaunchKernelGGL(k_targets_all, g256(n), dim3(256), 0, st, n, t->perm, t->tgt_sorted, t->tgt_slot);
        SR_HIP(hipGetLastError());
        return SR_OK;
    }
    hipLaunchKernelGGL(k_fill_i32w, g256(n), dim3(256), 0, st, t->mark, n, 0);
    hipLaunchKernelGGL(k_fill_i32w, g256(ST_WORDS), dim3(256), 0, st, t->status, (int64_t)ST_WORDS, 0);
    hipLaunchKernelGGL(k_mark_active, g256(n_active), dim3(256), 0, st, active, n_active, n, t->invperm, t->mark,
                       t->status);
    hipLaunchKernelGGL(k_flag_marked, g256(n), dim3(256), 0, st, n, t->mark, t->tgt_flag);
    int rc = sr_scan_exclusive(t->tgt_flag, (uint32_t*)t->tgt_pos, n, t->scan_tmp, st);
    if (rc) return rc;
    hipLaunchKernelGGL(k_compact_targets, g256(n), dim3(256), 0, st, n, t->mark, t->tgt_pos, t->tgt_sorted,
                       t->tgt_slot);
    int32_t flags = 0;
    SR_HIP(hipMemcpyAsync(&flags, t->status + ST_FLAGS, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    SR_HIP(hipStreamSynchronize(st));
    if (flags & 2) return sr_fail(SR_EINVAL, "active: index out of range [0, n)");
    if (flags & 4) return sr_fail(SR_EINVAL, "active: repeated index");
    return SR_OK;
}

int sr_axpy_device(void* y, int y_type, const void* x, int x_type, double a, int64_t n, hipStream_t st)
{
    const dim3 g = g256(n);
    if (y_type == SR_F64 && x_type == SR_F64) hipLaunchKernelGGL((k_axpy<double, double>), g, dim3(256), 0, st, (double*)y, (const double*)x, a, n);
    else if (y_type == SR_F64) hipLaunchKernelGGL((k_axpy<double, float>), g, dim3(256), 0, st, (double*)y, (const float*)x, a, n);
    else if (x_type == SR_F64) hipLaunchKernelGGL((k_axpy<float, double>), g, dim3(256), 0, st, (float*)y, (const double*)x, a, n);
    else hipLaunchKernelGGL((k_axpy<float, float>), g, dim3(256), 0, st, (float*)y, (const float*)x, a, n);
    SR_HIP(hipGetLastError());
    return SR_OK;
}

int sr_walk_forward(sr_tree* t, const sr_params* p, int64_t n_t, const int32_t* active, const double* a_old,
                    void* acc, int32_t* counts, hipStream_t st)
{
    if (n_t == 0) return SR_OK;
    WalkArgs a = make_args(t, p, n_t, a_old);
    a.acc = acc;
    a.counts = counts;
    if (t->n_nodes == 0) {
        // a single particle: no sources, every group list is empty
        const int64_t groups = (n_t + WAVE - 1) / WAVE;
        int rc = sr_list_reserve(t, groups, 1, 1, st);
        if (rc) return rc;
        t->n_units = 0;
        t->lkey.valid = false;
        hipLaunchKernelGGL(k_fill_i32w, g256(groups), dim3(256), 0, st, t->group_head, groups, -1);
        return eval_and_reduce<false>(p, a, handle_store(t), 0, 0, st);
    }
    // traversal, evaluation and reduction go to the stream back to back, the
    // evaluation sized by the previous unit count; the counters are checked once
    // at the end (units beyond the estimate are evaluated then, an overflow
    // grows the lists and starts again)
    int64_t want = initial_want(n_t);
    int64_t fcap = t->cap_front > 4096 ? t->cap_front : 4096;
    for (int attempt = 0; attempt < 8; ++attempt) {
        int rc = traverse_launch(t, p, n_t, active, a_old, want, fcap, st);
        if (rc) return rc;
        const int64_t guess = t->unit_hint > 0 && t->unit_hint < t->cap_units ? t->unit_hint : t->cap_units;
        if ((rc = eval_and_reduce<false>(p, a, handle_store(t), 0, guess, st))) return rc;
        bool overflow = false;
        if ((rc = traverse_finish(t, p, n_t, active, a_old, st, overflow))) return rc;
        if (!overflow) {
            if (t->n_units > guess) {
                if ((rc = eval_and_reduce<false>(p, a, handle_store(t), guess, t->n_units - guess, st))) return rc;
            }
            t->unit_hint = t->n_units + t->n_units / 8 + 64;
            return SR_OK;
        }
        want = 2 * t->cap_chunks * 64;
        fcap = 2 * t->cap_front;
    }
    return sr_fail(SR_ENOMEM, "interaction lists did not fit after repeated growth");
}

int sr_walk_adjoint(sr_tree* t, const sr_params* p, int64_t n_t, const int32_t* active, const double* a_old,
                    const void* w, double* dLdx, double* dLdm, int64_t list_token, hipStream_t st)
{
    const int64_t n = t->n, m = t->n_nodes;
    hipLaunchKernelGGL(k_zero3_f64, g256(7 * n + 4 * m), dim3(256), 0, st, t->pbar, 4 * n, t->tbar, 3 * n, t->nbar,
                       4 * m);
    if (n_t > 0 && m > 0) {
        // the forward's lists (named by the token, checked by the caller) carry the frozen
        // decisions; without a token the same deterministic walk is repeated
        if (list_token == 0) {
            int rc = traverse(t, p, n_t, active, a_old, st);
            if (rc) return rc;
        }
        WalkArgs a = make_args(t, p, n_t, a_old);
        a.w = w;
        a.pbar = t->pbar;
        a.tbar = t->tbar;
        a.nbar = t->nbar;
        int rc = eval_and_reduce<true>(p, a, handle_store(t), 0, t->n_units, st);
        if (rc) return rc;
    }
    double sx = 1.0, sm = 1.0;
    if (p->precision != SR_FP64) {
        // FP32 terms carry masses scaled by 2^64 and integer-coordinate lengths
        const double L = t->box;
        sx = p->G * TWO32 / (L * L * L);
        sm = p->G * TWO32 * TWO32 / (L * L);
    }
    sr_timing_mark(SR_T_PUSHDOWN, true, st);
    hipLaunchKernelGGL(k_pushdown, g256(n), dim3(256), 0, st, n, t->perm, t->pparent, t->n_parent, t->prec64,
                       t->nrec64, t->pbar, t->tbar, t->nbar, sx, sm, dLdx, dLdm);
    sr_timing_mark(SR_T_PUSHDOWN, false, st);
    SR_HIP(hipGetLastError());
    return SR_OK;
}

// ----------------------------------------------------------------------------------
// the allocation-free forward
// ----------------------------------------------------------------------------------
//
// Everything the forward needs beyond the tree, the targets' workspace of the
// handle and the outputs -- list counters, group heads, the traversal frontier,
// chunks, units and partial sums -- lives in one fixed device buffer.  Each GPU
// that runs the library holds its own copy until the process ends, and every
// call on that GPU shares it.

static __device__ __align__(256) char scratch[SR_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int SCRATCH_MAX_DEVICES = 64;
constexpr int64_t NOALLOC_FRONT = 2048;   // frontier entries per wave and level
std::mutex g_scratch_mu;
char* g_scratch_addr[SCRATCH_MAX_DEVICES] = {};

// Device address of the current device's copy of `scratch`, looked up once per
// device with that device current.  Host code passes this address, never the
// array's name, to kernels and copies.
int scratch_address(char** out)
{
    int dev = -1;
    SR_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= SCRATCH_MAX_DEVICES)
        return sr_fail(SR_EUNSUPPORTED, "the allocation-free forward supports device ids below %d (current: %d)",
                       SCRATCH_MAX_DEVICES, dev);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_addr[dev]) {
        void* ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr) {
            (void)hipGetLastError();
            return sr_fail(SR_EHIP, "hipGetSymbolAddress of the scratch buffer failed on device %d: %s", dev,
                           hipGetErrorString(e));
        }
        g_scratch_addr[dev] = (char*)ptr;
    }
    *out = g_scratch_addr[dev];
    return SR_OK;
}

// Lays out a list store for n_t targets and `wgs` traversal workgroups in the
// buffer at `base`: counters, group heads and the frontier first, then units
// and chunks in proportion (UCH chunks per unit, plus the units
// every wave may open or leave reserved).
int carve_scratch(char* base, int64_t n_t, int64_t wgs, ListStore& S)
{
    auto up = [](int64_t b) { return (b + 255) & ~(int64_t)255; };
    const int64_t groups = (n_t + WAVE - 1) / WAVE;
    S = ListStore{};
    int64_t off = 0;
    S.counters = (int32_t*)(base + off);
    off += up(8 * sizeof(int32_t));
    S.group_head = (int32_t*)(base + off);
    off += up(groups * (int64_t)sizeof(int32_t));
    S.cap_front = NOALLOC_FRONT;
    S.chunk_batch = TRAV_CHUNK_BATCH_NOALLOC;
    S.unit_batch = TRAV_UNIT_BATCH_NOALLOC;
    S.frontier = (uint32_t*)(base + off);
    off += up(wgs * TW * S.cap_front * 6 * (int64_t)sizeof(uint32_t));
    const int64_t per_chunk = 64 * 4 + 64 * 8 + 2 * 4;   // ent_src, ent_mask, next, count
    const int64_t per_unit = 4 * 4 + PARTIAL_BYTES;       // group, chunk, nch, next, partials
    const int64_t unit_fixed = TW * groups + TW * wgs * TRAV_UNIT_BATCH_NOALLOC + 1;
    const int64_t slack = 10 * 256;                       // alignment of the ten arrays below
    const int64_t left = SR_NOALLOC_SCRATCH_BYTES - off - slack - unit_fixed * per_unit;
    const int64_t chunks = left > 0 ? left * UCH / (UCH * per_chunk + per_unit) : 0;
    const int64_t min_chunks = TW * wgs * (TRAV_CHUNK_BATCH_NOALLOC + 2) + 1;
    if (chunks < min_chunks)
        return sr_fail(SR_EINVAL, "%lld targets leave no room for interaction lists in the %lld-byte scratch buffer",
                       (long long)n_t, (long long)SR_NOALLOC_SCRATCH_BYTES);
    const int64_t units = unit_fixed + chunks / UCH;
    auto take = [&](int64_t bytes) {
        char* q = base + off;
        off += up(bytes);
        return q;
    };
    S.ent_src = (uint32_t*)take(64 * chunks * 4);
    S.ent_mask = (uint64_t*)take(64 * chunks * 8);
    S.chunk_next = (int32_t*)take(chunks * 4);
    S.chunk_cnt = (int32_t*)take(chunks * 4);
    S.unit_group = (int32_t*)take(units * 4);
    S.unit_chunk = (int32_t*)take(units * 4);
    S.unit_nch = (int32_t*)take(units * 4);
    S.unit_next = (int32_t*)take(units * 4);
    S.partials = take(units * PARTIAL_BYTES);
    if (off > SR_NOALLOC_SCRATCH_BYTES)
        return sr_fail(SR_EINVAL, "internal: scratch layout of %lld bytes exceeds the buffer", (long long)off);
    S.cap_chunks = chunks;
    S.cap_units = units;
    return SR_OK;
}

}  // namespace

int sr_walk_forward_noalloc(sr_tree* t, const sr_params* p, int64_t n_t, const int32_t* active, const double* a_old,
                            void* acc, int32_t* counts, hipStream_t st)
{
    t->lkey.valid = false;   // the targets changed; the handle's lists no longer match them
    if (n_t == 0) return SR_OK;
    if (n_t > SR_NOALLOC_MAX_TARGETS)
        return sr_fail(SR_EINVAL, "the allocation-free forward takes at most %lld targets (got %lld)",
                       (long long)SR_NOALLOC_MAX_TARGETS, (long long)n_t);
    char* base = nullptr;
    int rc = scratch_address(&base);
    if (rc) return rc;
    const int64_t groups = (n_t + WAVE - 1) / WAVE;
    int64_t wgs = 1;
    if ((rc = traversal_workgroups(groups, 1, wgs))) return rc;
    ListStore S;
    if ((rc = carve_scratch(base, n_t, wgs, S))) return rc;
    WalkArgs a = make_args(t, p, n_t, a_old);
    a.acc = acc;
    a.counts = counts;
    if (t->n_nodes == 0) {
        // a single particle: no sources, every group list is empty
        hipLaunchKernelGGL(k_fill_i32w, g256(groups), dim3(256), 0, st, S.group_head, groups, -1);
        return eval_and_reduce<false>(p, a, S, 0, 0, st);
    }
    if ((rc = launch_traversal(t, p, n_t, active, a_old, S, wgs, st))) return rc;
    const int64_t guess = t->unit_hint > 0 && t->unit_hint < S.cap_units ? t->unit_hint : S.cap_units;
    if ((rc = eval_and_reduce<false>(p, a, S, 0, guess, st))) return rc;
    bool overflow = false;
    rc = traverse_finish(t, p, n_t, active, a_old, st, overflow);
    t->lkey.valid = false;   // these lists are not the handle's: no token names them
    if (rc) return rc;
    if (overflow)
        return sr_fail(SR_ENOMEM, "the interaction lists of %lld targets do not fit the %lld-byte scratch buffer "
                       "of the allocation-free forward (acc and counts are not valid)",
                       (long long)n_t, (long long)SR_NOALLOC_SCRATCH_BYTES);
    if (t->n_units > guess) return eval_and_reduce<false>(p, a, S, guess, t->n_units - guess, st);
    return SR_OK;
}
