// Tree build on the device: wrap + quantise + Morton keys, LDS radix sort,
// compressed octree topology, pre-order numbering, FP64 node moments.
//
// All integer steps are exact, and the FP64 moment fold follows the fixed
// child order with no fused multiply-add (the file is compiled with
// -ffp-contract=off), so the result is reproducible bit for bit.
#include <stdarg.h>
#include <stdio.h>

#include "internal.h"
#include "sort.h"

namespace {

constexpr int TPB = 256;                 // threads per block for elementwise kernels
// Radix-sort tiles hold TPB * ITEMS keys; ITEMS is chosen by N (2, 4 or 8) so
// that a pass has several hundred blocks.
constexpr int SCAN_ITEMS = 8;
constexpr int SCAN_TILE = TPB * SCAN_ITEMS;
constexpr double TWO32 = 4294967296.0;

__host__ __device__ inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

// ------------------------------------------------------------------------------------
// wrap, quantise, key
// ------------------------------------------------------------------------------------

// u = x/L - floor(x/L) in [0, 1) (a rounding to 1 maps to 0), X = floor(u 2^32).
__device__ inline double wrap_unit(double x, double box)
{
    double u = x / box;
    u = u - floor(u);
    if (u >= 1.0) u = 0.0;
    return u;
}

// Spread the low 15 bits of v to every third bit (bit b -> bit 3b).
__device__ inline uint64_t spread3(uint64_t v)
{
    v &= 0x1fffffull;
    v = (v | (v << 32)) & 0x1f00000000ffffull;
    v = (v | (v << 16)) & 0x1f0000ff0000ffull;
    v = (v | (v << 8)) & 0x100f00f00f00f00full;
    v = (v | (v << 4)) & 0x10c30c30c30c30c3ull;
    v = (v | (v << 2)) & 0x1249249249249249ull;
    return v;
}

__global__ void k_keys(const double* __restrict__ pos, const double* __restrict__ mass,
                       const double* __restrict__ eps, double eps_scalar, int64_t n, double box,
                       uint64_t* __restrict__ khi, uint64_t* __restrict__ klo,
                       uint32_t* __restrict__ kidx, int32_t* __restrict__ status)
{
    int64_t i = blockIdx.x * (int64_t)TPB + threadIdx.x;
    if (i >= n) return;
    bool bad = false;
    uint32_t c[3];
    for (int k = 0; k < 3; ++k) {
        double x = pos[3 * i + k];
        if (!isfinite(x)) bad = true;
        double u = isfinite(x) ? wrap_unit(x, box) : 0.0;
        c[k] = ((uint32_t)floor(u * TWO32)) >> 2;   // 30-bit coordinate
    }
    double m = mass[i];
    double e = eps ? eps[i] : eps_scalar;
    if (!(isfinite(m) && m > 0.0) || !(isfinite(e) && e > 0.0)) bad = true;
    if (bad) atomicOr(&status[ST_FLAGS], 1);
    // bit 1: some softening differs from particle 0's (one atomic per wave at most)
    const bool differs = eps && e != eps[0];
    if (__ballot(differs) && (threadIdx.x & 63) == __builtin_ctzll(__ballot(differs))) atomicOr(&status[ST_FLAGS], 2);
    // digits 1..15 from coordinate bits 29..15, digits 16..30 from bits 14..0; x-major
    khi[i] = (spread3(c[0] >> 15) << 2) | (spread3(c[1] >> 15) << 1) | spread3(c[2] >> 15);
    klo[i] = (spread3(c[0] & 0x7fffu) << 2) | (spread3(c[1] & 0x7fffu) << 1) | spread3(c[2] & 0x7fffu);
    kidx[i] = (uint32_t)i;
}

// ------------------------------------------------------------------------------------
// exclusive scan of uint32 (three kernels: tile sums, scan of sums, tile scans)
// ------------------------------------------------------------------------------------

__device__ inline uint32_t wave_inclusive_scan(uint32_t v)
{
    const int lane = threadIdx.x & 63;
    for (int o = 1; o < 64; o <<= 1) {
        uint32_t y = __shfl_up(v, o, 64);
        if (lane >= o) v += y;
    }
    return v;
}

// Block-wide exclusive scan of one value per thread (TPB threads); returns the
// exclusive prefix and the block total.
__device__ inline uint32_t block_exclusive_scan(uint32_t v, uint32_t* total)
{
    __shared__ uint32_t s_w[TPB / 64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    uint32_t inc = wave_inclusive_scan(v);
    if (lane == 63) s_w[w] = inc;
    __syncthreads();
    uint32_t off = 0, tot = 0;
    for (int k = 0; k < TPB / 64; ++k) {
        if (k < w) off += s_w[k];
        tot += s_w[k];
    }
    __syncthreads();
    *total = tot;
    return off + inc - v;
}

__global__ void k_scan_sums(const uint32_t* __restrict__ in, int64_t n, uint32_t* __restrict__ sums)
{
    int64_t base = blockIdx.x * (int64_t)SCAN_TILE;
    uint32_t acc = 0;
    for (int r = 0; r < SCAN_ITEMS; ++r) {
        int64_t i = base + (int64_t)threadIdx.x * SCAN_ITEMS + r;
        if (i < n) acc += in[i];
    }
    uint32_t tot;
    block_exclusive_scan(acc, &tot);
    if (threadIdx.x == 0) sums[blockIdx.x] = tot;
}

// Exclusive scan of n <= 64 * 1024 values by one workgroup of 1024 threads, total
// at out[n]; in place is allowed.  Thread t takes a contiguous run of `per`
// values (a multiple of 4), loaded as 16-byte vectors in one unrolled burst.
constexpr int SCAN1_TPB = 1024;
constexpr int SCAN1_MAXPER = 64;
__global__ __launch_bounds__(SCAN1_TPB) void k_scan_one(const uint32_t* in, uint32_t* out, int64_t n)
{
    __shared__ uint32_t s_w[SCAN1_TPB / 64];
    const int64_t per = ((n + SCAN1_TPB - 1) / SCAN1_TPB + 3) & ~(int64_t)3;
    const int64_t b = threadIdx.x * per;
    uint32_t v[SCAN1_MAXPER];
    uint32_t acc = 0;
#pragma unroll
    for (int q = 0; q < SCAN1_MAXPER / 4; ++q) {
        const int64_t i = b + 4 * q;
        uint4 x = make_uint4(0, 0, 0, 0);
        if (4 * q < per) {
            if (i + 3 < n) {
                x = *(const uint4*)(in + i);
            } else {
                x.x = i < n ? in[i] : 0u;
                x.y = i + 1 < n ? in[i + 1] : 0u;
                x.z = i + 2 < n ? in[i + 2] : 0u;
            }
        }
        v[4 * q] = x.x;
        v[4 * q + 1] = x.y;
        v[4 * q + 2] = x.z;
        v[4 * q + 3] = x.w;
        acc += (x.x + x.y) + (x.z + x.w);
    }
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const uint32_t inc = wave_inclusive_scan(acc);
    if (lane == 63) s_w[w] = inc;
    __syncthreads();
    uint32_t off = inc - acc;
    for (int k = 0; k < w; ++k) off += s_w[k];
#pragma unroll
    for (int q = 0; q < SCAN1_MAXPER / 4; ++q) {
        const int64_t i = b + 4 * q;
        uint4 y;
        y.x = off;
        y.y = y.x + v[4 * q];
        y.z = y.y + v[4 * q + 1];
        y.w = y.z + v[4 * q + 2];
        off = y.w + v[4 * q + 3];
        if (4 * q < per) {
            if (i + 3 < n) {
                *(uint4*)(out + i) = y;
            } else {
                if (i < n) out[i] = y.x;
                if (i + 1 < n) out[i + 1] = y.y;
                if (i + 2 < n) out[i + 2] = y.z;
            }
        }
    }
    if (threadIdx.x == SCAN1_TPB - 1) out[n] = off;
}

// One block scans all tile sums in place (exclusive).
__global__ void k_scan_top(uint32_t* __restrict__ sums, int64_t nb)
{
    __shared__ uint32_t s_carry;
    if (threadIdx.x == 0) s_carry = 0;
    __syncthreads();
    for (int64_t b0 = 0; b0 < nb; b0 += TPB) {
        int64_t i = b0 + threadIdx.x;
        uint32_t v = i < nb ? sums[i] : 0;
        uint32_t tot;
        uint32_t ex = block_exclusive_scan(v, &tot);
        uint32_t carry = s_carry;
        if (i < nb) sums[i] = carry + ex;
        __syncthreads();
        if (threadIdx.x == 0) s_carry = carry + tot;
        __syncthreads();
    }
    if (threadIdx.x == 0) sums[nb] = s_carry;
}

__global__ void k_scan_tiles(const uint32_t* __restrict__ in, uint32_t* __restrict__ out, int64_t n,
                             const uint32_t* __restrict__ sums)
{
    int64_t base = blockIdx.x * (int64_t)SCAN_TILE;
    uint32_t v[SCAN_ITEMS];
    uint32_t acc = 0;
    for (int r = 0; r < SCAN_ITEMS; ++r) {
        int64_t i = base + (int64_t)threadIdx.x * SCAN_ITEMS + r;
        v[r] = i < n ? in[i] : 0;
        acc += v[r];
    }
    uint32_t tot;
    uint32_t off = block_exclusive_scan(acc, &tot) + sums[blockIdx.x];
    for (int r = 0; r < SCAN_ITEMS; ++r) {
        int64_t i = base + (int64_t)threadIdx.x * SCAN_ITEMS + r;
        if (i < n) out[i] = off;
        off += v[r];
    }
    if (blockIdx.x == gridDim.x - 1 && threadIdx.x == TPB - 1) out[n] = off;
}

// ------------------------------------------------------------------------------------
// LSD radix sort of 90-bit keys (two 45-bit words) with the original index as payload
// ------------------------------------------------------------------------------------

// Digit `pass` of a key: with HI, the 96-bit tree key (lo word bits 0..47, then
// hi word bits 0..47); without, byte `pass` of a single 64-bit key.
template <bool HI>
__device__ inline uint32_t rs_digit(uint64_t hi, uint64_t lo, int pass)
{
    if (!HI) return (uint32_t)(lo >> (8 * pass)) & 0xffu;
    return pass < 6 ? (uint32_t)(lo >> (8 * pass)) & 0xffu : (uint32_t)(hi >> (8 * (pass - 6))) & 0xffu;
}

template <int RS_ITEMS, bool HI>
__global__ void k_rs_hist(const uint64_t* __restrict__ hi, const uint64_t* __restrict__ lo, int64_t n,
                          int pass, uint32_t* __restrict__ hist, int64_t nb)
{
    __shared__ uint32_t h[256];
    h[threadIdx.x] = 0;
    __syncthreads();
    int64_t base = blockIdx.x * (int64_t)(TPB * RS_ITEMS);
    for (int r = 0; r < RS_ITEMS; ++r) {
        int64_t i = base + r * TPB + threadIdx.x;
        if (i < n) atomicAdd(&h[rs_digit<HI>(HI ? hi[i] : 0, lo[i], pass)], 1u);
    }
    __syncthreads();
    hist[threadIdx.x * nb + blockIdx.x] = h[threadIdx.x];
}

// Per digit (one block each): exclusive scan, in place, of the digit's tile
// counts (row d of the digit-major histogram), and the digit's total into
// tot[d].  The scatter adds the digits' base offsets (the exclusive scan of tot)
// itself, so a pass needs no device-wide scan.
__global__ void k_rs_digit_scan(uint32_t* __restrict__ hist, int64_t nb, uint32_t* __restrict__ tot)
{
    uint32_t* row = hist + blockIdx.x * nb;
    const int64_t per = (nb + TPB - 1) / TPB;
    const int64_t b = threadIdx.x * per, e = b + per < nb ? b + per : nb;
    uint32_t acc = 0;
    for (int64_t i = b; i < e; ++i) acc += row[i];
    uint32_t total;
    uint32_t off = block_exclusive_scan(acc, &total);
    for (int64_t i = b; i < e; ++i) {
        const uint32_t v = row[i];
        row[i] = off;
        off += v;
    }
    if (threadIdx.x == 0) tot[blockIdx.x] = total;
}

// Stable scatter: within a tile, keys keep their order (rounds in order, waves
// in order, lanes in order); a tile's offset for digit d is the digit's base
// (keys with a smaller digit) plus the keys of digit d in earlier tiles.
template <int RS_ITEMS, bool HI>
__global__ void k_rs_scatter(const uint64_t* __restrict__ hi, const uint64_t* __restrict__ lo,
                             const uint32_t* __restrict__ idx, uint64_t* __restrict__ ohi,
                             uint64_t* __restrict__ olo, uint32_t* __restrict__ oidx, int64_t n,
                             int pass, const uint32_t* __restrict__ offs, int64_t nb,
                             const uint32_t* __restrict__ tot)
{
    static_assert(TPB == 256, "one thread per digit");
    __shared__ uint32_t s_off[256];
    __shared__ uint32_t s_w[TPB / 64][256];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    uint32_t all;
    const uint32_t dbase = block_exclusive_scan(tot[threadIdx.x], &all);
    s_off[threadIdx.x] = dbase + offs[threadIdx.x * nb + blockIdx.x];
    const uint64_t lt = (1ull << lane) - 1ull;
    int64_t base = blockIdx.x * (int64_t)(TPB * RS_ITEMS);
    for (int r = 0; r < RS_ITEMS; ++r) {
        int64_t i = base + r * TPB + threadIdx.x;
        bool valid = i < n;
        uint64_t h = 0, l = 0;
        uint32_t v = 0, d = 0;
        if (valid) {
            if (HI) h = hi[i];
            l = lo[i];
            v = idx[i];
            d = rs_digit<HI>(h, l, pass);
        }
        uint64_t peers = __ballot(valid);
        for (int b = 0; b < 8; ++b) {
            uint64_t bits = __ballot(valid && ((d >> b) & 1u));
            peers &= ((d >> b) & 1u) ? bits : ~bits;
        }
        uint32_t rank = (uint32_t)__popcll(peers & lt);
        for (int k = 0; k < 4; ++k) s_w[w][lane * 4 + k] = 0;
        __syncthreads();
        if (valid && rank == 0) s_w[w][d] = (uint32_t)__popcll(peers);
        __syncthreads();
        uint32_t p = 0;
        if (valid) {
            p = s_off[d] + rank;
            for (int k = 0; k < w; ++k) p += s_w[k][d];
        }
        __syncthreads();
        uint32_t add = 0;
        for (int k = 0; k < TPB / 64; ++k) add += s_w[k][threadIdx.x];
        s_off[threadIdx.x] += add;
        __syncthreads();
        if (valid) {
            if (HI) ohi[p] = h;
            olo[p] = l;
            oidx[p] = v;
        }
    }
}

// ------------------------------------------------------------------------------------
// single-pass radix sort of the tree keys (decoupled look-back)
// ------------------------------------------------------------------------------------
//
// One launch histograms all 12 digits; then one launch per 8-bit digit, LSD
// order.  A pass's workgroups take tiles of OS_TPB x OS_ITEMS consecutive keys in ticket
// order (a device counter) and rank their keys in the tile (stable: wave w holds
// a contiguous run, rounds in order, lanes in order, per-wave digit counters in
// LDS).  Per digit, a tile publishes its count, then, once the counts of all
// earlier tiles are known, its inclusive prefix; it learns its own prefix by
// reading back over the earlier tiles' words, OS_WIN at a time, adding counts
// until it meets an inclusive prefix.  A tile only waits for tiles with smaller
// tickets, which are already running and publish their counts before they wait
// themselves, so every wait ends; a wait that sees no progress for OS_SPIN_MAX
// rounds gives up and flags the build as failed.  The words are 64-bit: the
// pass's tag and state (count or inclusive prefix) in the high half, the value
// in the low half; the tag changes every pass, so the words need no clearing
// between sorts.  The tile is then reordered by digit in LDS and written out
// with consecutive threads on consecutive output positions.
constexpr int OS_TPB = 1024;
#ifndef SR_OS_WIN
#define SR_OS_WIN 16
#endif
// keys per thread: 2 (tiles of 2048) up to OS_SMALL_N keys, else 4 (tiles of 4096):
// 0.399 -> 0.389 ms per build on clustered 262k, while 2048-key tiles cost the
// 2M-particle build 1.31 -> 1.47 ms (twice the tiles to look back over)
constexpr int64_t OS_SMALL_N = 512 * 1024;
constexpr int OS_ITEMS_MIN = 2;
constexpr int OS_WAVES = OS_TPB / 64;
constexpr int OS_TILE_MIN = OS_TPB * OS_ITEMS_MIN;
constexpr int OS_WIN = SR_OS_WIN;
constexpr uint32_t OS_AGG = 1u, OS_INC = 2u;
constexpr int64_t OS_SPIN_MAX = int64_t(1) << 20;

__global__ __launch_bounds__(TPB) void k_os_hist(const uint64_t* __restrict__ hi, const uint64_t* __restrict__ lo,
                                                 int64_t n, uint32_t* __restrict__ hist)
{
    __shared__ uint32_t h[12 * 256];
    for (int i = threadIdx.x; i < 12 * 256; i += TPB) h[i] = 0;
    __syncthreads();
    for (int64_t i = blockIdx.x * (int64_t)TPB + threadIdx.x; i < n; i += (int64_t)gridDim.x * TPB) {
        const uint64_t H = hi[i], L = lo[i];
#pragma unroll
        for (int p = 0; p < 12; ++p) atomicAdd(&h[p * 256 + rs_digit<true>(H, L, p)], 1u);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < 12 * 256; i += TPB)
        if (h[i]) atomicAdd(&hist[i], h[i]);
}

// Exclusive scan over the 256 digits held by threads 0 .. 255 (the others pass
// 0 and get garbage); every thread of the block must call it.
__device__ inline uint32_t digit_exclusive_scan(uint32_t v, uint32_t* s_w)
{
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const uint32_t inc = wave_inclusive_scan(v);
    if (w < 4 && lane == 63) s_w[w] = inc;
    __syncthreads();
    uint32_t off = 0;
    for (int k = 0; k < 4; ++k)
        if (k < w) off += s_w[k];
    __syncthreads();
    return off + inc - v;
}

template <int OS_ITEMS>
__global__ __launch_bounds__(OS_TPB) void k_os_pass(const uint64_t* __restrict__ hi, const uint64_t* __restrict__ lo,
                                                    const uint32_t* __restrict__ idx, uint64_t* __restrict__ ohi,
                                                    uint64_t* __restrict__ olo, uint32_t* __restrict__ oidx,
                                                    int64_t n, int pass, const uint32_t* __restrict__ hist,
                                                    uint32_t* __restrict__ ticket, uint64_t* __restrict__ look,
                                                    uint32_t tag, int32_t* __restrict__ flags)
{
    __shared__ uint32_t s_cnt[OS_WAVES][256];   // per wave: digit counts, then offsets in the tile
    __shared__ uint32_t s_base[256];             // output position of the tile's first key of each digit
    __shared__ uint32_t s_start[256];            // tile position of the first key of each digit
    __shared__ uint32_t s_w[4];
    constexpr int OS_TILE = OS_TPB * OS_ITEMS;
    __shared__ uint64_t s_hi[OS_TILE], s_lo[OS_TILE];
    __shared__ uint32_t s_ix[OS_TILE];
    __shared__ int64_t s_tile;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, d = threadIdx.x;
    if (threadIdx.x == 0) s_tile = atomicAdd(ticket, 1u);
    for (int k = lane; k < 256; k += 64) s_cnt[w][k] = 0;
    // keys with a smaller digit (threads 0 .. 255)
    const uint32_t dbase = digit_exclusive_scan(d < 256 ? hist[d] : 0u, s_w);
    const int64_t tile = s_tile;
    const int64_t e0 = tile * OS_TILE + (int64_t)w * 64 * OS_ITEMS;
    const uint64_t lt = (1ull << lane) - 1ull;
    uint64_t H[OS_ITEMS], L[OS_ITEMS];
    uint32_t V[OS_ITEMS], R[OS_ITEMS], D[OS_ITEMS];
#pragma unroll
    for (int r = 0; r < OS_ITEMS; ++r) {
        const int64_t i = e0 + r * 64 + lane;
        const bool valid = i < n;
        H[r] = valid ? hi[i] : 0;
        L[r] = valid ? lo[i] : 0;
        V[r] = valid ? idx[i] : 0;
    }
#pragma unroll
    for (int r = 0; r < OS_ITEMS; ++r) {
        const bool valid = e0 + r * 64 + lane < n;
        const uint32_t dg = rs_digit<true>(H[r], L[r], pass);
        D[r] = dg;
        uint64_t peers = __ballot(valid);
        for (int b = 0; b < 8; ++b) {
            const uint64_t bits = __ballot(valid && ((dg >> b) & 1u));
            peers &= ((dg >> b) & 1u) ? bits : ~bits;
        }
        const uint32_t rank = (uint32_t)__popcll(peers & lt);
        uint32_t before = 0;
        if (valid) before = s_cnt[w][dg];
        R[r] = before + rank;
        // the lowest lane of each digit group moves the wave's counter on; the
        // wave's LDS accesses happen in program order
        if (valid && rank == 0) s_cnt[w][dg] = before + (uint32_t)__popcll(peers);
    }
    __syncthreads();
    // per digit: the tile's count and each wave's offset among the digit's keys
    uint32_t cnt = 0;
    if (d < 256) {
        for (int k = 0; k < OS_WAVES; ++k) {
            const uint32_t c = s_cnt[k][d];
            s_cnt[k][d] = cnt;
            cnt += c;
        }
    }
    const uint32_t start = digit_exclusive_scan(d < 256 ? cnt : 0u, s_w);
    if (d < 256) {
        s_start[d] = start;
        uint64_t* word = look + tile * 256 + d;
        const uint64_t hi_agg = (uint64_t)(4u * tag + OS_AGG) << 32, hi_inc = (uint64_t)(4u * tag + OS_INC) << 32;
        uint32_t prefix = 0;
        if (tile == 0) {
            __hip_atomic_store(word, hi_inc | cnt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        } else {
            __hip_atomic_store(word, hi_agg | cnt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            int64_t j = tile - 1, idle = 0;
            for (;;) {
                uint64_t v[OS_WIN];
#pragma unroll
                for (int k = 0; k < OS_WIN; ++k)
                    v[k] = j - k >= 0 ? __hip_atomic_load(look + (j - k) * 256 + d, __ATOMIC_RELAXED,
                                                          __HIP_MEMORY_SCOPE_AGENT)
                                      : hi_inc;
                int k = 0;
                bool done = false;
                for (; k < OS_WIN; ++k) {
                    const uint32_t h = (uint32_t)(v[k] >> 32);
                    if ((h >> 2) != tag) break;   // not published yet
                    prefix += (uint32_t)v[k];
                    if ((h & 3u) == OS_INC) {
                        done = true;
                        break;
                    }
                }
                if (done) break;
                j -= k;
                if (k == 0 && ++idle > OS_SPIN_MAX) {
                    atomicOr(flags, 4);
                    break;
                }
            }
            __hip_atomic_store(word, hi_inc | (prefix + cnt), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        s_base[d] = dbase + prefix;
    }
    __syncthreads();
    // the tile in digit order in LDS
#pragma unroll
    for (int r = 0; r < OS_ITEMS; ++r) {
        if (e0 + r * 64 + lane >= n) continue;
        const uint32_t q = s_start[D[r]] + s_cnt[w][D[r]] + R[r];
        s_hi[q] = H[r];
        s_lo[q] = L[r];
        s_ix[q] = V[r];
    }
    __syncthreads();
    const int64_t rem = n - tile * OS_TILE;
    const int m = rem < OS_TILE ? (int)rem : OS_TILE;
    for (int q = threadIdx.x; q < m; q += OS_TPB) {
        const uint64_t Hq = s_hi[q], Lq = s_lo[q];
        const uint32_t dg = rs_digit<true>(Hq, Lq, pass);
        const uint32_t p = s_base[dg] + (uint32_t)q - s_start[dg];
        ohi[p] = Hq;
        olo[p] = Lq;
        oidx[p] = s_ix[q];
    }
}

// ------------------------------------------------------------------------------------
// sorted records
// ------------------------------------------------------------------------------------

__global__ void k_gather(const double* __restrict__ pos, const double* __restrict__ mass,
                         const double* __restrict__ eps, double eps_scalar, int64_t n, double box,
                         const uint32_t* __restrict__ sidx, int32_t* __restrict__ perm,
                         int32_t* __restrict__ invperm, Rec64* __restrict__ r64,
                         double* __restrict__ h64, Rec32* __restrict__ r32, float* __restrict__ h32)
{
    int64_t s = blockIdx.x * (int64_t)TPB + threadIdx.x;
    if (s >= n) return;
    uint32_t i = sidx[s];
    perm[s] = (int32_t)i;
    invperm[i] = (int32_t)s;
    double u[3];
    uint32_t X[3];
    for (int k = 0; k < 3; ++k) {
        u[k] = wrap_unit(pos[3 * i + k], box);
        X[k] = (uint32_t)floor(u[k] * TWO32);
    }
    double m = mass[i];
    double h = 2.8 * (eps ? eps[i] : eps_scalar);
    r64[s] = Rec64{u[0] * box, u[1] * box, u[2] * box, m};
    h64[s] = h;
    r32[s] = Rec32{X[0], X[1], X[2], (float)m};
    h32[s] = (float)(h / box * TWO32);
}

// ------------------------------------------------------------------------------------
// topology: binary radix tree of the keys (index-augmented), then its octree nodes
// ------------------------------------------------------------------------------------

// Common-prefix length in bits of sorted keys a and b, ties broken by position
// (90 + leading equal bits of the positions); -1 outside [0, n).
__device__ inline int delta(const uint64_t* __restrict__ hi, const uint64_t* __restrict__ lo,
                            int64_t n, int64_t a, int64_t b)
{
    if (b < 0 || b >= n) return -1;
    uint64_t x = hi[a] ^ hi[b];
    if (x) return __clzll(x) - 19;
    x = lo[a] ^ lo[b];
    if (x) return 45 + __clzll(x) - 19;
    return 90 + __clz((uint32_t)a ^ (uint32_t)b);
}

__device__ inline int level_of(int lambda) { return (lambda < 90 ? lambda : 90) / 3; }

__global__ void k_radix_tree(const uint64_t* __restrict__ hi, const uint64_t* __restrict__ lo,
                             int64_t n, int32_t* __restrict__ b_lo, int32_t* __restrict__ b_hi,
                             int32_t* __restrict__ b_lambda, int32_t* __restrict__ b_parent,
                             int32_t* __restrict__ leaf_bparent)
{
    int64_t i = blockIdx.x * (int64_t)TPB + threadIdx.x;
    if (i >= n - 1) return;
    int d = delta(hi, lo, n, i, i + 1) - delta(hi, lo, n, i, i - 1) > 0 ? 1 : -1;
    int dmin = delta(hi, lo, n, i, i - d);
    int64_t lmax = 2;
    while (delta(hi, lo, n, i, i + lmax * d) > dmin) lmax <<= 1;
    int64_t l = 0;
    for (int64_t t = lmax >> 1; t >= 1; t >>= 1)
        if (delta(hi, lo, n, i, i + (l + t) * d) > dmin) l += t;
    int64_t j = i + l * d;
    int dnode = delta(hi, lo, n, i, j);
    int64_t s = 0, t = l;
    do {
        t = (t + 1) >> 1;
        if (delta(hi, lo, n, i, i + (s + t) * d) > dnode) s += t;
    } while (t > 1);
    int64_t g = i + s * d + (d < 0 ? -1 : 0);
    int64_t a = i < j ? i : j, b = i < j ? j : i;
    b_lo[i] = (int32_t)a;
    b_hi[i] = (int32_t)b;
    b_lambda[i] = dnode;
    if (a == g) leaf_bparent[g] = (int32_t)i;
    else b_parent[g] = (int32_t)i;
    if (b == g + 1) leaf_bparent[g + 1] = (int32_t)i;
    else b_parent[g + 1] = (int32_t)i;
    if (i == 0) b_parent[0] = -1;
}

// A binary node is an octree node when it is the root or its octree level is
// deeper than its binary parent's: it is then the whole of its octree cell.
__global__ void k_octree_flags(int64_t n, const int32_t* __restrict__ b_lo,
                               const int32_t* __restrict__ b_lambda, const int32_t* __restrict__ b_parent,
                               uint32_t* __restrict__ levelmask, int32_t* __restrict__ b_pre)
{
    int64_t i = blockIdx.x * (int64_t)TPB + threadIdx.x;
    if (i >= n - 1) return;
    int lev = level_of(b_lambda[i]);
    bool oct = i == 0 || lev > level_of(b_lambda[b_parent[i]]);
    b_pre[i] = oct ? 0 : -1;
    if (oct) atomicOr(&levelmask[b_lo[i]], 1u << lev);
}

__global__ void k_popcount(const uint32_t* __restrict__ mask, int64_t n, uint32_t* __restrict__ cnt)
{
    int64_t s = blockIdx.x * (int64_t)TPB + threadIdx.x;
    if (s < n) cnt[s] = (uint32_t)__popc(mask[s]);
}

// Pre-order = order by (first, level): all nodes that start before `first`, plus
// the enclosing nodes that start at `first` with a smaller level.
__global__ void k_preorder(int64_t n, const int32_t* __restrict__ b_lo, const int32_t* __restrict__ b_lambda,
                           const uint32_t* __restrict__ levelmask, const int32_t* __restrict__ base,
                           int32_t* __restrict__ b_pre)
{
    int64_t i = blockIdx.x * (int64_t)TPB + threadIdx.x;
    if (i >= n - 1 || b_pre[i] < 0) return;
    int lev = level_of(b_lambda[i]);
    int32_t f = b_lo[i];
    b_pre[i] = base[f] + __popc(levelmask[f] & ((1u << lev) - 1u));
}

__global__ void k_node_arrays(int64_t n, const int32_t* __restrict__ b_lo, const int32_t* __restrict__ b_hi,
                              const int32_t* __restrict__ b_lambda, const int32_t* __restrict__ b_parent,
                              const int32_t* __restrict__ b_pre, const int32_t* __restrict__ base,
                              const Rec32* __restrict__ r32, int32_t* __restrict__ n_level,
                              int32_t* __restrict__ n_first, int32_t* __restrict__ n_count,
                              int32_t* __restrict__ n_parent, int32_t* __restrict__ n_skip,
                              uint32_t* __restrict__ n_corner)
{
    int64_t i = blockIdx.x * (int64_t)TPB + threadIdx.x;
    if (i >= n - 1) return;
    int32_t pre = b_pre[i];
    if (pre < 0) return;
    int lev = level_of(b_lambda[i]);
    int32_t f = b_lo[i], c = b_hi[i] - b_lo[i] + 1;
    int32_t p = b_parent[i];
    while (p >= 0 && b_pre[p] < 0) p = b_parent[p];
    n_level[pre] = lev;
    n_first[pre] = f;
    n_count[pre] = c;
    n_parent[pre] = p >= 0 ? b_pre[p] : -1;
    n_skip[pre] = base[f + c];
    uint64_t keep = lev == 0 ? 0ull : (~((1ull << (32 - lev)) - 1ull)) & 0xffffffffull;
    Rec32 q = r32[f];
    n_corner[3 * pre + 0] = (uint32_t)(q.X & keep);
    n_corner[3 * pre + 1] = (uint32_t)(q.Y & keep);
    n_corner[3 * pre + 2] = (uint32_t)(q.Z & keep);
}

// Launched for the N - 1 node bound; the node count m is read on the device.
__global__ void k_node_depth(const int32_t* __restrict__ m_dev, const int32_t* __restrict__ n_parent,
                             const int32_t* __restrict__ n_first,
                             const int32_t* __restrict__ n_count, const int32_t* __restrict__ base,
                             int32_t* __restrict__ n_depth, Item* __restrict__ items,
                             int32_t* __restrict__ status)
{
    // the deepest depth of the block in LDS, one global atomic per block
    __shared__ int32_t dmax;
    if (threadIdx.x == 0) dmax = 0;
    __syncthreads();
    const int64_t m = *m_dev;
    int64_t nd = blockIdx.x * (int64_t)TPB + threadIdx.x;
    if (nd < m) {
        int d = 0;
        for (int32_t p = n_parent[nd]; p >= 0; p = n_parent[p]) ++d;
        n_depth[nd] = d;
        int32_t f = n_first[nd], c = n_count[nd];
        items[f + nd] = Item{(uint32_t)nd, (uint32_t)(f + c + base[f + c]), (uint32_t)d, 0u};
        atomicMax(&dmax, d);
    }
    __syncthreads();
    if (threadIdx.x == 0) atomicMax(&status[ST_MAXDEPTH], dmax);
}

__global__ void k_particle_items(int64_t n, const int32_t* __restrict__ leaf_bparent,
                                 const int32_t* __restrict__ b_parent, const int32_t* __restrict__ b_pre,
                                 const int32_t* __restrict__ base, const int32_t* __restrict__ n_depth,
                                 int32_t* __restrict__ pparent, Item* __restrict__ items)
{
    int64_t s = blockIdx.x * (int64_t)TPB + threadIdx.x;
    if (s >= n) return;
    int32_t pp = -1;
    uint32_t depth = 0;
    if (n > 1) {
        int32_t p = leaf_bparent[s];
        while (b_pre[p] < 0) p = b_parent[p];
        pp = b_pre[p];
        depth = (uint32_t)n_depth[pp] + 1u;
    }
    pparent[s] = pp;
    uint32_t it = (uint32_t)(s + (n > 1 ? base[s + 1] : 0));
    items[it] = Item{(uint32_t)s | ITEM_PARTICLE, it + 1u, depth, 0u};
}

// ------------------------------------------------------------------------------------
// node moments, bottom-up in one launch
// ------------------------------------------------------------------------------------

// Child table of every node: its children in digit order, at most 8 (node
// index, or sorted particle index | ITEM_PARTICLE); a level-30 bucket keeps its
// particle range (first, count) with META_BUCKET.  Launched for the N - 1 node
// bound; the node count is read on the device.
__global__ void k_child_table(const int32_t* __restrict__ m_dev, const Item* __restrict__ items,
                              const int32_t* __restrict__ n_first, const int32_t* __restrict__ n_level,
                              const int32_t* __restrict__ n_count, uint32_t* __restrict__ kids,
                              uint32_t* __restrict__ meta)
{
    const int64_t nd = blockIdx.x * (int64_t)TPB + threadIdx.x;
    if (nd >= *m_dev) return;
    if (n_level[nd] == 30) {
        kids[8 * nd + 0] = (uint32_t)n_first[nd];
        kids[8 * nd + 1] = (uint32_t)n_count[nd];
        meta[nd] = META_BUCKET;
        return;
    }
    const uint32_t it = (uint32_t)(n_first[nd] + nd);
    const uint32_t end = items[it].next;
    uint32_t nk = 0;
    for (uint32_t j = it + 1; j < end;) {
        const Item c = items[j];
        kids[8 * nd + nk] = c.ref;
        ++nk;
        j = (c.ref & ITEM_PARTICLE) ? j + 1 : c.next;
    }
    meta[nd] = nk;
}

// Moments of one node whose children are done: M, S = sum m x, COM = S / M,
// folded left to right over the children in digit order without FMA, the
// support range, the cube geometry and the FP32 record.  All children's data
// are loaded before the fold.
//
// DRIFT (a tree whose particles moved after the build, topology kept): also the
// bounding box of the node's particles, folded with min / max (exact), and the
// node's half side grown to max(l/2, max over members and axes of |x - c|)
// about the fixed cell centre c; that maximum is attained at a box corner
// because rounding is monotone, so the result equals the per-member maximum.
// The opening tests then use twice the grown half side.
struct MomArgs {
    double box;
    const int32_t *n_first, *n_level, *n_count, *n_parent;
    const uint32_t *n_corner, *kids, *meta;
    const Rec64* r64;
    const double* h64;
    Rec64* nrec64;
    double* nS;
    Geo64* geo;
    double *nhmax, *nhmin;
    Rec32* nrec32;
    float* nhmax32;
    WalkRec32* w32;
    WalkRec64* w64;
    double* nbox;
};

// A node's fold of its children: M, S = sum m x, the support range and (DRIFT)
// the bounding box of its particles.
struct NodeFold {
    double M, S0, S1, S2, hx, hn;
    double blo[3], bhi[3];
};

// Everything stored for a folded node: COM = S / M, the cube geometry (grown
// with DRIFT), the FP32-path record and the walk's records.
template <bool DRIFT>
__device__ void node_store(const MomArgs& A, int32_t nd, const NodeFold& f)
{
    const double box = A.box;
    const int32_t* n_level = A.n_level;
    const uint32_t* n_corner = A.n_corner;
    Rec64* nrec64 = A.nrec64;
    double* nS = A.nS;
    Geo64* geo = A.geo;
    double* nhmax = A.nhmax;
    double* nhmin = A.nhmin;
    Rec32* nrec32 = A.nrec32;
    float* nhmax32 = A.nhmax32;
    WalkRec32* w32 = A.w32;
    WalkRec64* w64 = A.w64;
    double* nbox = A.nbox;
    const uint32_t mt = A.meta[nd];
    const uint4 ka = ((const uint4*)(A.kids + 8 * (int64_t)nd))[0];
    const uint4 kb = ((const uint4*)(A.kids + 8 * (int64_t)nd))[1];
    const double M = f.M, S0 = f.S0, S1 = f.S1, S2 = f.S2, hx = f.hx, hn = f.hn;
    const double* blo = f.blo;
    const double* bhi = f.bhi;
    double com[3] = {S0 / M, S1 / M, S2 / M};
    nrec64[nd] = Rec64{com[0], com[1], com[2], M};
    nS[3 * nd + 0] = S0;
    nS[3 * nd + 1] = S1;
    nS[3 * nd + 2] = S2;
    nhmax[nd] = hx;
    nhmin[nd] = hn;
    int lev = n_level[nd];
    const double lcell = ldexp(box, -lev);
    double half = ldexp(1.0, -lev - 1);
    const double cc[3] = {box * (ldexp((double)n_corner[3 * nd + 0], -32) + half),
                          box * (ldexp((double)n_corner[3 * nd + 1], -32) + half),
                          box * (ldexp((double)n_corner[3 * nd + 2], -32) + half)};
    double l = lcell;
    bool grown = false;
    if constexpr (DRIFT) {
        double hs = 0.5 * lcell;
        for (int k = 0; k < 3; ++k) {
            nbox[6 * (int64_t)nd + k] = blo[k];
            nbox[6 * (int64_t)nd + 3 + k] = bhi[k];
            const double e0 = fabs(blo[k] - cc[k]), e1 = fabs(bhi[k] - cc[k]);
            if (e0 > hs) hs = e0;
            if (e1 > hs) hs = e1;
        }
        grown = hs != 0.5 * lcell;
        l = 2.0 * hs;
    }
    const Geo64 gg{cc[0], cc[1], cc[2], l};
    geo[nd] = gg;
    // ticks modulo 2^32 through a signed integer (a drifted centre of mass may lie
    // just outside the box)
    uint32_t q[3];
    for (int k = 0; k < 3; ++k) q[k] = (uint32_t)(int64_t)rint(com[k] / box * TWO32);
    const float M32 = (float)M, hx32 = (float)(hx / box * TWO32);
    nrec32[nd] = Rec32{q[0], q[1], q[2], M32};
    nhmax32[nd] = hx32;
    // the walk's record of this node (one 128-byte line per precision)
    const uint32_t halfi = 1u << (31 - lev);
    const uint64_t lint = 1ull << (32 - lev);
    WalkRec32 a{};
    a.cX = n_corner[3 * nd + 0] + halfi;
    a.cY = n_corner[3 * nd + 1] + halfi;
    a.cZ = n_corner[3 * nd + 2] + halfi;
    a.tin = (uint32_t)((3ull * lint - 1ull) / 5ull);   // largest integer below 0.6 l
    a.X = q[0];
    a.Y = q[1];
    a.Z = q[2];
    a.l2 = __float_as_uint((float)lint * (float)lint);
    a.half = __float_as_uint((float)halfi);
    if (grown) {
        // the grown cube in ticks: half side rounded up (the prune stays conservative),
        // the largest integer below 0.6 side, and the side squared
        const double ht = 0.5 * l / box * TWO32, sd = 2.0 * ht;
        float hf = (float)ht;
        if ((double)hf < ht) hf = nextafterf(hf, INFINITY);
        const double tin = ceil(0.6 * sd) - 1.0;
        a.tin = tin >= 4294967295.0 ? 0xffffffffu : (uint32_t)tin;
        a.l2 = __float_as_uint((float)sd * (float)sd);
        a.half = __float_as_uint(hf);
    }
    a.M = __float_as_uint(M32);
    a.hx = __float_as_uint(hx32);
    a.mixed = hn != hx ? 1u : 0u;
    a.meta = mt;
    a.kids[0] = ka.x;
    a.kids[1] = ka.y;
    a.kids[2] = ka.z;
    a.kids[3] = ka.w;
    a.kids[4] = kb.x;
    a.kids[5] = kb.y;
    a.kids[6] = kb.z;
    a.kids[7] = kb.w;
    w32[nd] = a;
    WalkRec64 b{};
    b.cx = gg.cx;
    b.cy = gg.cy;
    b.cz = gg.cz;
    b.l = l;
    b.X = com[0];
    b.Y = com[1];
    b.Z = com[2];
    b.M = M;
    b.hx = hx;
    b.hn = hn;
    b.meta = mt;
    for (int k = 0; k < 8; ++k) b.kids[k] = a.kids[k];
    w64[nd] = b;
}

// A node that reaches past the end of the particle partition its first particle
// lies in (partitions of P sorted particles).
__device__ inline bool crosses(const MomArgs& A, int32_t nd, int64_t P)
{
    const int64_t f = A.n_first[nd];
    return (f + A.n_count[nd] - 1) / P != f / P;
}

// All node moments, deepest depth first, in a few launches and without
// device-wide waits.  Every node is folded exactly once, after all of its
// children, with the fold above (same order, same operations), so the result
// is that of a depth-by-depth fold.
//
// First pass (k_moments_leaves): block b owns the sorted particles
// [bP1, (b+1)P1) and the nodes whose first particle lies there, the pre-order
// run [base[bP1], base[(b+1)P1]) of at most P1 + 30 nodes (a forest of nodes
// with two or more children each, plus the chain of nodes that reach past the
// partition's end).  The nodes that stay inside the partition only have
// children inside it: the block stages the partition's particles and those
// nodes' child tables in LDS and folds the nodes one depth at a time, their sums
// kept in LDS, a block barrier between depths, then stores them.  The nodes that
// reach past the end contain its last particle and the next one: they are
// ancestors of one node, at consecutive depths, at most 31, and go to the
// block's slots of a list in depth order, which is pre-order.
//
// Later passes (k_moments_list), partitions growing by MP_FAN: block w takes
// the listed nodes of its MP_FAN sub-partitions (pre-order, with their child
// tables, in LDS), folds those that stay inside its own partition one depth at
// a time, a block barrier between depths, and lists the others for the next
// pass the same way.  A child of a folded node is either listed in this block
// (its sums in LDS; `slot` maps it there) or was folded by an earlier pass
// (global memory).  The pass whose partition holds all N particles lists
// nothing.
constexpr int MP_P1 = 512;                               // particles per block of the first pass
constexpr int MP_TPB = 256;
constexpr int MP_NODES = MP_P1 + 32;                     // nodes whose first particle is in a partition
constexpr int MP_OWN = (MP_NODES + MP_TPB - 1) / MP_TPB;
constexpr int MP_SLOTS = 32;                             // list slots per partition (at most 31 used)
constexpr int MP_FAN = 32;                               // sub-partitions per partition of a later pass
constexpr int ML_TPB = 512;
constexpr int ML_CAND = MP_FAN * MP_SLOTS;
constexpr int ML_POOL = 1024;   // children staged in LDS by a later pass (without DRIFT)

struct MomList {
    int32_t* nodes;    // MP_SLOTS per partition
    int32_t* count;    // per partition
};

// One child's terms: M, S (= m x for a particle), hmax, hmin.
struct ChildTerms {
    double cm, c0, c1, c2, cx, cn;
};

__device__ inline void fold_child(NodeFold& f, bool first, const ChildTerms& c)
{
    if (first) {
        f.M = c.cm;
        f.S0 = c.c0;
        f.S1 = c.c1;
        f.S2 = c.c2;
        f.hx = c.cx;
        f.hn = c.cn;
    } else {
        f.M = f.M + c.cm;
        f.S0 = f.S0 + c.c0;
        f.S1 = f.S1 + c.c1;
        f.S2 = f.S2 + c.c2;
        f.hx = c.cx > f.hx ? c.cx : f.hx;
        f.hn = c.cn < f.hn ? c.cn : f.hn;
    }
}

// DRIFT: a child's member box (a particle's position for both corners).
__device__ inline void grow_child(NodeFold& f, bool first, const double* lo, const double* hi)
{
    for (int e = 0; e < 3; ++e) {
        f.blo[e] = first || lo[e] < f.blo[e] ? lo[e] : f.blo[e];
        f.bhi[e] = first || hi[e] > f.bhi[e] ? hi[e] : f.bhi[e];
    }
}

__device__ inline ChildTerms particle_terms(double m, double x, double y, double z, double h)
{
    return ChildTerms{m, m * x, m * y, m * z, h, h};
}

// Terms of child r from its raw data: a particle's m, x, y, z, h or a node's sums.
__device__ inline ChildTerms child_terms(uint32_t r, const double* raw)
{
    if (r & ITEM_PARTICLE) return particle_terms(raw[0], raw[1], raw[2], raw[3], raw[4]);
    return ChildTerms{raw[0], raw[1], raw[2], raw[3], raw[4], raw[5]};
}

// LDS sums of the nodes a block folds: M, S0, S1, S2, hmax, hmin, then with
// DRIFT the box lo xyz, hi xyz.
template <bool DRIFT, int CAP>
struct NodeSums {
    double v[DRIFT ? 12 : 6][CAP];
    __device__ void put(int j, const NodeFold& f)
    {
        v[0][j] = f.M;
        v[1][j] = f.S0;
        v[2][j] = f.S1;
        v[3][j] = f.S2;
        v[4][j] = f.hx;
        v[5][j] = f.hn;
        if constexpr (DRIFT)
            for (int e = 0; e < 3; ++e) {
                v[6 + e][j] = f.blo[e];
                v[9 + e][j] = f.bhi[e];
            }
    }
    __device__ ChildTerms terms(int j) const { return ChildTerms{v[0][j], v[1][j], v[2][j], v[3][j], v[4][j], v[5][j]}; }
    __device__ void box(int j, double* lo, double* hi) const
    {
        for (int e = 0; e < 3; ++e) {
            lo[e] = v[6 + e][j];
            hi[e] = v[9 + e][j];
        }
    }
    __device__ NodeFold fold(int j) const
    {
        NodeFold f{v[0][j], v[1][j], v[2][j], v[3][j], v[4][j], v[5][j], {}, {}};
        if constexpr (DRIFT) box(j, f.blo, f.bhi);
        return f;
    }
};

template <bool DRIFT>
__global__ __launch_bounds__(MP_TPB) void k_moments_leaves(MomArgs A, const int32_t* __restrict__ base,
                                                          const int32_t* __restrict__ depth, int64_t n,
                                                          MomList out)
{
    __shared__ double s_p[5][MP_P1];                    // m, x, y, z, h
    __shared__ NodeSums<DRIFT, MP_NODES> s_n;
    __shared__ uint32_t s_meta[MP_NODES];
    __shared__ uint4 s_kids[MP_NODES][2];
    __shared__ int32_t s_dmin, s_dmax, s_cmin, s_out;
    const int64_t s0 = blockIdx.x * (int64_t)MP_P1, s1 = s0 + MP_P1 < n ? s0 + MP_P1 : n;
    const int32_t nb = base[s0], ne = base[s1];
    if (threadIdx.x == 0) {
        s_dmin = s_cmin = 1 << 30;
        s_dmax = -1;
        s_out = 0;
    }
    for (int64_t k = threadIdx.x; k < s1 - s0; k += MP_TPB) {
        const Rec64 q = A.r64[s0 + k];
        s_p[0][k] = q.m;
        s_p[1][k] = q.x;
        s_p[2][k] = q.y;
        s_p[3][k] = q.z;
        s_p[4][k] = A.h64[s0 + k];
    }
    __syncthreads();
    // own nodes nb + tid + k MP_TPB: depth, or -1 when outside / reaching past the end
    int32_t dep[MP_OWN];
    bool cross[MP_OWN];
    int32_t lmin = 1 << 30, lmax = -1, cmin = 1 << 30;
#pragma unroll
    for (int k = 0; k < MP_OWN; ++k) {
        const int32_t i = nb + (int32_t)threadIdx.x + k * MP_TPB;
        dep[k] = -1;
        cross[k] = false;
        if (i < ne) {
            const int32_t d = depth[i];
            if (crosses(A, i, MP_P1)) {
                cross[k] = true;
                dep[k] = d;
                cmin = d < cmin ? d : cmin;
            } else {
                dep[k] = d;
                lmin = d < lmin ? d : lmin;
                lmax = d > lmax ? d : lmax;
                const int j = i - nb;
                s_meta[j] = A.meta[i];
                s_kids[j][0] = ((const uint4*)(A.kids + 8 * (int64_t)i))[0];
                s_kids[j][1] = ((const uint4*)(A.kids + 8 * (int64_t)i))[1];
            }
        }
    }
    if (lmax >= 0) {
        atomicMin(&s_dmin, lmin);
        atomicMax(&s_dmax, lmax);
    }
    if (cmin < (1 << 30)) atomicMin(&s_cmin, cmin);
    __syncthreads();
    const int32_t dmin = s_dmin, dmax = s_dmax, dtop = s_cmin;
#pragma unroll
    for (int k = 0; k < MP_OWN; ++k)
        if (cross[k]) {
            out.nodes[blockIdx.x * (int64_t)MP_SLOTS + dep[k] - dtop] = nb + (int32_t)threadIdx.x + k * MP_TPB;
            atomicAdd(&s_out, 1);
        }
    for (int32_t d = dmax; d >= dmin; --d) {
#pragma unroll
        for (int k = 0; k < MP_OWN; ++k) {
            if (cross[k] || dep[k] != d) continue;
            const int j = (int)threadIdx.x + k * MP_TPB;
            const uint32_t mt = s_meta[j];
            const uint4 ka = s_kids[j][0], kb = s_kids[j][1];
            const uint32_t kr[8] = {ka.x, ka.y, ka.z, ka.w, kb.x, kb.y, kb.z, kb.w};
            NodeFold f{};
            if (mt == META_BUCKET) {
                for (uint32_t c = 0; c < kr[1]; ++c) {
                    const int64_t q = (int64_t)(kr[0] + c) - s0;
                    fold_child(f, c == 0, particle_terms(s_p[0][q], s_p[1][q], s_p[2][q], s_p[3][q], s_p[4][q]));
                    if constexpr (DRIFT) {
                        const double x[3] = {s_p[1][q], s_p[2][q], s_p[3][q]};
                        grow_child(f, c == 0, x, x);
                    }
                }
            } else {
                // all children's data read before the fold (a particle: m, x, y, z, h;
                // a node: its sums), the products formed in the fold
                // (the read addresses are selected, not the data, and slots past the
                // last child read the partition's first particle, so that no read waits
                // for another)
                double raw[8][6];
#pragma unroll
                for (int c = 0; c < 8; ++c) {
                    const uint32_t r = (uint32_t)c < mt ? kr[c] : (uint32_t)s0 | ITEM_PARTICLE;
                    const bool pt = (r & ITEM_PARTICLE) != 0;
                    const int q = pt ? (int)((int64_t)(r & ~ITEM_PARTICLE) - s0) : 0;
                    const int j = pt ? 0 : (int)r - nb;
#pragma unroll
                    for (int e = 0; e < 6; ++e) raw[c][e] = *(pt ? &s_p[e < 5 ? e : 4][q] : &s_n.v[e][j]);
                }
#pragma unroll
                for (int c = 0; c < 8; ++c)
                    if ((uint32_t)c < mt) fold_child(f, c == 0, child_terms(kr[c], raw[c]));
                if constexpr (DRIFT) {
                    for (uint32_t c = 0; c < mt; ++c) {
                        const uint32_t r = kr[c];
                        double lo[3], hi[3];
                        if (r & ITEM_PARTICLE) {
                            const int64_t q = (int64_t)(r & ~ITEM_PARTICLE) - s0;
                            lo[0] = hi[0] = s_p[1][q];
                            lo[1] = hi[1] = s_p[2][q];
                            lo[2] = hi[2] = s_p[3][q];
                        } else {
                            s_n.box((int)r - nb, lo, hi);
                        }
                        grow_child(f, c == 0, lo, hi);
                    }
                }
            }
            s_n.put(j, f);
        }
        __syncthreads();
    }
#pragma unroll
    for (int k = 0; k < MP_OWN; ++k)
        if (!cross[k] && dep[k] >= 0) {
            const int j = (int)threadIdx.x + k * MP_TPB;
            node_store<DRIFT>(A, nb + j, s_n.fold(j));
        }
    if (threadIdx.x == 0) out.count[blockIdx.x] = s_out;
}

template <bool DRIFT>
__global__ __launch_bounds__(ML_TPB) void k_moments_list(MomArgs A, const int32_t* __restrict__ depth,
                                                        int32_t* __restrict__ slot, int64_t P, int64_t n_sub,
                                                        MomList in, MomList out)
{
    __shared__ NodeSums<DRIFT, ML_CAND> s_n;
    __shared__ int32_t s_nd[ML_CAND], s_dp[ML_CAND];
    __shared__ uint32_t s_meta[ML_CAND];
    __shared__ uint4 s_kids[ML_CAND][2];
    __shared__ int32_t s_off[MP_FAN + 1];
    __shared__ int32_t s_dmin, s_dmax, s_cmin, s_out, s_pool_n;
    // without DRIFT: the children's data staged once for the folds of every depth --
    // per child of a listed node, a pool slot (particle or node folded earlier) or
    // -1 - the listed node's index; nodes whose children do not fit fold from global
    // memory
    __shared__ double s_pool[6][DRIFT ? 1 : ML_POOL];
    __shared__ int16_t s_cref[DRIFT ? 1 : ML_CAND][8];
    __shared__ uint8_t s_staged[DRIFT ? 1 : ML_CAND];
    if (threadIdx.x < 64) {
        // candidate offsets: the sub-partitions' lists concatenated (pre-order), an
        // exclusive scan of their counts over the first wave
        const int q = threadIdx.x;
        const int64_t sub = blockIdx.x * (int64_t)MP_FAN + q;
        const uint32_t c = q < MP_FAN && sub < n_sub ? (uint32_t)in.count[sub] : 0u;
        const uint32_t inc = wave_inclusive_scan(c);
        if (q <= MP_FAN) s_off[q] = (int32_t)(inc - c);
        if (q == 0) {
            s_pool_n = 0;
            s_dmin = s_cmin = 1 << 30;
            s_dmax = -1;
            s_out = 0;
        }
    }
    __syncthreads();
    const int32_t cnt = s_off[MP_FAN];
    int32_t lmin = 1 << 30, lmax = -1, cmin = 1 << 30;
    for (int t = threadIdx.x; t < ML_CAND; t += ML_TPB) {
        const int q = t / MP_SLOTS, j = t % MP_SLOTS;
        if (j >= s_off[q + 1] - s_off[q]) continue;
        const int64_t sub = blockIdx.x * (int64_t)MP_FAN + q;
        const int k = s_off[q] + j;
        const int32_t nd = in.nodes[sub * MP_SLOTS + j];
        const int32_t d = depth[nd];
        s_nd[k] = nd;
        if (crosses(A, nd, P)) {
            s_dp[k] = -1 - d;   // listed for the next pass
            cmin = d < cmin ? d : cmin;
        } else {
            s_dp[k] = d;
            lmin = d < lmin ? d : lmin;
            lmax = d > lmax ? d : lmax;
            slot[nd] = k;
            s_meta[k] = A.meta[nd];
            s_kids[k][0] = ((const uint4*)(A.kids + 8 * (int64_t)nd))[0];
            s_kids[k][1] = ((const uint4*)(A.kids + 8 * (int64_t)nd))[1];
        }
    }
    if (lmax >= 0) {
        atomicMin(&s_dmin, lmin);
        atomicMax(&s_dmax, lmax);
    }
    if (cmin < (1 << 30)) atomicMin(&s_cmin, cmin);
    __syncthreads();
    const int32_t dmin = s_dmin, dmax = s_dmax, dtop = s_cmin;
    // a node child listed in this block (its slot points back at it) is read from
    // LDS, one folded by an earlier pass from global memory
    auto here = [&](uint32_t r, int32_t j) { return j >= 0 && j < cnt && s_nd[j] == (int32_t)r; };
    for (int k = threadIdx.x; k < cnt; k += ML_TPB)
        if (s_dp[k] < 0) {
            out.nodes[blockIdx.x * (int64_t)MP_SLOTS + (-1 - s_dp[k]) - dtop] = s_nd[k];
            atomicAdd(&s_out, 1);
        }
    if constexpr (!DRIFT) {
        for (int k = threadIdx.x; k < cnt; k += ML_TPB) {
            s_staged[k] = 0;
            const uint32_t mt = s_meta[k];
            if (s_dp[k] < 0 || mt == META_BUCKET) continue;
            const uint4 ka = s_kids[k][0], kb = s_kids[k][1];
            const uint32_t kr[8] = {ka.x, ka.y, ka.z, ka.w, kb.x, kb.y, kb.z, kb.w};
            // every child's data and slot loaded at once (addresses selected; slots past
            // the last child load particle 0)
            double raw[8][6];
            int32_t js[8];
#pragma unroll
            for (int c = 0; c < 8; ++c) {
                const uint32_t r = (uint32_t)c < mt ? kr[c] : ITEM_PARTICLE;
                const bool pt = (r & ITEM_PARTICLE) != 0;
                const uint32_t q = pt ? r & ~ITEM_PARTICLE : 0u, nd = pt ? 0u : r;
                const Rec64* pr = A.r64 + q;
                const double* src[6] = {pt ? &pr->m : &A.nrec64[nd].m, pt ? &pr->x : A.nS + 3 * nd,
                                        pt ? &pr->y : A.nS + 3 * nd + 1, pt ? &pr->z : A.nS + 3 * nd + 2,
                                        pt ? A.h64 + q : A.nhmax + nd, pt ? A.h64 + q : A.nhmin + nd};
#pragma unroll
                for (int e = 0; e < 6; ++e) raw[c][e] = *src[e];
                js[c] = slot[nd];
            }
            int need = 0;
#pragma unroll
            for (int c = 0; c < 8; ++c)
                need += (uint32_t)c < mt && ((kr[c] & ITEM_PARTICLE) || !here(kr[c], js[c])) ? 1 : 0;
            const int base = atomicAdd(&s_pool_n, need);
            if (base + need > ML_POOL) continue;
            int used = 0;
#pragma unroll
            for (int c = 0; c < 8; ++c) {
                if ((uint32_t)c >= mt) continue;
                if (!(kr[c] & ITEM_PARTICLE) && here(kr[c], js[c])) {
                    s_cref[k][c] = (int16_t)(-1 - js[c]);
                } else {
#pragma unroll
                    for (int e = 0; e < 6; ++e) s_pool[e][base + used] = raw[c][e];
                    s_cref[k][c] = (int16_t)(base + used);
                    ++used;
                }
            }
            s_staged[k] = 1;
        }
        __syncthreads();
    }
    for (int32_t d = dmax; d >= dmin; --d) {
        for (int k = threadIdx.x; k < cnt; k += ML_TPB) {
            if (s_dp[k] != d) continue;
            const uint32_t mt = s_meta[k];
            const uint4 ka = s_kids[k][0], kb = s_kids[k][1];
            const uint32_t kr[8] = {ka.x, ka.y, ka.z, ka.w, kb.x, kb.y, kb.z, kb.w};
            NodeFold f{};
            bool staged = false;
            if constexpr (!DRIFT) staged = s_staged[k] != 0;
            if (staged) {
                if constexpr (!DRIFT) {
                    double raw[8][6];
#pragma unroll
                    for (int c = 0; c < 8; ++c) {
                        if ((uint32_t)c >= mt) continue;
                        const int ref = s_cref[k][c];
#pragma unroll
                        for (int e = 0; e < 6; ++e) raw[c][e] = *(ref >= 0 ? &s_pool[e][ref] : &s_n.v[e][-1 - ref]);
                    }
#pragma unroll
                    for (int c = 0; c < 8; ++c)
                        if ((uint32_t)c < mt) fold_child(f, c == 0, child_terms(kr[c], raw[c]));
                }
            } else if (mt == META_BUCKET) {
                for (uint32_t c = 0; c < kr[1]; ++c) {
                    const Rec64 p = A.r64[kr[0] + c];
                    fold_child(f, c == 0, particle_terms(p.m, p.x, p.y, p.z, A.h64[kr[0] + c]));
                    if constexpr (DRIFT) {
                        const double x[3] = {p.x, p.y, p.z};
                        grow_child(f, c == 0, x, x);
                    }
                }
            } else {
                // all children's data loaded before the fold (a particle: m, x, y, z, h;
                // a node: its sums), the products formed in the fold
                // (the load addresses are selected, not the data, so that no load
                // waits for another; a particle's slot entry is not used)
                double raw[8][6];
                int32_t js[8];
#pragma unroll
                for (int c = 0; c < 8; ++c) {
                    // slots past the last child load particle 0 (always there)
                    const uint32_t r = (uint32_t)c < mt ? kr[c] : ITEM_PARTICLE;
                    const bool pt = (r & ITEM_PARTICLE) != 0;
                    const uint32_t q = pt ? r & ~ITEM_PARTICLE : 0u, nd = pt ? 0u : r;
                    const Rec64* pr = A.r64 + q;
                    const double* src[6] = {pt ? &pr->m : &A.nrec64[nd].m, pt ? &pr->x : A.nS + 3 * nd,
                                            pt ? &pr->y : A.nS + 3 * nd + 1, pt ? &pr->z : A.nS + 3 * nd + 2,
                                            pt ? A.h64 + q : A.nhmax + nd, pt ? A.h64 + q : A.nhmin + nd};
#pragma unroll
                    for (int e = 0; e < 6; ++e) raw[c][e] = *src[e];
                    js[c] = slot[nd];
                }
#pragma unroll
                for (int c = 0; c < 8; ++c)
                    if ((uint32_t)c < mt && !(kr[c] & ITEM_PARTICLE) && here(kr[c], js[c]))
                        for (int e = 0; e < 6; ++e) raw[c][e] = s_n.v[e][js[c]];
#pragma unroll
                for (int c = 0; c < 8; ++c)
                    if ((uint32_t)c < mt) fold_child(f, c == 0, child_terms(kr[c], raw[c]));
                if constexpr (DRIFT) {
                    for (uint32_t c = 0; c < mt; ++c) {
                        const uint32_t r = kr[c];
                        double lo[3], hi[3];
                        if (r & ITEM_PARTICLE) {
                            const Rec64 p = A.r64[r & ~ITEM_PARTICLE];
                            lo[0] = hi[0] = p.x;
                            lo[1] = hi[1] = p.y;
                            lo[2] = hi[2] = p.z;
                        } else if (here(r, js[c])) {
                            s_n.box(js[c], lo, hi);
                        } else {
                            for (int e = 0; e < 3; ++e) {
                                lo[e] = A.nbox[6 * (int64_t)r + e];
                                hi[e] = A.nbox[6 * (int64_t)r + 3 + e];
                            }
                        }
                        grow_child(f, c == 0, lo, hi);
                    }
                }
            }
            s_n.put(k, f);
        }
        __syncthreads();
    }
    for (int k = threadIdx.x; k < cnt; k += ML_TPB)
        if (s_dp[k] >= 0) node_store<DRIFT>(A, s_nd[k], s_n.fold(k));
    if (threadIdx.x == 0 && out.count) out.count[blockIdx.x] = s_out;
}

MomArgs mom_args(const sr_tree* t, double* nbox)
{
    return MomArgs{t->box, t->n_first, t->n_level, t->n_count, t->n_parent, t->n_corner, t->n_kids, t->n_meta,
                   t->prec64, t->ph64, t->nrec64, t->nS, t->ngeo64, t->nhmax, t->nhmin, t->nrec32, t->nhmax32,
                   t->wrec32, t->wrec64, nbox};
}

// The moment passes of a tree of n particles.  The lists live in two build
// scratch arrays of cap >= n words: partition slots in `ucount`, counts in
// `levelmask`, one region per pass (for n > MP_P1 fewer than n / 15 + 192 and
// n / 500 + 6 words for all passes together); the later passes' LDS slots of
// the listed nodes go to a third (`b_lambda`, one word per node), which the
// topology pass no longer needs.
template <bool DRIFT>
int launch_moments_t(const sr_tree* t, int64_t n, double* nbox, hipStream_t st)
{
    const MomArgs A = mom_args(t, nbox);
    int32_t* lists = (int32_t*)t->ucount;
    int32_t* counts = (int32_t*)t->levelmask;
    int64_t P = MP_P1, parts = cdiv(n, P);
    MomList in{lists, counts};
    hipLaunchKernelGGL(k_moments_leaves<DRIFT>, dim3((unsigned)parts), dim3(MP_TPB), 0, st, A, t->base, t->n_depth,
                       n, in);
    while (P < n) {
        const int64_t Pn = P * MP_FAN, pn = cdiv(n, Pn);
        MomList out{nullptr, nullptr};
        if (Pn < n) out = MomList{in.nodes + parts * MP_SLOTS, in.count + parts};
        hipLaunchKernelGGL(k_moments_list<DRIFT>, dim3((unsigned)pn), dim3(ML_TPB), 0, st, A, t->n_depth,
                           t->b_lambda, Pn, parts, in, out);
        in = out;
        P = Pn;
        parts = pn;
    }
    SR_HIP(hipGetLastError());
    return SR_OK;
}

int launch_moments(const sr_tree* t, int64_t n, double* nbox, bool drift, hipStream_t st)
{
    return drift ? launch_moments_t<true>(t, n, nbox, st) : launch_moments_t<false>(t, n, nbox, st);
}

__global__ void k_fill_i32(int32_t* p, int64_t n, int32_t v)
{
    int64_t i = blockIdx.x * (int64_t)TPB + threadIdx.x;
    if (i < n) p[i] = v;
}

__global__ void k_fill_u32(uint32_t* p, int64_t n, uint32_t v)
{
    int64_t i = blockIdx.x * (int64_t)TPB + threadIdx.x;
    if (i < n) p[i] = v;
}

inline dim3 grid_for(int64_t n) { return dim3((unsigned)cdiv(n > 0 ? n : 1, TPB)); }

}  // namespace

int sr_scan_exclusive(const uint32_t* in, uint32_t* out, int64_t n, uint32_t* tmp, hipStream_t st)
{
    if (n <= (int64_t)8 * SCAN1_TPB) {
        hipLaunchKernelGGL(k_scan_one, dim3(1), dim3(SCAN1_TPB), 0, st, in, out, n);
        SR_HIP(hipGetLastError());
        return SR_OK;
    }
    int64_t nb = cdiv(n > 0 ? n : 1, SCAN_TILE);
    hipLaunchKernelGGL(k_scan_sums, dim3((unsigned)nb), dim3(TPB), 0, st, in, n, tmp);
    hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(TPB), 0, st, tmp, nb);
    hipLaunchKernelGGL(k_scan_tiles, dim3((unsigned)nb), dim3(TPB), 0, st, in, out, n, tmp);
    SR_HIP(hipGetLastError());
    return SR_OK;
}

namespace {

template <int ITEMS>
void sort64_pass(uint64_t* const keys[2], uint32_t* const idx[2], int cur, int64_t n, int pass, uint32_t* hist,
                 int64_t nb, hipStream_t st)
{
    const dim3 gb((unsigned)nb), tb(TPB);
    uint32_t* tot = hist + 256 * nb;
    hipLaunchKernelGGL((k_rs_hist<ITEMS, false>), gb, tb, 0, st, nullptr, keys[cur], n, pass, hist, nb);
    hipLaunchKernelGGL(k_rs_digit_scan, dim3(256), tb, 0, st, hist, nb, tot);
    hipLaunchKernelGGL((k_rs_scatter<ITEMS, false>), gb, tb, 0, st, nullptr, keys[cur], idx[cur], nullptr,
                       keys[cur ^ 1], idx[cur ^ 1], n, pass, hist, nb, tot);
}

int sort_items(int64_t n) { return n <= 384 * 1024 ? 2 : n <= 1536 * 1024 ? 4 : 8; }

}  // namespace

int64_t sr_tree_sort_status_words(int64_t cap)
{
    return 256 * cdiv(cap > 0 ? cap : 1, (int64_t)OS_TILE_MIN);
}

int64_t sr_sort_hist_words(int64_t n)
{
    return 256 * cdiv(n > 0 ? n : 1, (int64_t)TPB * sort_items(n)) + 256 + 1;
}

int sr_sort_keys64(uint64_t* const keys[2], uint32_t* const idx[2], int64_t n, int passes, uint32_t* hist,
                   hipStream_t st)
{
    const int items = sort_items(n);
    const int64_t nb = cdiv(n > 0 ? n : 1, (int64_t)TPB * items);
    for (int pass = 0; pass < passes; ++pass) {
        const int cur = pass & 1;
        if (items == 2)
            sort64_pass<2>(keys, idx, cur, n, pass, hist, nb, st);
        else if (items == 4)
            sort64_pass<4>(keys, idx, cur, n, pass, hist, nb, st);
        else
            sort64_pass<8>(keys, idx, cur, n, pass, hist, nb, st);
    }
    SR_HIP(hipGetLastError());
    return SR_OK;
}

int sr_build_device(sr_tree* t, const double* pos, const double* mass, const double* eps,
                    double eps_scalar, hipStream_t st)
{
    const int64_t n = t->n;
    const double box = t->box;
    t->drift_base = false;   // a drift after this build starts from its records
    hipLaunchKernelGGL(k_fill_i32, grid_for(ST_ALLOC), dim3(TPB), 0, st, t->status, (int64_t)ST_ALLOC, 0);
    hipLaunchKernelGGL(k_keys, grid_for(n), dim3(TPB), 0, st, pos, mass, eps, eps_scalar, n, box,
                       t->khi[0], t->klo[0], t->kidx[0], t->status);
    // 12 passes of 8 bits: lo word bits 0..47, then hi word bits 0..47
    {
        const bool small = n <= OS_SMALL_N;
        const int64_t tiles = cdiv(n, (int64_t)OS_TPB * (small ? 2 : 4));
        if (t->rs_epoch > (1u << 29)) {
            // tags about to run out: clear the words and start again
            SR_HIP(hipMemsetAsync(t->rs_status, 0, sizeof(uint64_t) * sr_tree_sort_status_words(t->cap), st));
            t->rs_epoch = 0;
        }
        uint32_t* hist = (uint32_t*)(t->status + ST_RS_HIST);
        uint32_t* tickets = (uint32_t*)(t->status + ST_RS_TICKET);
        const int64_t hb = cdiv(n, (int64_t)TPB * 16);
        hipLaunchKernelGGL(k_os_hist, dim3((unsigned)(hb < 1024 ? hb : 1024)), dim3(TPB), 0, st, t->khi[0],
                           t->klo[0], n, hist);
        for (int pass = 0; pass < 12; ++pass) {
            const int cur = pass & 1;
            if (small)
                hipLaunchKernelGGL(k_os_pass<2>, dim3((unsigned)tiles), dim3(OS_TPB), 0, st, t->khi[cur],
                                   t->klo[cur], t->kidx[cur], t->khi[cur ^ 1], t->klo[cur ^ 1], t->kidx[cur ^ 1], n,
                                   pass, hist + 256 * pass, tickets + pass, t->rs_status,
                                   t->rs_epoch + 1 + (uint32_t)pass, t->status + ST_FLAGS);
            else
                hipLaunchKernelGGL(k_os_pass<4>, dim3((unsigned)tiles), dim3(OS_TPB), 0, st, t->khi[cur],
                                   t->klo[cur], t->kidx[cur], t->khi[cur ^ 1], t->klo[cur ^ 1], t->kidx[cur ^ 1], n,
                                   pass, hist + 256 * pass, tickets + pass, t->rs_status,
                                   t->rs_epoch + 1 + (uint32_t)pass, t->status + ST_FLAGS);
        }
        t->rs_epoch += 12;
    }
    // 12 passes leave the sorted keys in buffer 0
    hipLaunchKernelGGL(k_gather, grid_for(n), dim3(TPB), 0, st, pos, mass, eps, eps_scalar, n, box,
                       t->kidx[0], t->perm, t->invperm, t->prec64, t->ph64, t->prec32, t->ph32);
    if (n > 1) {
        hipLaunchKernelGGL(k_radix_tree, grid_for(n - 1), dim3(TPB), 0, st, t->khi[0], t->klo[0], n, t->b_lo,
                           t->b_hi, t->b_lambda, t->b_parent, t->leaf_bparent);
        hipLaunchKernelGGL(k_fill_u32, grid_for(n), dim3(TPB), 0, st, t->levelmask, n, 0u);
        hipLaunchKernelGGL(k_octree_flags, grid_for(n - 1), dim3(TPB), 0, st, n, t->b_lo, t->b_lambda,
                           t->b_parent, t->levelmask, t->b_pre);
        hipLaunchKernelGGL(k_popcount, grid_for(n), dim3(TPB), 0, st, t->levelmask, n, t->ucount);
        int rc = sr_scan_exclusive(t->ucount, (uint32_t*)t->base, n, t->scan_tmp, st);
        if (rc) return rc;
        hipLaunchKernelGGL(k_preorder, grid_for(n - 1), dim3(TPB), 0, st, n, t->b_lo, t->b_lambda, t->levelmask,
                           t->base, t->b_pre);
        hipLaunchKernelGGL(k_node_arrays, grid_for(n - 1), dim3(TPB), 0, st, n, t->b_lo, t->b_hi, t->b_lambda,
                           t->b_parent, t->b_pre, t->base, t->prec32, t->n_level, t->n_first, t->n_count,
                           t->n_parent, t->n_skip, t->n_corner);
        // the node count is base[n]; it is read back with the status words, and the
        // depth pass (sized for the N - 1 bound) reads it on the device
        SR_HIP(hipMemcpyAsync(t->status + ST_NODES, t->base + n, sizeof(int32_t), hipMemcpyDeviceToDevice, st));
        hipLaunchKernelGGL(k_node_depth, grid_for(n - 1), dim3(TPB), 0, st, t->status + ST_NODES, t->n_parent,
                           t->n_first, t->n_count, t->base, t->n_depth, t->items, t->status);
    }
    hipLaunchKernelGGL(k_particle_items, grid_for(n), dim3(TPB), 0, st, n, t->leaf_bparent, t->b_parent,
                       t->b_pre, t->base, t->n_depth, t->pparent, t->items);
    if (n > 1) {
        // child tables (for the N - 1 node bound, the node count read on the
        // device), then every node's moments, deepest first, in two launches
        hipLaunchKernelGGL(k_child_table, grid_for(n - 1), dim3(TPB), 0, st, t->status + ST_NODES, t->items,
                           t->n_first, t->n_level, t->n_count, t->n_kids, t->n_meta);
        int rc = launch_moments(t, n, nullptr, false, st);
        if (rc) return rc;
    }
    // the build's one synchronisation, at its end: input flags, node count and the
    // deepest depth go to pinned host memory
    SR_HIP(hipMemcpyAsync(t->h_status, t->status, ST_WORDS * sizeof(int32_t), hipMemcpyDeviceToHost, st));
    SR_HIP(hipEventRecord(t->ev_status, st));
    SR_HIP(hipGetLastError());
    SR_HIP(hipEventSynchronize(t->ev_status));
    const int32_t* hstat = t->h_status;
    if (hstat[ST_FLAGS] & 1) return sr_fail(SR_EINVAL, "tree_build: non-finite position or non-positive / non-finite mass or softening");
    if (hstat[ST_FLAGS] & 4) return sr_fail(SR_EHIP, "tree_build: the key sort's look-back made no progress");
    // softenings that are not all equal select the walk's mixed-softening opening rule
    t->mixed_soft = (hstat[ST_FLAGS] & 2) != 0;
    const int64_t m = n > 1 ? hstat[ST_NODES] : 0;
    t->n_nodes = m;
    if (m == 0) {
        t->max_depth = 0;
        t->mixed_soft = false;
        return SR_OK;
    }
    t->max_depth = hstat[ST_MAXDEPTH];
    if (t->max_depth >= SR_MAX_DEPTH) return sr_fail(SR_EUNSUPPORTED, "tree_build: tree deeper than %d", SR_MAX_DEPTH);
    return SR_OK;
}

namespace {

// A drifted particle: its built (wrapped) position plus the displacement, not
// wrapped again; its integer coordinates are those of the moved position.
__global__ void k_drift_particles(int64_t n, double box, const int32_t* __restrict__ perm,
                                  const Rec64* __restrict__ r0, const double* __restrict__ disp,
                                  Rec64* __restrict__ r64, Rec32* __restrict__ r32, int32_t* __restrict__ status)
{
    int64_t s = blockIdx.x * (int64_t)TPB + threadIdx.x;
    if (s >= n) return;
    const int64_t i = perm[s];
    const Rec64 b = r0[s];
    const double x[3] = {b.x + disp[3 * i + 0], b.y + disp[3 * i + 1], b.z + disp[3 * i + 2]};
    uint32_t X[3];
    bool bad = false;
    for (int k = 0; k < 3; ++k) {
        if (!isfinite(x[k])) bad = true;
        X[k] = isfinite(x[k]) ? (uint32_t)floor(wrap_unit(x[k], box) * TWO32) : 0u;
    }
    if (bad) atomicOr(&status[ST_FLAGS], 1);
    r64[s] = Rec64{x[0], x[1], x[2], b.m};
    r32[s] = Rec32{X[0], X[1], X[2], r32[s].m};
}

}  // namespace

int sr_drift_device(sr_tree* t, const double* disp, hipStream_t st)
{
    const int64_t n = t->n, m = t->n_nodes;
    if (!t->drift_base) {
        // the first drift after a build keeps the built particle records
        SR_HIP(hipMemcpyAsync(t->prec64_0, t->prec64, (size_t)n * sizeof(Rec64), hipMemcpyDeviceToDevice, st));
        t->drift_base = true;
    }
    hipLaunchKernelGGL(k_fill_i32, grid_for(1), dim3(TPB), 0, st, t->status, (int64_t)1, 0);
    hipLaunchKernelGGL(k_drift_particles, grid_for(n), dim3(TPB), 0, st, n, t->box, t->perm, t->prec64_0, disp,
                       t->prec64, t->prec32, t->status);
    SR_HIP(hipMemcpyAsync(t->h_status, t->status, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    SR_HIP(hipEventRecord(t->ev_status, st));
    if (m > 0) {
        int rc = launch_moments(t, n, t->nbox, true, st);
        if (rc) return rc;
    }
    SR_HIP(hipGetLastError());
    SR_HIP(hipEventSynchronize(t->ev_status));
    if (t->h_status[ST_FLAGS] & 1) return sr_fail(SR_EINVAL, "tree_drift: non-finite displacement");
    return SR_OK;
}
