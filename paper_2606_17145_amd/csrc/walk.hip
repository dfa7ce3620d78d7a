// Group-wise Barnes-Hut walk (forward and adjoint) for the short-range force.
//
// One wavefront walks the tree for up to 64 targets that are consecutive in
// Morton order.  Each lane takes exactly the decisions a depth-first walk of
// its own target would take (prune, open, accept); the wave only shares the
// traversal: it scans the combined pre-order item sequence, entering a node's
// children when at least one lane opened it (a ballot), and skipping the whole
// subtree otherwise.  The open masks of the current path sit in LDS, indexed
// by depth.  Accepted nodes and reached particles are appended, with the mask
// of lanes they apply to, to an interaction list in LDS; when the list holds a
// wavefront's worth of entries their records are staged in LDS with one
// coalesced load and every lane sweeps the list, evaluating the pair force for
// the entries whose mask holds it.  This is the chunked neighbour processing
// of the paper's GPU port (chunks of neighbours evaluated before the walk
// continues, its GPU-porting subsection) mapped onto a 64-wide wavefront.
#include <stdio.h>

#include <type_traits>

#include "gpoly.h"
#include "internal.h"

namespace {

constexpr int WAVE = 64;
constexpr int CHUNK = 64;               // list entries per flush (one per lane when staging)
constexpr double TWO32 = 4294967296.0;
constexpr double TWO_OVER_SQRTPI = 1.12837916709551257390;
constexpr float LOG2E_F = 1.44269504088896340736f;
constexpr float TWO_OVER_SQRTPI_F = 1.12837916709551257390f;
constexpr float TWO64_F = 18446744073709551616.0f;

enum { PR64 = 0, PR32 = 1, PR32A = 2 };
enum { D_PRUNE = 0, D_ACCEPT = 1, D_ACCEPT_FAR = 2, D_OPEN = 3 };

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
    float rc2t, theta2f, inv2rs_t;
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

__device__ inline uint64_t uniform64(uint64_t v)
{
    uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
    return ((uint64_t)hi << 32) | lo;
}

__device__ inline uint32_t uniform32(uint32_t v) { return __builtin_amdgcn_readfirstlane(v); }

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

// Softened branch in FP32: h^3 S as a function of q, written around q = 1 in the
// outer part so that nothing cancels; also q dS/dq-type term for the adjoint.
__device__ inline float spline_h3S_32(float q)
{
    if (q < 0.5f) return __builtin_fmaf(q * q, __builtin_fmaf(32.0f, q, -38.4f), 10.6666666667f);
    float t = 1.0f - q;
    float poly = __builtin_fmaf(t, __builtin_fmaf(t, __builtin_fmaf(t, 10.6666666667f, 6.4f), 3.2f), 1.06666666667f);
    return poly - 1.0f / (15.0f * q * q * q);
}

// h^4 dS/dr as a function of q.
__device__ inline float spline_h4dS_32(float q)
{
    if (q < 0.5f) return q * __builtin_fmaf(96.0f, q, -76.8f);
    float t = 1.0f - q;
    float q2 = q * q;
    return __builtin_fmaf(t, __builtin_fmaf(t, -32.0f, -12.8f), -3.2f) + 1.0f / (5.0f * q2 * q2);
}

// ---- wave reduction --------------------------------------------------------------

template <class T>
__device__ inline T wave_sum(T v)
{
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// ----------------------------------------------------------------------------------
// the walk
// ----------------------------------------------------------------------------------

template <int PREC>
struct Stage;

template <>
struct Stage<PR64> {
    double x[CHUNK], y[CHUNK], z[CHUNK], m[CHUNK], h[CHUNK];
};

template <>
struct Stage<PR32> {
    uint32_t X[CHUNK], Y[CHUNK], Z[CHUNK];
    float m[CHUNK], h[CHUNK];
};

template <>
struct Stage<PR32A> : Stage<PR32> {};

template <int PREC>
struct WalkShared {
    uint64_t open[SR_MAX_DEPTH];
    uint64_t mask[CHUNK];
    uint32_t src[CHUNK];
    Stage<PREC> rec;
};

template <int PREC, bool ADJ>
__global__ __launch_bounds__(WAVE) void k_walk(WalkArgs a)
{
    using acc_t = typename std::conditional<PREC == PR32, float, double>::type;
    __shared__ WalkShared<PREC> sh;
    const int lane = threadIdx.x;
    const int64_t t = (int64_t)blockIdx.x * WAVE + lane;
    const bool valid = t < a.n_t;

    // target state
    int32_t s_i = valid ? a.tgt_sorted[t] : 0;
    int32_t slot = valid ? a.tgt_slot[t] : 0;
    double x64 = 0, y64 = 0, z64 = 0, h64 = 0, aold = 0;
    uint32_t X = 0, Y = 0, Z = 0;
    float h32 = 0;
    double atau = 0;
    if (valid) {
        if constexpr (PREC == PR64) {
            Rec64 r = a.prec64[s_i];
            x64 = r.x;
            y64 = r.y;
            z64 = r.z;
            h64 = a.ph64[s_i];
        } else {
            Rec32 r = a.prec32[s_i];
            X = r.X;
            Y = r.Y;
            Z = r.Z;
            h32 = a.ph32[s_i];
        }
        if (a.relative) {
            aold = a.a_old[a.perm[s_i]];
            atau = (a.alpha * aold) * a.tau2;
        }
    }
    acc_t ax = 0, ay = 0, az = 0;
    int npp = 0, npn = 0;
    // adjoint cotangent and target-side adjoint
    acc_t wx = 0, wy = 0, wz = 0, tbx = 0, tby = 0, tbz = 0;
    if (ADJ && valid) {
        const acc_t* w = (const acc_t*)a.w;
        wx = w[3 * slot];
        wy = w[3 * slot + 1];
        wz = w[3 * slot + 2];
    }
    const uint64_t active = __ballot(valid);
    const bool mixed = a.n_nodes > 0 && a.nhmax[0] != a.nhmin[0];

    auto flush = [&](int nl) {
        __syncthreads();
        if (lane < nl) {
            uint32_t src = sh.src[lane];
            if constexpr (PREC == PR64) {
                Rec64 r;
                double h;
                if (src & ITEM_PARTICLE) {
                    r = a.prec64[src & ~ITEM_PARTICLE];
                    h = a.ph64[src & ~ITEM_PARTICLE];
                } else {
                    r = a.nrec64[src];
                    h = a.nhmax[src];
                }
                sh.rec.x[lane] = r.x;
                sh.rec.y[lane] = r.y;
                sh.rec.z[lane] = r.z;
                sh.rec.m[lane] = r.m;
                sh.rec.h[lane] = h;
            } else {
                Rec32 r;
                float h;
                if (src & ITEM_PARTICLE) {
                    r = a.prec32[src & ~ITEM_PARTICLE];
                    h = a.ph32[src & ~ITEM_PARTICLE];
                } else {
                    r = a.nrec32[src];
                    h = a.nhmax32[src];
                }
                sh.rec.X[lane] = r.X;
                sh.rec.Y[lane] = r.Y;
                sh.rec.Z[lane] = r.Z;
                sh.rec.m[lane] = r.m * TWO64_F;
                sh.rec.h[lane] = h;
            }
        }
        __syncthreads();
        for (int e = 0; e < nl; ++e) {
            const uint64_t m = uniform64(sh.mask[e]);
            const uint32_t src = uniform32(sh.src[e]);
            const bool isp = (src & ITEM_PARTICLE) != 0;
            const bool on = (m >> lane) & 1ull;
            // source-side adjoint terms of this entry (0 on lanes that do not use it)
            acc_t vx = 0, vy = 0, vz = 0, vm = 0;
            if (on) {
                if constexpr (PREC == PR64) {
                    double dx = min_image(sh.rec.x[e] - x64, a.box);
                    double dy = min_image(sh.rec.y[e] - y64, a.box);
                    double dz = min_image(sh.rec.z[e] - z64, a.box);
                    double r2 = (dx * dx + dy * dy) + dz * dz;
                    if (r2 < a.rc2) {
                        if (isp) ++npp;
                        else ++npn;
                        double r = sqrt(r2);
                        double u = r * a.inv2rs;
                        double ex = exp(-u * u);
                        double g = erfc(u) + TWO_OVER_SQRTPI * u * ex;
                        double hp = h64 > sh.rec.h[e] ? h64 : sh.rec.h[e];
                        double S, dS;
                        spline64(r, hp, S, dS);
                        double K = a.G * S * g;
                        double Mg = sh.rec.m[e];
                        if constexpr (!ADJ) {
                            double f = Mg * K;
                            ax += f * dx;
                            ay += f * dy;
                            az += f * dz;
                        } else {
                            double dg = -2.0 * TWO_OVER_SQRTPI * u * u * ex;
                            double dK = a.G * (dS * g + S * dg * a.inv2rs);
                            double c2 = r > 0.0 ? dK / r : 0.0;
                            double wd = (wx * dx + wy * dy) + wz * dz;
                            vx = Mg * (K * wx + c2 * wd * dx);
                            vy = Mg * (K * wy + c2 * wd * dy);
                            vz = Mg * (K * wz + c2 * wd * dz);
                            vm = K * wd;
                            tbx -= vx;
                            tby -= vy;
                            tbz -= vz;
                        }
                    }
                } else {
                    float dx = (float)(int32_t)(sh.rec.X[e] - X);
                    float dy = (float)(int32_t)(sh.rec.Y[e] - Y);
                    float dz = (float)(int32_t)(sh.rec.Z[e] - Z);
                    float r2 = r2_ticks(dx, dy, dz);
                    if (r2 < a.rc2t) {
                        if (isp) ++npp;
                        else ++npn;
                        float rinv = __builtin_amdgcn_rsqf(r2);
                        float r = r2 > 0.0f ? r2 * rinv : 0.0f;
                        float u = r * a.inv2rs_t;
                        float ex;
                        float g = gshort32(u, ex);
                        float hp = fmaxf(h32, sh.rec.h[e]);
                        float S, Srd;   // S and r dS/dr
                        if (r2 < hp * hp) {
                            float ih = __builtin_amdgcn_rcpf(hp);
                            float q = r * ih;
                            float ih3 = ih * ih * ih;
                            S = spline_h3S_32(q) * ih3;
                            Srd = ADJ ? spline_h4dS_32(q) * q * ih3 : 0.0f;
                        } else {
                            S = rinv * rinv * rinv;
                            Srd = -3.0f * S;
                        }
                        float Mg = sh.rec.m[e];
                        float K = S * g;
                        if constexpr (!ADJ) {
                            float f = Mg * K;
                            ax += (acc_t)(f * dx);
                            ay += (acc_t)(f * dy);
                            az += (acc_t)(f * dz);
                        } else {
                            // K' r = r dS/dr g + S g'(u) u
                            float dg = -2.0f * TWO_OVER_SQRTPI_F * u * u * ex;
                            float Kr = Srd * g + S * dg * u;
                            float nrm = r2 > 0.0f ? rinv : 0.0f;
                            float nx = dx * nrm, ny = dy * nrm, nz = dz * nrm;
                            float fw = (float)wx, fy = (float)wy, fz = (float)wz;
                            float wn = __builtin_fmaf(fw, nx, __builtin_fmaf(fy, ny, fz * nz));
                            float wd = __builtin_fmaf(fw, dx, __builtin_fmaf(fy, dy, fz * dz));
                            float c = Kr * wn;
                            float px = Mg * __builtin_fmaf(K, fw, c * nx);
                            float py = Mg * __builtin_fmaf(K, fy, c * ny);
                            float pz = Mg * __builtin_fmaf(K, fz, c * nz);
                            vx = px;
                            vy = py;
                            vz = pz;
                            vm = K * wd;
                            tbx -= (acc_t)px;
                            tby -= (acc_t)py;
                            tbz -= (acc_t)pz;
                        }
                    }
                }
            }
            if constexpr (ADJ) {
                // one atomic per (wave, source) after a wave reduction
                double sx, sy, sz, smass;
                if constexpr (PREC == PR64) {
                    sx = wave_sum<double>(vx);
                    sy = wave_sum<double>(vy);
                    sz = wave_sum<double>(vz);
                    smass = wave_sum<double>(vm);
                } else {
                    sx = wave_sum<float>((float)vx);
                    sy = wave_sum<float>((float)vy);
                    sz = wave_sum<float>((float)vz);
                    smass = wave_sum<float>((float)vm);
                }
                if (lane == 0) {
                    double* dst = isp ? a.pbar + 4 * (int64_t)(src & ~ITEM_PARTICLE) : a.nbar + 4 * (int64_t)src;
                    unsafeAtomicAdd(dst + 0, sx);
                    unsafeAtomicAdd(dst + 1, sy);
                    unsafeAtomicAdd(dst + 2, sz);
                    unsafeAtomicAdd(dst + 3, smass);
                }
            }
        }
        __syncthreads();
    };

    if (a.n_nodes > 0) {
        int nl = 0;
        uint32_t k = 0;
        while (k < a.n_items) {
            const Item it = a.items[k];
            const uint32_t ref = uniform32(it.ref), depth = uniform32(it.depth), next = uniform32(it.next);
            const uint64_t reach = depth ? uniform64(sh.open[depth - 1]) : active;
            if (ref & ITEM_PARTICLE) {
                const uint64_t self = __ballot(valid && (uint32_t)s_i == (ref & ~ITEM_PARTICLE));
                const uint64_t m = reach & ~self;
                if (m) {
                    if (lane == 0) {
                        sh.src[nl] = ref;
                        sh.mask[nl] = m;
                    }
                    ++nl;
                }
                ++k;
            } else {
                const uint32_t nd = ref;
                int dec = D_PRUNE;
                if ((reach >> lane) & 1ull) {
                    if constexpr (PREC == PR64) {
                        const Geo64 g = a.ngeo64[nd];
                        const Rec64 c = a.nrec64[nd];
                        const double l = g.l;
                        double dcx = min_image(g.cx - x64, a.box);
                        double dcy = min_image(g.cy - y64, a.box);
                        double dcz = min_image(g.cz - z64, a.box);
                        double t2 = 0.0, tt;
                        tt = fabs(dcx) - 0.5 * l;
                        if (tt > 0) t2 += tt * tt;
                        tt = fabs(dcy) - 0.5 * l;
                        if (tt > 0) t2 += tt * tt;
                        tt = fabs(dcz) - 0.5 * l;
                        if (tt > 0) t2 += tt * tt;
                        if (!(t2 > a.rc2 * (1.0 + 1e-6))) {
                            bool inside = fabs(dcx) < 0.6 * l && fabs(dcy) < 0.6 * l && fabs(dcz) < 0.6 * l;
                            double dx = min_image(c.x - x64, a.box);
                            double dy = min_image(c.y - y64, a.box);
                            double dz = min_image(c.z - z64, a.box);
                            double r2 = (dx * dx + dy * dy) + dz * dz;
                            bool open = inside || l * l > a.theta2 * r2;
                            if (a.relative && (a.G * c.m) * (l * l) > (a.alpha * aold) * (r2 * r2)) open = true;
                            if (mixed) {
                                double hx = a.nhmax[nd];
                                if (a.nhmin[nd] != hx && r2 < hx * hx) open = true;
                            }
                            dec = open ? D_OPEN : (r2 < a.rc2 ? D_ACCEPT : D_ACCEPT_FAR);
                        }
                    } else {
                        const Rec32 c = a.nrec32[nd];
                        const int lev = a.n_level[nd];
                        const uint32_t half = 1u << (31 - lev);
                        const float lt = (float)(1ull << (32 - lev));
                        const uint64_t lint = 1ull << (32 - lev);
                        int32_t dcx = (int32_t)(a.n_corner[3 * nd + 0] + half - X);
                        int32_t dcy = (int32_t)(a.n_corner[3 * nd + 1] + half - Y);
                        int32_t dcz = (int32_t)(a.n_corner[3 * nd + 2] + half - Z);
                        uint64_t ax_ = (uint64_t)(dcx < 0 ? -(int64_t)dcx : (int64_t)dcx);
                        uint64_t ay_ = (uint64_t)(dcy < 0 ? -(int64_t)dcy : (int64_t)dcy);
                        uint64_t az_ = (uint64_t)(dcz < 0 ? -(int64_t)dcz : (int64_t)dcz);
                        float tx = fmaxf((float)ax_ - 0.5f * lt, 0.0f);
                        float ty = fmaxf((float)ay_ - 0.5f * lt, 0.0f);
                        float tz = fmaxf((float)az_ - 0.5f * lt, 0.0f);
                        float t2 = tx * tx + ty * ty + tz * tz;
                        if (!(t2 > a.rc2t * 1.0001f)) {
                            bool inside = 5 * ax_ < 3 * lint && 5 * ay_ < 3 * lint && 5 * az_ < 3 * lint;
                            float dx = (float)(int32_t)(c.X - X);
                            float dy = (float)(int32_t)(c.Y - Y);
                            float dz = (float)(int32_t)(c.Z - Z);
                            float r2 = r2_ticks(dx, dy, dz);
                            bool open = inside || lt * lt > a.theta2f * r2;
                            if (a.relative) {
                                double r2d = (double)r2;
                                if ((a.G * (double)c.m) * ((double)lt * (double)lt) > atau * (r2d * r2d)) open = true;
                            }
                            if (mixed) {
                                float hx = a.nhmax32[nd];
                                if (a.nhmin[nd] != a.nhmax[nd] && r2 < hx * hx) open = true;
                            }
                            dec = open ? D_OPEN : (r2 < a.rc2t ? D_ACCEPT : D_ACCEPT_FAR);
                        }
                    }
                }
                const uint64_t om = __ballot(dec == D_OPEN);
                const uint64_t am = __ballot(dec == D_ACCEPT);
                if (am) {
                    if (lane == 0) {
                        sh.src[nl] = nd;
                        sh.mask[nl] = am;
                    }
                    ++nl;
                }
                if (om) {
                    if (lane == 0) sh.open[depth] = om;
                    ++k;
                } else {
                    k = next;
                }
            }
            if (nl == CHUNK) {
                flush(nl);
                nl = 0;
            }
        }
        if (nl) flush(nl);
    }

    if (!valid) return;
    if constexpr (!ADJ) {
        if constexpr (PREC == PR64) {
            double* o = (double*)a.acc;
            o[3 * (int64_t)slot + 0] = ax;
            o[3 * (int64_t)slot + 1] = ay;
            o[3 * (int64_t)slot + 2] = az;
        } else if constexpr (PREC == PR32) {
            float* o = (float*)a.acc;
            const float sc = (float)a.out_scale;
            o[3 * (int64_t)slot + 0] = (float)ax * sc;
            o[3 * (int64_t)slot + 1] = (float)ay * sc;
            o[3 * (int64_t)slot + 2] = (float)az * sc;
        } else {
            double* o = (double*)a.acc;
            o[3 * (int64_t)slot + 0] = (double)ax * a.out_scale;
            o[3 * (int64_t)slot + 1] = (double)ay * a.out_scale;
            o[3 * (int64_t)slot + 2] = (double)az * a.out_scale;
        }
        if (a.counts) {
            a.counts[2 * (int64_t)slot] = npp;
            a.counts[2 * (int64_t)slot + 1] = npn;
        }
    } else {
        a.tbar[3 * (int64_t)s_i + 0] = (double)tbx;
        a.tbar[3 * (int64_t)s_i + 1] = (double)tby;
        a.tbar[3 * (int64_t)s_i + 2] = (double)tbz;
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

__global__ void k_zero_f64(double* p, int64_t n)
{
    int64_t i = blockIdx.x * (int64_t)256 + threadIdx.x;
    if (i < n) p[i] = 0.0;
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
    a.theta2f = (float)(p->theta * p->theta);
    a.inv2rs_t = (float)(tick / (2.0 * p->r_s));
    a.tau2 = tick * tick;
    a.out_scale = p->G / (t->box * t->box);
    return a;
}

template <bool ADJ>
int launch_walk(const sr_tree* t, const sr_params* p, const WalkArgs& a, hipStream_t st)
{
    dim3 grid((unsigned)((a.n_t + WAVE - 1) / WAVE));
    if (a.n_t == 0) return SR_OK;
    switch (p->precision) {
    case SR_FP64: hipLaunchKernelGGL((k_walk<PR64, ADJ>), grid, dim3(WAVE), 0, st, a); break;
    case SR_FP32: hipLaunchKernelGGL((k_walk<PR32, ADJ>), grid, dim3(WAVE), 0, st, a); break;
    default: hipLaunchKernelGGL((k_walk<PR32A, ADJ>), grid, dim3(WAVE), 0, st, a); break;
    }
    SR_HIP(hipGetLastError());
    (void)t;
    return SR_OK;
}

}  // namespace

int sr_prepare_targets(sr_tree* t, const int32_t* active, int64_t n_active, hipStream_t st)
{
    const int64_t n = t->n;
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

int sr_walk_forward(sr_tree* t, const sr_params* p, int64_t n_t, const double* a_old, void* acc,
                    int32_t* counts, hipStream_t st)
{
    WalkArgs a = make_args(t, p, n_t, a_old);
    a.acc = acc;
    a.counts = counts;
    return launch_walk<false>(t, p, a, st);
}

int sr_walk_adjoint(sr_tree* t, const sr_params* p, int64_t n_t, const double* a_old, const void* w,
                    double* dLdx, double* dLdm, hipStream_t st)
{
    const int64_t n = t->n, m = t->n_nodes;
    hipLaunchKernelGGL(k_zero_f64, g256(4 * n), dim3(256), 0, st, t->pbar, 4 * n);
    hipLaunchKernelGGL(k_zero_f64, g256(3 * n), dim3(256), 0, st, t->tbar, 3 * n);
    if (m) hipLaunchKernelGGL(k_zero_f64, g256(4 * m), dim3(256), 0, st, t->nbar, 4 * m);
    WalkArgs a = make_args(t, p, n_t, a_old);
    a.w = w;
    a.pbar = t->pbar;
    a.tbar = t->tbar;
    a.nbar = t->nbar;
    int rc = launch_walk<true>(t, p, a, st);
    if (rc) return rc;
    double sx = 1.0, sm = 1.0;
    if (p->precision != SR_FP64) {
        // FP32 terms carry masses scaled by 2^64 and integer-coordinate lengths
        const double L = t->box;
        sx = p->G * TWO32 / (L * L * L);
        sm = p->G * TWO32 * TWO32 / (L * L);
    }
    hipLaunchKernelGGL(k_pushdown, g256(n), dim3(256), 0, st, n, t->perm, t->pparent, t->n_parent, t->prec64,
                       t->nrec64, t->pbar, t->tbar, t->nbar, sx, sm, dLdx, dLdm);
    SR_HIP(hipGetLastError());
    return SR_OK;
}
