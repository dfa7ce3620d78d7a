// SPH density with an iterated smoothing length, on the tree of tree_build.
//
// The paper's density module iterates each particle's smoothing length until
// its kernel sphere holds a fixed number of neighbours (Sec. 2).  With Gadget-2's
// cubic spline of support h, W(r, h) = 8 / (pi h^3) w(r / h), the density
// rho_i(h) = sum_j m_j W(r_ij, h) (self included, minimum image) and the
// mass-weighted neighbour number N_i(h) = (4 pi / 3) h^3 rho_i(h) / m_i =
// (32/3) sum_j (m_j / m_i) w(r_ij / h), h_i is the root of N_i(h) = T.  N_i is
// strictly increasing in h once a neighbour lies inside, so the root is unique.
//
// One thread per particle in Morton order; the 64 lanes of a wave share one
// walk of the pre-order node sequence without a stack: a node whose cube meets
// any lane's ball |x - x_i| < h (minimum image) is entered (each lane sums the
// direct particle children within its own h, and the walk continues at the
// next node in pre-order, its first child node or, if it has none, the node
// after its subtree); any other node is skipped with n_skip.  The sums give
// N(h) and dN/dh, and a safeguarded Newton step in h^3 updates h inside the
// bracket the iterations have found.
#include <math.h>

#include "internal.h"

namespace {

constexpr int SPH_TPB = 256;
constexpr int SPH_MAX_ITER = 100;
constexpr double SPH_OVERFULL = 4.0;        // a partial neighbour number above 4 T ends a lane's walk
constexpr double SPH_INIT_FRACTION = 0.25;   // the initial density from the smallest ancestor with T/4 particles
constexpr double SPH_GROW = 2.0;             // largest growth of h per step before an upper bound is known

enum : int32_t { SPH_ACTIVE = 0, SPH_DONE = 1, SPH_FAILED = 2 };

inline dim3 sph_grid(int64_t n) { return dim3((unsigned)((n + SPH_TPB - 1) / SPH_TPB)); }

// w(q) and q w'(q) of the cubic spline (zero beyond q = 1).
__device__ inline void spline_w(double q, double& wq, double& qdw)
{
    if (q <= 0.5) {
        wq = 1.0 - 6.0 * q * q + 6.0 * q * q * q;
        qdw = q * (-12.0 * q + 18.0 * q * q);
    } else if (q <= 1.0) {
        const double u = 1.0 - q;
        wq = 2.0 * u * u * u;
        qdw = -6.0 * q * u * u;
    } else {
        wq = 0.0;
        qdw = 0.0;
    }
}

// Minimum image of a separation; inv_box = 1 / L (a product instead of an FP64
// division; the image can differ from d / L rounding only at an exact half-box
// tie, where both images are equally far).
__device__ inline double min_image(double d, double box, double inv_box) { return d - box * rint(d * inv_box); }

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

__global__ void k_sph_iterate(int64_t n, int64_t m, const WalkRec64* __restrict__ wrec,
                              const int32_t* __restrict__ n_skip, const Rec64* __restrict__ prec, double box,
                              double target, double h_max, double* __restrict__ h, double* __restrict__ lo,
                              double* __restrict__ hi, int32_t* __restrict__ state, double* __restrict__ rho,
                              int32_t* __restrict__ active)
{
    const int64_t s = blockIdx.x * (int64_t)SPH_TPB + threadIdx.x;
    const bool act = s < n && state[s] == SPH_ACTIVE;
    if (__ballot(act) == 0) return;         // the whole wave is done
    Rec64 me{0.0, 0.0, 0.0, 0.0};
    double hh = 0.0;
    if (act) {
        me = prec[s];
        hh = h[s];
    }
    // an inactive lane has h2 = 0: it meets no node and no particle.  A lane
    // whose partial sum already exceeds SPH_OVERFULL T neighbours (so h lies above
    // the root) drops out of the walk the same way.
    double h2 = hh * hh;
    const double inv_h = act ? 1.0 / hh : 0.0, inv_box = 1.0 / box;
    const double a_cut = SPH_OVERFULL * target * (3.0 / 32.0) * (act ? me.m : 0.0);
    bool overfull = false;
    double A = 0.0, D = 0.0;       // sum m_j w(q_j), sum m_j q_j w'(q_j)
    auto pair = [&](int64_t j) {
        const Rec64 p = prec[j];
        const double dx = min_image(p.x - me.x, box, inv_box), dy = min_image(p.y - me.y, box, inv_box),
                     dz = min_image(p.z - me.z, box, inv_box);
        const double r2 = (dx * dx + dy * dy) + dz * dz;
        if (r2 < h2) {
            double wq, qdw;
            spline_w(sqrt(r2) * inv_h, wq, qdw);
            A += p.m * wq;
            D += p.m * qdw;
            if (A > a_cut && me.m > 0.0) {
                overfull = true;
                h2 = 0.0;
            }
        }
    };
    if (m == 0) {
        if (act) pair(s);
    } else {
        // The walk is shared by the wave: node k (the same on every lane) is
        // entered when any lane's ball meets its cube; each lane then sums the
        // node's particle children that lie within its own h.
        int64_t k = 0;
        while (k < m) {
            const WalkRec64* r = wrec + k;
            const int64_t skip = n_skip[k];          // loaded with the record, not after the test
            const double half = 0.5 * r->l;
            const double ex = fmax(fabs(min_image(me.x - r->cx, box, inv_box)) - half, 0.0);
            const double ey = fmax(fabs(min_image(me.y - r->cy, box, inv_box)) - half, 0.0);
            const double ez = fmax(fabs(min_image(me.z - r->cz, box, inv_box)) - half, 0.0);
            if (__ballot((ex * ex + ey * ey) + ez * ez < h2) != 0) {
                const uint32_t meta = r->meta;
                if (meta == META_BUCKET) {
                    const int64_t f = r->kids[0], c = r->kids[1];
                    for (int64_t j = f; j < f + c; ++j) pair(j);
                } else {
                    for (uint32_t c = 0; c < meta; ++c) {
                        const uint32_t kid = r->kids[c];
                        if (kid & ITEM_PARTICLE) pair(kid & ~ITEM_PARTICLE);
                    }
                }
                ++k;
            } else {
                k = skip;
            }
        }
    }
    if (!act) return;
    const double mi = me.m;
    if (overfull) {
        // N(hh) > SPH_OVERFULL T: hh bounds the root from above; halve h, or
        // bisect once a lower bound is known
        const double l = lo[s];
        hi[s] = hh;
        h[s] = l > 0.0 ? 0.5 * (l + hh) : 0.5 * hh;
        atomicAdd(active, 1);
        return;
    }
    rho[s] = 8.0 / M_PI * inv_h * inv_h * inv_h * A;
    if (!(mi > 0.0)) {
        state[s] = SPH_FAILED;
        return;
    }
    const double N = 32.0 / 3.0 * A / mi;
    const double f = N - target;
    double l = lo[s], u = hi[s];
    if (fabs(f) <= 1e-13 * target) {
        state[s] = SPH_DONE;
        return;
    }
    if (f < 0.0)
        l = hh;
    else
        u = hh;
    if (u > 0.0 && u - l <= 4e-16 * u) {     // the bracket has closed
        state[s] = SPH_DONE;
        return;
    }
    // Newton in v = h^3, where N is close to linear: dN/dv = (dN/dh) / (3 h^2)
    const double dN = -32.0 / 3.0 * D / (mi * hh);
    double hn = -1.0;
    if (dN > 0.0) {
        const double v = hh * hh * hh - f * 3.0 * hh * hh / dN;
        if (v > 0.0) hn = cbrt(v);
    }
    if (u < 0.0) {
        if (!(hn > hh)) hn = SPH_GROW * hh;
        hn = fmin(hn, SPH_GROW * hh);
        if (hn > h_max) {
            if (hh >= h_max) {              // N(h_max) < T: no root within h_max
                state[s] = SPH_FAILED;
                return;
            }
            hn = h_max;
        }
    } else if (!(hn > l && hn < u)) {
        hn = 0.5 * (l + u);
    }
    lo[s] = l;
    hi[s] = u;
    h[s] = hn;
    atomicAdd(active, 1);
}

// Launched with one thread; the lane-indexed address keeps it a vector store.
__global__ void k_sph_zero(int32_t* p) { p[threadIdx.x] = 0; }

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

}  // namespace

extern "C" {

int sph_density(sr_tree* t, double n_ngb, double* h, double* rho, int64_t* unconverged, void* stream)
{
    if (!t) return sr_fail(SR_ESTATE, "sph_density: tree is NULL");
    if (t->n <= 0) return sr_fail(SR_ESTATE, "sph_density: the tree holds no particles");
    if (!(n_ngb > 32.0 / 3.0) || !isfinite(n_ngb))
        return sr_fail(SR_EINVAL, "sph_density: n_ngb must be finite and above 32/3 (got %g)", n_ngb);
    if (!h || !rho) return sr_fail(SR_EINVAL, "sph_density: h and rho are required");
    int dev = 0;
    SR_HIP(hipGetDevice(&dev));
    if (dev != t->device) return sr_fail(SR_ESTATE, "sph_density: tree belongs to device %d, current is %d", t->device, dev);
    hipStream_t st = (hipStream_t)stream;
    const int64_t n = t->n, m = t->n_nodes;
    const double box = t->box, h_max = 0.25 * box;
    // workspace (stream-ordered): h, lo, hi, rho in sorted order; state; two counters
    double* buf = nullptr;
    int32_t* ibuf = nullptr;
    if (hipMallocAsync((void**)&buf, sizeof(double) * 4 * n, st) != hipSuccess ||
        hipMallocAsync((void**)&ibuf, sizeof(int32_t) * (n + 2), st) != hipSuccess) {
        if (buf) (void)hipFreeAsync(buf, st);
        return sr_fail(SR_ENOMEM, "sph_density: workspace allocation for %lld particles failed", (long long)n);
    }
    double *hs = buf, *lo = buf + n, *hi = buf + 2 * n, *rs = buf + 3 * n;
    int32_t *state = ibuf, *active = ibuf + n, *failed = ibuf + n + 1;
    int32_t count = 0;
    int rc = SR_OK;
    hipLaunchKernelGGL(k_sph_init, sph_grid(n), dim3(SPH_TPB), 0, st, n, m, t->pparent, t->n_parent, t->n_count,
                       t->wrec64, n_ngb, box, h_max, hs, lo, hi, state);
    for (int it = 0; it < SPH_MAX_ITER; ++it) {
        hipLaunchKernelGGL(k_sph_zero, dim3(1), dim3(1), 0, st, active);
        sr_timing_mark(SR_T_SPH_ITER, true, st);
        hipLaunchKernelGGL(k_sph_iterate, sph_grid(n), dim3(SPH_TPB), 0, st, n, m, t->wrec64, t->n_skip, t->prec64,
                           box, n_ngb, h_max, hs, lo, hi, state, rs, active);
        sr_timing_mark(SR_T_SPH_ITER, false, st);
        if (hipGetLastError() != hipSuccess ||
            hipMemcpyAsync(&count, active, sizeof(int32_t), hipMemcpyDeviceToHost, st) != hipSuccess ||
            hipStreamSynchronize(st) != hipSuccess) {
            rc = sr_fail(SR_EHIP, "sph_density: iteration %d failed", it);
            break;
        }
        if (count == 0) break;
    }
    if (rc == SR_OK) {
        hipLaunchKernelGGL(k_sph_zero, dim3(1), dim3(1), 0, st, failed);
        hipLaunchKernelGGL(k_sph_out, sph_grid(n), dim3(SPH_TPB), 0, st, n, t->perm, hs, rs, state, h, rho, failed);
        if (hipGetLastError() != hipSuccess ||
            hipMemcpyAsync(&count, failed, sizeof(int32_t), hipMemcpyDeviceToHost, st) != hipSuccess ||
            hipStreamSynchronize(st) != hipSuccess)
            rc = sr_fail(SR_EHIP, "sph_density: output failed");
        else if (unconverged)
            *unconverged = count;
    }
    (void)hipFreeAsync(buf, st);
    (void)hipFreeAsync(ibuf, st);
    return rc;
}

}  // extern "C"
