// Particle-mesh (PM) long-range force of the TreePM split on the device.
//
// The long-range half of the force that the tree walk's erfc split leaves out:
// periodic cloud-in-cell (CIC) assignment to an N^3 mesh, a real-to-complex 3D
// FFT (hipFFT), the Gaussian-filtered Green's function -4 pi G exp(-k^2 r_s^2)
// / k^2 with the CIC window divided out twice, one complex-to-real FFT to the
// potential, and per particle the fourth-order central difference of the
// potential at its eight CIC mesh points, weighted as in the assignment.  The
// paper runs this half on the host with FFTW (Sec. 3.1); the scheme is
// Gadget-2's periodic PM.
//
// Mesh point (i, j, k) sits at (i, j, k) L / N and is stored at (i N + j) N + k;
// the spectrum has N x N x (N/2 + 1) complex values in the same order.
#include <math.h>

#include <new>

#include <hipfft/hipfft.h>

#include "internal.h"
#include "sort.h"

#define PM_TRY(call)                     \
    do {                                 \
        const int rc_ = (call);          \
        if (rc_ != SR_OK) return rc_;    \
    } while (0)

struct sr_pm {
    int32_t n = 0;
    int device = 0;
    hipfftHandle r2c = 0, c2r = 0;
    bool have_r2c = false, have_c2r = false;
    double* mesh = nullptr;                   // N^3: the density, then N^3 times the potential
    hipfftDoubleComplex* spec = nullptr;      // N^2 (N/2 + 1): its spectrum, then the potential's
    double* axis = nullptr;                   // N: the per-axis filter factor of the Green's function
    double* work = nullptr;                   // N^3, adjoint only: one component of the assigned weights, then psi
    double* chi = nullptr;                    // N^3, adjoint only: the differenced weights
    // particle workspace, grown on demand: base-cell keys and particle indices
    // (two buffers each for the radix sort) and the sort's histogram
    int64_t cap = 0;
    uint64_t* key[2] = {};
    uint32_t* idx[2] = {};
    uint32_t* hist = nullptr;
    int sorted = 0;                           // the buffer that holds the sorted keys
};

namespace {

constexpr int PM_TPB = 256;

inline dim3 pm_grid(int64_t n) { return dim3((unsigned)((n + PM_TPB - 1) / PM_TPB)); }

// u = x/L - floor(x/L) in [0, 1), a rounding to 1 maps to 0; s = u N; the lower
// mesh index (mod N) and the weight f of the upper one.  A non-finite coordinate
// is placed at 0, so that every index stays on the mesh.
__device__ inline void cic_axis(double x, double box, int n, int& i0, double& f)
{
    double u = x / box;
    u = u - floor(u);
    if (!(u >= 0.0 && u < 1.0)) u = 0.0;
    const double s = u * (double)n;
    const double fl = floor(s);
    f = s - fl;
    i0 = (int)fl % n;
}

__global__ void k_pm_clear(double* __restrict__ p, int64_t count)
{
    const int64_t i = blockIdx.x * (int64_t)PM_TPB + threadIdx.x;
    if (i < count) p[i] = 0.0;
}

// Key of a particle: the linear index of its lower CIC mesh point.
__global__ void k_pm_keys(const double* __restrict__ pos, int64_t np, double box, int n,
                          uint64_t* __restrict__ key, uint32_t* __restrict__ idx)
{
    const int64_t p = blockIdx.x * (int64_t)PM_TPB + threadIdx.x;
    if (p >= np) return;
    int i[3];
    double f[3];
    for (int d = 0; d < 3; ++d) cic_axis(pos[3 * p + d], box, n, i[d], f[d]);
    key[p] = ((uint64_t)i[0] * (uint64_t)n + (uint64_t)i[1]) * (uint64_t)n + (uint64_t)i[2];
    idx[p] = (uint32_t)p;
}

// Mass (or weight) assignment in key order: particle idx[q] adds v w * scale to
// its eight mesh points, v = val[idx[q] * stride].  Lanes of a wave whose
// particles share a lower mesh point (a run of equal keys) share all eight
// targets: a segmented sum over the run leaves the totals in its last lane,
// which alone issues the eight FP64 atomics.  A wave without such runs adds
// directly.
__global__ void k_pm_deposit(const double* __restrict__ pos, const double* __restrict__ val, int stride,
                             const uint64_t* __restrict__ key, const uint32_t* __restrict__ idx, int64_t np,
                             double box, int n, double scale, double* __restrict__ mesh)
{
    const int64_t q = blockIdx.x * (int64_t)PM_TPB + threadIdx.x;
    const int lane = (int)(threadIdx.x & 63);
    const bool valid = q < np;
    const uint64_t k = valid ? key[q] : ~0ull;
    const uint64_t k_prev = __shfl_up(k, 1);
    const bool head = !valid || lane == 0 || k != k_prev;
    const uint64_t heads = __ballot(head);
    int i[3] = {0, 0, 0};
    double f[3] = {0.0, 0.0, 0.0}, v = 0.0;
    if (valid) {
        const int64_t p = idx[q];
        for (int d = 0; d < 3; ++d) cic_axis(pos[3 * p + d], box, n, i[d], f[d]);
        v = val[p * stride] * scale;
    }
    double c[8];
    for (int cx = 0; cx < 2; ++cx)
        for (int cy = 0; cy < 2; ++cy)
            for (int cz = 0; cz < 2; ++cz) {
                const double wx = cx ? f[0] : 1.0 - f[0], wy = cy ? f[1] : 1.0 - f[1], wz = cz ? f[2] : 1.0 - f[2];
                c[(cx * 2 + cy) * 2 + cz] = v * ((wx * wy) * wz);
            }
    bool issue = valid;
    if (heads != ~0ull) {          // some run spans lanes (uniform over the wave)
        const uint64_t upto = lane == 63 ? heads : heads & ((2ull << lane) - 1ull);
        const int start = 63 - __clzll(upto);          // first lane of this lane's run
        for (int off = 1; off < 64; off <<= 1)
            for (int r = 0; r < 8; ++r) {
                const double t = __shfl_up(c[r], off);
                if (lane - off >= start) c[r] += t;
            }
        issue = valid && (lane == 63 || ((heads >> (lane + 1)) & 1ull));
    }
    if (!issue) return;
    for (int cx = 0; cx < 2; ++cx) {
        const int64_t ix = (i[0] + cx) % n;
        for (int cy = 0; cy < 2; ++cy) {
            const int64_t iy = (i[1] + cy) % n;
            for (int cz = 0; cz < 2; ++cz)
                unsafeAtomicAdd(mesh + (ix * n + iy) * n + (i[2] + cz) % n, c[(cx * 2 + cy) * 2 + cz]);
        }
    }
}

// The filter exp(-k^2 r_s^2) / prod_d sinc(pi n_d / N)^4 is a product over the
// axes; entry i of the table is the factor of signed wavenumber n = i (i <= N/2)
// or i - N: exp(-(2 pi n / L)^2 r_s^2) / sinc(pi n / N)^4.
__global__ void k_pm_axis_table(double* __restrict__ t, int n, double box, double r_s)
{
    const int i = blockIdx.x * PM_TPB + threadIdx.x;
    if (i >= n) return;
    const int m = i <= n / 2 ? i : i - n;
    const double k = 2.0 * M_PI / box * m;
    double s = 1.0;
    if (m != 0) {
        const double x = M_PI * (double)m / (double)n;
        s = sin(x) / x;
    }
    const double s2 = s * s;
    t[i] = exp(-(k * r_s) * (k * r_s)) / (s2 * s2);
}

// In place: rho_hat -> phi_hat = -4 pi G rho_hat t(n_x) t(n_y) t(n_z) / k^2,
// phi_hat(0) = 0.
__global__ void k_pm_green(hipfftDoubleComplex* __restrict__ spec, const double* __restrict__ t, int n,
                           double box, double G)
{
    const int nh = n / 2 + 1;
    const int64_t idx = blockIdx.x * (int64_t)PM_TPB + threadIdx.x;
    if (idx >= (int64_t)n * n * nh) return;
    const int iz = (int)(idx % nh);
    const int iy = (int)((idx / nh) % n);
    const int ix = (int)(idx / ((int64_t)nh * n));
    const int nx = ix <= n / 2 ? ix : ix - n, ny = iy <= n / 2 ? iy : iy - n, nz = iz;
    const double tpl = 2.0 * M_PI / box;
    const double kx = tpl * nx, ky = tpl * ny, kz = tpl * nz;
    const double k2 = (kx * kx + ky * ky) + kz * kz;
    hipfftDoubleComplex z{0.0, 0.0};
    if (idx != 0) {
        const double green = -4.0 * M_PI * G * ((t[ix] * t[iy]) * t[iz]) / k2;
        const hipfftDoubleComplex r = spec[idx];
        z = hipfftDoubleComplex{r.x * green, r.y * green};
    }
    spec[idx] = z;
}

// 8 (p[1] - p[3]) - (p[0] - p[4]): 12 h times -dphi/dx at p[2] from the potential
// at offsets -2..+2 along one axis.
__device__ inline double fd4(double p0, double p1, double p3, double p4)
{
    return 8.0 * (p1 - p3) - (p0 - p4);
}

// a_i = scale * sum over the eight CIC mesh points c of w_c * fd4 along each
// axis at c.  Along axis d the two corners that differ in d share one line of
// six potential values (offsets -2..+3 from the lower corner).
// Particles are taken in key order (idx), so the lanes of a wave read nearby
// mesh points.
__global__ void k_pm_interp(const double* __restrict__ pos, const uint32_t* __restrict__ order, int64_t np,
                            double box, int n, const double* __restrict__ phi, double scale,
                            double* __restrict__ acc)
{
    const int64_t q = blockIdx.x * (int64_t)PM_TPB + threadIdx.x;
    if (q >= np) return;
    const int64_t p = order[q];
    int i[3];
    double f[3];
    for (int d = 0; d < 3; ++d) cic_axis(pos[3 * p + d], box, n, i[d], f[d]);
    const int64_t s[3] = {(int64_t)n * n, n, 1};      // element stride of each axis
    double a[3] = {0.0, 0.0, 0.0};
    for (int d = 0; d < 3; ++d) {
        const int e = d == 0 ? 1 : 0, g = d == 2 ? 1 : 2;      // the two other axes
        for (int ce = 0; ce < 2; ++ce) {
            const double we = ce ? f[e] : 1.0 - f[e];
            const int64_t oe = (int64_t)((i[e] + ce) % n) * s[e];
            for (int cg = 0; cg < 2; ++cg) {
                const double wg = cg ? f[g] : 1.0 - f[g];
                const int64_t base = oe + (int64_t)((i[g] + cg) % n) * s[g];
                double line[6];
                for (int k = 0; k < 6; ++k) line[k] = phi[base + (int64_t)((i[d] + k - 2 + n) % n) * s[d]];
                const double wo = we * wg;
                a[d] += ((1.0 - f[d]) * wo) * fd4(line[0], line[1], line[3], line[4]) +
                        (f[d] * wo) * fd4(line[1], line[2], line[4], line[5]);
            }
        }
    }
    acc[3 * p + 0] = a[0] * scale;
    acc[3 * p + 1] = a[1] * scale;
    acc[3 * p + 2] = a[2] * scale;
}

// chi (+)= -fd4 of `a` along axis d at every mesh point: the transpose of the
// difference rule (an odd stencil) applied to one weight component.
__global__ void k_pm_stencil(const double* __restrict__ a, double* __restrict__ chi, int n, int d, int accumulate)
{
    const int64_t n3 = (int64_t)n * n * n;
    const int64_t c = blockIdx.x * (int64_t)PM_TPB + threadIdx.x;
    if (c >= n3) return;
    const int64_t stride = d == 0 ? (int64_t)n * n : d == 1 ? n : 1;
    const int id = (int)((c / stride) % n);
    const int64_t row = c - (int64_t)id * stride;
    auto at = [&](int k) { return a[row + (int64_t)((id + k + n) % n) * stride]; };
    const double v = -fd4(at(-2), at(-1), at(1), at(2));
    chi[c] = accumulate ? chi[c] + v : v;
}

// Per particle j, with W_j(c) its CIC weights and grad W_j(c) their position
// derivatives (+-N/L along one axis times the other two weights):
//   dmass_j = inv_h3 scale sum_c W_j(c) psi(c)
//   dpos_j  = scale [sum_d w_j,d sum_c grad W_j(c) fd4_d phi(c) + m_j inv_h3 sum_c grad W_j(c) psi(c)]
// phi and psi are the unnormalised potential and adjoint meshes, so one scale
// 1 / (12 h N^3) covers both.
__global__ void k_pm_adjoint_gather(const double* __restrict__ pos, const double* __restrict__ mass,
                                    const double* __restrict__ w, const uint32_t* __restrict__ order, int64_t np,
                                    double box, int n, const double* __restrict__ phi,
                                    const double* __restrict__ psi, double scale, double inv_h3,
                                    double* __restrict__ dpos, double* __restrict__ dmass)
{
    const int64_t q = blockIdx.x * (int64_t)PM_TPB + threadIdx.x;
    if (q >= np) return;
    const int64_t p = order[q];          // key order, as in the interpolation
    int i[3];
    double f[3];
    for (int d = 0; d < 3; ++d) cic_axis(pos[3 * p + d], box, n, i[d], f[d]);
    const double inv_h = (double)n / box;
    const int64_t s[3] = {(int64_t)n * n, n, 1};
    // weight and derivative of the lower (0) and upper (1) mesh point on each axis
    double wt[3][2], dw[3][2];
    for (int d = 0; d < 3; ++d) {
        wt[d][0] = 1.0 - f[d];
        wt[d][1] = f[d];
        dw[d][0] = -inv_h;
        dw[d][1] = inv_h;
    }
    double gt[3] = {0.0, 0.0, 0.0};      // target term: sum_d w_d grad(sum_c W fd4_d phi)
    for (int d = 0; d < 3; ++d) {
        const double wd = w[3 * p + d];
        const int e = d == 0 ? 1 : 0, g = d == 2 ? 1 : 2;
        for (int ce = 0; ce < 2; ++ce) {
            const int64_t oe = (int64_t)((i[e] + ce) % n) * s[e];
            for (int cg = 0; cg < 2; ++cg) {
                const int64_t base = oe + (int64_t)((i[g] + cg) % n) * s[g];
                double line[6];
                for (int k = 0; k < 6; ++k) line[k] = phi[base + (int64_t)((i[d] + k - 2 + n) % n) * s[d]];
                const double fc[2] = {fd4(line[0], line[1], line[3], line[4]), fd4(line[1], line[2], line[4], line[5])};
                for (int cd = 0; cd < 2; ++cd) {
                    const double v = wd * fc[cd];
                    gt[d] += dw[d][cd] * (wt[e][ce] * wt[g][cg]) * v;
                    gt[e] += wt[d][cd] * (dw[e][ce] * wt[g][cg]) * v;
                    gt[g] += wt[d][cd] * (wt[e][ce] * dw[g][cg]) * v;
                }
            }
        }
    }
    double pv = 0.0, gs[3] = {0.0, 0.0, 0.0};   // source term
    for (int cx = 0; cx < 2; ++cx) {
        const int64_t ix = (i[0] + cx) % n;
        for (int cy = 0; cy < 2; ++cy) {
            const int64_t iy = (i[1] + cy) % n;
            for (int cz = 0; cz < 2; ++cz) {
                const double v = psi[(ix * n + iy) * n + (i[2] + cz) % n];
                pv += (wt[0][cx] * wt[1][cy]) * wt[2][cz] * v;
                gs[0] += (dw[0][cx] * wt[1][cy]) * wt[2][cz] * v;
                gs[1] += (wt[0][cx] * dw[1][cy]) * wt[2][cz] * v;
                gs[2] += (wt[0][cx] * wt[1][cy]) * dw[2][cz] * v;
            }
        }
    }
    const double ms = mass[p] * inv_h3;
    for (int e = 0; e < 3; ++e) dpos[3 * p + e] = (gt[e] + ms * gs[e]) * scale;
    dmass[p] = pv * inv_h3 * scale;
}

int fft_fail(const char* what, hipfftResult r) { return sr_fail(SR_EHIP, "%s failed (hipFFT status %d)", what, (int)r); }

void pm_release(sr_pm* m)
{
    if (m->have_r2c) (void)hipfftDestroy(m->r2c);
    if (m->have_c2r) (void)hipfftDestroy(m->c2r);
    m->have_r2c = m->have_c2r = false;
    (void)hipFree(m->mesh);
    (void)hipFree(m->spec);
    (void)hipFree(m->axis);
    (void)hipFree(m->work);
    (void)hipFree(m->chi);
    for (int b = 0; b < 2; ++b) {
        (void)hipFree(m->key[b]);
        (void)hipFree(m->idx[b]);
        m->key[b] = nullptr;
        m->idx[b] = nullptr;
    }
    (void)hipFree(m->hist);
    m->hist = nullptr;
    m->cap = 0;
    m->mesh = nullptr;
    m->spec = nullptr;
    m->axis = nullptr;
    m->work = nullptr;
    m->chi = nullptr;
}

}  // namespace

extern "C" {

int pm_create(int32_t n_mesh, sr_pm** out)
{
    if (!out) return sr_fail(SR_EINVAL, "pm_create: out is NULL");
    *out = nullptr;
    if (n_mesh < 2 || n_mesh > 2048 || (n_mesh & 1))
        return sr_fail(SR_EINVAL, "pm_create: n_mesh must be even and in [2, 2048] (got %d)", (int)n_mesh);
    int dev = 0;
    SR_HIP(hipGetDevice(&dev));
    sr_pm* m = new (std::nothrow) sr_pm();
    if (!m) return sr_fail(SR_ENOMEM, "pm_create: host allocation failed");
    m->n = n_mesh;
    m->device = dev;
    const int64_t n3 = (int64_t)n_mesh * n_mesh * n_mesh, nc = (int64_t)n_mesh * n_mesh * (n_mesh / 2 + 1);
    const bool ok = sr_device_malloc((void**)&m->mesh, sizeof(double) * n3) == hipSuccess &&
                    sr_device_malloc((void**)&m->spec, sizeof(hipfftDoubleComplex) * nc) == hipSuccess &&
                    sr_device_malloc((void**)&m->axis, sizeof(double) * n_mesh) == hipSuccess;
    if (!ok) {
        pm_release(m);
        delete m;
        return sr_fail(SR_ENOMEM, "pm_create: device allocation of the %d^3 mesh failed", (int)n_mesh);
    }
    hipfftResult r = hipfftPlan3d(&m->r2c, n_mesh, n_mesh, n_mesh, HIPFFT_D2Z);
    m->have_r2c = r == HIPFFT_SUCCESS;
    if (r == HIPFFT_SUCCESS) {
        r = hipfftPlan3d(&m->c2r, n_mesh, n_mesh, n_mesh, HIPFFT_Z2D);
        m->have_c2r = r == HIPFFT_SUCCESS;
    }
    if (r != HIPFFT_SUCCESS) {
        pm_release(m);
        delete m;
        return fft_fail("pm_create: hipfftPlan3d", r);
    }
    *out = m;
    return SR_OK;
}

}  // extern "C"

namespace {

int pm_check(sr_pm* m, const char* fn, const double* pos, const double* mass, int64_t n, double box, double r_s,
             double G)
{
    if (!m) return sr_fail(SR_ESTATE, "%s: handle is NULL", fn);
    if (n < 0 || (n > 0 && (!pos || !mass))) return sr_fail(SR_EINVAL, "%s: bad particle arrays", fn);
    if (!(box > 0.0 && isfinite(box))) return sr_fail(SR_EINVAL, "%s: box must be finite and > 0", fn);
    if (!(r_s > 0.0 && isfinite(r_s) && isfinite(G))) return sr_fail(SR_EINVAL, "%s: r_s > 0 and finite G required", fn);
    if (n > INT32_MAX) return sr_fail(SR_EINVAL, "%s: at most 2^31 - 1 particles", fn);
    int dev = 0;
    SR_HIP(hipGetDevice(&dev));
    if (dev != m->device) return sr_fail(SR_ESTATE, "%s: handle belongs to device %d, current is %d", fn, m->device, dev);
    return SR_OK;
}

// The spectral half shared by the force and its adjoint: the real mesh `src`
// -> spectrum -> times the filtered Green's function -> N^3 times K src in `dst`.
int pm_convolve(sr_pm* m, double* src, double* dst, double box, double r_s, double G, hipStream_t st,
                const char* fn)
{
    const int N = m->n;
    const int64_t nc = (int64_t)N * N * (N / 2 + 1);
    hipfftResult r = hipfftSetStream(m->r2c, st);
    if (r == HIPFFT_SUCCESS) r = hipfftSetStream(m->c2r, st);
    if (r != HIPFFT_SUCCESS) return fft_fail(fn, r);
    sr_timing_mark(SR_T_PM_FFT, true, st);
    r = hipfftExecD2Z(m->r2c, (hipfftDoubleReal*)src, m->spec);
    sr_timing_mark(SR_T_PM_FFT, false, st);
    if (r != HIPFFT_SUCCESS) return fft_fail(fn, r);
    sr_timing_mark(SR_T_PM_GREEN, true, st);
    hipLaunchKernelGGL(k_pm_axis_table, pm_grid(N), dim3(PM_TPB), 0, st, m->axis, N, box, r_s);
    hipLaunchKernelGGL(k_pm_green, pm_grid(nc), dim3(PM_TPB), 0, st, m->spec, m->axis, N, box, G);
    sr_timing_mark(SR_T_PM_GREEN, false, st);
    SR_HIP(hipGetLastError());
    sr_timing_mark(SR_T_PM_FFT, true, st);
    r = hipfftExecZ2D(m->c2r, m->spec, (hipfftDoubleReal*)dst);
    sr_timing_mark(SR_T_PM_FFT, false, st);
    if (r != HIPFFT_SUCCESS) return fft_fail(fn, r);
    return SR_OK;
}

// Particle workspace for n particles; a larger n frees and reallocates it (the
// free waits for the call's stream).
int pm_reserve(sr_pm* m, int64_t n, const char* fn, hipStream_t st)
{
    if (n <= m->cap) return SR_OK;
    if (m->cap > 0) SR_HIP(hipStreamSynchronize(st));   // earlier calls may still use the buffers
    for (int b = 0; b < 2; ++b) {
        (void)hipFree(m->key[b]);
        (void)hipFree(m->idx[b]);
        m->key[b] = nullptr;
        m->idx[b] = nullptr;
    }
    (void)hipFree(m->hist);
    m->hist = nullptr;
    m->cap = 0;
    bool ok = sr_device_malloc((void**)&m->hist, sizeof(uint32_t) * sr_sort_hist_words(n)) == hipSuccess;
    for (int b = 0; b < 2 && ok; ++b)
        ok = sr_device_malloc((void**)&m->key[b], sizeof(uint64_t) * n) == hipSuccess &&
             sr_device_malloc((void**)&m->idx[b], sizeof(uint32_t) * n) == hipSuccess;
    if (!ok) return sr_fail(SR_ENOMEM, "%s: device allocation for %lld particles failed", fn, (long long)n);
    m->cap = n;
    return SR_OK;
}

// Deposit val (stride apart, times scale) into `mesh`, cleared first, in the
// key order of the last pm_sort.
void pm_deposit(sr_pm* m, const double* pos, const double* val, int stride, int64_t n, double box, double scale,
                double* mesh, hipStream_t st)
{
    const int N = m->n;
    const int64_t n3 = (int64_t)N * N * N;
    sr_timing_mark(SR_T_PM_DEPOSIT, true, st);
    hipLaunchKernelGGL(k_pm_clear, pm_grid(n3), dim3(PM_TPB), 0, st, mesh, n3);
    hipLaunchKernelGGL(k_pm_deposit, pm_grid(n), dim3(PM_TPB), 0, st, pos, val, stride, m->key[m->sorted],
                       m->idx[m->sorted], n, box, N, scale, mesh);
    sr_timing_mark(SR_T_PM_DEPOSIT, false, st);
}

// Sort the particles by lower mesh point, then m->mesh = N^3 times their
// long-range potential.
int pm_potential(sr_pm* m, const double* pos, const double* mass, int64_t n, double box, double r_s, double G,
                 hipStream_t st, const char* fn)
{
    const int N = m->n;
    const double h = box / N;
    PM_TRY(pm_reserve(m, n, fn, st));
    const uint64_t n3 = (uint64_t)N * N * N;
    int bits = 1;
    while (bits < 64 && (n3 - 1) >> bits) ++bits;
    const int passes = (bits + 7) / 8;
    sr_timing_mark(SR_T_PM_SORT, true, st);
    hipLaunchKernelGGL(k_pm_keys, pm_grid(n), dim3(PM_TPB), 0, st, pos, n, box, N, m->key[0], m->idx[0]);
    SR_HIP(hipGetLastError());
    PM_TRY(sr_sort_keys64(m->key, m->idx, n, passes, m->hist, st));
    sr_timing_mark(SR_T_PM_SORT, false, st);
    m->sorted = passes & 1;
    pm_deposit(m, pos, mass, 1, n, box, 1.0 / (h * h * h), m->mesh, st);
    SR_HIP(hipGetLastError());
    return pm_convolve(m, m->mesh, m->mesh, box, r_s, G, st, fn);
}

}  // namespace

extern "C" {

int pm_accel(sr_pm* m, const double* pos, const double* mass, int64_t n, double box, double r_s, double G,
             double* acc, void* stream)
{
    PM_TRY(pm_check(m, "pm_accel", pos, mass, n, box, r_s, G));
    if (n > 0 && !acc) return sr_fail(SR_EINVAL, "pm_accel: acc is NULL");
    if (n == 0) return SR_OK;
    hipStream_t st = (hipStream_t)stream;
    const int N = m->n;
    const double h = box / N;
    PM_TRY(pm_potential(m, pos, mass, n, box, r_s, G, st, "pm_accel"));
    sr_timing_mark(SR_T_PM_INTERP, true, st);
    hipLaunchKernelGGL(k_pm_interp, pm_grid(n), dim3(PM_TPB), 0, st, pos, m->idx[m->sorted], n, box, N, m->mesh,
                       1.0 / (12.0 * h * (double)N * N * N), acc);
    sr_timing_mark(SR_T_PM_INTERP, false, st);
    SR_HIP(hipGetLastError());
    return SR_OK;
}

int pm_accel_adjoint(sr_pm* m, const double* pos, const double* mass, int64_t n, double box, double r_s, double G,
                     const double* w, double* dpos, double* dmass, void* stream)
{
    PM_TRY(pm_check(m, "pm_accel_adjoint", pos, mass, n, box, r_s, G));
    if (n > 0 && (!w || !dpos || !dmass)) return sr_fail(SR_EINVAL, "pm_accel_adjoint: w, dpos and dmass required");
    if (n == 0) return SR_OK;
    const int N = m->n;
    const int64_t n3 = (int64_t)N * N * N;
    if (!m->work) {
        if (sr_device_malloc((void**)&m->work, sizeof(double) * n3) != hipSuccess ||
            sr_device_malloc((void**)&m->chi, sizeof(double) * n3) != hipSuccess) {
            (void)hipFree(m->work);
            m->work = nullptr;
            m->chi = nullptr;
            return sr_fail(SR_ENOMEM, "pm_accel_adjoint: device allocation of two %d^3 meshes failed", N);
        }
    }
    hipStream_t st = (hipStream_t)stream;
    const double h = box / N;
    PM_TRY(pm_potential(m, pos, mass, n, box, r_s, G, st, "pm_accel_adjoint"));
    // chi = -sum_d fd4_d (the weights' component d assigned to the mesh)
    for (int d = 0; d < 3; ++d) {
        pm_deposit(m, pos, w + d, 3, n, box, 1.0, m->work, st);
        sr_timing_mark(SR_T_PM_STENCIL, true, st);
        hipLaunchKernelGGL(k_pm_stencil, pm_grid(n3), dim3(PM_TPB), 0, st, m->work, m->chi, N, d, d > 0 ? 1 : 0);
        sr_timing_mark(SR_T_PM_STENCIL, false, st);
        SR_HIP(hipGetLastError());
    }
    PM_TRY(pm_convolve(m, m->chi, m->work, box, r_s, G, st, "pm_accel_adjoint"));
    sr_timing_mark(SR_T_PM_ADJ_GATHER, true, st);
    hipLaunchKernelGGL(k_pm_adjoint_gather, pm_grid(n), dim3(PM_TPB), 0, st, pos, mass, w, m->idx[m->sorted], n,
                       box, N, m->mesh,
                       m->work, 1.0 / (12.0 * h * (double)n3), 1.0 / (h * h * h), dpos, dmass);
    sr_timing_mark(SR_T_PM_ADJ_GATHER, false, st);
    SR_HIP(hipGetLastError());
    return SR_OK;
}

void pm_free(sr_pm* m)
{
    if (!m) return;
    (void)hipDeviceSynchronize();
    pm_release(m);
    delete m;
}

}  // extern "C"
