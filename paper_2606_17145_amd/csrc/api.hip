// C ABI of the short-range gravity library: argument checks, handle and
// workspace management, and the calls into the build and walk launchers.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <atomic>
#include <mutex>
#include <new>
#include <vector>

#include "internal.h"
#include "gpoly.h"

namespace {
thread_local char g_err[512] = "";

// allocation-failure injection for tests: -1 off, k >= 0 fails the allocation
// after the next k successful ones
std::atomic<int64_t> g_alloc_fail_after{-1};

// phase timing state (process-wide)
struct TimedLaunch {
    int phase;
    hipEvent_t start, stop;
};
std::mutex g_tmu;
bool g_timing = false;
std::vector<TimedLaunch> g_pending;
std::vector<hipEvent_t> g_open(SR_T_COUNT, nullptr);
std::vector<hipEvent_t> g_free;   // recorded-and-read events, reused
double g_ms[SR_T_COUNT] = {};
int64_t g_calls[SR_T_COUNT] = {};

template <class T>
int alloc(T** p, int64_t count)
{
    *p = nullptr;
    if (count <= 0) count = 1;
    hipError_t e = sr_device_malloc((void**)p, sizeof(T) * (size_t)count);
    if (e != hipSuccess) {
        *p = nullptr;
        (void)hipGetLastError();
        return sr_fail(SR_ENOMEM, "hipMalloc of %lld bytes failed: %s", (long long)(sizeof(T) * count),
                       hipGetErrorString(e));
    }
    return SR_OK;
}

template <class T>
void release(T*& p)
{
    if (p) (void)hipFree((void*)p);
    p = nullptr;
}

void free_lists(sr_tree* t)
{
    release(t->ent_src);
    release(t->ent_mask);
    release(t->chunk_next);
    release(t->chunk_cnt);
    release(t->unit_group);
    release(t->unit_chunk);
    release(t->unit_nch);
    release(t->unit_next);
    release(t->group_head);
    release(t->list_counters);
    release(t->partials);
    t->cap_chunks = t->cap_units = t->cap_groups = 0;
    t->lkey.valid = false;
}

void free_workspace(sr_tree* t)
{
    for (int k = 0; k < 2; ++k) {
        release(t->khi[k]);
        release(t->klo[k]);
        release(t->kidx[k]);
    }
    release(t->hist);
    release(t->rs_status);
    release(t->scan_tmp);
    release(t->levelmask);
    release(t->ucount);
    release(t->base);
    release(t->b_lo);
    release(t->b_hi);
    release(t->b_lambda);
    release(t->b_parent);
    release(t->b_pre);
    release(t->leaf_bparent);
    release(t->status);
    if (t->h_status) (void)hipHostFree(t->h_status);
    if (t->h_counters) (void)hipHostFree(t->h_counters);
    if (t->ev_status) (void)hipEventDestroy(t->ev_status);
    if (t->ev_counters) (void)hipEventDestroy(t->ev_counters);
    t->h_status = t->h_counters = nullptr;
    t->ev_status = t->ev_counters = nullptr;
    release(t->perm);
    release(t->invperm);
    release(t->pparent);
    release(t->prec64);
    release(t->ph64);
    release(t->prec32);
    release(t->ph32);
    release(t->n_level);
    release(t->n_first);
    release(t->n_count);
    release(t->n_parent);
    release(t->n_skip);
    release(t->n_depth);
    release(t->n_corner);
    release(t->nrec64);
    release(t->nS);
    release(t->ngeo64);
    release(t->nhmax);
    release(t->nhmin);
    release(t->nrec32);
    release(t->nhmax32);
    release(t->items);
    release(t->n_kids);
    release(t->n_meta);
    release(t->wrec32);
    release(t->wrec64);
    release(t->prec64_0);
    release(t->nbox);
    t->drift_base = false;
    release(t->tgt_sorted);
    release(t->tgt_slot);
    release(t->mark);
    release(t->tgt_flag);
    release(t->tgt_pos);
    release(t->pbar);
    release(t->tbar);
    release(t->nbar);
    t->cap = 0;
    free_lists(t);
    release(t->frontier);
    t->cap_front = t->n_front_waves = 0;
}

int allocate_workspace(sr_tree* t, int64_t cap)
{
    const int64_t nb_rs = (cap + 255) / 256;             // radix-sort tiles (at least 256 keys each)
    const int64_t hist = 256 * nb_rs + 256 + 1;          // per-tile digit counts, then the digit totals
    const int64_t scan_tiles = (hist > cap + 1 ? hist : cap + 1) / 2048 + 2;
    const int64_t nodes = cap > 1 ? cap - 1 : 1;
    int rc = SR_OK;
#define A(ptr, count)                     \
    if ((rc = alloc(&(ptr), (count))) != SR_OK) { \
        free_workspace(t);                \
        return rc;                        \
    }
    for (int k = 0; k < 2; ++k) {
        A(t->khi[k], cap);
        A(t->klo[k], cap);
        A(t->kidx[k], cap);
    }
    A(t->hist, hist);
    A(t->scan_tmp, scan_tiles + 1);
    A(t->levelmask, cap);
    A(t->ucount, cap);
    A(t->base, cap + 1);
    A(t->b_lo, nodes);
    A(t->b_hi, nodes);
    A(t->b_lambda, nodes);
    A(t->b_parent, nodes);
    A(t->b_pre, nodes);
    A(t->leaf_bparent, cap);
    A(t->status, ST_ALLOC);
    A(t->rs_status, sr_tree_sort_status_words(cap));
    // the look-back words start untagged (tag 0 is never used)
    if (hipMemset(t->rs_status, 0, sizeof(uint64_t) * sr_tree_sort_status_words(cap)) != hipSuccess) {
        free_workspace(t);
        return sr_fail(SR_EHIP, "hipMemset of the sort's look-back words failed");
    }
    t->rs_epoch = 0;
    if (hipHostMalloc((void**)&t->h_status, ST_WORDS * sizeof(int32_t), hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void**)&t->h_counters, 8 * sizeof(int32_t), hipHostMallocDefault) != hipSuccess ||
        hipEventCreateWithFlags(&t->ev_status, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&t->ev_counters, hipEventDisableTiming) != hipSuccess) {
        free_workspace(t);
        return sr_fail(SR_ENOMEM, "pinned host read-back buffers or their events could not be created");
    }
    A(t->perm, cap);
    A(t->invperm, cap);
    A(t->pparent, cap);
    A(t->prec64, cap);
    A(t->ph64, cap);
    A(t->prec32, cap);
    A(t->ph32, cap);
    A(t->n_level, nodes);
    A(t->n_first, nodes);
    A(t->n_count, nodes);
    A(t->n_parent, nodes);
    A(t->n_skip, nodes);
    A(t->n_depth, nodes);
    A(t->n_corner, 3 * nodes);
    A(t->nrec64, nodes);
    A(t->nS, 3 * nodes);
    A(t->ngeo64, nodes);
    A(t->nhmax, nodes);
    A(t->nhmin, nodes);
    A(t->nrec32, nodes);
    A(t->nhmax32, nodes);
    A(t->items, 2 * cap);
    A(t->n_kids, 8 * nodes);
    A(t->n_meta, nodes);
    A(t->wrec32, nodes);
    A(t->wrec64, nodes);
    A(t->tgt_sorted, cap);
    A(t->tgt_slot, cap);
    A(t->mark, cap);
    A(t->tgt_flag, cap);
    A(t->tgt_pos, cap + 1);
    A(t->pbar, 4 * cap);
    A(t->tbar, 3 * cap);
    A(t->nbar, 4 * nodes);
#undef A
    t->cap = cap;
    return SR_OK;
}

int check_params(const sr_tree* t, const sr_params* p)
{
    if (!p) return sr_fail(SR_EINVAL, "params is NULL");
    if (!(isfinite(p->G) && isfinite(p->r_s) && p->r_s > 0.0))
        return sr_fail(SR_EINVAL, "G must be finite and r_s > 0");
    if (!(p->r_cut > 0.0 && p->r_cut < 0.5 * t->box))
        return sr_fail(SR_EINVAL, "r_cut must satisfy 0 < r_cut < box / 2 (got %g, box %g)", p->r_cut, t->box);
    if (!(p->theta >= 0.0 && isfinite(p->theta))) return sr_fail(SR_EINVAL, "theta must be finite and >= 0");
    if (p->criterion != SR_OPEN_BH && p->criterion != SR_OPEN_RELATIVE)
        return sr_fail(SR_EINVAL, "unknown opening criterion %d", p->criterion);
    if (p->criterion == SR_OPEN_RELATIVE && !(p->alpha >= 0.0 && isfinite(p->alpha)))
        return sr_fail(SR_EINVAL, "alpha must be finite and >= 0");
    if (p->precision != SR_FP64 && p->precision != SR_FP32 && p->precision != SR_FP32_ACC64)
        return sr_fail(SR_EINVAL, "unknown precision %d", p->precision);
    // the FP32 split factor is a polynomial fitted for u = r / (2 r_s) <= GPOLY_U_MAX
    if (p->precision != SR_FP64 && p->r_cut > 2.0 * GPOLY_U_MAX * p->r_s)
        return sr_fail(SR_EUNSUPPORTED, "FP32 precisions need r_cut <= %g r_s (got r_cut / r_s = %g)",
                       2.0 * GPOLY_U_MAX, p->r_cut / p->r_s);
    return SR_OK;
}

int check_call(sr_tree* t, const sr_params* p, const int32_t* active, int64_t n_active, const double* a_old)
{
    if (!t || t->n <= 0) return sr_fail(SR_ESTATE, "tree handle is NULL or was never built");
    int dev = -1;
    SR_HIP(hipGetDevice(&dev));
    if (dev != t->device)
        return sr_fail(SR_ESTATE, "the tree was built on device %d, the current device is %d", t->device, dev);
    int rc = check_params(t, p);
    if (rc) return rc;
    if (!active && n_active != t->n)
        return sr_fail(SR_EINVAL, "n_active (%lld) must equal n (%lld) when active is NULL", (long long)n_active,
                       (long long)t->n);
    if (active && (n_active < 0 || n_active > t->n))
        return sr_fail(SR_EINVAL, "n_active must lie in [0, n]");
    if (p->criterion == SR_OPEN_RELATIVE && !a_old) return sr_fail(SR_EINVAL, "relative criterion needs a_old");
    return SR_OK;
}
}  // namespace

hipError_t sr_device_malloc(void** p, size_t bytes)
{
    if (g_alloc_fail_after.load() >= 0 && g_alloc_fail_after.fetch_sub(1) == 0) {
        *p = nullptr;
        return hipErrorOutOfMemory;
    }
    return hipMalloc(p, bytes);
}

int sr_front_reserve(sr_tree* t, int64_t waves, int64_t cap, hipStream_t st)
{
    if (waves <= t->n_front_waves && cap <= t->cap_front) return SR_OK;
    // the old frontier may still be read by work queued on the call's stream
    SR_HIP(hipStreamSynchronize(st));
    release(t->frontier);
    // per wave: two levels of node ids (u32) and masks (u64)
    int rc = alloc(&t->frontier, waves * cap * 6);
    if (rc) {
        t->cap_front = t->n_front_waves = 0;
        return rc;
    }
    t->n_front_waves = waves;
    t->cap_front = cap;
    return SR_OK;
}

int sr_list_reserve(sr_tree* t, int64_t groups, int64_t chunks, int64_t units, hipStream_t st)
{
    if (groups <= t->cap_groups && chunks <= t->cap_chunks && units <= t->cap_units) return SR_OK;
    // the old lists may still be read by work queued on the call's stream
    SR_HIP(hipStreamSynchronize(st));
    free_lists(t);
    int rc = SR_OK;
#define A(ptr, count)                              \
    if ((rc = alloc(&(ptr), (count))) != SR_OK) { \
        free_lists(t);                             \
        return rc;                                 \
    }
    A(t->ent_src, 64 * chunks);
    A(t->ent_mask, 64 * chunks);
    A(t->chunk_next, chunks);
    A(t->chunk_cnt, chunks);
    A(t->unit_group, units);
    A(t->unit_chunk, units);
    A(t->unit_nch, units);
    A(t->unit_next, units);
    A(t->group_head, groups);
    A(t->list_counters, 8);
    A(t->partials, 64 * (3 * 8 + 2 * 4) * units);
#undef A
    t->cap_groups = groups;
    t->cap_chunks = chunks;
    t->cap_units = units;
    return SR_OK;
}

bool sr_timing_on() { return g_timing; }

void sr_timing_mark(int phase, bool start, hipStream_t st)
{
    std::lock_guard<std::mutex> lk(g_tmu);
    if (!g_timing) return;
    hipEvent_t e;
    if (!g_free.empty()) {
        e = g_free.back();
        g_free.pop_back();
    } else if (hipEventCreate(&e) != hipSuccess) {
        return;
    }
    (void)hipEventRecord(e, st);
    if (start) {
        g_open[phase] = e;
    } else if (g_open[phase]) {
        g_pending.push_back(TimedLaunch{phase, g_open[phase], e});
        g_open[phase] = nullptr;
    } else {
        g_free.push_back(e);
    }
}

int sr_fail(int code, const char* fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
    return code;
}

extern "C" {

const char* srgrav_last_error(void) { return g_err; }

int tree_build(const double* pos, const double* mass, const double* eps, double eps_scalar, int64_t n, double box,
               int32_t leaf_size, void* stream, sr_tree** tree)
{
    g_err[0] = 0;
    if (!tree) return sr_fail(SR_EINVAL, "tree out-pointer is NULL");
    if (!pos || !mass) return sr_fail(SR_EINVAL, "pos and mass are required");
    if (n < 1 || n > SR_N_MAX) return sr_fail(SR_EINVAL, "n must lie in [1, 2^30] (got %lld)", (long long)n);
    if (!(box > 0.0 && isfinite(box))) return sr_fail(SR_EINVAL, "box must be finite and > 0");
    if (leaf_size != 1) return sr_fail(SR_EUNSUPPORTED, "only leaf_size == 1 is supported");
    if (!eps && !(eps_scalar > 0.0 && isfinite(eps_scalar)))
        return sr_fail(SR_EINVAL, "eps_scalar must be finite and > 0 when eps is NULL");
    hipStream_t st = (hipStream_t)stream;
    sr_tree* t = *tree;
    bool fresh = false;
    if (!t) {
        t = new (std::nothrow) sr_tree();
        if (!t) return sr_fail(SR_ENOMEM, "host allocation of the handle failed");
        fresh = true;
        SR_HIP(hipGetDevice(&t->device));
    }
    if (n > t->cap) {
        // wait for in-flight work on the old workspace before releasing it
        if (!fresh) SR_HIP(hipStreamSynchronize(st));
        free_workspace(t);
        int rc = allocate_workspace(t, n);
        if (rc) {
            // the old tree is gone with its workspace: the handle reads as never built
            if (fresh) delete t;
            else t->n = 0;
            return rc;
        }
    }
    t->n = n;
    t->box = box;
    ++t->build_gen;
    sr_timing_mark(SR_T_BUILD, true, st);
    int rc = sr_build_device(t, pos, mass, eps, eps_scalar, st);
    sr_timing_mark(SR_T_BUILD, false, st);
    if (rc) {
        t->n = 0;
        if (fresh) {
            free_workspace(t);
            delete t;
        }
        return rc;
    }
    *tree = t;
    return SR_OK;
}

int shortrange_accel(sr_tree* t, const sr_params* p, const int32_t* active, int64_t n_active, const double* a_old,
                     void* acc, int32_t* counts, int64_t* list_token, void* stream)
{
    g_err[0] = 0;
    if (list_token) *list_token = 0;
    int rc = check_call(t, p, active, n_active, a_old);
    if (rc) return rc;
    if (!acc && n_active > 0) return sr_fail(SR_EINVAL, "acc is NULL");
    hipStream_t st = (hipStream_t)stream;
    if ((rc = sr_prepare_targets(t, active, n_active, st))) return rc;
    if ((rc = sr_walk_forward(t, p, n_active, active, a_old, acc, counts, st))) return rc;
    if (list_token && t->lkey.valid) *list_token = t->lkey.token;
    return SR_OK;
}

int shortrange_accel_noalloc(sr_tree* t, const sr_params* p, const int32_t* active, int64_t n_active,
                             const double* a_old, void* acc, int32_t* counts, void* stream)
{
    g_err[0] = 0;
    int rc = check_call(t, p, active, n_active, a_old);
    if (rc) return rc;
    if (!acc && n_active > 0) return sr_fail(SR_EINVAL, "acc is NULL");
    if (n_active > SR_NOALLOC_MAX_TARGETS)
        return sr_fail(SR_EINVAL, "the allocation-free forward takes at most %lld targets (got %lld)",
                       (long long)SR_NOALLOC_MAX_TARGETS, (long long)n_active);
    hipStream_t st = (hipStream_t)stream;
    if ((rc = sr_prepare_targets(t, active, n_active, st))) return rc;
    return sr_walk_forward_noalloc(t, p, n_active, active, a_old, acc, counts, st);
}

int shortrange_accel_adjoint(sr_tree* t, const sr_params* p, const int32_t* active, int64_t n_active,
                             const double* a_old, const void* w, double* dLdx, double* dLdm, int64_t list_token,
                             void* stream)
{
    g_err[0] = 0;
    if (list_token < 0) return sr_fail(SR_EINVAL, "list_token must be 0 or a token from shortrange_accel");
    if (list_token > 0) {
        // the targets and decisions come from the forward call that issued the token:
        // active and a_old are not read
        if (!t || t->n <= 0) return sr_fail(SR_ESTATE, "tree handle is NULL or was never built");
        int dev = -1;
        SR_HIP(hipGetDevice(&dev));
        if (dev != t->device)
            return sr_fail(SR_ESTATE, "the tree was built on device %d, the current device is %d", t->device, dev);
        int rc = check_params(t, p);
        if (rc) return rc;
        if (n_active < 0 || n_active > t->n) return sr_fail(SR_EINVAL, "n_active must lie in [0, n]");
        if ((rc = sr_check_list_token(t, p, n_active, list_token))) return rc;
    } else {
        int rc = check_call(t, p, active, n_active, a_old);
        if (rc) return rc;
    }
    if (!w || !dLdx || !dLdm) return sr_fail(SR_EINVAL, "w, dLdx and dLdm are required");
    hipStream_t st = (hipStream_t)stream;
    int rc = SR_OK;
    if (list_token == 0 && (rc = sr_prepare_targets(t, active, n_active, st))) return rc;
    return sr_walk_adjoint(t, p, n_active, active, a_old, w, dLdx, dLdm, list_token, st);
}

int tree_drift(sr_tree* t, const double* disp, void* stream)
{
    g_err[0] = 0;
    if (!t || t->n <= 0) return sr_fail(SR_ESTATE, "tree handle is NULL or was never built");
    int dev = -1;
    SR_HIP(hipGetDevice(&dev));
    if (dev != t->device)
        return sr_fail(SR_ESTATE, "the tree was built on device %d, the current device is %d", t->device, dev);
    if (!disp) return sr_fail(SR_EINVAL, "disp is NULL");
    hipStream_t st = (hipStream_t)stream;
    int rc = SR_OK;
    if (!t->prec64_0) {
        // drift buffers, sized for the workspace capacity (kept across rebuilds)
        const int64_t nodes = t->cap > 1 ? t->cap - 1 : 1;
        if ((rc = alloc(&t->prec64_0, t->cap)) || (rc = alloc(&t->nbox, 6 * nodes))) {
            release(t->prec64_0);
            release(t->nbox);
            return rc;
        }
        t->drift_base = false;
    }
    // the interaction lists belong to the undrifted particles: no token names them now
    t->lkey.valid = false;
    ++t->build_gen;
    sr_timing_mark(SR_T_DRIFT, true, st);
    rc = sr_drift_device(t, disp, st);
    sr_timing_mark(SR_T_DRIFT, false, st);
    return rc;
}

int tree_walk_stats(const sr_tree* t, int64_t* stats)
{
    if (!t || t->n <= 0) return sr_fail(SR_ESTATE, "tree handle is NULL or was never built");
    if (!stats) return sr_fail(SR_EINVAL, "stats is NULL");
    stats[0] = t->n_tests;
    stats[1] = t->n_chunks;
    stats[2] = t->n_units;
    stats[3] = t->lkey.valid ? t->lkey.n_t : 0;
    return SR_OK;
}

int tree_node_count(const sr_tree* t, int64_t* n_nodes)
{
    if (!t || t->n <= 0) return sr_fail(SR_ESTATE, "tree handle is NULL or was never built");
    if (!n_nodes) return sr_fail(SR_EINVAL, "n_nodes is NULL");
    *n_nodes = t->n_nodes;
    return SR_OK;
}

int tree_export(const sr_tree* t, const sr_tree_export* ex, void* stream)
{
    if (!t || t->n <= 0) return sr_fail(SR_ESTATE, "tree handle is NULL or was never built");
    if (!ex) return sr_fail(SR_EINVAL, "export record is NULL");
    hipStream_t st = (hipStream_t)stream;
    const int64_t n = t->n, m = t->n_nodes;
    auto cp = [&](void* dst, const void* src, size_t bytes) -> int {
        if (dst && bytes) SR_HIP(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, st));
        return SR_OK;
    };
    int rc = SR_OK;
    if ((rc = cp(ex->key_hi, t->khi[0], 8 * n)) || (rc = cp(ex->key_lo, t->klo[0], 8 * n)) ||
        (rc = cp(ex->perm, t->perm, 4 * n)) || (rc = cp(ex->level, t->n_level, 4 * m)) ||
        (rc = cp(ex->first, t->n_first, 4 * m)) || (rc = cp(ex->count, t->n_count, 4 * m)) ||
        (rc = cp(ex->parent, t->n_parent, 4 * m)) || (rc = cp(ex->skip, t->n_skip, 4 * m)) ||
        (rc = cp(ex->corner, t->n_corner, 12 * m)))
        return rc;
    if (m && (ex->M || ex->com || ex->M32 || ex->comX)) {
        // strided fields: copy through a 2D copy of the records
        if (ex->M) SR_HIP(hipMemcpy2DAsync(ex->M, 8, &t->nrec64[0].m, sizeof(Rec64), 8, m, hipMemcpyDeviceToDevice, st));
        if (ex->com) SR_HIP(hipMemcpy2DAsync(ex->com, 24, t->nrec64, sizeof(Rec64), 24, m, hipMemcpyDeviceToDevice, st));
        if (ex->M32) SR_HIP(hipMemcpy2DAsync(ex->M32, 4, &t->nrec32[0].m, sizeof(Rec32), 4, m, hipMemcpyDeviceToDevice, st));
        if (ex->comX) SR_HIP(hipMemcpy2DAsync(ex->comX, 12, t->nrec32, sizeof(Rec32), 12, m, hipMemcpyDeviceToDevice, st));
    }
    if (m && ex->side)
        SR_HIP(hipMemcpy2DAsync(ex->side, 8, &t->ngeo64[0].l, sizeof(Geo64), 8, m, hipMemcpyDeviceToDevice, st));
    return SR_OK;
}

int sr_axpy(void* y, int32_t y_type, const void* x, int32_t x_type, double a, int64_t n, void* stream)
{
    g_err[0] = 0;
    if (n < 0) return sr_fail(SR_EINVAL, "n must be >= 0");
    if (n == 0) return SR_OK;
    if (!y || !x) return sr_fail(SR_EINVAL, "x and y are required");
    if ((y_type != SR_F64 && y_type != SR_F32) || (x_type != SR_F64 && x_type != SR_F32))
        return sr_fail(SR_EINVAL, "element types must be SR_F64 or SR_F32");
    return sr_axpy_device(y, y_type, x, x_type, a, n, (hipStream_t)stream);
}

int srgrav_inject_alloc_failure(int64_t after)
{
    g_alloc_fail_after.store(after < 0 ? -1 : after);
    return SR_OK;
}

int srgrav_timing(int32_t enable)
{
    std::lock_guard<std::mutex> lk(g_tmu);
    for (auto& p : g_pending) {
        g_free.push_back(p.start);
        g_free.push_back(p.stop);
    }
    g_pending.clear();
    for (auto& e : g_open)
        if (e) g_free.push_back(e), e = nullptr;
    if (enable)
        for (int k = 0; k < SR_T_COUNT; ++k) g_ms[k] = 0.0, g_calls[k] = 0;
    g_timing = enable != 0;
    return SR_OK;
}

int srgrav_timing_read(double* ms, int64_t* calls)
{
    if (!ms || !calls) return sr_fail(SR_EINVAL, "ms and calls are required");
    std::lock_guard<std::mutex> lk(g_tmu);
    for (auto& p : g_pending) {
        float x = 0.0f;
        SR_HIP(hipEventSynchronize(p.stop));
        SR_HIP(hipEventElapsedTime(&x, p.start, p.stop));
        g_ms[p.phase] += x;
        g_calls[p.phase] += 1;
        g_free.push_back(p.start);
        g_free.push_back(p.stop);
    }
    g_pending.clear();
    for (int k = 0; k < SR_T_COUNT; ++k) {
        ms[k] = g_ms[k];
        calls[k] = g_calls[k];
    }
    return SR_OK;
}

void tree_free(sr_tree* t)
{
    if (!t) return;
    (void)hipDeviceSynchronize();
    free_workspace(t);
    delete t;
}

}  // extern "C"
