/*
 * srgrav.h -- short-range TreePM gravity on AMD Instinct MI355X (gfx950).
 *
 * The short-range half of a Gadget-style TreePM gravity solver: for every
 * target particle, a Barnes-Hut walk of an octree, opened by an angular (or
 * relative) criterion, applying each accepted node or particle on the fly
 * (the module the paper ports, Sec. 2 "OpenGadget3 infrastructure" and its
 * GPU-porting subsection; the TreePM split with the long-range mesh on the
 * CPU is stated in Sec. 3.1).  Per target i:
 *
 *   a_i = sum over accepted sources s with |d| < r_cut of  G M_s S_h(|d|) g(|d| / 2 r_s) d,
 *   d   = min-image(x_s - x_i),   h = max(h_i, h_s),   h = 2.8 eps,
 *   g(u) = erfc(u) + 2u/sqrt(pi) exp(-u^2)         (short-range part of the erfc split)
 *   S_h(r) = cubic-spline softened 1/r^3           (= 1/r^3 for r >= h)
 *
 * The library builds the tree on the device (integer coordinates, 90-bit
 * Morton keys, LDS radix sort, compressed octree, FP64 node moments) and
 * walks it by wavefront-sized target groups.  The paper builds the tree on
 * the host and re-uploads it every step (its GPU-porting subsection and
 * Appendix A); here nothing but launches and one small status read cross the
 * host-device boundary.
 *
 * Conventions for every entry point:
 *   - Pointers marked DEVICE are device memory (HIP / torch.cuda tensors) of
 *     the current device, contiguous, owned by the caller.  Nothing is
 *     retained after a call except inside an sr_tree handle.
 *   - Work is enqueued on `stream` (a hipStream_t; NULL = the null stream).
 *     The host waits only where stated, and then for one point of the
 *     stream (an event behind a small copy), not for all work queued on it.
 *   - Every call returns SR_OK (0) or a negative error code and never throws;
 *     srgrav_last_error() gives a message for the calling thread.
 *   - Outputs are overwritten, never accumulated into.
 *   - Particle arrays are in the caller's (input) order; outputs for a target
 *     subset follow the order of the `active` array.
 */
#ifndef SRGRAV_H
#define SRGRAV_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* return codes */
enum {
    SR_OK = 0,
    SR_EINVAL = -1,        /* invalid argument or input value (NaN/Inf, range) */
    SR_ENOMEM = -2,        /* device allocation failed */
    SR_EHIP = -3,          /* a HIP runtime call failed */
    SR_ESTATE = -4,        /* handle does not match the call (e.g. never built) */
    SR_EUNSUPPORTED = -5   /* argument combination not implemented */
};

/* opening criterion */
enum {
    SR_OPEN_BH = 0,        /* open iff l^2 > theta^2 r^2 (r to the node's centre of mass) */
    SR_OPEN_RELATIVE = 1   /* open iff G M l^2 > alpha |a_old| r^4, or l^2 > theta^2 r^2 */
};

/* arithmetic of the walk */
enum {
    SR_FP64 = 0,           /* FP64 positions, decisions, forces and sums */
    SR_FP32 = 1,           /* integer coordinates, FP32 decisions, forces and sums */
    SR_FP32_ACC64 = 2      /* as SR_FP32 but every target sums its forces in FP64 */
};

typedef struct sr_tree sr_tree;

typedef struct {
    double G;              /* gravitational constant (1 in all synthetic workloads) */
    double r_s;            /* PM split scale, r_s = 1.25 L / N_mesh in Gadget's default */
    double r_cut;          /* short-range cutoff (4.5 r_s by default); 0 < r_cut < L/2, and
                              r_cut <= 4.6 r_s for SR_FP32 / SR_FP32_ACC64 (SR_EUNSUPPORTED otherwise:
                              the FP32 split factor is fitted on r / 2 r_s <= 2.3) */
    int32_t criterion;     /* SR_OPEN_BH or SR_OPEN_RELATIVE */
    double theta;          /* opening angle (BH), or the geometric guard (RELATIVE); >= 0 */
    double alpha;          /* relative tolerance (RELATIVE only); >= 0 */
    int32_t precision;     /* SR_FP64, SR_FP32 or SR_FP32_ACC64 */
} sr_params;

/*
 * tree_build -- keys, sort, octree and node moments for n particles.
 *
 *   pos   DEVICE double[n*3]  positions, any real values; wrapped into [0, box)
 *   mass  DEVICE double[n]    masses (> 0)
 *   eps   DEVICE double[n]    Plummer-equivalent softening per particle (> 0),
 *                             or NULL to use eps_scalar for every particle
 *   n     1 <= n <= 2^30
 *   box   periodic box side L > 0
 *   leaf_size  must be 1 (every particle is its own leaf)
 *   tree  in/out: if *tree is NULL a new handle is created; otherwise that
 *         handle is rebuilt in place, growing its workspace only when n
 *         exceeds what it holds.  The handle keeps its own copy of every
 *         sorted particle record, so callers may change pos/mass afterwards.
 *
 * The node set is the compressed octree of the 90-bit Morton keys (cells with
 * at least two non-empty children, and level-30 buckets of identical keys), in
 * pre-order.  The host waits once, for the point of `stream` where the node
 * count, the depth histogram and the input flags have been copied back (the
 * remaining build kernels are queued afterwards and run asynchronously).
 * SR_EINVAL on NaN/Inf positions, masses or softenings.
 */
int tree_build(const double* pos, const double* mass, const double* eps, double eps_scalar,
               int64_t n, double box, int32_t leaf_size, void* stream, sr_tree** tree);

/*
 * shortrange_accel -- short-range accelerations of the targets.
 *
 *   active    DEVICE int32[n_active] distinct input indices of the targets, or
 *             NULL for all particles (then n_active must equal n)
 *   a_old     DEVICE double[n]  |a| of the previous step per particle (input
 *             order); read only for SR_OPEN_RELATIVE, else may be NULL
 *   acc       DEVICE [n_active*3] output, double unless p->precision == SR_FP32
 *             (then float); may be NULL only when n_active == 0
 *   counts    DEVICE int32[n_active*2] output (particle-particle, particle-node
 *             interactions per target), or NULL
 *   list_token  HOST int64 output, or NULL: a positive token naming the
 *             interaction lists this call made (0 when none were made, e.g.
 *             n_active == 0 or a single particle).  Passing it to
 *             shortrange_accel_adjoint differentiates exactly this call.
 *
 * Per-target semantics are those of a depth-first walk of one particle; the
 * group walk only shares the traversal.  The host waits once for the
 * traversal's list counters (the point right behind the traversal kernel; the
 * evaluation is already queued and may still run when the call returns), and
 * once more when `active` is given, to report out-of-range or repeated
 * indices.  Lists that outgrow their reservation are grown and the traversal
 * repeated within the call; the reservation is kept on the handle.
 */
int shortrange_accel(sr_tree* tree, const sr_params* p, const int32_t* active, int64_t n_active,
                     const double* a_old, void* acc, int32_t* counts, int64_t* list_token, void* stream);

/*
 * shortrange_accel_noalloc -- shortrange_accel for callers that cannot allocate
 * device memory (code under stream capture, tight serving loops, harnesses that
 * forbid hipMalloc).  Same arguments, targets, decisions and results as
 * shortrange_accel (bit for bit: the same kernels make the same lists), but the
 * interaction lists, traversal frontier, list counters and per-unit partial sums
 * live in one fixed device buffer of SR_NOALLOC_SCRATCH_BYTES that the library
 * holds on each GPU it runs on until the process ends; the call allocates and
 * frees nothing (with phase timing on, srgrav_timing may still create events).
 * The tree handle must already have been built; its per-target workspace is
 * reused.
 *
 *   n_active  at most SR_NOALLOC_MAX_TARGETS, else SR_EINVAL before any device work
 *
 * Lists that do not fit the buffer give SR_ENOMEM (acc and counts are then not
 * valid): the list size depends on the clustering, not only on n_active.  No
 * list token is issued (the adjoint repeats the walk for token 0), and a token
 * from an earlier shortrange_accel on this handle is invalidated.  Every call
 * on one GPU shares that GPU's buffer: calls that overlap on one GPU (on
 * different streams or host threads) race and give wrong results; calls in
 * stream order on one stream are safe.
 */
#define SR_NOALLOC_SCRATCH_BYTES (128ll << 20)
#define SR_NOALLOC_MAX_TARGETS (1ll << 18)
int shortrange_accel_noalloc(sr_tree* tree, const sr_params* p, const int32_t* active,
                             int64_t n_active, const double* a_old, void* acc, int32_t* counts,
                             void* stream);

/*
 * shortrange_accel_adjoint -- gradient of L = sum_t w_t . a_t.
 *
 * The tree topology, node membership, opening decisions and cutoff membership
 * are those of the forward pass and L is differentiated with all of them held
 * fixed.
 *
 *   list_token  0: prepare the targets from `active` and repeat the forward's
 *               deterministic walk (decisions from `a_old` for the relative
 *               criterion).
 *               > 0: a token returned by shortrange_accel on this handle; its
 *               interaction lists and targets are reused and `active` and
 *               `a_old` are not read (the gradient is that of the call that
 *               issued the token, whatever the caller did to those arrays
 *               since).  SR_ESTATE if the token no longer names the handle's
 *               lists (a later shortrange_accel, an adjoint without a token or
 *               a rebuild replaced them), SR_EINVAL if n_active or the decision
 *               parameters (everything but the precision's accumulator) differ
 *               from that call.
 *   w     DEVICE [n_active*3] cotangent, same element type as `acc`
 *   dLdx  DEVICE double[n*3]  output, input order (w.r.t. the wrapped positions,
 *                             which is the same as w.r.t. pos)
 *   dLdm  DEVICE double[n]    output, input order
 *
 * Node terms are scattered with device atomics, so the low bits of the result
 * may differ from run to run.  The host does not wait when the forward's lists
 * are reused; otherwise it waits for the repeated traversal's counters as
 * shortrange_accel does.
 */
int shortrange_accel_adjoint(sr_tree* tree, const sr_params* p, const int32_t* active,
                             int64_t n_active, const double* a_old, const void* w, double* dLdx,
                             double* dLdm, int64_t list_token, void* stream);

/*
 * tree_drift -- reuse a built tree after its particles moved (paper App. A:
 * between rebuilds the GPU step drifts the tree nodes with their particles).
 * The topology, particle order and node order stay those of the last
 * tree_build; every particle is placed at its built (wrapped) position plus
 * disp, not wrapped again (its integer coordinates are those of the moved
 * position); the node moments are refolded in the build's order; and each
 * node's cube, centred on its cell centre c, grows to the half side
 * max(l/2, max over its particles and axes of |x - c|), which every opening
 * test then uses in place of the cell.  disp is measured from the built
 * positions, so drifting twice is not cumulative.  The walks and the adjoint
 * then run on the drifted tree; list tokens issued before are void.
 *
 *   disp   DEVICE double[n*3] displacement per particle, input order (finite)
 *
 * The first drift after a build allocates the drift buffers (kept by the
 * handle).  The host waits once, for the finiteness flag.  SR_EINVAL for a
 * non-finite displacement (the tree is then not usable until rebuilt).
 */
int tree_drift(sr_tree* tree, const double* disp, void* stream);

/*
 * sr_axpy -- y[i] += a * x[i] for i < n, the elementwise update of a
 * kick-drift-kick leapfrog step (kick: v += dt/2 a(x); drift: x += dt v) and
 * of its transpose in a rollout's backward pass.  (The paper's GPU steps drift
 * every particle at the start of the step: its GPU-porting subsection and
 * Appendix A.)  Errors: SR_EINVAL for n < 0, NULL pointers or unknown types.
 *
 *   y       DEVICE, element type y_type (SR_F64 or SR_F32), n elements, updated in place
 *   x       DEVICE, element type x_type, n elements (may not alias y)
 */
enum { SR_F64 = 0, SR_F32 = 1 };
int sr_axpy(void* y, int32_t y_type, const void* x, int32_t x_type, double a, int64_t n, void* stream);

/*
 * Phase timing with HIP events recorded on the launch stream around every
 * phase of the path (for profiling; off by default).  srgrav_timing(1) resets
 * the accumulators and starts recording, srgrav_timing(0) stops;
 * srgrav_timing_read() waits for the recorded events and returns, per phase,
 * the summed duration in milliseconds and the number of launches.
 *   ms, calls  HOST arrays of SR_T_COUNT entries
 */
enum {
    SR_T_BUILD = 0,        /* tree_build: keys, sort, topology, moments */
    SR_T_TRAVERSE = 1,     /* walk decisions -> interaction lists */
    SR_T_EVAL = 2,         /* pair forces of the lists */
    SR_T_REDUCE = 3,       /* per-target sums of the evaluation units */
    SR_T_ADJ_EVAL = 4,     /* adjoint pair terms */
    SR_T_ADJ_REDUCE = 5,   /* per-target adjoint sums */
    SR_T_PUSHDOWN = 6,     /* node adjoints to particles */
    SR_T_PM_DEPOSIT = 7,   /* PM: mesh clear and CIC assignment (masses, or adjoint weights) */
    SR_T_PM_FFT = 8,       /* PM: one 3D FFT (two per pm_accel) */
    SR_T_PM_GREEN = 9,     /* PM: Green's function applied to the density spectrum */
    SR_T_PM_INTERP = 10,   /* PM: finite-difference force and CIC interpolation */
    SR_T_PM_STENCIL = 11,  /* PM adjoint: transposed difference rule on one weight mesh */
    SR_T_PM_ADJ_GATHER = 12, /* PM adjoint: per-particle position and mass gradients */
    SR_T_PM_SORT = 13,     /* PM: particles sorted by mesh cell for the assignment */
    SR_T_SPH_ITER = 14,    /* SPH density: one iteration (neighbour walk, Halley step) */
    SR_T_DRIFT = 15,       /* tree_drift: moved particle records, refolded moments and cubes */
    SR_T_COUNT = 16
};
int srgrav_timing(int32_t enable);
int srgrav_timing_read(double* ms, int64_t* calls);

/*
 * srgrav_inject_alloc_failure -- test hook for the out-of-memory paths: with
 * after >= 0, the library's device allocation that follows the next `after`
 * successful ones fails as if hipMalloc had (SR_ENOMEM), once; a negative
 * value switches the injection off.  Process-wide; host-pinned buffers,
 * hipFFT's own plan memory and sph_density's stream-ordered workspace are not
 * covered.  Always SR_OK.
 */
int srgrav_inject_alloc_failure(int64_t after);

/* Internal arrays of a built tree, copied into caller buffers (DEVICE; any may
 * be NULL).  Node arrays need room for tree_node_count() entries. */
typedef struct {
    uint64_t* key_hi;      /* [n] sorted keys, digits 1..15 (45 bits) */
    uint64_t* key_lo;      /* [n] digits 16..30 */
    int32_t* perm;         /* [n] sorted position -> input index */
    int32_t* level;        /* [nodes] octree level 0..30 */
    int32_t* first;        /* [nodes] first sorted position */
    int32_t* count;        /* [nodes] particles in the node */
    int32_t* parent;       /* [nodes] parent node, -1 for the root */
    int32_t* skip;         /* [nodes] first node after the subtree (pre-order) */
    uint32_t* corner;      /* [nodes*3] cube corner in integer coordinates */
    double* M;             /* [nodes] mass */
    double* com;           /* [nodes*3] centre of mass */
    float* M32;            /* [nodes] (float)M */
    uint32_t* comX;        /* [nodes*3] rint(com / L * 2^32) mod 2^32 */
    double* side;          /* [nodes] cube side the opening tests use: the cell side
                              L 2^-level, or after tree_drift twice the grown half side */
} sr_tree_export;

int tree_node_count(const sr_tree* tree, int64_t* n_nodes);

/* Work statistics of the handle's last walk (HOST int64[4]): node-target
 * opening tests, 64-entry list chunks, evaluation units, targets. */
int tree_walk_stats(const sr_tree* tree, int64_t* stats);
int tree_export(const sr_tree* tree, const sr_tree_export* out, void* stream);

/* Frees the handle and its device workspace (NULL is allowed). */
void tree_free(sr_tree* tree);

/* Message of the last failed call on this thread ("" if none). */
const char* srgrav_last_error(void);

/*
 * PM long-range force -- the mesh half of the TreePM split, the complement of
 * the short-range erfc force above (the paper computes it on the host with
 * FFTW, Sec. 3.1; the scheme is Gadget-2's periodic PM):
 *
 *   rho   = CIC assignment of the masses to an n_mesh^3 periodic mesh (mesh
 *           points at (i, j, k) L / n_mesh), mass per cell / h^3
 *   phi^  = -4 pi G rho^ exp(-k^2 r_s^2) / k^2 / W(k)^2,  phi^(0) = 0,
 *           W(k) = prod_d sinc(pi n_d / n_mesh)^2 the CIC window
 *   phi   = inverse transform of phi^ on the mesh
 *   F_d   = -dphi/dx_d on the mesh by the fourth-order central difference
 *           [8 (phi(i - e_d) - phi(i + e_d)) - (phi(i - 2 e_d) - phi(i + 2 e_d))] / 12h
 *   a_i   = CIC interpolation of F at particle i (the assignment weights)
 *
 * The two 3D FFTs are hipFFT's; everything else is this library's kernels.
 *
 * pm_create -- mesh workspace (about 16 n_mesh^3 bytes plus hipFFT's work
 *   area) and FFT plans on the
 *   current device.  n_mesh even, in [2, 2048].  *pm is NULL on failure.
 */
typedef struct sr_pm sr_pm;
int pm_create(int32_t n_mesh, sr_pm** pm);

/*
 * pm_accel -- long-range accelerations of all n particles.
 *
 *   pos   DEVICE double[n*3]  positions (any real values, wrapped into the box; a
 *                             non-finite coordinate is taken as 0, not reported)
 *   mass  DEVICE double[n]
 *   acc   DEVICE double[n*3]  output, input order, overwritten
 *   box   L > 0;  r_s the split scale (> 0), the same as the short-range call's
 *
 * Work is enqueued on `stream`; the host does not wait.  The mass assignment
 * uses device atomics, so the low bits may differ from run to run.  Calls on
 * one handle must not overlap (the mesh is shared).  SR_ESTATE for a handle of
 * another device.
 */
int pm_accel(sr_pm* pm, const double* pos, const double* mass, int64_t n, double box, double r_s,
             double G, double* acc, void* stream);

/*
 * pm_accel_adjoint -- gradient of L = sum_i w_i . a_i, a the pm_accel
 * accelerations of the same arguments, with respect to the positions and the
 * masses.  With W_j(c) the CIC weights, D_d the difference rule above (an odd
 * operator) and K the filtered Green's convolution (a symmetric one):
 *
 *   omega_d = sum_i w_i,d W_i        (the weights assigned to the mesh)
 *   psi     = -K sum_d D_d omega_d
 *   dmass_j = sum_c W_j(c) psi(c) / h^3
 *   dpos_j  = sum_d w_j,d sum_c grad W_j(c) F_d(c) + m_j / h^3 sum_c grad W_j(c) psi(c)
 *
 * grad W is the derivative inside a mesh cell (the CIC weights are piecewise
 * linear); the second term of dpos is particle j as a source, the first as a
 * target.
 *
 *   w      DEVICE double[n*3]  the cotangent of acc
 *   dpos   DEVICE double[n*3]  output dL/dpos, overwritten
 *   dmass  DEVICE double[n]    output dL/dmass, overwritten
 *
 * The other arguments, the stream and the host behaviour are pm_accel's.  The
 * first call on a handle allocates two more n_mesh^3 meshes (16 n_mesh^3 bytes),
 * kept until pm_free; SR_ENOMEM if that fails.
 */
int pm_accel_adjoint(sr_pm* pm, const double* pos, const double* mass, int64_t n, double box, double r_s,
                     double G, const double* w, double* dpos, double* dmass, void* stream);

/* pm_free -- waits for the device and releases the handle (NULL is ignored). */
void pm_free(sr_pm* pm);

/*
 * sph_density -- SPH smoothing lengths and densities of the particles of a
 * built tree (the paper's density module iterates each smoothing length to a
 * fixed neighbour number, Sec. 2; the definitions are Gadget-2's):
 *
 *   W(r, h) = 8 / (pi h^3) w(r/h),  w(q) = 1 - 6q^2 + 6q^3 (q <= 1/2),
 *             2 (1 - q)^3 (1/2 < q <= 1), 0 beyond      (cubic spline, support h)
 *   rho_i(h) = sum_j m_j W(|x_j - x_i|, h)               (all j, self included,
 *                                                         minimum image)
 *   N_i(h)   = (4 pi / 3) h^3 rho_i(h) / m_i
 *
 * h_i is the root of N_i(h) = n_ngb (unique: N_i is strictly increasing once a
 * neighbour lies within h), found by safeguarded Halley iterations (in h^3) to
 * |N_i - n_ngb| <= 1e-13 n_ngb or a closed bracket, or ended by a bracketed
 * Halley step taken from |N_i - n_ngb| <= 1e-5 n_ngb (whose error is of the
 * order of the cube of that); rho_i = rho_i(h_i), which at the root is
 * 3 n_ngb m_i / (4 pi h_i^3).
 *
 *   tree         built by tree_build; its positions, masses and box are used
 *   n_ngb        the neighbour number, finite and > 32/3 (the particle alone)
 *   h, rho       DEVICE double[n] outputs, input order, overwritten
 *   unconverged  HOST int64 (may be NULL): particles without a root below L/4
 *                (or with mass <= 0), whose h is L/4 (or the last iterate)
 *
 * Neighbours are gathered per group of 64 Morton-consecutive particles into
 * candidate lists that are kept across iterations while the group's smoothing
 * lengths stay within the gathered radius.  The host waits once per iteration
 * (at most 100) for an event behind the copy of a few counters to the handle's
 * pinned read-back buffer, which the walk entry points use too: calls on one
 * handle must not overlap.  The workspace (about 36 bytes per particle plus
 * the candidate lists, grown on demand) comes from the stream-ordered allocator
 * and is released before the call returns; the sums are deterministic.
 */
int sph_density(sr_tree* tree, double n_ngb, double* h, double* rho, int64_t* unconverged, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* SRGRAV_H */
