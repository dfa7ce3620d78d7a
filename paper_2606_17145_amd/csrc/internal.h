// Internal data layout of the short-range gravity library (device side and handle).
//
// Particle data live in Morton order ("sorted position" s); nodes of the
// compressed octree live in pre-order.  The walk reads a single combined
// pre-order "item" sequence in which every internal node is followed by its
// children -- particles and nodes interleaved in digit order -- so that one
// forward scan with skip pointers visits exactly what a depth-first walk
// visits.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "srgrav.h"

// Sorted particle record, FP64 path: wrapped position and mass (32 B).
struct Rec64 {
    double x, y, z, m;
};

// Sorted particle / node record, FP32 path: integer position and FP32 mass (16 B).
struct Rec32 {
    uint32_t X, Y, Z;
    float m;
};

// Node geometry for FP64 decisions: cube centre and side.
struct Geo64 {
    double cx, cy, cz, l;
};

// Everything the walk reads about one node, packed into one 128-byte line
// (written by the build after the moments): decision data and child table.
struct alignas(16) WalkRec32 {
    uint32_t cX, cY, cZ, tin;     // cube centre (ticks), 0.6 side rounded down (ticks)
    uint32_t X, Y, Z, l2;         // centre of mass (ticks), side^2 (float bits, ticks^2)
    uint32_t half, M, hx, mixed;  // half side, mass, h_max (float bits), mixed softening flag
    uint32_t meta, r0, r1, r2;    // child count or META_BUCKET
    uint32_t kids[8];
    uint32_t pad[8];
};
struct alignas(16) WalkRec64 {
    double cx, cy, cz, l;         // cube centre and side
    double X, Y, Z, M;            // centre of mass and mass
    double hx, hn;                // largest and smallest support h below the node
    uint32_t meta, r0, r1, r2;    // child count or META_BUCKET
    uint32_t kids[8];
};
static_assert(sizeof(WalkRec32) == 128 && sizeof(WalkRec64) == 128, "one line per node");

// One entry of the combined pre-order sequence.
//   ref:   node index, or (sorted particle position | ITEM_PARTICLE)
//   next:  item index after this entry's subtree
//   depth: depth below the root (root = 0)
struct Item {
    uint32_t ref;
    uint32_t next;
    uint32_t depth;
    uint32_t pad;
};

#define ITEM_PARTICLE 0x80000000u
// node meta word: number of children (<= 8), or META_BUCKET for a level-30 bucket
// whose children are the particles kids[0] .. kids[0] + kids[1] - 1
#define META_BUCKET 0x100u
#define SR_MAX_DEPTH 32
#define SR_N_MAX (int64_t(1) << 30)

// Device status words written by the build and read back once per build.
enum {
    ST_FLAGS = 0,      // bit 0: non-finite / non-positive input
    ST_NODES = 1,      // number of internal nodes
    ST_MAXDEPTH = 2,   // deepest node depth
    ST_WORDS = 3,      // the words read back by the host
    // tree-key sort: digit totals of its 12 passes (256 each), then its tile tickets
    ST_RS_HIST = 4,
    ST_RS_TICKET = ST_RS_HIST + 12 * 256,
    ST_ALLOC = ST_RS_TICKET + 16   // words allocated and cleared at the start of a build

};

// What a traversal's lists were made for.  `token` names them: shortrange_accel
// hands it to the caller, and the adjoint reuses these lists (and the targets they
// were made for) only when it is given the same token and the same decision
// parameters; any later target preparation or traversal invalidates it.
struct ListKey {
    bool valid = false;
    int64_t token = 0;
    int64_t gen = -1;
    int dec64 = 0;
    double G = 0, r_s = 0, r_cut = 0, theta = 0, alpha = 0;
    int criterion = 0;
    int64_t n_t = 0;
};

struct sr_tree {
    int64_t n = 0;            // particles in the current tree
    int64_t cap = 0;          // particle capacity of the workspace
    double box = 1.0;
    int device = 0;

    // build workspace (cap)
    uint64_t *khi[2] = {}, *klo[2] = {};
    uint32_t* kidx[2] = {};
    uint32_t* hist = nullptr;         // radix histograms / offsets
    uint32_t* scan_tmp = nullptr;     // block sums of the scans
    uint32_t* levelmask = nullptr;    // levels of the nodes starting at each sorted position
    uint32_t* ucount = nullptr;       // per-position counts for the scans
    int32_t* base = nullptr;          // (cap+1) nodes with first < s
    int32_t *b_lo = nullptr, *b_hi = nullptr, *b_lambda = nullptr, *b_parent = nullptr;
    int32_t* b_pre = nullptr;         // pre-order index, -1 if not an octree node
    int32_t* leaf_bparent = nullptr;
    int32_t* status = nullptr;        // ST_ALLOC
    uint64_t* rs_status = nullptr;    // tree-key sort: per tile and digit, look-back word
    uint32_t rs_epoch = 0;            // tags of the look-back words of the last sort
    // pinned host copies of the status words and of the list counters, and the
    // events recorded after those copies: the host waits for these points only
    int32_t* h_status = nullptr;      // ST_WORDS
    int32_t* h_counters = nullptr;    // 8
    hipEvent_t ev_status = nullptr, ev_counters = nullptr;

    // tree (particles: cap, nodes: cap - 1, items: 2 cap)
    int32_t *perm = nullptr, *invperm = nullptr, *pparent = nullptr;
    Rec64* prec64 = nullptr;
    double* ph64 = nullptr;           // spline support h = 2.8 eps
    Rec32* prec32 = nullptr;
    float* ph32 = nullptr;            // h in integer-coordinate units
    int32_t *n_level = nullptr, *n_first = nullptr, *n_count = nullptr, *n_parent = nullptr,
            *n_skip = nullptr, *n_depth = nullptr;
    uint32_t* n_corner = nullptr;
    Rec64* nrec64 = nullptr;          // centre of mass and mass
    double* nS = nullptr;             // first moments (3 per node)
    Geo64* ngeo64 = nullptr;
    double *nhmax = nullptr, *nhmin = nullptr;
    Rec32* nrec32 = nullptr;
    float* nhmax32 = nullptr;
    Item* items = nullptr;
    uint32_t* n_kids = nullptr;       // 8 per node: children (node index or particle | ITEM_PARTICLE)
    uint32_t* n_meta = nullptr;
    WalkRec32* wrec32 = nullptr;      // per node, for the walk
    WalkRec64* wrec64 = nullptr;
    // node drift (allocated at the first drift): the built particle records, and
    // per node the bounding box of its particles (lo xyz, hi xyz)
    Rec64* prec64_0 = nullptr;
    double* nbox = nullptr;
    bool drift_base = false;          // prec64_0 holds the current build's records

    // walk workspace (cap)
    int32_t *tgt_sorted = nullptr, *tgt_slot = nullptr, *mark = nullptr;
    uint32_t* tgt_flag = nullptr;
    int32_t* tgt_pos = nullptr;       // (cap+1)
    // adjoint workspace
    double* pbar = nullptr;           // 4 per particle (x, y, z, m) source terms
    double* tbar = nullptr;           // 3 per particle target terms
    double* nbar = nullptr;           // 4 per node

    // interaction lists of the last traversal (capacity-managed)
    int64_t cap_chunks = 0, cap_units = 0, cap_groups = 0;
    uint32_t* ent_src = nullptr;      // 64 per chunk
    uint64_t* ent_mask = nullptr;
    int32_t *chunk_next = nullptr, *chunk_cnt = nullptr;
    int32_t *unit_group = nullptr, *unit_chunk = nullptr, *unit_nch = nullptr, *unit_next = nullptr;
    int32_t* group_head = nullptr;
    int32_t* list_counters = nullptr;  // chunks, units, overflow, -, node tests (u64 at [4])
    char* partials = nullptr;          // per unit
    uint32_t* frontier = nullptr;      // per traversal wave: 2 x cap_front node ids + 2 x cap_front masks
    int64_t cap_front = 0, n_front_waves = 0;
    int64_t n_units = 0, n_chunks = 0, n_tests = 0;
    int64_t unit_hint = 0;             // unit count expected from the previous traversal
    ListKey lkey;
    int64_t list_serial = 0;           // last token issued on this handle
    int64_t build_gen = 0;

    // host mirrors
    int64_t n_nodes = 0;
    bool mixed_soft = false;      // softening lengths differ between particles
    int max_depth = 0;
};

// error helpers shared by the host files
int sr_fail(int code, const char* fmt, ...);
#define SR_HIP(call)                                                                   \
    do {                                                                               \
        hipError_t e_ = (call);                                                        \
        if (e_ != hipSuccess)                                                          \
            return sr_fail(SR_EHIP, "%s failed: %s", #call, hipGetErrorString(e_));   \
    } while (0)

// build.hip: move the particles of a built tree to their built positions plus
// disp (input order) and refold the moments and node cubes; topology kept
int sr_drift_device(sr_tree* t, const double* disp, hipStream_t st);
// build.hip
int sr_build_device(sr_tree* t, const double* pos, const double* mass, const double* eps,
                    double eps_scalar, hipStream_t st);
int sr_scan_exclusive(const uint32_t* in, uint32_t* out, int64_t n, uint32_t* tmp, hipStream_t st);
// build.hip: look-back words the tree-key sort needs for a capacity of cap keys
int64_t sr_tree_sort_status_words(int64_t cap);

// walk.hip
int sr_prepare_targets(sr_tree* t, const int32_t* active, int64_t n_active, hipStream_t st);
int sr_walk_forward(sr_tree* t, const sr_params* p, int64_t n_t, const int32_t* active, const double* a_old,
                    void* acc, int32_t* counts, hipStream_t st);
int sr_walk_adjoint(sr_tree* t, const sr_params* p, int64_t n_t, const int32_t* active, const double* a_old,
                    const void* w, double* dLdx, double* dLdm, int64_t list_token, hipStream_t st);
// walk.hip: the forward with its lists in the fixed scratch buffer (allocates nothing)
int sr_walk_forward_noalloc(sr_tree* t, const sr_params* p, int64_t n_t, const int32_t* active, const double* a_old,
                            void* acc, int32_t* counts, hipStream_t st);
// walk.hip: SR_OK if `token` names the handle's current lists and they were made
// with the decision parameters of `p` for n_t targets, else an error code
int sr_check_list_token(const sr_tree* t, const sr_params* p, int64_t n_t, int64_t token);

// walk.hip: elementwise y += a x
int sr_axpy_device(void* y, int y_type, const void* x, int x_type, double a, int64_t n, hipStream_t st);

// api.hip: phase timing (HIP events around launches while enabled)
bool sr_timing_on();
void sr_timing_mark(int phase, bool start, hipStream_t st);

// api.hip: make room for the lists of `groups` target groups, `chunks` chunks and `units`
// units (waits for stream st before it frees smaller lists)
int sr_list_reserve(sr_tree* t, int64_t groups, int64_t chunks, int64_t units, hipStream_t st);
// api.hip: frontier scratch of `waves` persistent traversal waves, `cap` entries per level
int sr_front_reserve(sr_tree* t, int64_t waves, int64_t cap, hipStream_t st);
// api.hip: every device allocation of the library (hipMalloc, or the injected failure
// of srgrav_inject_alloc_failure)
hipError_t sr_device_malloc(void** p, size_t bytes);
