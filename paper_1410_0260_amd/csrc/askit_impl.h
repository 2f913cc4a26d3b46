// Internal declarations of the gfx950 ASKIT library: the handle, device
// helpers shared by the kernel files, and the host-side launchers.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <functional>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/askit.h"

namespace askit {

// ---------------------------------------------------------------- errors
struct Error {
    askit_status code;
    std::string msg;
};

[[noreturn]] void fail(askit_status code, const std::string &msg);
void hip_check(hipError_t e, const char *what);
#define HIPC(x) ::askit::hip_check((x), #x)

// ---------------------------------------------------------------- working memory
// Stream-ordered working buffers.  Inside an ArenaScope (a setup holding the
// device's working-memory arena) ws_alloc bumps an offset in the arena and
// ws_free of an arena buffer does nothing; the scope resets the arena when it
// ends.  Elsewhere, and for what does not fit, they are hipMallocAsync and
// hipFreeAsync.  The arena is one allocation per device that grows (up to
// ARENA_CAP) to what the largest setup asked for and is kept for the
// process; one setup at a time holds it (the others allocate as usual).
constexpr size_t ARENA_CAP = 16ull << 30;
hipError_t ws_alloc(void **p, size_t bytes, hipStream_t s);
hipError_t ws_free(void *p, hipStream_t s);
template <typename T>
inline hipError_t ws_alloc(T **p, size_t bytes, hipStream_t s)
{
    return ws_alloc(reinterpret_cast<void **>(p), bytes, s);
}
struct ArenaScope {
    explicit ArenaScope(hipStream_t s);
    ~ArenaScope();
    ArenaScope(const ArenaScope &) = delete;
    ArenaScope &operator=(const ArenaScope &) = delete;
    hipStream_t stream;
    int dev = -1;
    bool held = false;
    char *base = nullptr;
    size_t cap = 0, off = 0, need = 0;
};

// ---------------------------------------------------------------- sizes
constexpr int WAVE = 64;
constexpr int SLAB = 64;           // target rows per evaluation work item (one bit per row)
constexpr int KNN_CAND = 64;       // candidates kept per row by the approximate pass
constexpr int MAX_RHS = 64;

inline int round_up(int x, int a) { return (x + a - 1) / a * a; }

// ---------------------------------------------------------------- device helpers
// Canonical squared distance: FP64, increasing k, no fused multiply-add.
// Rows are 16-byte aligned (stride dp, a multiple of 16), so they are read
// four coordinates at a time; the sum still runs over k in order.
__device__ __forceinline__ double canon_sqdist(const float *a, const float *b, int d)
{
#pragma clang fp contract(off)
    double s = 0.0;
    int k = 0;
    for (; k + 4 <= d; k += 4) {
        const float4 x = *reinterpret_cast<const float4 *>(a + k);
        const float4 y = *reinterpret_cast<const float4 *>(b + k);
        double t;
        t = (double)x.x - (double)y.x;
        s += t * t;
        t = (double)x.y - (double)y.y;
        s += t * t;
        t = (double)x.z - (double)y.z;
        s += t * t;
        t = (double)x.w - (double)y.w;
        s += t * t;
    }
    for (; k < d; ++k) {
        double t = (double)a[k] - (double)b[k];
        s += t * t;
    }
    return s;
}

__device__ __forceinline__ double canon_sqdist_c(const float *a, const double *c, int d)
{
#pragma clang fp contract(off)
    double s = 0.0;
    int k = 0;
    for (; k + 4 <= d; k += 4) {
        const float4 x = *reinterpret_cast<const float4 *>(a + k);
        double t;
        t = (double)x.x - c[k];
        s += t * t;
        t = (double)x.y - c[k + 1];
        s += t * t;
        t = (double)x.z - c[k + 2];
        s += t * t;
        t = (double)x.w - c[k + 3];
        s += t * t;
    }
    for (; k < d; ++k) {
        double t = (double)a[k] - c[k];
        s += t * t;
    }
    return s;
}

// Order-preserving map of a double onto uint64 (total order for non-NaN).
__device__ __forceinline__ uint64_t dkey(double x)
{
    uint64_t b = (uint64_t)__double_as_longlong(x);
    return (b >> 63) ? ~b : (b | 0x8000000000000000ull);
}

// ---------------------------------------------------------------- tree node
struct Node {
    int32_t lo, hi, level, parent, left, right;
    int64_t path;
};
static_assert(sizeof(Node) == sizeof(askit_node), "node layout");

// ---------------------------------------------------------------- handle
struct Buf {
    void *p = nullptr;
    size_t bytes = 0;
};

struct Slab {              // SLAB consecutive tree positions of one leaf
    int32_t row0, nrows, leaf, pad;
};

// Weights of one evaluation: W in tree order and the skeleton weights.
struct WeightSet {
    float *Wt = nullptr;       // N x R
    float *Wsk = nullptr;      // nn x smax x R
    float *part = nullptr;     // npairs x R partial sums of the evaluation
    int R = 0;
};

// Evaluation work item: up to 64 targets of one source node.
struct Chunk {
    int32_t node;
    int32_t kind;              // 0: near (the leaf's points), 1: far (the skeleton); + 2 x instance (batch)
    int32_t first, count;      // pairs [first, first + count) of the pair lists
};

// (target, source node) pairs grouped by source node and kind.
struct PairLists {
    int64_t npairs = 0, nchunk = 0, ntarget = 0;
    int32_t *tpos = nullptr;   // target row of each pair
    int32_t *tslot = nullptr;  // partial-sum slot of each pair
    int32_t *sbase = nullptr;  // ntarget + 1: first slot of each target (slots of a target are contiguous)
    int32_t *snear = nullptr;  // ntarget: first far slot of each target (its near slots come first)
    Chunk *chunks = nullptr;
    int64_t near_lists = 0, far_lists = 0;   // sum over targets of |near(i)| and |far(i)|
};

// Strided samples of the tree-ordered points for neighbour searches of new
// points: level j holds every (8^(L-j))-th position (bf16 hi / lo rows and
// FP32 squared norms copied from the full set), so level 0 is the coarsest
// and each level is a subset of the next.
struct KnnSample {
    static constexpr int MAXL = 10;
    int levels = 0;
    uint16_t *h[MAXL] = {}, *l[MAXL] = {};
    float *n[MAXL] = {};
    int64_t rows[MAXL] = {};
};

}  // namespace askit

struct askit_handle {
    // problem
    int64_t N = 0;
    int d = 0, dp = 0;                 // dp: coordinate stride (d rounded up to 16)
    askit_params prm{};
    int kappa = 0, m = 0, smax = 0, ell = 0, ncol_max = 0;
    int minlev = 0;                    // first level whose nodes may be pruned (level restriction)
    bool varh = false;
    float maxnorm = 0.0f;              // largest FP32 squared norm of the points
    int device = 0;

    // tree (host copy; shape depends only on N and m)
    std::vector<askit::Node> nodes;
    std::vector<std::vector<int>> level_nodes;   // node ids per level
    std::vector<int> leaves;                     // leaf node ids in position order
    int depth = 0;                               // deepest level
    std::vector<askit::Slab> slabs;
    std::vector<int64_t> pslot;                  // per node offset of its P slot (floats)
    int64_t pslot_total = 0;

    // device state (owned)
    std::vector<void *> allocs;
    float *Xo = nullptr;          // N x dp, original order (FP32, zero padded)
    uint16_t *Xh = nullptr, *Xl = nullptr;   // bf16 hi / lo split of Xo (N x dp)
    float *Xn = nullptr;          // FP32 squared norms of Xo rows
    float *Xt = nullptr;          // N x dp, tree order
    float *gt = nullptr;          // per tree position: -log2(e) / (2 h^2)
    double *hsrc = nullptr;       // per original id bandwidth
    int32_t *perm = nullptr, *iperm = nullptr;
    int32_t *knn_idx = nullptr;   // N x kappa original ids
    double *knn_d = nullptr;      // N x kappa
    askit::Node *d_nodes = nullptr;
    int32_t *leaf_of = nullptr;   // per tree position: leaf node id
    int32_t *nl_pos = nullptr;    // nn x ell
    double *nl_key = nullptr;
    int32_t *nl_cnt = nullptr;
    int32_t *T = nullptr, *T_cnt = nullptr;   // nn x ell
    int32_t *S = nullptr, *skk = nullptr;     // nn x smax, nn
    int32_t *colperm = nullptr, *ncols = nullptr;   // nn x ncol_max, nn
    float *P = nullptr;           // pslot_total floats
    int64_t *d_pslot = nullptr;
    float *Xs = nullptr;          // nn x smax x dp skeleton coordinates
    float *gs = nullptr;          // nn x smax skeleton bandwidth factors
    askit::WeightSet ws;          // weights of askit_update_weights / askit_evaluate
    int wcap = 0;                 // columns allocated in ws
    int32_t *up_ids = nullptr;    // non-root node ids, deepest level first
    std::vector<std::pair<int, int>> up_seg;   // (offset, count) per level, bottom-up
    askit::Slab *d_slabs = nullptr;
    int32_t *sl_ptr = nullptr;    // 2*nslab+2: near offsets [0..nslab], far offsets [nslab+1..]
    int32_t *sl_node = nullptr;
    uint64_t *sl_mask = nullptr;
    int64_t near_entries = 0, far_entries = 0;
    askit::PairLists pairs;       // the same pairs grouped by source node (evaluation work)
    askit::KnnSample ksamp;       // query threshold samples (levels == 0: none)

    // diagnostics
    int64_t near_pairs = 0, far_pairs = 0, knn_uncertified = 0;
    double t_knn = 0, t_tree = 0, t_lists = 0, t_skel = 0, t_inter = 0, t_update = 0;
    double t_knn_sweep = 0, t_qr = 0, t_knn_filter = 0;
    int knn_filter_launches = 0, knn_retry_rows = 0;
    int64_t knn_tiles_swept = -1;      // (wave, tile) sweeps of the symmetric sweep; -1: no skipping
    std::vector<int32_t> knn_retry_list;   // their tree positions
    hipEvent_t ev_up0 = nullptr, ev_up1 = nullptr;
    bool up_pending = false;

    ~askit_handle();
    void *alloc(size_t bytes, bool zero = true);
    std::mutex alloc_mu;               // alloc may be called from two host threads during setup
    hipStream_t astream = nullptr;     // stream that orders alloc's zero fill (the calling API's)
    bool skel_pending = false;         // set up without skeletons (a batch's fused pass completes it)
};

namespace askit {

// ---------------------------------------------------------------- launchers
// points.hip
void pack_points(const float *X, int64_t N, int d, int64_t ldx, int dp, float *out, int32_t *bad,
                 hipStream_t s);
void split_bf16(const float *X, int64_t N, int dp, uint16_t *hi, uint16_t *lo, float *nrm,
                hipStream_t s);
void gather_rows(const float *src, const int32_t *idx, int64_t n, int dp, float *dst, hipStream_t s);

// knn.hip -- references are tree-ordered points (positions); idmap maps a
// position to its point id (ties are broken by point id); rowmap maps a query
// row to its output row (NULL = identity).
// candidates + threshold per row; rows that need the exact scan are appended to
// bad_rows (count in *bad_count, device)
void knn_candidates(const uint16_t *Qh, const uint16_t *Ql, const float *Qn, int64_t M,
                    const uint16_t *Xh, const uint16_t *Xl, const float *Xn, int64_t N, int dp,
                    bool exclude_self, bool start_local, int32_t *cand, float *thr,
                    int32_t *bad_rows, int32_t *bad_count, hipStream_t s,
                    float *t_filter_ms = nullptr, int *n_filter = nullptr, int *n_retry = nullptr,
                    const KnnSample *samp = nullptr, std::vector<int32_t> *retry_rows = nullptr,
                    const float *Xf = nullptr, int d = 0, int64_t *tiles_swept = nullptr,
                    int nsel = KNN_CAND);
// Candidates the threshold filter keeps per row for kappa neighbours: enough
// above kappa that the FP64 certificate (the kappa-th exact distance below the
// nsel-th approximate one, less the error bound) holds for most rows, and no
// more, since the threshold sets how many points survive the filter.
inline int knn_nsel(int kappa) { return std::min(KNN_CAND, kappa + std::max(16, kappa / 2)); }
// Fills h->ksamp from the tree-ordered bf16 points when the point set is large
// enough for the sampled query search (allocations owned by the handle).
void knn_build_sample(askit_handle *h, hipStream_t s);
void knn_refine(const float *Q, int64_t M, const float *X, int64_t N, int d, int dp, int kappa,
                const int32_t *cand, const float *thr, const float *Qn, float maxnorm,
                const int32_t *idmap, const int32_t *rowmap, int32_t *idx, double *dist,
                int32_t *bad_rows, int32_t *bad_count, float *tbound, hipStream_t s);
// Exact lists of the rows refine could not certify: threshold sweep at each
// row's bound (tbound), FP64 re-rank of the survivors, full scan for rows whose
// survivors overflow.
void knn_fallback(const float *Q, const uint16_t *Qh, const uint16_t *Ql, const float *Qn, const float *X,
                  const uint16_t *Xh, const uint16_t *Xl, const float *Xn, int64_t N, int d, int dp, int kappa,
                  bool exclude_self, const int32_t *rows, int nrows, const float *tbound, const int32_t *idmap,
                  const int32_t *rowmap, int32_t *idx, double *dist, hipStream_t s);
void knn_exact_rows(const float *Q, const float *X, int64_t N, int d, int dp, int kappa,
                    bool exclude_self, const int32_t *rows, int nrows, const int32_t *idmap,
                    const int32_t *rowmap, int32_t *idx, double *dist, hipStream_t s);
float max_norm(const float *nrm, int64_t N, hipStream_t s);

// tree.hip
void build_tree(askit_handle *h, hipStream_t s);
// refinement of the tree order (leaves split on until cells of <= mfine points)
// used as the sweep order of the neighbour search
void build_fine_order(const askit_handle *h, int mfine, int32_t *perm_f, hipStream_t s);
// nodes visited per target (original order) under neighbour and distance pruning
void prune_visits(const askit_handle *h, int32_t *vk, int32_t *vd, hipStream_t s);
// approximate kappa nearest neighbours by iterated random projection trees
// (Xo: N x dp points, original order); idx/dist: N x kappa, sorted by (distance, id)
void rp_knn(const float *Xo, int64_t N, int d, int dp, int kappa, int leaf, int iters, uint64_t seed,
            int32_t *idx, double *dist, hipStream_t s);

// lists.hip
void build_node_lists(askit_handle *h, hipStream_t s);
void sample_rows(askit_handle *h, hipStream_t s);
void build_interactions(askit_handle *h, hipStream_t s);
// algorithmic (target, source) pair counts of one evaluation (needs the skeleton sizes)
void count_pairs(askit_handle *h, hipStream_t s);
// query lists: nb is M x kappa neighbour positions; slabs of consecutive queries
// query lists: nb is M x kappa neighbour positions (sorted queries); slabs of
// consecutive queries that stay within one segment (segs: segment lengths,
// NULL = one segment); nslab receives their number
void build_query_interactions(askit_handle *h, const int32_t *nb, int64_t M, Slab *&slabs,
                              int32_t *&ptr, int32_t *&node, uint64_t *&mask, int64_t &ne_near,
                              int64_t &ne_far, std::vector<void *> &tmp, hipStream_t s,
                              const std::vector<int64_t> *segs, int64_t &nslab);

void gather_f64(const double *src, const int32_t *idx, int64_t n, double *dst, hipStream_t s);

// queries sorted by (segment, leaf of the nearest source, index): order[M],
// nb rows permuted; seg (device, M) gives each query's segment (NULL: one)
void sort_queries(askit_handle *h, const int32_t *nb, int64_t M, int32_t *order, int32_t *nb_sorted,
                  std::vector<void *> &tmp, hipStream_t s, const int32_t *seg = nullptr);

// skel.hip
void skeletonize(askit_handle *h, hipStream_t s);
// Ascending bitonic sort of n2 (a power of two) 64-bit keys in place.
void sort_u64_pow2(uint64_t *key, int64_t n2, hipStream_t s);
// The skeletons of several handles (same ell, s_max and tolerance) in one
// pass over the tree levels: each kernel launched once per level for the
// nodes of every handle.
void skeletonize_multi(const std::vector<askit_handle *> &hs, hipStream_t s);
// askit_setup up to (not including) the skeletons; finish_deferred completes
// a handle after its skeletons are built.  Throws Error.
askit_handle *setup_deferred(const float *X, int64_t N, int32_t d, int64_t ldx, const askit_params *p,
                             hipStream_t s);
void finish_deferred(askit_handle *h, hipStream_t s);

// A handle's arrays as the skeletonization kernels read them (one entry per
// handle; work items are (entry, node) pairs).
struct SkelInst {
    const Node *nodes;
    const float *Xt, *gt;
    const int32_t *T, *T_cnt;
    int32_t *S, *skk, *ncols, *colperm;
    const int64_t *pslot;
    float *P, *Xs, *gs;
    const double *hpos;        // per tree position bandwidth (variable h), else NULL
    double h;                  // the fixed bandwidth
    int dp, d, ncol_max;       // ncol_max: the handle's column bound (row stride of colperm)
};
// columns [r0, r1) of ws (r1 < 0: all); no host sync
void upward(askit_handle *h, const WeightSet &ws, hipStream_t s, int r0 = 0, int r1 = -1);
void prepare_upward(askit_handle *h);                                  // once, after setup
void permute_weights(askit_handle *h, const float *W, int64_t ldw, WeightSet &ws, hipStream_t s);
// W (N x rb, original order) into columns [c0, c0 + rb) of Wt (tree order, row stride ldt)
void permute_weight_cols(askit_handle *h, const float *W, int64_t ldw, int rb, float *Wt, int ldt, int c0,
                         hipStream_t s);

// eval.hip
// Pair lists of the targets described by slab lists (ptr: near offsets
// [0..nslab], far offsets [nslab+1 .. 2 nslab + 1] into node/mask); `al`
// allocates the outputs (persistent or temporary).
// With nseg > 1 the slabs carry their segment in `pad`, and no chunk mixes
// targets of two segments (a served request's result then does not depend on
// the requests batched with it).
void build_pairs(const askit_handle *h, const Slab *d_slabs, int64_t nslab, int64_t ntarget, const int32_t *ptr,
                 const int32_t *node, const uint64_t *mask, int64_t ne_near, int64_t ne_far, PairLists &L,
                 const std::function<void *(size_t)> &al, hipStream_t s, int64_t nseg = 1);
// u at the targets Y (rows of stride dp) for the weights ws: partial sums per
// pair slot into part (>= npairs x R floats), then per-target sums into
// U[outmap[i]] (identity when NULL).
void evaluate(const askit_handle *h, const WeightSet &ws, const float *Y, const PairLists &L,
              const int32_t *outmap, float *U, int64_t ldu, float *part, hipStream_t s,
              float *Unear = nullptr, int64_t ldun = 0);

// The evaluation's chunks [ch0, ch1) for the weight columns [c0, c1) of ws
// (row stride ws.R): their pair slots of part (row stride ws.R).
void evaluate_chunk_range(const askit_handle *h, const WeightSet &ws, const PairLists &L, int64_t ch0, int64_t ch1,
                          int c0, int c1, float *part, hipStream_t s);
// Per-target sums of the slot columns [c0, c0 + rb) of part (row stride R) into
// U[outmap[i]] columns [0, rb).
void sum_slot_cols(const askit_handle *h, const PairLists &L, const float *part, int R, int c0, int rb,
                   const int32_t *outmap, float *U, int64_t ldu, hipStream_t s);

// ---------------------------------------------------------------- batched form
// One entry per instance of a batch (device tables).  Weights of all
// instances live in shared buffers: the instance's tree-order weights start
// at row wt_off (times R) and its skeleton weights at slot wsk_off (times R).
struct EvalInst {
    const Node *nodes;
    const float *Y, *Xt, *gt, *Xs, *gs;
    const int32_t *skk;
    int64_t wt_off, wsk_off;
    int smax, dp;
};
struct UpInst {
    const Node *nodes;
    const int32_t *skk, *ncols, *colperm;
    const int64_t *pslot;
    const float *P;
    int64_t wt_off, wsk_off;
    int ncol_max, smax;
};
struct BatchEvalArgs {
    const EvalInst *inst;
    const Chunk *chunks;       // kind = 2 x instance + kind
    int64_t nchunk;
    const int32_t *tpos, *tslot;   // tpos: row in the instance's targets; tslot: batch-wide slot
    const int32_t *sbase;      // batch rows + 1
    const int32_t *outrow;     // batch output row of each batch tree row
    int64_t rows;
    const float *Wt, *Wsk;
    float *part;
    float *U;
    int64_t ldu;
    int R;
    bool bf;
    int persistent;            // 0: one workgroup per chunk; else the persistent grid size
    int32_t *queue;            // persistent: work counter (cleared by a kernel before the launch)
    int plan;                  // column passes: 0 wide (64/32 MFMA, 4/1 vector), 1 narrow (32 MFMA, 1 vector)
};
void evaluate_batch(const BatchEvalArgs &b, hipStream_t s);
// One launch per level (deepest first): items are (instance, node) pairs.
void upward_batch(const UpInst *inst, const int2 *items, const std::vector<std::pair<int64_t, int64_t>> &levels,
                  int smax, const float *Wt, float *Wsk, int R, hipStream_t s);
// Wt[t, r] = W[gperm[t], r] over all rows of a batch (gperm: original row of tree row t).
void permute_rows(const float *W, int64_t ldw, const int32_t *gperm, int64_t rows, int R, float *Wt,
                  hipStream_t s);
// queries at M new points against the weights ws (U: M x ws.R, row stride ldu);
// segs: lengths of consecutive independent requests (NULL = one)
void query_points(askit_handle *h, const WeightSet &ws, const float *Y, int64_t M, int64_t ldy,
                  float *U, int64_t ldu, hipStream_t s, const std::vector<int64_t> *segs = nullptr);

}  // namespace askit
