// C ABI of the library: argument checks, host orchestration of the setup
// phases (Alg. 5), the upward pass, evaluation and queries.
#include "askit_impl.h"

#include <algorithm>
#include <cstdlib>
#include <chrono>
#include <cmath>
#include <cstring>
#include <memory>
#include <exception>
#include <new>
#include <thread>

using namespace askit;

namespace askit {

// ---------------------------------------------------------------- working-memory arena
namespace {
struct ArenaState {
    std::mutex mu;                 // held by the setup using the arena
    char *base = nullptr;
    size_t cap = 0;
};
ArenaState g_arena[64];
thread_local ArenaScope *tl_scope = nullptr;
constexpr size_t ARENA_ALIGN = 256;
}  // namespace

ArenaScope::ArenaScope(hipStream_t s) : stream(s)
{
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64 || tl_scope) return;
    if (!g_arena[dev].mu.try_lock()) return;
    held = true;
    base = g_arena[dev].base;
    cap = g_arena[dev].cap;
    tl_scope = this;
}

ArenaScope::~ArenaScope()
{
    if (!held) return;
    tl_scope = nullptr;
    // the setup's kernels are done with the arena before the next one takes
    // it (its stream is already idle on success; after an error it is waited
    // for here)
    (void)hipStreamSynchronize(stream);
    ArenaState &A = g_arena[dev];
    const size_t want = std::min(ARENA_CAP, need);
    if (want > A.cap) {
        // grow for the next setup to what this one asked for
        if (A.base) (void)hipFree(A.base);
        A.base = nullptr;
        A.cap = 0;
        void *nb = nullptr;
        if (hipMalloc(&nb, want) == hipSuccess) {
            A.base = (char *)nb;
            A.cap = want;
        } else {
            (void)hipGetLastError();           // no arena: later setups allocate as before
        }
    }
    A.mu.unlock();
}

hipError_t ws_alloc(void **p, size_t bytes, hipStream_t s)
{
    ArenaScope *u = tl_scope;
    if (u) {
        const size_t b = (std::max<size_t>(bytes, 1) + ARENA_ALIGN - 1) / ARENA_ALIGN * ARENA_ALIGN;
        u->need += b;
        if (u->base && u->off + b <= u->cap) {
            *p = u->base + u->off;
            u->off += b;
            return hipSuccess;
        }
    }
    return hipMallocAsync(p, bytes, s);
}

hipError_t ws_free(void *p, hipStream_t s)
{
    int dev = 0;
    if (p && hipGetDevice(&dev) == hipSuccess && dev >= 0 && dev < 64) {
        // arena buffers are released with their scope (the range is only
        // read here while the scope's thread holds the arena)
        const ArenaScope *u = tl_scope;
        if (u && u->base && (const char *)p >= u->base && (const char *)p < u->base + u->cap) return hipSuccess;
    }
    return hipFreeAsync(p, s);
}

thread_local std::string g_err;

void fail(askit_status code, const std::string &msg) { throw Error{code, msg}; }

void hip_check(hipError_t e, const char *what)
{
    if (e == hipSuccess) return;
    askit_status c = (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) ? ASKIT_ERR_OUT_OF_MEMORY
                                                                              : ASKIT_ERR_DEVICE;
    fail(c, std::string(what) + ": " + hipGetErrorString(e));
}

__global__ void k_gather_f64(const double *__restrict__ src, const int32_t *__restrict__ idx, int64_t n,
                             double *__restrict__ dst)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = src[idx[i]];
}

void gather_f64(const double *src, const int32_t *idx, int64_t n, double *dst, hipStream_t s)
{
    if (n == 0) return;
    hipLaunchKernelGGL(k_gather_f64, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, src, idx, n, dst);
    HIPC(hipGetLastError());
}

// Bandwidth per source: fixed h, or the distance to the b-th neighbour.
__global__ void k_bandwidth(const double *__restrict__ knn_d, int64_t N, int kappa, int b, double h,
                            double *__restrict__ hs, int32_t *bad)
{
    int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= N) return;
    double v = b > 0 ? sqrt(knn_d[j * kappa + (b - 1)]) : h;
    if (!(v > 0.0)) atomicOr(bad, 1);
    hs[j] = v;
}

// g = -log2(e) / (2 h^2) per tree position (FP32 exponent factor of exp2).
// list[i] <- ip[p[list[i]]] (a row of one order as a position of another)
__global__ void k_map_rows(int32_t *__restrict__ list, int64_t n, const int32_t *__restrict__ p,
                           const int32_t *__restrict__ ip)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) list[i] = ip[p[list[i]]];
}

__global__ void k_gfactor(const double *__restrict__ hs, const int32_t *__restrict__ perm, int64_t N,
                          float *__restrict__ g)
{
    int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= N) return;
    double h = hs[perm[p]];
    g[p] = (float)(-1.4426950408889634 / (2.0 * h * h));
}

__global__ void k_leaf_of(const Node *__restrict__ nodes, const int32_t *__restrict__ leaves, int nl,
                          int32_t *__restrict__ leaf_of)
{
    int q = blockIdx.x;
    if (q >= nl) return;
    Node nd = nodes[leaves[q]];
    for (int p = nd.lo + threadIdx.x; p < nd.hi; p += blockDim.x) leaf_of[p] = leaves[q];
}

__global__ void k_permute_w(const float *__restrict__ W, int64_t ldw, const int32_t *__restrict__ perm,
                            int64_t N, int R, float *__restrict__ Wt)
{
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t p = t / R;
    if (p >= N) return;
    int r = (int)(t - p * R);
    Wt[t] = W[(int64_t)perm[p] * ldw + r];
}

__global__ void k_map_pos(const int32_t *__restrict__ ids, int64_t n, const int32_t *__restrict__ iperm,
                          int32_t *__restrict__ out)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = iperm[ids[i]];
}

// Neighbour lists given by the caller (ASKIT takes N(X) as an input, Alg. 5):
// per row, validate the kappa ids (in range, not the row itself, distinct),
// compute their canonical FP64 squared distances and store the row sorted by
// (distance, id).  Xo holds the points in original order (stride dp).
__global__ void k_knn_import(const int32_t *__restrict__ in, int64_t ldk, int64_t N, int kappa,
                             const float *__restrict__ Xo, int dp, int d, int32_t *__restrict__ idx,
                             double *__restrict__ dist, int32_t *__restrict__ bad)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    int32_t li[64];
    double ld[64];
    bool ok = true;
    for (int t = 0; t < kappa; ++t) {
        const int32_t j = in[i * ldk + t];
        if (j < 0 || j >= N || j == i) {
            ok = false;
            li[t] = 0;
            ld[t] = 0.0;
            continue;
        }
        const double D = canon_sqdist(Xo + i * dp, Xo + (int64_t)j * dp, d);
        int q = t;
        while (q > 0 && (ld[q - 1] > D || (ld[q - 1] == D && li[q - 1] > j))) {
            ld[q] = ld[q - 1];
            li[q] = li[q - 1];
            --q;
        }
        ld[q] = D;
        li[q] = j;
    }
    for (int t = 1; t < kappa && ok; ++t)
        if (li[t] == li[t - 1]) ok = false;
    if (!ok) atomicOr(bad, 1);
    for (int t = 0; t < kappa; ++t) {
        idx[i * kappa + t] = li[t];
        dist[i * kappa + t] = ld[t];
    }
}

void permute_rows(const float *W, int64_t ldw, const int32_t *gperm, int64_t rows, int R, float *Wt,
                  hipStream_t s)
{
    const int64_t tot = rows * R;
    if (tot == 0) return;
    hipLaunchKernelGGL(k_permute_w, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, W, ldw, gperm, rows,
                       R, Wt);
    HIPC(hipGetLastError());
}

void permute_weights(askit_handle *h, const float *W, int64_t ldw, WeightSet &ws, hipStream_t s)
{
    int64_t tot = h->N * ws.R;
    hipLaunchKernelGGL(k_permute_w, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, W, ldw,
                       h->perm, h->N, ws.R, ws.Wt);
    HIPC(hipGetLastError());
}

__global__ void k_permute_w_cols(const float *__restrict__ W, int64_t ldw, const int32_t *__restrict__ perm,
                                 int64_t N, int rb, float *__restrict__ Wt, int ldt, int c0)
{
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t p = t / rb;
    if (p >= N) return;
    int r = (int)(t - p * rb);
    Wt[p * ldt + c0 + r] = W[(int64_t)perm[p] * ldw + r];
}

void permute_weight_cols(askit_handle *h, const float *W, int64_t ldw, int rb, float *Wt, int ldt, int c0,
                         hipStream_t s)
{
    int64_t tot = h->N * rb;
    hipLaunchKernelGGL(k_permute_w_cols, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, W, ldw, h->perm,
                       h->N, rb, Wt, ldt, c0);
    HIPC(hipGetLastError());
}

// Exact kappa nearest sources of M new points (original ids and FP64 squared
// distances, M x kappa each); Yp receives the packed points.  Temporaries come
// from ta (freed by the caller's guard).
static void query_knn(askit_handle *h, const float *Y, int64_t M, int64_t ldy, float *Yp, int32_t *qidx,
                      double *qd, const std::function<void *(size_t)> &ta, hipStream_t s)
{
    const int dp = h->dp, kappa = h->kappa;
    uint16_t *Yh = (uint16_t *)ta(sizeof(uint16_t) * M * dp);
    uint16_t *Yl = (uint16_t *)ta(sizeof(uint16_t) * M * dp);
    float *Yn = (float *)ta(sizeof(float) * M);
    int32_t *flag = (int32_t *)ta(sizeof(int32_t) * (M + 1));
    int32_t *cand = (int32_t *)ta(sizeof(int32_t) * M * KNN_CAND);
    float *thr = (float *)ta(sizeof(float) * M);
    HIPC(hipMemsetAsync(flag, 0, sizeof(int32_t), s));
    pack_points(Y, M, h->d, ldy, dp, Yp, flag, s);
    int32_t hflag = 0;
    HIPC(hipMemcpyAsync(&hflag, flag, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    HIPC(hipStreamSynchronize(s));
    if (hflag) fail(ASKIT_ERR_INVALID_ARG, "Y holds a non-finite value");
    HIPC(hipMemsetAsync(flag, 0, sizeof(int32_t), s));
    split_bf16(Yp, M, dp, Yh, Yl, Yn, s);
    knn_candidates(Yh, Yl, Yn, M, h->Xh, h->Xl, h->Xn, h->N, dp, false, false, cand, thr, flag + 1,
                   flag, s, nullptr, nullptr, nullptr, &h->ksamp, nullptr, nullptr, 0, nullptr, knn_nsel(kappa));
    float *tb = (float *)ta(sizeof(float) * M);
    knn_refine(Yp, M, h->Xt, h->N, h->d, dp, kappa, cand, thr, Yn, h->maxnorm, h->perm, nullptr, qidx,
               qd, flag + 1, flag, tb, s);
    int32_t nbad = 0;
    HIPC(hipMemcpyAsync(&nbad, flag, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    HIPC(hipStreamSynchronize(s));
    knn_fallback(Yp, Yh, Yl, Yn, h->Xt, h->Xh, h->Xl, h->Xn, h->N, h->d, dp, kappa, false, flag + 1, nbad, tb,
                 h->perm, nullptr, qidx, qd, s);
}

void query_points(askit_handle *h, const WeightSet &ws, const float *Y, int64_t M, int64_t ldy, float *U,
                  int64_t ldu, hipStream_t s, const std::vector<int64_t> *segs)
{
    const int dp = h->dp, kappa = h->kappa;
    std::vector<void *> tmp;
    struct Guard {
        std::vector<void *> &t;
        hipStream_t s;
        ~Guard() { for (void *p : t) (void)ws_free(p, s); }
    } guard{tmp, s};
    auto ta = [&](size_t b) {
        void *p;
        HIPC(ws_alloc(&p, std::max<size_t>(b, 16), s));
        tmp.push_back(p);
        return p;
    };
    float *Yp = (float *)ta(sizeof(float) * M * dp);
    int32_t *qidx = (int32_t *)ta(sizeof(int32_t) * M * kappa);
    double *qd = (double *)ta(sizeof(double) * M * kappa);
    int32_t *nb = (int32_t *)ta(sizeof(int32_t) * M * kappa);
    int32_t *nbs = (int32_t *)ta(sizeof(int32_t) * M * kappa);
    int32_t *order = (int32_t *)ta(sizeof(int32_t) * M);
    float *Ys = (float *)ta(sizeof(float) * M * dp);
    query_knn(h, Y, M, ldy, Yp, qidx, qd, ta, s);
    hipLaunchKernelGGL(k_map_pos, dim3((unsigned)((M * kappa + 255) / 256)), dim3(256), 0, s, qidx,
                       M * kappa, h->iperm, nb);
    HIPC(hipGetLastError());
    // requests of a served batch are kept apart: each sorts, forms slabs and
    // chunks among its own points only, so its result is the one it gets alone
    const int64_t nseg = segs ? (int64_t)segs->size() : 1;
    int32_t *dseg = nullptr;
    if (nseg > 1) {
        if ((uint64_t)nseg * (uint64_t)h->nodes.size() >= (1ull << 32))
            fail(ASKIT_ERR_UNSUPPORTED, "too many requests in one query batch");
        std::vector<int32_t> hseg;
        hseg.reserve(M);
        for (int64_t sg = 0; sg < nseg; ++sg) hseg.insert(hseg.end(), (size_t)(*segs)[sg], (int32_t)sg);
        if ((int64_t)hseg.size() != M) fail(ASKIT_ERR_INVALID_ARG, "query segments do not add up to the query count");
        dseg = (int32_t *)ta(sizeof(int32_t) * M);
        HIPC(hipMemcpyAsync(dseg, hseg.data(), sizeof(int32_t) * M, hipMemcpyHostToDevice, s));
        HIPC(hipStreamSynchronize(s));         // hseg is released on return of this block
    }
    sort_queries(h, nb, M, order, nbs, tmp, s, dseg);
    gather_rows(Yp, order, M, dp, Ys, s);
    int32_t *ptr, *node;
    uint64_t *mask;
    Slab *qslabs;
    int64_t nen, nef, nqslab = 0;
    build_query_interactions(h, nbs, M, qslabs, ptr, node, mask, nen, nef, tmp, s, nseg > 1 ? segs : nullptr,
                             nqslab);
    PairLists L;
    build_pairs(h, qslabs, nqslab, M, ptr, node, mask, nen, nef, L, ta, s, nseg);
    float *part = (float *)ta(sizeof(float) * std::max<int64_t>(L.npairs, 1) * ws.R);
    evaluate(h, ws, Ys, L, order, U, ldu, part, s);
    HIPC(hipStreamSynchronize(s));
}

}  // namespace askit

#define API_BEGIN                                                                                 \
    try {                                                                                         \
        g_err.clear();
#define API_END                                                                                   \
    }                                                                                             \
    catch (const Error &e)                                                                        \
    {                                                                                             \
        g_err = e.msg;                                                                            \
        return e.code;                                                                            \
    }                                                                                             \
    catch (const std::bad_alloc &)                                                                \
    {                                                                                             \
        g_err = "host allocation failed";                                                         \
        return ASKIT_ERR_OUT_OF_MEMORY;                                                           \
    }                                                                                             \
    catch (...)                                                                                   \
    {                                                                                             \
        g_err = "internal error";                                                                 \
        return ASKIT_ERR_DEVICE;                                                                  \
    }                                                                                             \
    return ASKIT_OK;

askit_handle::~askit_handle()
{
    if (ev_up0) (void)hipEventDestroy(ev_up0);
    if (ev_up1) (void)hipEventDestroy(ev_up1);
    for (void *p : allocs) (void)hipFree(p);
}

void *askit_handle::alloc(size_t bytes, bool zero)
{
    std::lock_guard<std::mutex> lk(alloc_mu);
    void *p = nullptr;
    HIPC(hipMalloc(&p, std::max<size_t>(bytes, 16)));
    allocs.push_back(p);
    if (zero) HIPC(hipMemsetAsync(p, 0, std::max<size_t>(bytes, 16), astream));
    return p;
}

static void check_device()
{
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || n < 1) fail(ASKIT_ERR_DEVICE, "no HIP device");
    int dev = 0;
    HIPC(hipGetDevice(&dev));
    hipDeviceProp_t prop;
    HIPC(hipGetDeviceProperties(&prop, dev));
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
        fail(ASKIT_ERR_DEVICE, std::string("library is built for gfx950, device is ") + prop.gcnArchName);
}

// Tree shape (depends on N and m only): breadth-first, left before right.
static void make_shape(askit_handle *h)
{
    h->nodes.clear();
    h->nodes.push_back(Node{0, (int32_t)h->N, 0, -1, -1, -1, 0});
    for (size_t a = 0; a < h->nodes.size(); ++a) {
        Node nd = h->nodes[a];
        int n = nd.hi - nd.lo;
        if (n <= h->m) continue;
        int nl = (n + 1) / 2;
        int L = (int)h->nodes.size();
        h->nodes.push_back(Node{nd.lo, nd.lo + nl, nd.level + 1, (int32_t)a, -1, -1, nd.path << 1});
        h->nodes.push_back(Node{nd.lo + nl, nd.hi, nd.level + 1, (int32_t)a, -1, -1, (nd.path << 1) | 1});
        h->nodes[a].left = L;
        h->nodes[a].right = L + 1;
    }
    h->depth = 0;
    for (auto &nd : h->nodes) h->depth = std::max(h->depth, (int)nd.level);
    h->level_nodes.assign(h->depth + 1, {});
    h->leaves.clear();
    for (size_t a = 0; a < h->nodes.size(); ++a) {
        h->level_nodes[h->nodes[a].level].push_back((int)a);
        if (h->nodes[a].left < 0) h->leaves.push_back((int)a);
    }
    std::sort(h->leaves.begin(), h->leaves.end(),
              [&](int x, int y) { return h->nodes[x].lo < h->nodes[y].lo; });
    int maxleaf = 0;
    for (int a : h->leaves) maxleaf = std::max(maxleaf, h->nodes[a].hi - h->nodes[a].lo);
    h->ncol_max = std::max(maxleaf, 2 * h->smax);
    h->slabs.clear();
    for (int a : h->leaves)
        for (int r0 = h->nodes[a].lo; r0 < h->nodes[a].hi; r0 += SLAB)
            h->slabs.push_back(Slab{r0, std::min(SLAB, h->nodes[a].hi - r0), a, 0});
    h->pslot.assign(h->nodes.size() + 1, 0);
    int64_t off = 0;
    for (size_t a = 0; a < h->nodes.size(); ++a) {
        h->pslot[a] = off;
        if (a == 0) continue;
        const Node &nd = h->nodes[a];
        int64_t n = nd.hi - nd.lo;
        int64_t ncap = nd.left < 0 ? n : 2 * (int64_t)h->smax;
        int64_t rows = std::min<int64_t>(h->ell, h->N - n);
        int64_t kcap = std::min<int64_t>(std::min<int64_t>(h->smax, rows), ncap);
        off += kcap * ncap;
    }
    h->pslot[h->nodes.size()] = off;
    h->pslot_total = off;
}

extern "C" {

askit_status askit_params_default(askit_params *p)
{
    if (!p) return ASKIT_ERR_INVALID_ARG;
    std::memset(p, 0, sizeof(*p));
    p->struct_size = sizeof(askit_params);
    p->abi_version = ASKIT_ABI_VERSION;
    p->leaf_size = 128;
    p->kappa = 16;
    p->max_skeleton = 64;
    p->sample_rows = 0;
    p->id_tol = 1e-6;
    p->bandwidth = 1.0;
    p->bw_neighbor = 0;
    p->precision = ASKIT_PREC_FP32;
    p->seed = 0;
    return ASKIT_OK;
}

const char *askit_last_error(void) { return g_err.c_str(); }

}  // extern "C"

// Alg. 5 setup steps; knn_in (device, N x kappa original ids, row stride ldk)
// replaces the exact neighbour search when given.
// defer_skel: stop before the skeletons (the fused skeletonization of a batch
// runs them for many handles at once; finish_deferred completes the setup).
static void setup_impl(const float *X, int64_t N, int32_t d, int64_t ldx, const int32_t *knn_in, int64_t ldk,
                       const askit_params *p, void *stream, askit_handle **out, bool defer_skel = false)
{
    if (!out) fail(ASKIT_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (!p || !X) fail(ASKIT_ERR_INVALID_ARG, "NULL argument");
    if (p->struct_size != sizeof(askit_params) || p->abi_version != ASKIT_ABI_VERSION)
        fail(ASKIT_ERR_INVALID_ARG, "askit_params size or ABI version mismatch");
    if (N < 2 || N >= (1ll << 31)) fail(ASKIT_ERR_INVALID_ARG, "N must be in [2, 2^31)");
    if (d < 1 || ldx < d) fail(ASKIT_ERR_INVALID_ARG, "need d >= 1 and ldx >= d");
    if (p->kappa < 1 || p->kappa >= N) fail(ASKIT_ERR_INVALID_ARG, "need 1 <= kappa < N");
    if (p->kappa > 64) fail(ASKIT_ERR_UNSUPPORTED, "kappa above 64 is not supported");
    if (p->leaf_size < 1 || p->max_skeleton < 1) fail(ASKIT_ERR_INVALID_ARG, "need m >= 1, s_max >= 1");
    int ell = p->sample_rows == 0 ? p->max_skeleton + 20 : p->sample_rows;
    if (ell < p->max_skeleton) fail(ASKIT_ERR_INVALID_ARG, "need sample_rows >= max_skeleton");
    if (!(p->id_tol >= 0.0)) fail(ASKIT_ERR_INVALID_ARG, "need id_tol >= 0");
    if (p->bw_neighbor < 0 || p->bw_neighbor > p->kappa)
        fail(ASKIT_ERR_INVALID_ARG, "need 0 <= bw_neighbor <= kappa");
    if (p->bw_neighbor == 0 && !(p->bandwidth > 0.0 && std::isfinite(p->bandwidth)))
        fail(ASKIT_ERR_INVALID_ARG, "need a positive finite bandwidth");
    if (p->precision != ASKIT_PREC_FP32 && p->precision != ASKIT_PREC_BF16X3)
        fail(ASKIT_ERR_INVALID_ARG, "unknown precision");
    if (d > 1024) fail(ASKIT_ERR_UNSUPPORTED, "d above 1024 is not supported");
    if (p->prune_levels < 0) fail(ASKIT_ERR_INVALID_ARG, "need prune_levels >= 0");
    if (knn_in && ldk < p->kappa) fail(ASKIT_ERR_INVALID_ARG, "need ldk >= kappa");
    check_device();
    hipStream_t s = (hipStream_t)stream;
    ArenaScope arena(s);               // this setup's working buffers (released on return)

    std::unique_ptr<askit_handle> h(new askit_handle());
    h->astream = s;
    HIPC(hipGetDevice(&h->device));
    h->N = N;
    h->d = d;
    h->dp = round_up(d, 16);
    h->prm = *p;
    h->prm.sample_rows = ell;
    h->kappa = p->kappa;
    h->m = p->leaf_size;
    h->smax = p->max_skeleton;
    h->ell = ell;
    h->varh = p->bw_neighbor > 0;
    make_shape(h.get());
    h->minlev = p->prune_levels > 0 ? std::max(1, h->depth - p->prune_levels + 1) : 0;
    const int64_t nn = (int64_t)h->nodes.size();
    const int dp = h->dp, kappa = h->kappa;

    hipEvent_t ev[6];
    for (auto &e : ev) HIPC(hipEventCreate(&e));
    struct EvGuard {
        hipEvent_t *e;
        ~EvGuard() { for (int i = 0; i < 6; ++i) (void)hipEventDestroy(e[i]); }
    } evg{ev};

    // device state
    h->Xo = (float *)h->alloc(sizeof(float) * N * dp, false);
    h->Xh = (uint16_t *)h->alloc(sizeof(uint16_t) * N * dp, false);
    h->Xl = (uint16_t *)h->alloc(sizeof(uint16_t) * N * dp, false);
    h->Xn = (float *)h->alloc(sizeof(float) * N, false);
    h->Xt = (float *)h->alloc(sizeof(float) * N * dp, false);
    h->gt = (float *)h->alloc(sizeof(float) * N, false);
    h->hsrc = (double *)h->alloc(sizeof(double) * N, false);
    h->perm = (int32_t *)h->alloc(sizeof(int32_t) * N, false);
    h->iperm = (int32_t *)h->alloc(sizeof(int32_t) * N, false);
    h->knn_idx = (int32_t *)h->alloc(sizeof(int32_t) * N * kappa, false);
    h->knn_d = (double *)h->alloc(sizeof(double) * N * kappa, false);
    h->d_nodes = (Node *)h->alloc(sizeof(Node) * nn, false);
    h->leaf_of = (int32_t *)h->alloc(sizeof(int32_t) * N, false);
    h->nl_pos = (int32_t *)h->alloc(sizeof(int32_t) * nn * ell, true);
    h->nl_key = (double *)h->alloc(sizeof(double) * nn * ell, true);
    h->nl_cnt = (int32_t *)h->alloc(sizeof(int32_t) * nn, true);
    h->T = (int32_t *)h->alloc(sizeof(int32_t) * nn * ell, true);
    h->T_cnt = (int32_t *)h->alloc(sizeof(int32_t) * nn, true);
    h->S = (int32_t *)h->alloc(sizeof(int32_t) * nn * h->smax, true);
    h->skk = (int32_t *)h->alloc(sizeof(int32_t) * nn, true);
    h->colperm = (int32_t *)h->alloc(sizeof(int32_t) * nn * h->ncol_max, true);
    h->ncols = (int32_t *)h->alloc(sizeof(int32_t) * nn, true);
    h->P = (float *)h->alloc(sizeof(float) * std::max<int64_t>(h->pslot_total, 1), false);
    h->d_pslot = (int64_t *)h->alloc(sizeof(int64_t) * (nn + 1), false);
    h->Xs = (float *)h->alloc(sizeof(float) * nn * h->smax * dp, true);
    h->gs = (float *)h->alloc(sizeof(float) * nn * h->smax, true);
    h->d_slabs = (Slab *)h->alloc(sizeof(Slab) * h->slabs.size(), false);
    HIPC(hipMemcpy(h->d_nodes, h->nodes.data(), sizeof(Node) * nn, hipMemcpyHostToDevice));
    HIPC(hipMemcpy(h->d_pslot, h->pslot.data(), sizeof(int64_t) * (nn + 1), hipMemcpyHostToDevice));
    HIPC(hipMemcpy(h->d_slabs, h->slabs.data(), sizeof(Slab) * h->slabs.size(), hipMemcpyHostToDevice));
    int32_t *flag = (int32_t *)h->alloc(sizeof(int32_t) * 4, true);

    HIPC(hipEventRecord(ev[0], s));
    // ---- points and tree (the tree needs only the coordinates)
    pack_points(X, N, d, ldx, dp, h->Xo, flag, s);
    int32_t hflag = 0;
    HIPC(hipMemcpyAsync(&hflag, flag, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    HIPC(hipStreamSynchronize(s));
    if (hflag) fail(ASKIT_ERR_INVALID_ARG, "X holds a non-finite value");
    build_tree(h.get(), s);
    gather_rows(h->Xo, h->perm, N, dp, h->Xt, s);
    {
        int32_t *dl;
        HIPC(ws_alloc((void **)&dl, sizeof(int32_t) * h->leaves.size(), s));
        HIPC(hipMemcpyAsync(dl, h->leaves.data(), sizeof(int32_t) * h->leaves.size(),
                            hipMemcpyHostToDevice, s));
        hipLaunchKernelGGL(k_leaf_of, dim3((unsigned)h->leaves.size()), dim3(256), 0, s, h->d_nodes, dl,
                           (int)h->leaves.size(), h->leaf_of);
        HIPC(hipGetLastError());
        HIPC(hipStreamSynchronize(s));
        HIPC(ws_free(dl, s));
    }
    HIPC(hipEventRecord(ev[1], s));
    // ---- exact neighbours, swept in tree order (each block starts at its own leaf)
    split_bf16(h->Xt, N, dp, h->Xh, h->Xl, h->Xn, s);
    knn_build_sample(h.get(), s);
    float mx = max_norm(h->Xn, N, s);
    h->maxnorm = mx;
    if (knn_in) {
        HIPC(hipMemsetAsync(flag, 0, sizeof(int32_t), s));
        hipLaunchKernelGGL(k_knn_import, dim3((unsigned)((N + 127) / 128)), dim3(128), 0, s, knn_in, ldk, N, kappa,
                           h->Xo, dp, d, h->knn_idx, h->knn_d, flag);
        HIPC(hipGetLastError());
        HIPC(hipMemcpyAsync(&hflag, flag, sizeof(int32_t), hipMemcpyDeviceToHost, s));
        HIPC(hipStreamSynchronize(s));
        if (hflag)
            fail(ASKIT_ERR_INVALID_ARG, "neighbour lists hold an id out of range, the row's own id or a repeated id");
    } else {
        int32_t *cand, *bad;
        float *thr;
        HIPC(ws_alloc((void **)&cand, sizeof(int32_t) * N * KNN_CAND, s));
        HIPC(ws_alloc((void **)&thr, sizeof(float) * N, s));
        HIPC(ws_alloc((void **)&bad, sizeof(int32_t) * (N + 1), s));
        HIPC(hipMemsetAsync(bad, 0, sizeof(int32_t), s));
        hipEvent_t k0, k1;
        HIPC(hipEventCreate(&k0));
        HIPC(hipEventCreate(&k1));
        // the search sweeps the points in a finer order than the tree's (leaves
        // split on into cells of at most 64 points): compact tiles, so far
        // (row block, tile) pairs are skipped; results are ids and exact
        // distances, independent of the order
        const bool fine = h->depth > 0 && N > 64 * 64 && !std::getenv("ASKIT_KNN_TREE_ORDER");
        int32_t *perm_f = h->perm;
        float *Xt_f = h->Xt, *Xn_f = h->Xn;
        uint16_t *Xh_f = h->Xh, *Xl_f = h->Xl;
        if (fine) {
            HIPC(ws_alloc((void **)&perm_f, sizeof(int32_t) * N, s));
            HIPC(ws_alloc((void **)&Xt_f, sizeof(float) * N * dp, s));
            HIPC(ws_alloc((void **)&Xn_f, sizeof(float) * N, s));
            HIPC(ws_alloc((void **)&Xh_f, sizeof(uint16_t) * N * dp, s));
            HIPC(ws_alloc((void **)&Xl_f, sizeof(uint16_t) * N * dp, s));
            build_fine_order(h.get(), 64, perm_f, s);
            gather_rows(h->Xo, perm_f, N, dp, Xt_f, s);
            split_bf16(Xt_f, N, dp, Xh_f, Xl_f, Xn_f, s);
        }
        HIPC(hipEventRecord(k0, s));
        float fms = 0.f;
        knn_candidates(Xh_f, Xl_f, Xn_f, N, Xh_f, Xl_f, Xn_f, N, dp, true, true, cand, thr,
                       bad + 1, bad, s, &fms, &h->knn_filter_launches, &h->knn_retry_rows, &h->ksamp,
                       &h->knn_retry_list, Xt_f, d, &h->knn_tiles_swept, knn_nsel(kappa));
        h->t_knn_filter = fms;
        HIPC(hipEventRecord(k1, s));
        if (fine && !h->knn_retry_list.empty()) {
            // retried rows are reported as tree positions: iperm[perm_f[r]]
            const int64_t nr = (int64_t)h->knn_retry_list.size();
            int32_t *dl;
            HIPC(ws_alloc((void **)&dl, sizeof(int32_t) * nr, s));
            HIPC(hipMemcpyAsync(dl, h->knn_retry_list.data(), sizeof(int32_t) * nr, hipMemcpyHostToDevice, s));
            hipLaunchKernelGGL(k_map_rows, dim3((unsigned)((nr + 255) / 256)), dim3(256), 0, s, dl, nr, perm_f,
                               h->iperm);
            HIPC(hipGetLastError());
            HIPC(hipMemcpyAsync(h->knn_retry_list.data(), dl, sizeof(int32_t) * nr, hipMemcpyDeviceToHost, s));
            HIPC(ws_free(dl, s));
            HIPC(hipStreamSynchronize(s));
        }
        float *tb;
        HIPC(ws_alloc((void **)&tb, sizeof(float) * N, s));
        knn_refine(Xt_f, N, Xt_f, N, d, dp, kappa, cand, thr, Xn_f, mx, perm_f, perm_f,
                   h->knn_idx, h->knn_d, bad + 1, bad, tb, s);
        int32_t nbad = 0;
        HIPC(hipMemcpyAsync(&nbad, bad, sizeof(int32_t), hipMemcpyDeviceToHost, s));
        HIPC(hipStreamSynchronize(s));
        h->knn_uncertified = nbad;
        float kms = 0.f;
        HIPC(hipEventElapsedTime(&kms, k0, k1));
        h->t_knn_sweep = kms;
        (void)hipEventDestroy(k0);
        (void)hipEventDestroy(k1);
        knn_fallback(Xt_f, Xh_f, Xl_f, Xn_f, Xt_f, Xh_f, Xl_f, Xn_f, N, d, dp, kappa, true, bad + 1, nbad,
                     tb, perm_f, perm_f, h->knn_idx, h->knn_d, s);
        HIPC(ws_free(tb, s));
        if (fine) {
            HIPC(ws_free(perm_f, s));
            HIPC(ws_free(Xt_f, s));
            HIPC(ws_free(Xn_f, s));
            HIPC(ws_free(Xh_f, s));
            HIPC(ws_free(Xl_f, s));
        }
        HIPC(ws_free(cand, s));
        HIPC(ws_free(thr, s));
        HIPC(ws_free(bad, s));
    }
    HIPC(hipMemsetAsync(flag, 0, sizeof(int32_t), s));
    hipLaunchKernelGGL(k_bandwidth, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, s, h->knn_d, N,
                       kappa, p->bw_neighbor, p->bandwidth, h->hsrc, flag);
    HIPC(hipGetLastError());
    HIPC(hipMemcpyAsync(&hflag, flag, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    HIPC(hipStreamSynchronize(s));
    if (hflag) fail(ASKIT_ERR_INVALID_ARG, "zero bandwidth (duplicate points with variable bandwidth)");
    hipLaunchKernelGGL(k_gfactor, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, s, h->hsrc, h->perm,
                       N, h->gt);
    HIPC(hipGetLastError());
    HIPC(hipEventRecord(ev[2], s));
    // ---- interaction lists and the same pairs grouped by source node: they
    // need the tree and the neighbours, not the skeletons, so a helper thread
    // builds them on a second stream while this one builds node lists, sampled
    // rows and skeletons
    float ms_inter = 0.f;
    if (defer_skel) {
        // a setup whose skeletons are built later (the batched form): the
        // lists follow on the same stream (no helper stream and thread per
        // instance; the instances' setups overlap each other instead)
        hipEvent_t ei[2] = {nullptr, nullptr};
        HIPC(hipEventCreate(&ei[0]));
        HIPC(hipEventCreate(&ei[1]));
        struct EvFree {
            hipEvent_t *e;
            ~EvFree()
            {
                (void)hipEventDestroy(e[0]);
                (void)hipEventDestroy(e[1]);
            }
        } evf{ei};
        build_node_lists(h.get(), s);
        sample_rows(h.get(), s);
        HIPC(hipEventRecord(ev[3], s));
        HIPC(hipEventRecord(ev[4], s));
        askit_handle *hp = h.get();
        HIPC(hipEventRecord(ei[0], s));
        build_interactions(hp, s);
        build_pairs(hp, hp->d_slabs, (int64_t)hp->slabs.size(), N, hp->sl_ptr, hp->sl_node, hp->sl_mask,
                    hp->near_entries, hp->far_entries, hp->pairs, [hp](size_t b) { return hp->alloc(b, false); }, s);
        HIPC(hipEventRecord(ei[1], s));
        HIPC(hipStreamSynchronize(s));
        HIPC(hipEventElapsedTime(&ms_inter, ei[0], ei[1]));
    } else {
        hipStream_t s2 = nullptr;
        hipEvent_t ei[2] = {nullptr, nullptr};
        HIPC(hipStreamCreateWithFlags(&s2, hipStreamNonBlocking));
        HIPC(hipEventCreate(&ei[0]));
        HIPC(hipEventCreate(&ei[1]));
        HIPC(hipStreamWaitEvent(s2, ev[2], 0));
        std::exception_ptr ierr;
        askit_handle *hp = h.get();
        std::thread ith([&, hp]() {
            try {
                HIPC(hipSetDevice(hp->device));
                HIPC(hipEventRecord(ei[0], s2));
                build_interactions(hp, s2);
                build_pairs(hp, hp->d_slabs, (int64_t)hp->slabs.size(), N, hp->sl_ptr, hp->sl_node, hp->sl_mask,
                            hp->near_entries, hp->far_entries, hp->pairs,
                            [hp](size_t b) { return hp->alloc(b, false); }, s2);
                HIPC(hipEventRecord(ei[1], s2));
                HIPC(hipStreamSynchronize(s2));
            } catch (...) {
                ierr = std::current_exception();
            }
        });
        struct Join {
            std::thread &t;
            hipStream_t s2;
            hipEvent_t *e;
            ~Join()
            {
                if (t.joinable()) t.join();
                (void)hipStreamSynchronize(s2);
                (void)hipStreamDestroy(s2);
                (void)hipEventDestroy(e[0]);
                (void)hipEventDestroy(e[1]);
            }
        };
        {
            Join jn{ith, s2, ei};
            // ---- node lists and sampled rows
            build_node_lists(h.get(), s);
            sample_rows(h.get(), s);
            HIPC(hipEventRecord(ev[3], s));
            // ---- skeletons
            if (!defer_skel) skeletonize(h.get(), s);
            HIPC(hipEventRecord(ev[4], s));
            ith.join();
            if (ierr) std::rethrow_exception(ierr);
            HIPC(hipEventElapsedTime(&ms_inter, ei[0], ei[1]));
        }
    }
    if (!defer_skel) count_pairs(h.get(), s);
    HIPC(hipEventRecord(ev[5], s));
    HIPC(hipStreamSynchronize(s));
    prepare_upward(h.get());
    HIPC(hipEventCreate(&h->ev_up0));
    HIPC(hipEventCreate(&h->ev_up1));
    float ms;
    HIPC(hipEventElapsedTime(&ms, ev[0], ev[1])); h->t_tree = ms;
    HIPC(hipEventElapsedTime(&ms, ev[1], ev[2])); h->t_knn = ms;
    HIPC(hipEventElapsedTime(&ms, ev[2], ev[3])); h->t_lists = ms;
    HIPC(hipEventElapsedTime(&ms, ev[3], ev[4])); h->t_skel = ms;
    h->t_inter = ms_inter;                 // on the second stream, overlapped with the above
    h->skel_pending = defer_skel;
    *out = h.release();
}

namespace askit {

askit_handle *setup_deferred(const float *X, int64_t N, int32_t d, int64_t ldx, const askit_params *p,
                             hipStream_t s)
{
    askit_handle *h = nullptr;
    setup_impl(X, N, d, ldx, nullptr, 0, p, s, &h, true);
    return h;
}

void finish_deferred(askit_handle *h, hipStream_t s)
{
    count_pairs(h, s);
    h->skel_pending = false;
}

}  // namespace askit

extern "C" {

askit_status askit_setup(const float *X, int64_t N, int32_t d, int64_t ldx, const askit_params *p,
                         void *stream, askit_handle **out)
{
    API_BEGIN
    setup_impl(X, N, d, ldx, nullptr, 0, p, stream, out);
    API_END
}

askit_status askit_setup_with_knn(const float *X, int64_t N, int32_t d, int64_t ldx, const int32_t *knn,
                                  int64_t ldk, const askit_params *p, void *stream, askit_handle **out)
{
    API_BEGIN
    if (!knn) fail(ASKIT_ERR_INVALID_ARG, "knn is NULL");
    setup_impl(X, N, d, ldx, knn, ldk, p, stream, out);
    API_END
}

askit_status askit_update_weights(askit_handle *h, const float *W, int64_t ldw, int32_t nrhs, void *stream)
{
    API_BEGIN
    if (!h || !W) fail(ASKIT_ERR_INVALID_ARG, "NULL argument");
    if (nrhs < 1 || nrhs > MAX_RHS) fail(ASKIT_ERR_INVALID_ARG, "need 1 <= nrhs <= 64");
    if (ldw < nrhs) fail(ASKIT_ERR_INVALID_ARG, "need ldw >= nrhs");
    hipStream_t s = (hipStream_t)stream;
    const int64_t nn = (int64_t)h->nodes.size();
    if (nrhs > h->wcap) {
        HIPC(hipStreamSynchronize(s));
        h->astream = s;
        auto drop = [&](void *p) {
            if (!p) return;
            (void)hipFree(p);
            h->allocs.erase(std::remove(h->allocs.begin(), h->allocs.end(), p), h->allocs.end());
        };
        drop(h->ws.Wt);
        drop(h->ws.Wsk);
        drop(h->ws.part);
        h->ws.Wt = (float *)h->alloc(sizeof(float) * h->N * nrhs, false);
        h->ws.Wsk = (float *)h->alloc(sizeof(float) * nn * h->smax * nrhs, true);
        h->ws.part = (float *)h->alloc(sizeof(float) * std::max<int64_t>(h->pairs.npairs, 1) * nrhs, false);
        h->wcap = nrhs;
    }
    h->ws.R = nrhs;
    HIPC(hipEventRecord(h->ev_up0, s));
    permute_weights(h, W, ldw, h->ws, s);
    upward(h, h->ws, s);
    HIPC(hipEventRecord(h->ev_up1, s));
    h->up_pending = true;
    API_END
}

askit_status askit_evaluate(askit_handle *h, float *U, int64_t ldu, void *stream)
{
    API_BEGIN
    if (!h || !U) fail(ASKIT_ERR_INVALID_ARG, "NULL argument");
    if (h->ws.R < 1) fail(ASKIT_ERR_NOT_READY, "askit_update_weights has not been called");
    if (ldu < h->ws.R) fail(ASKIT_ERR_INVALID_ARG, "need ldu >= nrhs");
    evaluate(h, h->ws, h->Xt, h->pairs, h->perm, U, ldu, h->ws.part, (hipStream_t)stream);
    API_END
}

askit_status askit_knn_rptree(const float *X, int64_t N, int32_t d, int64_t ldx, int32_t kappa, int32_t leaf_size,
                              int32_t iterations, uint64_t seed, int32_t *idx, double *dist, void *stream)
{
    API_BEGIN
    if (!X || !idx || !dist) fail(ASKIT_ERR_INVALID_ARG, "NULL argument");
    if (N < 2 || N >= (1ll << 31)) fail(ASKIT_ERR_INVALID_ARG, "N must be in [2, 2^31)");
    if (d < 1 || ldx < d) fail(ASKIT_ERR_INVALID_ARG, "need d >= 1 and ldx >= d");
    if (kappa < 1 || kappa >= N) fail(ASKIT_ERR_INVALID_ARG, "need 1 <= kappa < N");
    if (kappa > 64) fail(ASKIT_ERR_UNSUPPORTED, "kappa above 64 is not supported");
    if (d > 1024) fail(ASKIT_ERR_UNSUPPORTED, "d above 1024 is not supported");
    if (iterations < 1 || iterations > 2046) fail(ASKIT_ERR_INVALID_ARG, "need 1 <= iterations <= 2046");
    if (leaf_size < 2) fail(ASKIT_ERR_INVALID_ARG, "need leaf_size >= 2");
    check_device();
    hipStream_t s = (hipStream_t)stream;
    const int dp = round_up(d, 16);
    std::vector<void *> tmp;
    struct Guard {
        std::vector<void *> &t;
        hipStream_t s;
        ~Guard() { for (void *p : t) (void)ws_free(p, s); }
    } guard{tmp, s};
    float *Xo;
    int32_t *flag;
    HIPC(ws_alloc((void **)&Xo, sizeof(float) * N * dp, s));
    tmp.push_back(Xo);
    HIPC(ws_alloc((void **)&flag, 16, s));
    tmp.push_back(flag);
    HIPC(hipMemsetAsync(flag, 0, sizeof(int32_t), s));
    pack_points(X, N, d, ldx, dp, Xo, flag, s);
    int32_t hflag = 0;
    HIPC(hipMemcpyAsync(&hflag, flag, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    HIPC(hipStreamSynchronize(s));
    if (hflag) fail(ASKIT_ERR_INVALID_ARG, "X holds a non-finite value");
    rp_knn(Xo, N, d, dp, kappa, leaf_size, iterations, seed, idx, dist, s);
    API_END
}

askit_status askit_evaluate_parts(askit_handle *h, float *U, int64_t ldu, float *Unear, int64_t ldun, void *stream)
{
    API_BEGIN
    if (!h || !U || !Unear) fail(ASKIT_ERR_INVALID_ARG, "NULL argument");
    if (h->ws.R < 1) fail(ASKIT_ERR_NOT_READY, "askit_update_weights has not been called");
    if (ldu < h->ws.R || ldun < h->ws.R) fail(ASKIT_ERR_INVALID_ARG, "need ldu >= nrhs and ldun >= nrhs");
    evaluate(h, h->ws, h->Xt, h->pairs, h->perm, U, ldu, h->ws.part, (hipStream_t)stream, Unear, ldun);
    API_END
}

askit_status askit_query(askit_handle *h, const float *Y, int64_t M, int64_t ldy, float *U, int64_t ldu,
                         void *stream)
{
    API_BEGIN
    if (!h || !Y || !U) fail(ASKIT_ERR_INVALID_ARG, "NULL argument");
    if (M < 1 || M >= (1ll << 31)) fail(ASKIT_ERR_INVALID_ARG, "need 1 <= M < 2^31");
    if (ldy < h->d) fail(ASKIT_ERR_INVALID_ARG, "need ldy >= d");
    if (h->ws.R < 1) fail(ASKIT_ERR_NOT_READY, "askit_update_weights has not been called");
    if (ldu < h->ws.R) fail(ASKIT_ERR_INVALID_ARG, "need ldu >= nrhs");
    query_points(h, h->ws, Y, M, ldy, U, ldu, (hipStream_t)stream);
    API_END
}

askit_status askit_query_neighbors(askit_handle *h, const float *Y, int64_t M, int64_t ldy, int32_t *idx,
                                   double *dist, void *stream)
{
    API_BEGIN
    if (!h || !Y || !idx || !dist) fail(ASKIT_ERR_INVALID_ARG, "NULL argument");
    if (M < 1 || M >= (1ll << 31)) fail(ASKIT_ERR_INVALID_ARG, "need 1 <= M < 2^31");
    if (ldy < h->d) fail(ASKIT_ERR_INVALID_ARG, "need ldy >= d");
    hipStream_t s = (hipStream_t)stream;
    std::vector<void *> tmp;
    struct Guard {
        std::vector<void *> &t;
        hipStream_t s;
        ~Guard() { for (void *p : t) (void)ws_free(p, s); }
    } guard{tmp, s};
    auto ta = [&](size_t b) {
        void *p;
        HIPC(ws_alloc(&p, std::max<size_t>(b, 16), s));
        tmp.push_back(p);
        return p;
    };
    float *Yp = (float *)ta(sizeof(float) * M * h->dp);
    query_knn(h, Y, M, ldy, Yp, idx, dist, ta, s);
    HIPC(hipStreamSynchronize(s));
    API_END
}

void askit_destroy(askit_handle *h)
{
    if (!h) return;
    (void)hipDeviceSynchronize();
    delete h;
}

askit_status askit_pruning_visits(const askit_handle *h, int32_t *visits_kappa, int32_t *visits_dist, void *stream)
{
    API_BEGIN
    if (!h || !visits_kappa || !visits_dist) fail(ASKIT_ERR_INVALID_ARG, "NULL argument");
    prune_visits(h, visits_kappa, visits_dist, (hipStream_t)stream);
    API_END
}

askit_status askit_get_info(const askit_handle *h, askit_info *o)
{
    API_BEGIN
    if (!h || !o) fail(ASKIT_ERR_INVALID_ARG, "NULL argument");
    std::memset(o, 0, sizeof(*o));
    o->N = h->N;
    o->d = h->d;
    o->kappa = h->kappa;
    o->leaf_size = h->m;
    o->max_skeleton = h->smax;
    o->sample_rows = h->ell;
    o->nrhs = h->ws.R;
    o->num_nodes = (int32_t)h->nodes.size();
    o->num_leaves = (int32_t)h->leaves.size();
    o->depth = h->depth;
    o->ncol_max = h->ncol_max;
    o->num_slabs = (int32_t)h->slabs.size();
    o->near_entries = h->near_entries;
    o->far_entries = h->far_entries;
    o->near_pairs = h->near_pairs;
    o->far_pairs = h->far_pairs;
    o->knn_uncertified_rows = h->knn_uncertified;
    o->t_knn_ms = h->t_knn;
    o->t_tree_ms = h->t_tree;
    o->t_lists_ms = h->t_lists;
    o->t_skel_ms = h->t_skel;
    o->t_inter_ms = h->t_inter;
    if (h->up_pending) {
        float ms = 0.f;
        HIPC(hipEventSynchronize(h->ev_up1));
        HIPC(hipEventElapsedTime(&ms, h->ev_up0, h->ev_up1));
        const_cast<askit_handle *>(h)->t_update = ms;
        const_cast<askit_handle *>(h)->up_pending = false;
    }
    o->t_update_ms = h->t_update;
    o->t_knn_sweep_ms = h->t_knn_sweep;
    o->t_knn_filter_ms = h->t_knn_filter;
    o->knn_filter_launches = h->knn_filter_launches;
    o->eval_pairs = h->pairs.npairs;
    o->eval_chunks = h->pairs.nchunk;
    o->knn_retry_rows = h->knn_retry_rows;
    o->t_qr_ms = h->t_qr;
    o->knn_tiles_swept = h->knn_tiles_swept;
    o->near_lists = h->pairs.near_lists;
    o->far_lists = h->pairs.far_lists;
    API_END
}

askit_status askit_export(const askit_handle *h, int32_t what, void *dst, size_t cap, size_t *bytes)
{
    API_BEGIN
    if (!h) fail(ASKIT_ERR_INVALID_ARG, "NULL handle");
    const int64_t nn = (int64_t)h->nodes.size();
    const void *src = nullptr;
    size_t n = 0;
    bool host = false;
    const int64_t nslab = (int64_t)h->slabs.size();
    std::vector<int32_t> row0;
    switch (what) {
    case ASKIT_X_PERM: src = h->perm; n = 4 * h->N; break;
    case ASKIT_X_KNN_IDX: src = h->knn_idx; n = 4 * h->N * h->kappa; break;
    case ASKIT_X_KNN_DIST: src = h->knn_d; n = 8 * h->N * h->kappa; break;
    case ASKIT_X_NODES: src = h->nodes.data(); n = sizeof(Node) * nn; host = true; break;
    case ASKIT_X_NLIST_POS: src = h->nl_pos; n = 4 * nn * h->ell; break;
    case ASKIT_X_NLIST_KEY: src = h->nl_key; n = 8 * nn * h->ell; break;
    case ASKIT_X_NLIST_CNT: src = h->nl_cnt; n = 4 * nn; break;
    case ASKIT_X_ROWS: src = h->T; n = 4 * nn * h->ell; break;
    case ASKIT_X_ROWS_CNT: src = h->T_cnt; n = 4 * nn; break;
    case ASKIT_X_SKEL: src = h->S; n = 4 * nn * h->smax; break;
    case ASKIT_X_SKEL_K: src = h->skk; n = 4 * nn; break;
    case ASKIT_X_COLPERM: src = h->colperm; n = 4 * nn * h->ncol_max; break;
    case ASKIT_X_NCOLS: src = h->ncols; n = 4 * nn; break;
    case ASKIT_X_PROJ: src = h->P; n = 4 * h->pslot_total; break;
    case ASKIT_X_SKEL_W: src = h->ws.Wsk; n = h->ws.Wsk ? 4 * nn * h->smax * h->ws.R : 0; break;
    case ASKIT_X_SLAB_PTR: src = h->sl_ptr; n = 4 * (2 * nslab + 2); break;
    case ASKIT_X_SLAB_NODE: src = h->sl_node; n = 4 * (h->near_entries + h->far_entries); break;
    case ASKIT_X_SLAB_MASK: src = h->sl_mask; n = 8 * (h->near_entries + h->far_entries); break;
    case ASKIT_X_SLAB_ROW0:
        row0.resize(nslab);
        for (int64_t i = 0; i < nslab; ++i) row0[i] = h->slabs[i].row0;
        src = row0.data();
        n = 4 * nslab;
        host = true;
        break;
    case ASKIT_X_BANDWIDTH: src = h->hsrc; n = 8 * h->N; break;
    case ASKIT_X_KNN_RETRY:
        src = h->knn_retry_list.data();
        n = 4 * h->knn_retry_list.size();
        host = true;
        break;
    default: fail(ASKIT_ERR_INVALID_ARG, "unknown export item");
    }
    if (bytes) *bytes = n;
    if (!dst) return ASKIT_OK;
    if (cap < n) fail(ASKIT_ERR_INVALID_ARG, "destination buffer too small");
    if (n == 0) return ASKIT_OK;
    if (host) std::memcpy(dst, src, n);
    else {
        HIPC(hipDeviceSynchronize());
        HIPC(hipMemcpy(dst, src, n, hipMemcpyDeviceToHost));
    }
    API_END
}

}  // extern "C"
