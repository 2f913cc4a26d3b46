// Batched form: many independent problems (uneven sizes and dimensions)
// behind one handle.
//
// Setup runs the single-problem setup of every instance up to the skeletons,
// several at a time on worker threads with their own streams; then one fused
// skeletonization builds the IDs of every instance, level by level, each
// kernel launched once per level over the nodes of all instances (the small
// instances' per-node factorizations fill the device together instead of a
// few at a time).  The per-weight-vector work of
// all instances is then fused: one permutation launch over all rows, one
// upward launch per tree level across every instance (deepest level first,
// so each instance still sees its children before its parents), and one
// evaluation launch over the slabs of every instance, reading each slab's
// instance tables from a device array.  The evaluation runs either as one
// workgroup per slab or as a persistent grid that takes
// slabs from a work queue in decreasing cost order, with wide or narrow
// column tiles (the weight columns a pass contracts); an autotuner times the
// launch shapes once per problem class -- the bucket (d, m, s, R) -- and keeps
// the fastest.
// askit_batch_run captures the whole weights -> u sequence in a HIP graph
// (kernels only: the queue counters are cleared by a kernel) and replays it.
#include "askit_impl.h"

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <numeric>
#include <thread>

using namespace askit;

namespace askit {
extern thread_local std::string g_err;
}

namespace {

constexpr int MAX_PASSES = (MAX_RHS + 7) / 8;     // RHS passes of the evaluation (8 columns each)
constexpr int NUM_GRID = 4;                       // grid forms tried by the tuner
constexpr int CAND_BLOCKS_PER_CU[NUM_GRID] = {0, 2, 4, 8};   // 0: one workgroup per slab
constexpr int NUM_PLAN = 2;                       // column-tile plans (wide, narrow)
constexpr int NUM_CAND = NUM_GRID * NUM_PLAN;     // launch shapes, plan-major

struct GraphEntry {
    const float *W;
    int64_t ldw;
    int R;
    float *U;
    int64_t ldu;
    int blocks, plan;
    hipGraph_t graph;
    hipGraphExec_t exec;
};

struct Launch {
    int blocks = -1;     // -1: not tuned; 0: one workgroup per slab; else the persistent grid
    int plan = 0;
};

// Launch shapes already chosen in this process, by problem class.
std::mutex g_tune_mu;
std::map<std::string, std::pair<Launch, std::vector<double>>> g_tune_cache;

}  // namespace

struct askit_batch {
    std::vector<askit_handle *> inst;
    int device = 0;
    int num_cu = 256;
    askit_params prm{};
    int smax = 0;
    int64_t rows = 0, wsk_slots = 0, npairs = 0, nchunk = 0, ne = 0, fe = 0;
    int64_t near_pairs = 0, far_pairs = 0;
    double t_setup_ms = 0.0, t_skel_ms = 0.0;
    std::vector<void *> own;

    EvalInst *d_einst = nullptr;
    UpInst *d_uinst = nullptr;
    int2 *d_items = nullptr;
    std::vector<std::pair<int64_t, int64_t>> levels;
    Chunk *d_chunks = nullptr;
    int32_t *d_tpos = nullptr, *d_tslot = nullptr, *d_sbase = nullptr, *d_queue = nullptr, *d_outrow = nullptr;

    float *Wt = nullptr, *Wsk = nullptr, *part = nullptr;
    int wcap = 0, R = 0;

    Launch launch_for_R[MAX_RHS + 1];
    std::vector<double> cand_ms[MAX_RHS + 1];
    std::string tune_key_base;

    std::vector<GraphEntry> graphs;
    hipStream_t cap = nullptr;

    void *dev(size_t bytes)
    {
        void *p = nullptr;
        HIPC(hipMalloc(&p, std::max<size_t>(bytes, 16)));
        own.push_back(p);
        return p;
    }
    void drop_graphs()
    {
        for (auto &g : graphs) {
            (void)hipGraphExecDestroy(g.exec);
            (void)hipGraphDestroy(g.graph);
        }
        graphs.clear();
    }
    ~askit_batch()
    {
        (void)hipDeviceSynchronize();
        drop_graphs();
        if (cap) (void)hipStreamDestroy(cap);
        for (void *p : own) (void)hipFree(p);
        if (Wt) (void)hipFree(Wt);
        if (Wsk) (void)hipFree(Wsk);
        if (part) (void)hipFree(part);
        for (auto *h : inst) askit_destroy(h);
    }
    BatchEvalArgs eval_args(float *U, int64_t ldu, Launch l) const
    {
        BatchEvalArgs a{};
        a.inst = d_einst;
        a.chunks = d_chunks;
        a.nchunk = nchunk;
        a.tpos = d_tpos;
        a.tslot = d_tslot;
        a.sbase = d_sbase;
        a.outrow = d_outrow;
        a.rows = rows;
        a.Wt = Wt;
        a.Wsk = Wsk;
        a.part = part;
        a.U = U;
        a.ldu = ldu;
        a.R = R;
        a.bf = prm.precision == ASKIT_PREC_BF16X3;
        a.persistent = l.blocks > 0 ? l.blocks : 0;
        a.plan = l.plan;
        a.queue = d_queue;
        return a;
    }
    void update(const float *W, int64_t ldw, hipStream_t s)
    {
        permute_rows(W, ldw, d_outrow, rows, R, Wt, s);
        upward_batch(d_uinst, d_items, levels, smax, Wt, Wsk, R, s);
    }
};

__global__ void k_add_offset(int32_t *__restrict__ dst, const int32_t *__restrict__ src, int64_t n, int32_t off)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = src[i] + off;
}

static void add_offset(int32_t *dst, const int32_t *src, int64_t n, int32_t off)
{
    if (n <= 0) return;
    hipLaunchKernelGGL(k_add_offset, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, 0, dst, src, n, off);
    HIPC(hipGetLastError());
}

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
    catch (...)                                                                                   \
    {                                                                                             \
        g_err = "internal error";                                                                 \
        return ASKIT_ERR_DEVICE;                                                                  \
    }                                                                                             \
    return ASKIT_OK;

static void ensure_weights(askit_batch *b, int R, hipStream_t s)
{
    if (R > b->wcap) {
        HIPC(hipStreamSynchronize(s));
        b->drop_graphs();
        if (b->Wt) HIPC(hipFree(b->Wt));
        if (b->Wsk) HIPC(hipFree(b->Wsk));
        if (b->part) HIPC(hipFree(b->part));
        b->Wt = b->Wsk = b->part = nullptr;
        HIPC(hipMalloc((void **)&b->Wt, sizeof(float) * std::max<int64_t>(b->rows * R, 4)));
        HIPC(hipMalloc((void **)&b->Wsk, sizeof(float) * std::max<int64_t>(b->wsk_slots * R, 4)));
        HIPC(hipMalloc((void **)&b->part, sizeof(float) * std::max<int64_t>(b->npairs * R, 4)));
        b->wcap = R;
    }
    b->R = R;
}

// Times every launch shape of the evaluation for the current R (the weights
// must be in place) and keeps the fastest; all shapes give identical results.
// The choice is kept for the problem class (bucket) and reused by later
// batches of the same class.
static void autotune(askit_batch *b, float *U, int64_t ldu, hipStream_t s)
{
    const int R = b->R;
    const std::string key = b->tune_key_base + "/R" + std::to_string(R);
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto it = g_tune_cache.find(key);
        if (it != g_tune_cache.end()) {
            b->launch_for_R[R] = it->second.first;
            b->cand_ms[R] = it->second.second;
            return;
        }
    }
    hipEvent_t e0, e1;
    HIPC(hipEventCreate(&e0));
    HIPC(hipEventCreate(&e1));
    std::vector<double> ms(NUM_CAND, 0.0);
    int best = 0;
    auto cand = [&](int c) {
        Launch l;
        l.plan = c / NUM_GRID;
        l.blocks = CAND_BLOCKS_PER_CU[c % NUM_GRID] * b->num_cu;
        return l;
    };
    for (int c = 0; c < NUM_CAND; ++c) {
        const BatchEvalArgs a = b->eval_args(U, ldu, cand(c));
        evaluate_batch(a, s);                        // warm-up
        std::vector<float> t;
        for (int rep = 0; rep < 3; ++rep) {
            HIPC(hipEventRecord(e0, s));
            evaluate_batch(a, s);
            HIPC(hipEventRecord(e1, s));
            HIPC(hipEventSynchronize(e1));
            float v = 0.f;
            HIPC(hipEventElapsedTime(&v, e0, e1));
            t.push_back(v);
        }
        std::sort(t.begin(), t.end());
        ms[c] = t[1];
        if (ms[c] < ms[best]) best = c;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    b->launch_for_R[R] = cand(best);
    b->cand_ms[R] = ms;
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune_cache[key] = {b->launch_for_R[R], ms};
}

extern "C" {

askit_status askit_batch_setup(int32_t count, const float *const *X, const int64_t *N, const int32_t *d,
                               const int64_t *ldx, const askit_params *p, void *stream, askit_batch **out)
{
    API_BEGIN
    if (!out) fail(ASKIT_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (count < 1) fail(ASKIT_ERR_INVALID_ARG, "need count >= 1");
    if (!X || !N || !d || !ldx || !p) fail(ASKIT_ERR_INVALID_ARG, "NULL argument");
    for (int32_t i = 0; i < count; ++i)
        if (!X[i]) fail(ASKIT_ERR_INVALID_ARG, "NULL point set");
    hipStream_t s = (hipStream_t)stream;
    HIPC(hipStreamSynchronize(s));           // the point sets are written
    const auto t0 = std::chrono::steady_clock::now();
    std::unique_ptr<askit_batch> b(new askit_batch());
    HIPC(hipGetDevice(&b->device));
    hipDeviceProp_t prop;
    HIPC(hipGetDeviceProperties(&prop, b->device));
    b->num_cu = prop.multiProcessorCount;
    b->prm = *p;
    b->inst.assign(count, nullptr);

    // instance setups, several at once on worker threads with their own streams
    std::atomic<int32_t> next{0};
    std::mutex emu;
    askit_status first_code = ASKIT_OK;
    std::string first_msg;
    const int nthreads = std::min<int>(count, 16);
    std::vector<std::thread> th;
    for (int w = 0; w < nthreads; ++w)
        th.emplace_back([&, dev = b->device] {
            hipStream_t ws = nullptr;
            if (hipSetDevice(dev) != hipSuccess || hipStreamCreateWithFlags(&ws, hipStreamNonBlocking) != hipSuccess) {
                std::lock_guard<std::mutex> lk(emu);
                if (first_code == ASKIT_OK) {
                    first_code = ASKIT_ERR_DEVICE;
                    first_msg = "worker stream creation failed";
                }
                return;
            }
            for (;;) {
                const int32_t i = next++;
                if (i >= count) break;
                askit_status rc = ASKIT_OK;
                std::string msg;
                try {
                    if (!X[i]) fail(ASKIT_ERR_INVALID_ARG, "NULL point set");
                    b->inst[i] = setup_deferred(X[i], N[i], d[i], ldx[i], p, ws);
                } catch (const Error &e) {
                    rc = e.code;
                    msg = e.msg;
                } catch (const std::bad_alloc &) {
                    rc = ASKIT_ERR_OUT_OF_MEMORY;
                    msg = "host allocation failed";
                } catch (...) {
                    rc = ASKIT_ERR_DEVICE;
                    msg = "internal error";
                }
                if (rc != ASKIT_OK) {
                    std::lock_guard<std::mutex> lk(emu);
                    if (first_code == ASKIT_OK) {
                        first_code = rc;
                        first_msg = "instance " + std::to_string(i) + ": " + msg;
                    }
                    next = count;
                    break;
                }
            }
            (void)hipStreamSynchronize(ws);
            (void)hipStreamDestroy(ws);
        });
    for (auto &t : th) t.join();
    if (first_code != ASKIT_OK) fail(first_code, first_msg);
    // the fused skeletonization of all instances, then each setup's last step
    {
        const auto ts = std::chrono::steady_clock::now();
        skeletonize_multi(b->inst, s);
        for (auto *h : b->inst) finish_deferred(h, s);
        HIPC(hipStreamSynchronize(s));
        b->t_skel_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - ts).count();
    }

    // host tables: instance offsets of rows, skeleton-weight slots and pairs
    const int smax = b->inst[0]->smax;
    b->smax = smax;
    std::vector<int64_t> row_off(count + 1, 0), wsk_off(count + 1, 0), pair_off(count + 1, 0);
    int maxdepth = 0;
    for (int32_t i = 0; i < count; ++i) {
        const askit_handle *h = b->inst[i];
        row_off[i + 1] = row_off[i] + h->N;
        wsk_off[i + 1] = wsk_off[i] + (int64_t)h->nodes.size() * h->smax;
        pair_off[i + 1] = pair_off[i] + h->pairs.npairs;
        maxdepth = std::max(maxdepth, h->depth);
        b->near_pairs += h->near_pairs;
        b->far_pairs += h->far_pairs;
        b->ne += h->near_entries;
        b->fe += h->far_entries;
    }
    if (row_off[count] >= (1ll << 31)) fail(ASKIT_ERR_UNSUPPORTED, "batch above 2^31 points");
    if (pair_off[count] >= (1ll << 31)) fail(ASKIT_ERR_UNSUPPORTED, "batch above 2^31 evaluation pairs");
    b->rows = row_off[count];
    b->wsk_slots = wsk_off[count];
    b->npairs = pair_off[count];

    // concatenated pair lists: rows stay instance-local (targets are the
    // instance's own points), slots and chunk pair ranges become batch-wide
    std::vector<int32_t> outrow(b->rows);
    std::vector<Chunk> chunks;
    std::vector<EvalInst> einst(count);
    std::vector<UpInst> uinst(count);
    b->d_outrow = (int32_t *)b->dev(sizeof(int32_t) * b->rows);
    b->d_sbase = (int32_t *)b->dev(sizeof(int32_t) * (b->rows + 1));
    b->d_tpos = (int32_t *)b->dev(sizeof(int32_t) * std::max<int64_t>(b->npairs, 1));
    b->d_tslot = (int32_t *)b->dev(sizeof(int32_t) * std::max<int64_t>(b->npairs, 1));
    for (int32_t i = 0; i < count; ++i) {
        const askit_handle *h = b->inst[i];
        const PairLists &L = h->pairs;
        std::vector<int32_t> perm(h->N);
        std::vector<Chunk> hc(L.nchunk);
        HIPC(hipMemcpy(perm.data(), h->perm, sizeof(int32_t) * h->N, hipMemcpyDeviceToHost));
        if (L.nchunk > 0) HIPC(hipMemcpy(hc.data(), L.chunks, sizeof(Chunk) * L.nchunk, hipMemcpyDeviceToHost));
        for (int64_t t = 0; t < h->N; ++t) outrow[row_off[i] + t] = (int32_t)(row_off[i] + perm[t]);
        for (Chunk c : hc) {
            c.kind = (c.kind & 1) | (i << 1);
            c.first += (int32_t)pair_off[i];
            chunks.push_back(c);
        }
        if (L.npairs > 0) {
            HIPC(hipMemcpy(b->d_tpos + pair_off[i], L.tpos, sizeof(int32_t) * L.npairs, hipMemcpyDeviceToDevice));
            add_offset(b->d_tslot + pair_off[i], L.tslot, L.npairs, (int32_t)pair_off[i]);
        }
        add_offset(b->d_sbase + row_off[i], L.sbase, h->N + (i == count - 1 ? 1 : 0), (int32_t)pair_off[i]);
        einst[i] = EvalInst{h->d_nodes, h->Xt, h->Xt, h->gt, h->Xs, h->gs, h->skk, row_off[i], wsk_off[i], h->smax,
                            h->dp};
        uinst[i] = UpInst{h->d_nodes, h->skk, h->ncols, h->colperm, h->d_pslot, h->P, row_off[i], wsk_off[i],
                          h->ncol_max, h->smax};
    }
    b->nchunk = (int64_t)chunks.size();
    // upward items, deepest level first across all instances
    std::vector<int2> items;
    for (int lev = maxdepth; lev >= 1; --lev) {
        const int64_t first = (int64_t)items.size();
        for (int32_t i = 0; i < count; ++i) {
            const askit_handle *h = b->inst[i];
            if (lev > h->depth) continue;
            for (int a : h->level_nodes[lev]) items.push_back(int2{i, a});
        }
        b->levels.push_back({first, (int64_t)items.size() - first});
    }

    b->d_einst = (EvalInst *)b->dev(sizeof(EvalInst) * count);
    b->d_uinst = (UpInst *)b->dev(sizeof(UpInst) * count);
    b->d_items = (int2 *)b->dev(sizeof(int2) * std::max<size_t>(items.size(), 1));
    b->d_chunks = (Chunk *)b->dev(sizeof(Chunk) * std::max<int64_t>(b->nchunk, 1));
    b->d_queue = (int32_t *)b->dev(sizeof(int32_t) * 4);
    HIPC(hipMemcpy(b->d_einst, einst.data(), sizeof(EvalInst) * count, hipMemcpyHostToDevice));
    HIPC(hipMemcpy(b->d_uinst, uinst.data(), sizeof(UpInst) * count, hipMemcpyHostToDevice));
    if (!items.empty())
        HIPC(hipMemcpy(b->d_items, items.data(), sizeof(int2) * items.size(), hipMemcpyHostToDevice));
    if (b->nchunk > 0)
        HIPC(hipMemcpy(b->d_chunks, chunks.data(), sizeof(Chunk) * b->nchunk, hipMemcpyHostToDevice));
    HIPC(hipMemcpy(b->d_outrow, outrow.data(), sizeof(int32_t) * b->rows, hipMemcpyHostToDevice));
    HIPC(hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking));
    // problem class of the tuner: the bucket (largest padded dimension, leaf
    // size, skeleton bound; R is appended per tuning) and the precision form
    int maxdp = 0;
    for (auto *h : b->inst) maxdp = std::max(maxdp, h->dp);
    b->tune_key_base = "d" + std::to_string(maxdp) + "m" + std::to_string(p->leaf_size) + "s" +
                       std::to_string(smax) + "p" + std::to_string((int)p->precision);
    HIPC(hipDeviceSynchronize());
    b->t_setup_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    *out = b.release();
    API_END
}

askit_status askit_batch_update_weights(askit_batch *b, const float *W, int64_t ldw, int32_t nrhs, void *stream)
{
    API_BEGIN
    if (!b || !W) fail(ASKIT_ERR_INVALID_ARG, "NULL argument");
    if (nrhs < 1 || nrhs > MAX_RHS) fail(ASKIT_ERR_INVALID_ARG, "need 1 <= nrhs <= 64");
    if (ldw < nrhs) fail(ASKIT_ERR_INVALID_ARG, "need ldw >= nrhs");
    hipStream_t s = (hipStream_t)stream;
    ensure_weights(b, nrhs, s);
    b->update(W, ldw, s);
    API_END
}

askit_status askit_batch_evaluate(askit_batch *b, float *U, int64_t ldu, void *stream)
{
    API_BEGIN
    if (!b || !U) fail(ASKIT_ERR_INVALID_ARG, "NULL argument");
    if (b->R < 1) fail(ASKIT_ERR_NOT_READY, "askit_batch_update_weights has not been called");
    if (ldu < b->R) fail(ASKIT_ERR_INVALID_ARG, "need ldu >= nrhs");
    evaluate_batch(b->eval_args(U, ldu, b->launch_for_R[b->R]), (hipStream_t)stream);
    API_END
}

askit_status askit_batch_run(askit_batch *b, const float *W, int64_t ldw, int32_t nrhs, float *U, int64_t ldu,
                             void *stream)
{
    API_BEGIN
    if (!b || !W || !U) fail(ASKIT_ERR_INVALID_ARG, "NULL argument");
    if (nrhs < 1 || nrhs > MAX_RHS) fail(ASKIT_ERR_INVALID_ARG, "need 1 <= nrhs <= 64");
    if (ldw < nrhs || ldu < nrhs) fail(ASKIT_ERR_INVALID_ARG, "need ldw, ldu >= nrhs");
    hipStream_t s = (hipStream_t)stream;
    ensure_weights(b, nrhs, s);
    if (b->launch_for_R[nrhs].blocks < 0) {
        b->update(W, ldw, s);
        autotune(b, U, ldu, s);
    }
    const Launch ln = b->launch_for_R[nrhs];
    GraphEntry *ge = nullptr;
    for (auto &g : b->graphs)
        if (g.W == W && g.ldw == ldw && g.R == nrhs && g.U == U && g.ldu == ldu && g.blocks == ln.blocks &&
            g.plan == ln.plan)
            ge = &g;
    if (!ge) {
        if (b->graphs.size() >= 8) {
            HIPC(hipStreamSynchronize(s));
            (void)hipGraphExecDestroy(b->graphs.front().exec);
            (void)hipGraphDestroy(b->graphs.front().graph);
            b->graphs.erase(b->graphs.begin());
        }
        GraphEntry g{W, ldw, nrhs, U, ldu, ln.blocks, ln.plan, nullptr, nullptr};
        HIPC(hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal));
        try {
            b->update(W, ldw, b->cap);
            evaluate_batch(b->eval_args(U, ldu, ln), b->cap);
        } catch (...) {
            hipGraph_t junk = nullptr;
            (void)hipStreamEndCapture(b->cap, &junk);
            if (junk) (void)hipGraphDestroy(junk);
            throw;
        }
        HIPC(hipStreamEndCapture(b->cap, &g.graph));
        HIPC(hipGraphInstantiate(&g.exec, g.graph, nullptr, nullptr, 0));
        b->graphs.push_back(g);
        ge = &b->graphs.back();
    }
    HIPC(hipGraphLaunch(ge->exec, s));
    API_END
}

askit_status askit_batch_set_launch(askit_batch *b, int32_t nrhs, int32_t blocks, int32_t plan)
{
    API_BEGIN
    if (!b) fail(ASKIT_ERR_INVALID_ARG, "NULL argument");
    if (nrhs < 1 || nrhs > MAX_RHS) fail(ASKIT_ERR_INVALID_ARG, "need 1 <= nrhs <= 64");
    if (blocks < 0 || blocks > 64 * b->num_cu) fail(ASKIT_ERR_INVALID_ARG, "need 0 <= blocks <= 64 x CUs");
    if (plan < 0 || plan >= NUM_PLAN) fail(ASKIT_ERR_INVALID_ARG, "need plan 0 (wide) or 1 (narrow)");
    b->launch_for_R[nrhs].blocks = blocks;
    b->launch_for_R[nrhs].plan = plan;
    b->cand_ms[nrhs].clear();
    API_END
}

askit_status askit_batch_get_info(const askit_batch *b, askit_batch_info *o)
{
    API_BEGIN
    if (!b || !o) fail(ASKIT_ERR_INVALID_ARG, "NULL argument");
    std::memset(o, 0, sizeof(*o));
    o->count = (int32_t)b->inst.size();
    o->nrhs = b->R;
    o->total_points = b->rows;
    o->total_chunks = b->nchunk;
    o->near_entries = b->ne;
    o->far_entries = b->fe;
    o->near_pairs = b->near_pairs;
    o->far_pairs = b->far_pairs;
    o->t_setup_ms = b->t_setup_ms;
    o->t_skel_ms = b->t_skel_ms;
    const int R = b->R;
    o->tuned = R > 0 && b->launch_for_R[R].blocks >= 0;
    o->launch_blocks = o->tuned ? b->launch_for_R[R].blocks : 0;
    o->launch_plan = o->tuned ? b->launch_for_R[R].plan : 0;
    for (int c = 0; c < NUM_CAND && o->tuned && c < (int)b->cand_ms[R].size(); ++c) o->candidate_ms[c] = b->cand_ms[R][c];
    o->graphs = (int32_t)b->graphs.size();
    API_END
}

askit_handle *askit_batch_instance(askit_batch *b, int32_t i)
{
    if (!b || i < 0 || i >= (int32_t)b->inst.size()) return nullptr;
    return b->inst[i];
}

void askit_batch_destroy(askit_batch *b) { delete b; }

}  // extern "C"
