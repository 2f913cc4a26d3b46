// Serving: a resident setup answering weight and query requests with
// continuous batching under a device-memory budget (see include/askit.h).
//
// Scheduling: requests enter one FIFO.  A free worker takes the oldest
// pending request and appends the following pending requests of the same
// kind while the batch stays within its size limit and the memory budget;
// requests that do not fit stay queued ("deferred") and are admitted as soon
// as a finishing batch releases memory.  Each worker owns one stream, so
// batches of different workers overlap on the device.  A weight batch
// gathers the requests' columns side by side, runs the upward pass and the
// evaluation once for all of them and scatters the columns back; a query
// batch stacks the points, runs one query evaluation against the resident
// weights and scatters the rows back.
//
// Cyclic weights (weight_passes = K > 0): weight requests bypass the workers
// and go to one column engine that owns a resident pool of max_batch_rhs
// weight columns.  The evaluation's chunk list is cut into K ranges of about
// equal pair counts; the engine sweeps them round robin, one range per pass,
// over every column in flight.  Between passes it admits waiting requests
// into free columns (permutation to tree order and the upward pass for those
// columns only) and retires the columns that have now seen all K ranges
// (their per-target slot sums go straight to the request's output).  A
// request admitted mid-sweep therefore starts at whichever range comes next
// and finishes one full cycle later.  Every pair slot is written by exactly
// one pass and the slot sums run in a fixed order, so a request's result
// equals evaluating it alone up to the rounding of the contraction width (the
// run of live columns it rides in).
#include "askit_impl.h"

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>

using namespace askit;

namespace askit {
extern thread_local std::string g_err;
}

namespace {

using clk = std::chrono::steady_clock;

struct Request {
    uint64_t id;
    bool query;
    const float *in;
    int64_t ld_in;
    int64_t rows;     // query points (query) / N (weights)
    int32_t cols;     // nrhs (weights) / resident nrhs (query)
    float *out;
    int64_t ld_out;
    uint64_t bytes;
    clk::time_point t_submit;
    bool waited;      // counted once in `deferred`
};

struct Done {
    int32_t state;    // 1 done, -1 failed
    double ms;
    std::string err;
};

// A weight request holding pool columns [c0, c0 + r.cols).
struct Slot {
    Request r;
    int c0;
    int passes_left;
};

}  // namespace

struct askit_server {
    askit_handle *h = nullptr;
    askit_server_config cfg{};
    WeightSet ws0;                        // resident weights of query requests
    std::vector<void *> own;              // allocations of the resident weights
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<Request> pending;
    std::map<uint64_t, Done> done;
    std::vector<std::thread> workers;
    bool stopping = false;
    uint64_t next_id = 1;
    uint64_t mem_used = 0, peak_mem = 0;
    int64_t submitted = 0, completed = 0, failed = 0, deferred = 0, batches = 0, batched = 0, joined = 0;
    double targets_rhs = 0.0;
    std::vector<double> lat_all, lat_w, lat_q;
    bool any_submit = false;
    clk::time_point t_first, t_last;
    // cyclic weights
    std::deque<Request> wpending;         // weight requests waiting for pool columns
    WeightSet pool;                       // pool.R = max_batch_rhs columns; pool.part: the slots
    std::vector<int64_t> range_end;       // K + 1 chunk indices: pass p evaluates [range_end[p], range_end[p+1])
    std::thread engine;
    uint64_t pool_bytes = 0;

    uint64_t weights_bytes(int32_t R) const
    {
        const int64_t nn = (int64_t)h->nodes.size();
        return (uint64_t)R * (uint64_t)(12 * h->N + 4 * nn * h->smax + 4 * h->pairs.npairs) + (1u << 20);
    }
    uint64_t query_bytes(int64_t M) const
    {
        // per query: points, kNN work, lists, and its pairs (about npairs / N of them)
        const int64_t ppq = h->pairs.npairs / std::max<int64_t>(h->N, 1) + 1;
        return (uint64_t)M * (uint64_t)(24 * h->dp + 28 * h->kappa + 4 * KNN_CAND * 2 + 2048 + 4 * ws0.R +
                                        ppq * (8 + 4 * ws0.R + 40)) + (4u << 20);
    }
    void worker_loop(int wid);
    void run_batch(std::vector<Request> &b, hipStream_t s);
    void engine_loop();
    void finish(const std::vector<Request> &rs, int32_t state, const std::string &err);
};

static double percentile(std::vector<double> v, double q)
{
    if (v.empty()) return 0.0;
    std::sort(v.begin(), v.end());
    double pos = q * (double)(v.size() - 1);
    size_t i = (size_t)pos;
    double f = pos - (double)i;
    return i + 1 < v.size() ? v[i] * (1.0 - f) + v[i + 1] * f : v[i];
}

void askit_server::run_batch(std::vector<Request> &b, hipStream_t s)
{
    const int64_t N = h->N;
    std::vector<void *> tmp;
    struct Guard {
        std::vector<void *> &t;
        hipStream_t s;
        ~Guard()
        {
            (void)hipStreamSynchronize(s);
            for (void *p : t) (void)hipFreeAsync(p, s);
            (void)hipStreamSynchronize(s);
        }
    } guard{tmp, s};
    auto ta = [&](size_t bytes) {
        void *p;
        HIPC(hipMallocAsync(&p, std::max<size_t>(bytes, 16), s));
        tmp.push_back(p);
        return p;
    };
    if (!b[0].query) {
        int32_t R = 0;
        for (auto &r : b) R += r.cols;
        const int64_t nn = (int64_t)h->nodes.size();
        float *Wb = (float *)ta(sizeof(float) * N * R);
        float *Ub = (float *)ta(sizeof(float) * N * R);
        WeightSet ws;
        ws.R = R;
        ws.Wt = (float *)ta(sizeof(float) * N * R);
        ws.Wsk = (float *)ta(sizeof(float) * nn * h->smax * R);
        HIPC(hipMemsetAsync(ws.Wsk, 0, sizeof(float) * nn * h->smax * R, s));
        int32_t off = 0;
        for (auto &r : b) {
            HIPC(hipMemcpy2DAsync(Wb + off, sizeof(float) * R, r.in, sizeof(float) * r.ld_in,
                                  sizeof(float) * r.cols, N, hipMemcpyDeviceToDevice, s));
            off += r.cols;
        }
        permute_weights(h, Wb, R, ws, s);
        upward(h, ws, s);
        float *part = (float *)ta(sizeof(float) * std::max<int64_t>(h->pairs.npairs, 1) * R);
        evaluate(h, ws, h->Xt, h->pairs, h->perm, Ub, R, part, s);
        off = 0;
        for (auto &r : b) {
            HIPC(hipMemcpy2DAsync(r.out, sizeof(float) * r.ld_out, Ub + off, sizeof(float) * R,
                                  sizeof(float) * r.cols, N, hipMemcpyDeviceToDevice, s));
            off += r.cols;
        }
        HIPC(hipStreamSynchronize(s));
    } else {
        int64_t M = 0;
        for (auto &r : b) M += r.rows;
        const int d = h->d, R0 = ws0.R;
        float *Yb = (float *)ta(sizeof(float) * M * d);
        float *Ub = (float *)ta(sizeof(float) * M * R0);
        int64_t off = 0;
        for (auto &r : b) {
            HIPC(hipMemcpy2DAsync(Yb + off * d, sizeof(float) * d, r.in, sizeof(float) * r.ld_in,
                                  sizeof(float) * d, r.rows, hipMemcpyDeviceToDevice, s));
            off += r.rows;
        }
        std::vector<int64_t> segs;
        for (auto &r : b) segs.push_back(r.rows);
        query_points(h, ws0, Yb, M, d, Ub, R0, s, &segs);
        off = 0;
        for (auto &r : b) {
            HIPC(hipMemcpy2DAsync(r.out, sizeof(float) * r.ld_out, Ub + off * R0, sizeof(float) * R0,
                                  sizeof(float) * R0, r.rows, hipMemcpyDeviceToDevice, s));
            off += r.rows;
        }
        HIPC(hipStreamSynchronize(s));
    }
}

void askit_server::worker_loop(int wid)
{
    (void)wid;
    hipStream_t s = nullptr;
    if (hipSetDevice(h->device) != hipSuccess ||
        hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess)
        s = nullptr;
    for (;;) {
        std::vector<Request> batch;
        {
            std::unique_lock<std::mutex> lk(mu);
            for (;;) {
                if (!pending.empty()) {
                    Request &head = pending.front();
                    if (mem_used + head.bytes <= cfg.mem_budget) break;
                    if (!head.waited) {  // the oldest request waits for memory
                        head.waited = true;
                        ++deferred;
                    }
                } else if (stopping) {
                    break;
                }
                cv_work.wait(lk);
            }
            if (pending.empty() && stopping) break;
            // the oldest request, then later ones of the same kind that fit
            const bool q = pending.front().query;
            int64_t size = 0;
            const int64_t limit = q ? cfg.max_batch_queries : cfg.max_batch_rhs;
            for (auto it = pending.begin(); it != pending.end();) {
                if (it->query != q) { ++it; continue; }
                const int64_t sz = q ? it->rows : it->cols;
                if (!batch.empty() && (size + sz > limit || mem_used + it->bytes > cfg.mem_budget)) {
                    ++it;
                    continue;
                }
                size += sz;
                mem_used += it->bytes;
                batch.push_back(*it);
                it = pending.erase(it);
                if (size >= limit) break;
            }
            peak_mem = std::max(peak_mem, mem_used);
            ++batches;
            batched += (int64_t)batch.size();
        }
        std::string err;
        int32_t state = 1;
        if (!s) {
            state = -1;
            err = "worker stream creation failed";
        } else {
            try {
                run_batch(batch, s);
            } catch (const Error &e) {
                state = -1;
                err = e.msg;
            } catch (...) {
                state = -1;
                err = "internal error";
            }
        }
        finish(batch, state, err);
    }
    if (s) (void)hipStreamDestroy(s);
}

// Records the outcome of finished requests and releases their memory.
void askit_server::finish(const std::vector<Request> &rs, int32_t state, const std::string &err)
{
    if (rs.empty()) return;
    const auto t_end = clk::now();
    {
        std::lock_guard<std::mutex> lk(mu);
        for (auto &r : rs) {
            mem_used -= r.bytes;
            double ms = std::chrono::duration<double, std::milli>(t_end - r.t_submit).count();
            done[r.id] = Done{state, ms, err};
            if (state == 1) {
                ++completed;
                lat_all.push_back(ms);
                (r.query ? lat_q : lat_w).push_back(ms);
                targets_rhs += r.query ? (double)r.rows * ws0.R : (double)h->N * r.cols;
            } else {
                ++failed;
            }
        }
        t_last = t_end;
    }
    cv_done.notify_all();
    cv_work.notify_all();
}

void askit_server::engine_loop()
{
    hipStream_t s = nullptr;
    if (hipSetDevice(h->device) != hipSuccess ||
        hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess)
        s = nullptr;
    const int C = pool.R, K = (int)range_end.size() - 1;
    std::vector<char> used(C, 0);
    std::vector<Slot> live;
    int64_t pass = 0;
    auto fits = [&](int n) {
        for (int c0 = 0; c0 + n <= C; ++c0) {
            int c = c0;
            while (c < c0 + n && !used[c]) ++c;
            if (c == c0 + n) return c0;
            c0 = c;   // the loop's ++ moves past the used column
        }
        return -1;
    };
    for (;;) {
        std::vector<Slot> admitted;
        {
            std::unique_lock<std::mutex> lk(mu);
            for (;;) {
                // oldest first; a request that does not fit blocks those behind it
                while (!wpending.empty()) {
                    Request &head = wpending.front();
                    const int c0 = fits(head.cols);
                    if (c0 < 0) {
                        if (!head.waited) {
                            head.waited = true;
                            ++deferred;
                        }
                        break;
                    }
                    for (int c = c0; c < c0 + head.cols; ++c) used[c] = 1;
                    admitted.push_back(Slot{head, c0, K});
                    wpending.pop_front();
                }
                if (!admitted.empty() || !live.empty()) break;
                if (stopping && wpending.empty()) break;
                cv_work.wait(lk);
            }
            if (admitted.empty() && live.empty()) break;
            if (!admitted.empty()) {
                ++batches;
                batched += (int64_t)admitted.size();
                if (!live.empty()) joined += (int64_t)admitted.size();
            }
        }
        std::vector<Request> ok, bad;
        std::string err;
        try {
            if (!s) fail(ASKIT_ERR_DEVICE, "engine stream creation failed");
            for (auto &a : admitted) {
                permute_weight_cols(h, a.r.in, a.r.ld_in, a.r.cols, pool.Wt, C, a.c0, s);
                upward(h, pool, s, a.c0, a.c0 + a.r.cols);
                live.push_back(a);
            }
            admitted.clear();
            // this pass's range over every maximal run of live columns
            std::vector<char> on(C, 0);
            for (auto &l : live)
                for (int c = l.c0; c < l.c0 + l.r.cols; ++c) on[c] = 1;
            const int rg = (int)(pass % K);
            for (int c = 0; c < C;) {
                if (!on[c]) { ++c; continue; }
                int e = c;
                while (e < C && on[e]) ++e;
                evaluate_chunk_range(h, pool, h->pairs, range_end[rg], range_end[rg + 1], c, e, pool.part, s);
                c = e;
            }
            ++pass;
            std::vector<Slot> keep;
            for (auto &l : live) {
                if (--l.passes_left > 0) {
                    keep.push_back(l);
                    continue;
                }
                sum_slot_cols(h, h->pairs, pool.part, C, l.c0, l.r.cols, h->perm, l.r.out, l.r.ld_out, s);
                ok.push_back(l.r);
                for (int c = l.c0; c < l.c0 + l.r.cols; ++c) used[c] = 0;
            }
            HIPC(hipStreamSynchronize(s));
            live.swap(keep);
        } catch (const Error &e) {
            err = e.msg;
        } catch (...) {
            err = "internal error";
        }
        if (!err.empty()) {
            // every request in flight fails; the pool starts over empty
            if (s) (void)hipStreamSynchronize(s);
            for (auto &a : admitted) bad.push_back(a.r);
            for (auto &l : live) bad.push_back(l.r);
            bad.insert(bad.end(), ok.begin(), ok.end());
            ok.clear();
            live.clear();
            std::fill(used.begin(), used.end(), 0);
        }
        finish(ok, 1, "");
        finish(bad, -1, err);
    }
    if (s) (void)hipStreamDestroy(s);
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

extern "C" {

askit_status askit_server_config_default(askit_server_config *c)
{
    if (!c) return ASKIT_ERR_INVALID_ARG;
    std::memset(c, 0, sizeof(*c));
    c->struct_size = sizeof(askit_server_config);
    c->workers = 2;
    c->max_batch_rhs = 64;
    c->max_batch_queries = 65536;
    c->mem_budget = 8ull << 30;
    c->weight_passes = 0;
    c->max_pending = 0;
    return ASKIT_OK;
}

askit_status askit_server_create(askit_handle *h, const float *W0, int64_t ldw0, int32_t nrhs0,
                                 const askit_server_config *cfg, askit_server **out)
{
    API_BEGIN
    if (!out) fail(ASKIT_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (!h || !W0 || !cfg) fail(ASKIT_ERR_INVALID_ARG, "NULL argument");
    if (cfg->struct_size != sizeof(askit_server_config)) fail(ASKIT_ERR_INVALID_ARG, "config size mismatch");
    if (cfg->workers < 1 || cfg->workers > 16) fail(ASKIT_ERR_INVALID_ARG, "need 1 <= workers <= 16");
    if (cfg->max_batch_rhs < 1 || cfg->max_batch_rhs > MAX_RHS)
        fail(ASKIT_ERR_INVALID_ARG, "need 1 <= max_batch_rhs <= 64");
    if (cfg->max_batch_queries < 1) fail(ASKIT_ERR_INVALID_ARG, "need max_batch_queries >= 1");
    if (cfg->weight_passes < 0 || cfg->weight_passes > 4096)
        fail(ASKIT_ERR_INVALID_ARG, "need 0 <= weight_passes <= 4096");
    if (cfg->max_pending < 0) fail(ASKIT_ERR_INVALID_ARG, "need max_pending >= 0");
    if (nrhs0 < 1 || nrhs0 > MAX_RHS || ldw0 < nrhs0) fail(ASKIT_ERR_INVALID_ARG, "bad resident weights");
    std::unique_ptr<askit_server> sv(new askit_server());
    sv->h = h;
    sv->cfg = *cfg;
    if (sv->cfg.mem_budget == 0) sv->cfg.mem_budget = 8ull << 30;
    HIPC(hipSetDevice(h->device));
    const int64_t nn = (int64_t)h->nodes.size();
    sv->ws0.R = nrhs0;
    HIPC(hipMalloc((void **)&sv->ws0.Wt, sizeof(float) * h->N * nrhs0));
    sv->own.push_back(sv->ws0.Wt);
    HIPC(hipMalloc((void **)&sv->ws0.Wsk, sizeof(float) * nn * h->smax * nrhs0));
    sv->own.push_back(sv->ws0.Wsk);
    HIPC(hipMemset(sv->ws0.Wsk, 0, sizeof(float) * nn * h->smax * nrhs0));
    permute_weights(h, W0, ldw0, sv->ws0, nullptr);
    upward(h, sv->ws0, nullptr);
    if (sv->cfg.weight_passes > 0) {
        // the column pool stays allocated for the server's lifetime and is
        // charged to the budget up front
        const int C = sv->cfg.max_batch_rhs;
        sv->pool_bytes = sv->weights_bytes(C);
        if (sv->pool_bytes > sv->cfg.mem_budget)
            fail(ASKIT_ERR_OUT_OF_MEMORY, "the weight column pool exceeds the server memory budget");
        sv->pool.R = C;
        HIPC(hipMalloc((void **)&sv->pool.Wt, sizeof(float) * h->N * C));
        sv->own.push_back(sv->pool.Wt);
        HIPC(hipMalloc((void **)&sv->pool.Wsk, sizeof(float) * nn * h->smax * C));
        sv->own.push_back(sv->pool.Wsk);
        HIPC(hipMemset(sv->pool.Wsk, 0, sizeof(float) * nn * h->smax * C));
        HIPC(hipMalloc((void **)&sv->pool.part, sizeof(float) * std::max<int64_t>(h->pairs.npairs, 1) * C));
        sv->own.push_back(sv->pool.part);
        sv->mem_used = sv->peak_mem = sv->pool_bytes;
        // K ranges of the chunk list with about npairs / K pairs each
        const int K = sv->cfg.weight_passes;
        const int64_t nc = h->pairs.nchunk;
        std::vector<Chunk> ch((size_t)nc);
        if (nc > 0) HIPC(hipMemcpy(ch.data(), h->pairs.chunks, sizeof(Chunk) * nc, hipMemcpyDeviceToHost));
        int64_t tot = 0;
        for (auto &c : ch) tot += c.count;
        sv->range_end.assign(K + 1, nc);
        sv->range_end[0] = 0;
        int64_t acc = 0, i = 0;
        for (int k = 1; k < K; ++k) {
            const int64_t goal = (tot * k + K - 1) / K;
            while (i < nc && acc < goal) acc += ch[(size_t)i++].count;
            sv->range_end[k] = i;
        }
    }
    HIPC(hipDeviceSynchronize());
    for (int w = 0; w < sv->cfg.workers; ++w)
        sv->workers.emplace_back([p = sv.get(), w] { p->worker_loop(w); });
    if (sv->cfg.weight_passes > 0) sv->engine = std::thread([p = sv.get()] { p->engine_loop(); });
    *out = sv.release();
    API_END
}

static askit_status submit(askit_server *s, Request r, uint64_t *ticket)
{
    if (r.bytes > s->cfg.mem_budget) fail(ASKIT_ERR_OUT_OF_MEMORY, "request exceeds the server memory budget");
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->stopping) fail(ASKIT_ERR_INVALID_ARG, "server is stopping");
    const bool cyclic = !r.query && s->cfg.weight_passes > 0;
    if (s->cfg.max_pending > 0 && (int64_t)(s->pending.size() + s->wpending.size()) >= s->cfg.max_pending)
        fail(ASKIT_ERR_BUSY, "the server's queue is full; submit again later");
    r.id = s->next_id++;
    r.t_submit = clk::now();
    if (!s->any_submit) {
        s->any_submit = true;
        s->t_first = r.t_submit;
    }
    ++s->submitted;
    *ticket = r.id;
    if (cyclic) {
        s->wpending.push_back(r);
        s->cv_work.notify_all();   // the engine shares the condition with the workers
    } else {
        s->pending.push_back(r);
        s->cv_work.notify_one();
    }
    return ASKIT_OK;
}

askit_status askit_server_submit_weights(askit_server *s, const float *W, int64_t ldw, int32_t nrhs,
                                         float *U, int64_t ldu, uint64_t *ticket)
{
    API_BEGIN
    if (!s || !W || !U || !ticket) fail(ASKIT_ERR_INVALID_ARG, "NULL argument");
    if (nrhs < 1 || nrhs > s->cfg.max_batch_rhs) fail(ASKIT_ERR_INVALID_ARG, "need 1 <= nrhs <= max_batch_rhs");
    if (ldw < nrhs || ldu < nrhs) fail(ASKIT_ERR_INVALID_ARG, "need ldw, ldu >= nrhs");
    Request r{};
    r.query = false;
    r.in = W;
    r.ld_in = ldw;
    r.rows = s->h->N;
    r.cols = nrhs;
    r.out = U;
    r.ld_out = ldu;
    r.bytes = s->cfg.weight_passes > 0 ? 0 : s->weights_bytes(nrhs);   // cyclic: the pool is charged already
    return submit(s, r, ticket);
    API_END
}

askit_status askit_server_submit_query(askit_server *s, const float *Y, int64_t M, int64_t ldy, float *U,
                                       int64_t ldu, uint64_t *ticket)
{
    API_BEGIN
    if (!s || !Y || !U || !ticket) fail(ASKIT_ERR_INVALID_ARG, "NULL argument");
    if (M < 1 || M > s->cfg.max_batch_queries) fail(ASKIT_ERR_INVALID_ARG, "need 1 <= M <= max_batch_queries");
    if (ldy < s->h->d || ldu < s->ws0.R) fail(ASKIT_ERR_INVALID_ARG, "need ldy >= d and ldu >= nrhs0");
    Request r{};
    r.query = true;
    r.in = Y;
    r.ld_in = ldy;
    r.rows = M;
    r.cols = s->ws0.R;
    r.out = U;
    r.ld_out = ldu;
    r.bytes = s->query_bytes(M);
    return submit(s, r, ticket);
    API_END
}

static int32_t state_of(askit_server *s, uint64_t ticket)
{
    auto it = s->done.find(ticket);
    if (it == s->done.end()) return 0;
    if (it->second.state < 0) g_err = it->second.err;
    return it->second.state;
}

askit_status askit_server_poll(askit_server *s, uint64_t ticket, int32_t *state)
{
    API_BEGIN
    if (!s || !state) fail(ASKIT_ERR_INVALID_ARG, "NULL argument");
    std::lock_guard<std::mutex> lk(s->mu);
    if (ticket == 0 || ticket >= s->next_id) fail(ASKIT_ERR_INVALID_ARG, "unknown ticket");
    *state = state_of(s, ticket);
    API_END
}

askit_status askit_server_wait(askit_server *s, uint64_t ticket, double timeout_s, int32_t *state)
{
    API_BEGIN
    if (!s || !state) fail(ASKIT_ERR_INVALID_ARG, "NULL argument");
    std::unique_lock<std::mutex> lk(s->mu);
    if (ticket == 0 || ticket >= s->next_id) fail(ASKIT_ERR_INVALID_ARG, "unknown ticket");
    auto ready = [&] { return s->done.count(ticket) > 0; };
    if (timeout_s < 0) s->cv_done.wait(lk, ready);
    else s->cv_done.wait_for(lk, std::chrono::duration<double>(timeout_s), ready);
    *state = state_of(s, ticket);
    API_END
}

askit_status askit_server_stats(askit_server *s, askit_serving_stats *o)
{
    API_BEGIN
    if (!s || !o) fail(ASKIT_ERR_INVALID_ARG, "NULL argument");
    std::lock_guard<std::mutex> lk(s->mu);
    std::memset(o, 0, sizeof(*o));
    o->submitted = s->submitted;
    o->completed = s->completed;
    o->failed = s->failed;
    o->deferred = s->deferred;
    o->batches = s->batches;
    o->batched_requests = s->batched;
    o->p50_ms = percentile(s->lat_all, 0.50);
    o->p99_ms = percentile(s->lat_all, 0.99);
    double sum = 0.0;
    for (double v : s->lat_all) sum += v;
    o->mean_ms = s->lat_all.empty() ? 0.0 : sum / (double)s->lat_all.size();
    o->p50_weights_ms = percentile(s->lat_w, 0.50);
    o->p99_weights_ms = percentile(s->lat_w, 0.99);
    o->p50_query_ms = percentile(s->lat_q, 0.50);
    o->p99_query_ms = percentile(s->lat_q, 0.99);
    o->targets_rhs = s->targets_rhs;
    o->busy_s = s->any_submit ? std::chrono::duration<double>(s->t_last - s->t_first).count() : 0.0;
    o->peak_mem = s->peak_mem;
    o->joined_mid_cycle = s->joined;
    API_END
}

void askit_server_destroy(askit_server *s)
{
    if (!s) return;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stopping = true;
    }
    s->cv_work.notify_all();
    for (auto &t : s->workers) t.join();
    if (s->engine.joinable()) s->engine.join();
    for (void *p : s->own) (void)hipFree(p);
    delete s;
}

}  // extern "C"
