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
    int64_t submitted = 0, completed = 0, failed = 0, deferred = 0, batches = 0, batched = 0;
    double targets_rhs = 0.0;
    std::vector<double> lat_all, lat_w, lat_q;
    bool any_submit = false;
    clk::time_point t_first, t_last;

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
        const auto t_end = clk::now();
        {
            std::lock_guard<std::mutex> lk(mu);
            for (auto &r : batch) {
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
    HIPC(hipDeviceSynchronize());
    for (int w = 0; w < sv->cfg.workers; ++w)
        sv->workers.emplace_back([p = sv.get(), w] { p->worker_loop(w); });
    *out = sv.release();
    API_END
}

static askit_status submit(askit_server *s, Request r, uint64_t *ticket)
{
    if (r.bytes > s->cfg.mem_budget) fail(ASKIT_ERR_OUT_OF_MEMORY, "request exceeds the server memory budget");
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->stopping) fail(ASKIT_ERR_INVALID_ARG, "server is stopping");
    r.id = s->next_id++;
    r.t_submit = clk::now();
    if (!s->any_submit) {
        s->any_submit = true;
        s->t_first = r.t_submit;
    }
    ++s->submitted;
    *ticket = r.id;
    s->pending.push_back(r);
    s->cv_work.notify_one();
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
    r.bytes = s->weights_bytes(nrhs);
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
    for (void *p : s->own) (void)hipFree(p);
    delete s;
}

}  // extern "C"
