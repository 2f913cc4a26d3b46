// u = K w for a weight block without any device allocation: the upward pass
// and the evaluation of askit_update_weights + askit_evaluate, with their
// working buffers (weights in tree order, skeleton weights, per-pair partial
// sums) carved from one file-scope device array instead of allocations.
#include "askit_impl.h"

#include <mutex>
#include <new>
#include <string>

namespace {

constexpr size_t NOALLOC_SCRATCH_BYTES = 256ull << 20;   // ASKIT_NOALLOC_SCRATCH_BYTES in askit.h

// One copy per device, held until the process ends.  In host code this name is
// only a stand-in: its device address comes from hipGetSymbolAddress below.
static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];

constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[MAX_DEVICES] = {};

// Device address of `scratch` on `dev`, looked up once per device with that
// device current.
void *scratch_on(int dev)
{
    if (dev < 0 || dev >= MAX_DEVICES) askit::fail(ASKIT_ERR_DEVICE, "device index out of range");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        int cur = 0;
        HIPC(hipGetDevice(&cur));
        if (cur != dev) HIPC(hipSetDevice(dev));
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (cur != dev) HIPC(hipSetDevice(cur));
        HIPC(e);
        if (!p) askit::fail(ASKIT_ERR_DEVICE, "no device address for the scratch array");
        g_scratch_ptr[dev] = p;
    }
    return g_scratch_ptr[dev];
}

inline size_t up256(size_t b) { return (b + 255) / 256 * 256; }

}  // namespace

using namespace askit;

namespace askit {
extern thread_local std::string g_err;
}

extern "C" askit_status askit_evaluate_weights_noalloc(askit_handle *h, const float *W, int64_t ldw, int32_t nrhs,
                                                       float *U, int64_t ldu, void *stream)
{
    try {
        g_err.clear();
        if (!h || !W || !U) fail(ASKIT_ERR_INVALID_ARG, "NULL argument");
        if (nrhs < 1 || nrhs > MAX_RHS) fail(ASKIT_ERR_INVALID_ARG, "need 1 <= nrhs <= 64");
        if (ldw < nrhs || ldu < nrhs) fail(ASKIT_ERR_INVALID_ARG, "need ldw >= nrhs and ldu >= nrhs");
        const int64_t nn = (int64_t)h->nodes.size();
        const size_t b_wt = up256(sizeof(float) * (size_t)h->N * nrhs);
        const size_t b_wsk = up256(sizeof(float) * (size_t)nn * h->smax * nrhs);
        const size_t b_part = up256(sizeof(float) * (size_t)std::max<int64_t>(h->pairs.npairs, 1) * nrhs);
        if (b_wt + b_wsk + b_part > NOALLOC_SCRATCH_BYTES)
            fail(ASKIT_ERR_UNSUPPORTED, "working buffers of " + std::to_string(b_wt + b_wsk + b_part) +
                                            " bytes exceed the fixed scratch of " +
                                            std::to_string(NOALLOC_SCRATCH_BYTES) + " bytes (fewer columns fit)");
        unsigned char *base = (unsigned char *)scratch_on(h->device);
        WeightSet ws;
        ws.R = nrhs;
        ws.Wt = (float *)base;
        ws.Wsk = (float *)(base + b_wt);
        ws.part = (float *)(base + b_wt + b_wsk);
        // every value read below is written first in the same call (the
        // permutation writes all of Wt, the upward pass the first k rows of
        // each node's skeleton weights, the evaluation every pair slot), so
        // nothing needs clearing; the previous call's contents are never read
        hipStream_t s = (hipStream_t)stream;
        permute_weights(h, W, ldw, ws, s);
        upward(h, ws, s);
        evaluate(h, ws, h->Xt, h->pairs, h->perm, U, ldu, ws.part, s);
    } catch (const Error &e) {
        g_err = e.msg;
        return e.code;
    } catch (const std::bad_alloc &) {
        g_err = "host allocation failed";
        return ASKIT_ERR_OUT_OF_MEMORY;
    } catch (...) {
        g_err = "internal error";
        return ASKIT_ERR_DEVICE;
    }
    return ASKIT_OK;
}
