// Source-centric regrouping of the interaction lists for the evaluation.
//
// The slab lists (per 64 consecutive targets: near leaves and pruned nodes,
// each with a 64-bit mask of the targets that use it) describe the same
// (target, source node) pairs as Alg. 4's per-target recursion.  Here every
// source node and kind (near: the leaf's points; far: the node's skeleton)
// receives the list of its targets, so that the evaluation computes exactly
// the pairs the method needs (no masked-off rows), in dense chunks of 64
// targets.  Each (target, source node) pair also gets a slot: its rank in
// the target's own list (near entries, then far, in list order).  The
// evaluation writes one partial sum per slot, and a final pass adds a
// target's slots in slot order, so the result does not depend on the order
// in which chunks run.
#include "askit_impl.h"

namespace askit {

// ---- exclusive prefix sums of int32 counts (out[i] = in[0] + ... + in[i-1]):
// blocks of 1024 values scanned in registers and across waves, the block
// totals scanned the same way (recursively), then added back.
constexpr int SC_T = 256, SC_E = 4;

__global__ __launch_bounds__(SC_T) void k_scan_block(const int32_t *__restrict__ in, int64_t n,
                                                     int32_t *__restrict__ out, int32_t *__restrict__ bsum)
{
    __shared__ int32_t wsum[SC_T / 64];
    const int64_t b0 = (int64_t)blockIdx.x * SC_T * SC_E;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    int32_t v[SC_E];
    int32_t tsum = 0;
#pragma unroll
    for (int u = 0; u < SC_E; ++u) {
        const int64_t i = b0 + (int64_t)tid * SC_E + u;
        v[u] = i < n ? in[i] : 0;
        tsum += v[u];
    }
    int32_t x = tsum;                        // inclusive prefix over the wave's threads
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int32_t y = __shfl_up(x, o);
        if (lane >= o) x += y;
    }
    if (lane == 63) wsum[wv] = x;
    __syncthreads();
    int32_t run = x - tsum;
    for (int w = 0; w < wv; ++w) run += wsum[w];
#pragma unroll
    for (int u = 0; u < SC_E; ++u) {
        const int64_t i = b0 + (int64_t)tid * SC_E + u;
        if (i < n) out[i] = run;
        run += v[u];
    }
    if (tid == SC_T - 1) bsum[blockIdx.x] = run;
}

__global__ void k_scan_add(int32_t *__restrict__ out, int64_t n, const int32_t *__restrict__ boff)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] += boff[i / (SC_T * SC_E)];
}

static void exclusive_scan(const int32_t *in, int32_t *out, int64_t n, const std::function<void *(size_t)> &ta,
                           hipStream_t s)
{
    if (n <= 0) return;
    const int64_t per = SC_T * SC_E, nb = (n + per - 1) / per;
    int32_t *bsum = (int32_t *)ta(sizeof(int32_t) * nb);
    hipLaunchKernelGGL(k_scan_block, dim3((unsigned)nb), dim3(SC_T), 0, s, in, n, out, bsum);
    HIPC(hipGetLastError());
    if (nb > 1) {
        int32_t *boff = (int32_t *)ta(sizeof(int32_t) * nb);
        exclusive_scan(bsum, boff, nb, ta, s);
        hipLaunchKernelGGL(k_scan_add, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, out, n, boff);
        HIPC(hipGetLastError());
    }
}

// sort keys: (source key << 32) | entry; entries past ne are padding
__global__ void k_pair_sortkeys(const uint32_t *__restrict__ key, int64_t ne, int64_t n2, uint64_t *__restrict__ k64)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n2) return;
    k64[e] = e < ne ? (((uint64_t)key[e] << 32) | (uint64_t)e) : ~0ull;
}

__global__ void k_pair_sorted_idx(const uint64_t *__restrict__ k64, int64_t ne, int32_t *__restrict__ idx_s)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < ne) idx_s[i] = (int32_t)(k64[i] & 0xffffffffull);
}

// Segment of every list entry: the segment of its slab (`pad`).
__global__ void k_entry_seg(const Slab *__restrict__ slabs, int64_t nslab, const int32_t *__restrict__ ptr,
                            int32_t *__restrict__ eseg)
{
    const int64_t s = blockIdx.x;
    const int32_t sg = slabs[s].pad;
    for (int e = ptr[s] + threadIdx.x; e < ptr[s + 1]; e += blockDim.x) eseg[e] = sg;
    for (int e = ptr[nslab + 1 + s] + threadIdx.x; e < ptr[nslab + 2 + s]; e += blockDim.x) eseg[e] = sg;
}

__global__ void k_pair_keys(const int32_t *__restrict__ node, const uint64_t *__restrict__ mask,
                            int64_t ne_near, int64_t ne, const int32_t *__restrict__ eseg, int64_t nn,
                            uint32_t *__restrict__ key, int32_t *__restrict__ cnt)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= ne) return;
    const uint32_t k = (uint32_t)((eseg ? (int64_t)eseg[e] * nn : 0) + node[e]) * 2u + (e >= ne_near ? 1u : 0u);
    key[e] = k;
    atomicAdd(&cnt[k], __popcll(mask[e]));      // integer counts: order-independent
}

__global__ void k_sorted_popc(const int32_t *__restrict__ sorted_e, const uint64_t *__restrict__ mask,
                              int64_t ne, int32_t *__restrict__ pc)
{
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s < ne) pc[s] = __popcll(mask[sorted_e[s]]);
}

__global__ void k_scatter_off(const int32_t *__restrict__ sorted_e, const int32_t *__restrict__ off_sorted,
                              int64_t ne, int32_t *__restrict__ off_e)
{
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s < ne) off_e[sorted_e[s]] = off_sorted[s];
}

// One wave per slab; lane b counts the entries whose mask holds row b.
__global__ __launch_bounds__(64) void k_target_counts(const Slab *__restrict__ slabs, int64_t nslab,
                                                      const int32_t *__restrict__ ptr,
                                                      const uint64_t *__restrict__ mask,
                                                      int32_t *__restrict__ cnt_t)
{
    const int64_t s = blockIdx.x;
    const int b = threadIdx.x;
    const Slab sb = slabs[s];
    int c = 0;
    for (int part = 0; part < 2; ++part) {
        const int e0 = part ? ptr[nslab + 1 + s] : ptr[s], e1 = part ? ptr[nslab + 2 + s] : ptr[s + 1];
        for (int e = e0; e < e1; ++e) c += (int)((mask[e] >> b) & 1ull);
    }
    if (b < sb.nrows) cnt_t[sb.row0 + b] = c;
}

// One wave per slab; lane b places its row's pairs: position in the source's
// target list (entry offset + rank of b among the entry's rows) and slot
// (the row's slot base + rank of the entry among the row's entries).
__global__ __launch_bounds__(64) void k_pair_fill(const Slab *__restrict__ slabs, int64_t nslab,
                                                  const int32_t *__restrict__ ptr,
                                                  const uint64_t *__restrict__ mask,
                                                  const int32_t *__restrict__ off_e,
                                                  const int32_t *__restrict__ sbase,
                                                  int32_t *__restrict__ tpos, int32_t *__restrict__ tslot,
                                                  int32_t *__restrict__ snear)
{
    const int64_t s = blockIdx.x;
    const int b = threadIdx.x;
    const Slab sb = slabs[s];
    if (b >= sb.nrows) return;
    const uint64_t below = (b == 0) ? 0ull : (~0ull >> (64 - b));
    int r = 0;
    const int base = sbase[sb.row0 + b];
    for (int part = 0; part < 2; ++part) {
        const int e0 = part ? ptr[nslab + 1 + s] : ptr[s], e1 = part ? ptr[nslab + 2 + s] : ptr[s + 1];
        for (int e = e0; e < e1; ++e) {
            const uint64_t m = mask[e];
            if ((m >> b) & 1ull) {
                const int64_t i = (int64_t)off_e[e] + __popcll(m & below);
                tpos[i] = sb.row0 + b;
                tslot[i] = base + r;
                ++r;
            }
        }
        if (part == 0) snear[sb.row0 + b] = base + r;
    }
}

void build_pairs(const askit_handle *h, const Slab *d_slabs, int64_t nslab, int64_t ntarget, const int32_t *ptr,
                 const int32_t *node, const uint64_t *mask, int64_t ne_near, int64_t ne_far, PairLists &L,
                 const std::function<void *(size_t)> &al, hipStream_t s, int64_t nseg)
{
    const int64_t ne = ne_near + ne_far;
    const int64_t nn = (int64_t)h->nodes.size();
    if (nseg < 1 || nseg * 2 * nn >= (1ll << 31)) fail(ASKIT_ERR_UNSUPPORTED, "too many segments in one batch");
    const int64_t nkey = 2 * nn * nseg;
    L.ntarget = ntarget;
    std::vector<void *> tmp;
    auto ta = [&](size_t b) {
        void *p;
        HIPC(ws_alloc(&p, std::max<size_t>(b, 16), s));
        tmp.push_back(p);
        return p;
    };
    struct Guard {
        std::vector<void *> &t;
        hipStream_t s;
        ~Guard() { for (void *p : t) (void)ws_free(p, s); }
    } guard{tmp, s};
    int32_t *cnt = (int32_t *)ta(sizeof(int32_t) * nkey);
    HIPC(hipMemsetAsync(cnt, 0, sizeof(int32_t) * nkey, s));
    L.sbase = (int32_t *)al(sizeof(int32_t) * (ntarget + 1));
    L.snear = (int32_t *)al(sizeof(int32_t) * std::max<int64_t>(ntarget, 1));
    int32_t *cnt_t = (int32_t *)ta(sizeof(int32_t) * (ntarget + 1));
    HIPC(hipMemsetAsync(cnt_t, 0, sizeof(int32_t) * (ntarget + 1), s));
    if (nslab > 0)
        hipLaunchKernelGGL(k_target_counts, dim3((unsigned)nslab), dim3(64), 0, s, d_slabs, nslab, ptr, mask,
                           cnt_t);
    HIPC(hipGetLastError());
    exclusive_scan(cnt_t, L.sbase, ntarget + 1, ta, s);

    int32_t *off_e = (int32_t *)ta(sizeof(int32_t) * std::max<int64_t>(ne, 1));
    if (ne > 0) {
        uint32_t *key = (uint32_t *)ta(sizeof(uint32_t) * ne);
        int32_t *idx_s = (int32_t *)ta(sizeof(int32_t) * ne);
        int32_t *pc = (int32_t *)ta(sizeof(int32_t) * ne), *off_s = (int32_t *)ta(sizeof(int32_t) * ne);
        const unsigned g = (unsigned)((ne + 255) / 256);
        int32_t *eseg = nullptr;
        if (nseg > 1) {
            eseg = (int32_t *)ta(sizeof(int32_t) * ne);
            hipLaunchKernelGGL(k_entry_seg, dim3((unsigned)nslab), dim3(64), 0, s, d_slabs, nslab, ptr, eseg);
            HIPC(hipGetLastError());
        }
        hipLaunchKernelGGL(k_pair_keys, dim3(g), dim3(256), 0, s, node, mask, ne_near, ne, eseg, nn, key, cnt);
        HIPC(hipGetLastError());
        // entries by (source key, list position): the entry index in the low
        // bits keeps the entries of one source in list order
        int64_t n2 = 1;
        while (n2 < ne) n2 <<= 1;
        uint64_t *k64 = (uint64_t *)ta(sizeof(uint64_t) * n2);
        hipLaunchKernelGGL(k_pair_sortkeys, dim3((unsigned)((n2 + 255) / 256)), dim3(256), 0, s, key, ne, n2, k64);
        sort_u64_pow2(k64, n2, s);
        hipLaunchKernelGGL(k_pair_sorted_idx, dim3(g), dim3(256), 0, s, k64, ne, idx_s);
        hipLaunchKernelGGL(k_sorted_popc, dim3(g), dim3(256), 0, s, idx_s, mask, ne, pc);
        exclusive_scan(pc, off_s, ne, ta, s);
        hipLaunchKernelGGL(k_scatter_off, dim3(g), dim3(256), 0, s, idx_s, off_s, ne, off_e);
        HIPC(hipGetLastError());
    }
    // host: pair total and the chunk table (64 targets of one source per chunk)
    std::vector<int32_t> hc(nkey);
    HIPC(hipMemcpyAsync(hc.data(), cnt, sizeof(int32_t) * nkey, hipMemcpyDeviceToHost, s));
    HIPC(hipStreamSynchronize(s));
    int64_t npairs = 0;
    std::vector<Chunk> chunks;
    L.near_lists = L.far_lists = 0;
    for (int64_t k = 0; k < nkey; ++k) {
        (k & 1 ? L.far_lists : L.near_lists) += hc[k];
        for (int64_t j = 0; j < hc[k]; j += 64)
            chunks.push_back(Chunk{(int32_t)((k >> 1) % nn), (int32_t)(k & 1), (int32_t)(npairs + j),
                                   (int32_t)std::min<int64_t>(64, hc[k] - j)});
        npairs += hc[k];
    }
    if (npairs >= (1ll << 31)) fail(ASKIT_ERR_UNSUPPORTED, "more than 2^31 (target, source) pairs");
    L.npairs = npairs;
    L.nchunk = (int64_t)chunks.size();
    L.tpos = (int32_t *)al(sizeof(int32_t) * std::max<int64_t>(npairs, 1));
    L.tslot = (int32_t *)al(sizeof(int32_t) * std::max<int64_t>(npairs, 1));
    L.chunks = (Chunk *)al(sizeof(Chunk) * std::max<int64_t>(L.nchunk, 1));
    if (L.nchunk > 0)
        HIPC(hipMemcpyAsync(L.chunks, chunks.data(), sizeof(Chunk) * L.nchunk, hipMemcpyHostToDevice, s));
    if (nslab > 0 && npairs > 0)
        hipLaunchKernelGGL(k_pair_fill, dim3((unsigned)nslab), dim3(64), 0, s, d_slabs, nslab, ptr, mask, off_e,
                           L.sbase, L.tpos, L.tslot, L.snear);
    HIPC(hipGetLastError());
    HIPC(hipStreamSynchronize(s));          // the chunk table's host copy is released on return
}

}  // namespace askit
