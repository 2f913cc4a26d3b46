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

#include <hipcub/hipcub.hpp>

namespace askit {

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
                            uint32_t *__restrict__ key, int32_t *__restrict__ idx, int32_t *__restrict__ cnt)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= ne) return;
    const uint32_t k = (uint32_t)((eseg ? (int64_t)eseg[e] * nn : 0) + node[e]) * 2u + (e >= ne_near ? 1u : 0u);
    key[e] = k;
    idx[e] = (int32_t)e;
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
        HIPC(hipMallocAsync(&p, std::max<size_t>(b, 16), s));
        tmp.push_back(p);
        return p;
    };
    struct Guard {
        std::vector<void *> &t;
        hipStream_t s;
        ~Guard() { for (void *p : t) (void)hipFreeAsync(p, s); }
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
    size_t tb = 0;
    HIPC(hipcub::DeviceScan::ExclusiveSum(nullptr, tb, cnt_t, L.sbase, (int)(ntarget + 1), s));
    void *tstore = ta(tb);
    HIPC(hipcub::DeviceScan::ExclusiveSum(tstore, tb, cnt_t, L.sbase, (int)(ntarget + 1), s));

    int32_t *off_e = (int32_t *)ta(sizeof(int32_t) * std::max<int64_t>(ne, 1));
    if (ne > 0) {
        uint32_t *key = (uint32_t *)ta(sizeof(uint32_t) * ne), *key_s = (uint32_t *)ta(sizeof(uint32_t) * ne);
        int32_t *idx = (int32_t *)ta(sizeof(int32_t) * ne), *idx_s = (int32_t *)ta(sizeof(int32_t) * ne);
        int32_t *pc = (int32_t *)ta(sizeof(int32_t) * ne), *off_s = (int32_t *)ta(sizeof(int32_t) * ne);
        const unsigned g = (unsigned)((ne + 255) / 256);
        int32_t *eseg = nullptr;
        if (nseg > 1) {
            eseg = (int32_t *)ta(sizeof(int32_t) * ne);
            hipLaunchKernelGGL(k_entry_seg, dim3((unsigned)nslab), dim3(64), 0, s, d_slabs, nslab, ptr, eseg);
            HIPC(hipGetLastError());
        }
        hipLaunchKernelGGL(k_pair_keys, dim3(g), dim3(256), 0, s, node, mask, ne_near, ne, eseg, nn, key, idx, cnt);
        HIPC(hipGetLastError());
        int bits = 1;
        while (((int64_t)1 << bits) < nkey) ++bits;
        size_t sb = 0;
        HIPC(hipcub::DeviceRadixSort::SortPairs(nullptr, sb, key, key_s, idx, idx_s, (int)ne, 0, bits, s));
        void *sstore = ta(sb);
        // LSD radix sort is stable: the entries of one source stay in list order
        HIPC(hipcub::DeviceRadixSort::SortPairs(sstore, sb, key, key_s, idx, idx_s, (int)ne, 0, bits, s));
        hipLaunchKernelGGL(k_sorted_popc, dim3(g), dim3(256), 0, s, idx_s, mask, ne, pc);
        size_t eb = 0;
        HIPC(hipcub::DeviceScan::ExclusiveSum(nullptr, eb, pc, off_s, (int)ne, s));
        void *estore = ta(eb);
        HIPC(hipcub::DeviceScan::ExclusiveSum(estore, eb, pc, off_s, (int)ne, s));
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
