// Node neighbour lists (Alg. 2), sampled rows (Eq. e:sk_targets) and the
// interaction lists of the downward pass (Eq. e:prune, Alg. 4).
#include "askit_impl.h"

#include <algorithm>

namespace askit {

// ====================================================================
// Node neighbour lists.  A list is a set of (key, position) with key the
// FP64 squared distance (non-negative, so its bit pattern orders like the
// value).  reduce_list() drops positions inside [lo, hi), keeps the
// smallest key per position, sorts by (key, position) and cuts to l.
// A leaf's list is the reduction of all (D(x_i, x_j), pos j) over its
// points i and their neighbours j.  Applying the reduction to the leaf's
// points in chunks and feeding each chunk's result into the next gives the
// same list: an entry of the final l smallest is among the l smallest of
// the chunk that holds its smallest key.  An internal node reduces the
// union of its children's stored lists (Alg. 2, second line).
// ====================================================================
// CAP entries of LDS buffer per workgroup: 1024 (24 KiB, six workgroups per
// CU) when a chunk of neighbours plus a kept list (l + kappa) and the union
// of two children's lists (2 l) fit, else 2048 (48 KiB).
constexpr int NL_CAP = 2048;                // largest buffer
constexpr int NL_T = 256;

template <int CAP>
struct NLShared {
    uint64_t k[2][CAP];
    int32_t p[2][CAP];
    int32_t cnt;
    int32_t wsum[NL_T / 64];
};

__device__ __forceinline__ bool lt_pk(int32_t p1, uint64_t k1, int32_t p2, uint64_t k2)
{
    return p1 < p2 || (p1 == p2 && k1 < k2);
}
__device__ __forceinline__ bool lt_kp(uint64_t k1, int32_t p1, uint64_t k2, int32_t p2)
{
    return k1 < k2 || (k1 == k2 && p1 < p2);
}

template <bool BY_POS>
__device__ void bitonic_lds(uint64_t *k, int32_t *p, int n2)
{
    for (int kk = 2; kk <= n2; kk <<= 1) {
        for (int j = kk >> 1; j > 0; j >>= 1) {
            for (int t = threadIdx.x; t < n2 / 2; t += blockDim.x) {
                int i = 2 * t - (t & (j - 1));
                int q = i + j;
                bool up = (i & kk) == 0;
                bool gt = BY_POS ? lt_pk(p[q], k[q], p[i], k[i]) : lt_kp(k[q], p[q], k[i], p[i]);
                bool lt = BY_POS ? lt_pk(p[i], k[i], p[q], k[q]) : lt_kp(k[i], p[i], k[q], p[q]);
                if (up ? gt : lt) {
                    uint64_t tk = k[i]; k[i] = k[q]; k[q] = tk;
                    int32_t tp = p[i]; p[i] = p[q]; p[q] = tp;
                }
            }
            __syncthreads();
        }
    }
}

// Entries in buffer 0 [0, n); result (<= ell) in buffer 0 [0, return).
template <int CAP>
__device__ int reduce_list(NLShared<CAP> &S, int n, int ell)
{
    int n2 = 1;
    while (n2 < n) n2 <<= 1;
    for (int i = n + threadIdx.x; i < n2; i += blockDim.x) {
        S.k[0][i] = ~0ull;
        S.p[0][i] = 0x7fffffff;
    }
    __syncthreads();
    bitonic_lds<true>(S.k[0], S.p[0], n2);
    // keep the first entry of every position (its smallest key), compact to buffer 1
    const int per = (n2 + NL_T - 1) / NL_T;
    const int b0 = threadIdx.x * per;
    int mine = 0;
    for (int i = b0; i < min(b0 + per, n); ++i)
        mine += (i == 0 || S.p[0][i] != S.p[0][i - 1]);
    // block exclusive scan of `mine`
    int lane = threadIdx.x % 64, w = threadIdx.x / 64;
    int incl = mine;
    for (int o = 1; o < 64; o <<= 1) {
        int v = __shfl_up(incl, o);
        if (lane >= o) incl += v;
    }
    if (lane == 63) S.wsum[w] = incl;
    __syncthreads();
    int off = incl - mine;
    for (int v = 0; v < w; ++v) off += S.wsum[v];
    int total = 0;
    for (int v = 0; v < NL_T / 64; ++v) total += S.wsum[v];
    for (int i = b0; i < min(b0 + per, n); ++i)
        if (i == 0 || S.p[0][i] != S.p[0][i - 1]) {
            S.k[1][off] = S.k[0][i];
            S.p[1][off] = S.p[0][i];
            ++off;
        }
    __syncthreads();
    int u = total;
    int u2 = 1;
    while (u2 < u) u2 <<= 1;
    for (int i = u + threadIdx.x; i < u2; i += blockDim.x) {
        S.k[1][i] = ~0ull;
        S.p[1][i] = 0x7fffffff;
    }
    __syncthreads();
    if (u > 1) bitonic_lds<false>(S.k[1], S.p[1], u2);
    int keep = min(u, ell);
    for (int i = threadIdx.x; i < keep; i += blockDim.x) {
        S.k[0][i] = S.k[1][i];
        S.p[0][i] = S.p[1][i];
    }
    __syncthreads();
    return keep;
}

template <int CAP>
__global__ __launch_bounds__(NL_T) void k_leaf_nlists(const Node *__restrict__ nodes,
                                                      const int32_t *__restrict__ leaves,
                                                      const int32_t *__restrict__ perm,
                                                      const int32_t *__restrict__ iperm,
                                                      const int32_t *__restrict__ knn_idx,
                                                      const double *__restrict__ knn_d, int kappa,
                                                      int ell, int32_t *__restrict__ nl_pos,
                                                      double *__restrict__ nl_key,
                                                      int32_t *__restrict__ nl_cnt)
{
    __shared__ NLShared<CAP> S;
    const int a = leaves[blockIdx.x];
    const Node nd = nodes[a];
    const int chunk = max(1, (CAP - ell) / kappa);
    // Once the reduced list holds ell entries its ell-th (key, position) bounds
    // the final ell-th from above (more entries only lower a position's key or
    // add positions), so entries at or above it are dropped when read; the
    // buffer is reduced only when the next chunk might not fit, and at the end.
    uint64_t tk = ~0ull;
    int32_t tp = 0x7fffffff;
    int cur = 0;
    if (threadIdx.x == 0) S.cnt = 0;
    __syncthreads();
    for (int c0 = nd.lo; c0 < nd.hi; c0 += chunk) {
        const int c1 = min(nd.hi, c0 + chunk);
        const int tot = (c1 - c0) * kappa;
        for (int e = threadIdx.x; e < tot; e += blockDim.x) {
            const int i = c0 + e / kappa, t = e % kappa;
            const int64_t o = perm[i];
            const int pj = iperm[knn_idx[o * kappa + t]];
            if (pj >= nd.lo && pj < nd.hi) continue;
            const uint64_t key = (uint64_t)__double_as_longlong(knn_d[o * kappa + t]);
            if (!lt_kp(key, pj, tk, tp)) continue;
            const int slot = atomicAdd(&S.cnt, 1);
            S.p[0][slot] = pj;
            S.k[0][slot] = key;
        }
        __syncthreads();
        const int n = S.cnt;
        __syncthreads();
        if (c1 >= nd.hi || n + chunk * kappa > CAP) {
            cur = reduce_list(S, n, ell);
            if (cur == ell) {
                tk = S.k[0][ell - 1];
                tp = S.p[0][ell - 1];
            }
            if (threadIdx.x == 0) S.cnt = cur;
            __syncthreads();
        }
    }
    for (int t = threadIdx.x; t < cur; t += blockDim.x) {
        nl_pos[(int64_t)a * ell + t] = S.p[0][t];
        nl_key[(int64_t)a * ell + t] = __longlong_as_double((long long)S.k[0][t]);
    }
    if (threadIdx.x == 0) nl_cnt[a] = cur;
}

template <int CAP>
__global__ __launch_bounds__(NL_T) void k_internal_nlists(const Node *__restrict__ nodes,
                                                          const int32_t *__restrict__ ids, int ell,
                                                          int32_t *__restrict__ nl_pos,
                                                          double *__restrict__ nl_key,
                                                          int32_t *__restrict__ nl_cnt)
{
    __shared__ NLShared<CAP> S;
    const int a = ids[blockIdx.x];
    const Node nd = nodes[a];
    if (threadIdx.x == 0) S.cnt = 0;
    __syncthreads();
    const int ch[2] = {nd.left, nd.right};
    for (int c = 0; c < 2; ++c) {
        int n = nl_cnt[ch[c]];
        for (int t = threadIdx.x; t < n; t += blockDim.x) {
            int pj = nl_pos[(int64_t)ch[c] * ell + t];
            if (pj >= nd.lo && pj < nd.hi) continue;
            int slot = atomicAdd(&S.cnt, 1);
            S.p[0][slot] = pj;
            S.k[0][slot] = (uint64_t)__double_as_longlong(nl_key[(int64_t)ch[c] * ell + t]);
        }
    }
    __syncthreads();
    int n = S.cnt;
    __syncthreads();
    int cur = reduce_list(S, n, ell);
    for (int t = threadIdx.x; t < cur; t += blockDim.x) {
        nl_pos[(int64_t)a * ell + t] = S.p[0][t];
        nl_key[(int64_t)a * ell + t] = __longlong_as_double((long long)S.k[0][t]);
    }
    if (threadIdx.x == 0) nl_cnt[a] = cur;
}

void build_node_lists(askit_handle *h, hipStream_t s)
{
    if (h->ell > NL_CAP / 2 || h->kappa > NL_CAP / 2)
        fail(ASKIT_ERR_UNSUPPORTED, "sample_rows and kappa must be at most 1024");
    int nn = (int)h->nodes.size();
    HIPC(hipMemsetAsync(h->nl_cnt, 0, sizeof(int32_t) * nn, s));
    if (h->depth == 0) return;
    std::vector<int32_t> lv(h->leaves.begin(), h->leaves.end());
    int32_t *d_ids;
    HIPC(ws_alloc((void **)&d_ids, sizeof(int32_t) * nn, s));
    HIPC(hipMemcpyAsync(d_ids, lv.data(), sizeof(int32_t) * lv.size(), hipMemcpyHostToDevice, s));
    const bool small = h->ell + h->kappa <= NL_CAP / 2 && 2 * h->ell <= NL_CAP / 2;
    if (small)
        hipLaunchKernelGGL(k_leaf_nlists<NL_CAP / 2>, dim3((unsigned)lv.size()), dim3(NL_T), 0, s, h->d_nodes, d_ids,
                           h->perm, h->iperm, h->knn_idx, h->knn_d, h->kappa, h->ell, h->nl_pos, h->nl_key,
                           h->nl_cnt);
    else
        hipLaunchKernelGGL(k_leaf_nlists<NL_CAP>, dim3((unsigned)lv.size()), dim3(NL_T), 0, s, h->d_nodes, d_ids,
                           h->perm, h->iperm, h->knn_idx, h->knn_d, h->kappa, h->ell, h->nl_pos, h->nl_key,
                           h->nl_cnt);
    HIPC(hipGetLastError());
    // internal nodes bottom-up, root excluded (its list is empty by definition)
    std::vector<int32_t> ids;
    for (int lev = h->depth - 1; lev >= 1; --lev) {
        ids.clear();
        for (int a : h->level_nodes[lev])
            if (h->nodes[a].left >= 0) ids.push_back(a);
        if (ids.empty()) continue;
        HIPC(hipStreamSynchronize(s));   // d_ids is reused on the host side
        HIPC(hipMemcpyAsync(d_ids, ids.data(), sizeof(int32_t) * ids.size(), hipMemcpyHostToDevice, s));
        if (small)
            hipLaunchKernelGGL(k_internal_nlists<NL_CAP / 2>, dim3((unsigned)ids.size()), dim3(NL_T), 0, s,
                               h->d_nodes, d_ids, h->ell, h->nl_pos, h->nl_key, h->nl_cnt);
        else
            hipLaunchKernelGGL(k_internal_nlists<NL_CAP>, dim3((unsigned)ids.size()), dim3(NL_T), 0, s,
                               h->d_nodes, d_ids, h->ell, h->nl_pos, h->nl_key, h->nl_cnt);
        HIPC(hipGetLastError());
    }
    HIPC(hipStreamSynchronize(s));
    HIPC(ws_free(d_ids, s));
}

// ====================================================================
// Sampled rows (Eq. e:sk_targets).  T_alpha = N_alpha followed by
// r = min(l - |N_alpha|, N - n_alpha - |N_alpha|) positions drawn uniformly
// without replacement outside alpha and outside N_alpha, from the
// SplitMix64 stream of the node (Steele, Lea, Flood 2014): output t is
// mix(base + (t + 1) * 0x9E3779B97F4A7C15), base = seed ^ (key * golden),
// key = (level << 48) | path.  Draw: v = z mod (N - n_alpha), pos = v if
// v < lo else v + n_alpha, rejected if already in T_alpha.  When the pool
// holds at most 2r positions they are listed in increasing order and the
// first r of a Fisher-Yates shuffle (swap t with t + z_t mod (pool - t))
// are taken.  One wave per node; membership tests use the whole wave.
// ====================================================================
constexpr uint64_t GOLDEN = 0x9E3779B97F4A7C15ull;
constexpr int SMP_MAX_ELL = 1024;

__device__ __forceinline__ uint64_t sm64(uint64_t base, uint64_t t)
{
    uint64_t z = base + (t + 1) * GOLDEN;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

__device__ __forceinline__ bool wave_member(const int32_t *arr, int n, int32_t v, int lane)
{
    bool f = false;
    for (int i = lane; i < n; i += 64) f |= arr[i] == v;
    return __ballot(f) != 0;
}

__global__ __launch_bounds__(64) void k_sample(const Node *__restrict__ nodes, int nn, int64_t N, int ell,
                                               uint64_t seed, const int32_t *__restrict__ nl_pos,
                                               const int32_t *__restrict__ nl_cnt,
                                               int32_t *__restrict__ T, int32_t *__restrict__ T_cnt)
{
    __shared__ int32_t sT[SMP_MAX_ELL];
    __shared__ int32_t pool[3 * SMP_MAX_ELL];
    const int a = blockIdx.x + 1;               // the root has no sampled rows
    const int lane = threadIdx.x;
    const Node nd = nodes[a];
    const int64_t na = nd.hi - nd.lo;
    const int c = nl_cnt[a];
    for (int t = lane; t < c; t += 64) sT[t] = nl_pos[(int64_t)a * ell + t];
    __syncthreads();
    const int64_t npool = N - na - c;
    const int64_t r = min((int64_t)(ell - c), npool);
    const uint64_t key = ((uint64_t)nd.level << 48) | (uint64_t)nd.path;
    const uint64_t base = seed ^ (key * GOLDEN);
    if (r > 0 && npool <= 2 * r) {
        int q = 0;
        for (int64_t p = 0; p < N; ++p) {
            if (p >= nd.lo && p < nd.hi) {
                p = nd.hi - 1;
                continue;
            }
            if (wave_member(sT, c, (int32_t)p, lane)) continue;
            if (lane == 0) pool[q] = (int32_t)p;
            ++q;
        }
        __syncthreads();
        if (lane == 0)
            for (int64_t t = 0; t < r; ++t) {
                uint64_t z = sm64(base, (uint64_t)t);
                int64_t sidx = t + (int64_t)(z % (uint64_t)(npool - t));
                int32_t tmp = pool[t];
                pool[t] = pool[sidx];
                pool[sidx] = tmp;
                sT[c + t] = pool[t];
            }
        __syncthreads();
    } else if (r > 0) {
        // 64 draws at a time, draw t0 + i in lane i.  One at a time, a draw is
        // rejected exactly when its position is already listed; within a
        // batch that is: listed before the batch, or equal to an earlier draw
        // of the batch (which was either taken or itself rejected as listed).
        // The accepted draws, appended in draw order up to the r-th, are
        // therefore those of the one-at-a-time loop.
        int g = 0;
        for (uint64_t t0 = 0; g < r; t0 += 64) {
            const uint64_t z = sm64(base, t0 + (uint64_t)lane);
            const int64_t v = (int64_t)(z % (uint64_t)(N - na));
            const int32_t pos = (int32_t)(v < nd.lo ? v : v + na);
            const int n0 = c + g;
            bool dup = false;
            for (int i = 0; i < n0; ++i) dup |= sT[i] == pos;
            for (int j = 0; j < 63; ++j) {
                const int32_t pj = __shfl(pos, j);        // every lane takes part
                dup |= j < lane && pj == pos;
            }
            const uint64_t ok = __ballot(!dup);
            const int before = __popcll(ok & ((1ull << lane) - 1ull));
            const int take = (int)min<int64_t>((int64_t)__popcll(ok), r - g);
            __syncthreads();
            if (!dup && before < take) sT[n0 + before] = pos;
            g += take;
            __syncthreads();
        }
    }
    const int tot = c + (int)max((int64_t)0, r);
    __syncthreads();
    for (int t = lane; t < tot; t += 64) T[(int64_t)a * ell + t] = sT[t];
    if (lane == 0) T_cnt[a] = tot;
}

void sample_rows(askit_handle *h, hipStream_t s)
{
    int nn = (int)h->nodes.size();
    if (h->ell > SMP_MAX_ELL) fail(ASKIT_ERR_UNSUPPORTED, "sample_rows above 1024 is not supported");
    HIPC(hipMemsetAsync(h->T_cnt, 0, sizeof(int32_t) * nn, s));
    if (nn <= 1) return;
    hipLaunchKernelGGL(k_sample, dim3(nn - 1), dim3(64), 0, s, h->d_nodes, nn, h->N, h->ell,
                       h->prm.seed, h->nl_pos, h->nl_cnt, h->T, h->T_cnt);
    HIPC(hipGetLastError());
}

// ====================================================================
// Interaction lists.  For target i with neighbour positions nb(i) (its own
// position and those of its kappa neighbours; for a query point, its kappa
// neighbours), A(i) = the nodes holding at least one of nb(i).  Alg. 4
// evaluates the leaves in A(i) directly ("near") and the nodes beta not in
// A(i) whose parent is in A(i) by their skeletons ("far").  Targets are
// grouped in slabs of 64; each slab gets the union of its rows' near and far
// nodes, each with a 64-bit mask of the rows that use it.  Near entries are
// ordered by leaf id, far entries by node id.
// ====================================================================
__device__ __forceinline__ bool has_nb(const int32_t *nb, int n, int lo, int hi)
{
    int a = 0, b = n;                 // first entry >= lo
    while (a < b) {
        int mid = (a + b) >> 1;
        if (nb[mid] < lo) a = mid + 1;
        else b = mid;
    }
    return a < n && nb[a] < hi;
}

// mode 0: count entries per slab; mode 1: write them.  NW waves per slab:
// wave 0 builds the rows' sorted neighbour lists and marks A (the union of
// their ancestors); the node scan is split in NW contiguous word ranges (so
// the output keeps node order), with the per-wave entry counts of mode 0
// (cntw, prefix within the slab) placing each wave's entries in mode 1.
template <int NW>
__global__ __launch_bounds__(64 * NW) void k_interactions(const Node *__restrict__ nodes, int nn,
                                                          const int32_t *__restrict__ leaf_of,
                                                          const Slab *__restrict__ slabs,
                                                          const int32_t *__restrict__ nbpos, int nnb,
                                                          int mode, int32_t *__restrict__ cnt_near,
                                                          int32_t *__restrict__ cnt_far,
                                                          const int32_t *__restrict__ ptr, int64_t nslab,
                                                          int32_t *__restrict__ out_node,
                                                          uint64_t *__restrict__ out_mask,
                                                          int32_t *__restrict__ cntw, int minlev)
{
    extern __shared__ uint32_t sh[];
    __shared__ int nm[64];
    __shared__ int wcnt[2 * NW];
    const int nwords = (nn + 31) / 32;
    uint32_t *U = sh;
    int32_t *nbs = reinterpret_cast<int32_t *>(sh + nwords);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int64_t sl = blockIdx.x;
    const Slab sb = slabs[sl];
    const bool valid = lane < sb.nrows;
    for (int w = threadIdx.x; w < nwords; w += 64 * NW) U[w] = 0;
    int32_t *mine = nbs + lane * nnb;
    if (wv == 0) {
        int nmine = 0;
        if (valid) {
            const int32_t *src = nbpos + ((int64_t)sb.row0 + lane) * nnb;
            for (int t = 0; t < nnb; ++t) {
                int32_t v = src[t];
                if (v < 0) continue;
                int q = nmine++;
                while (q > 0 && mine[q - 1] > v) {
                    mine[q] = mine[q - 1];
                    --q;
                }
                mine[q] = v;
            }
        }
        nm[lane] = nmine;
    }
    __syncthreads();
    const int nmine = nm[lane];
    if (wv == 0) {
        for (int t = 0; t < nmine; ++t) {
            int a = leaf_of[mine[t]];
            while (a >= 0) {
                uint32_t bit = 1u << (a & 31);
                uint32_t old = atomicOr(&U[a >> 5], bit);
                if (old & bit) break;
                a = nodes[a].parent;
            }
        }
    }
    __syncthreads();
    const int per = (nwords + NW - 1) / NW;
    const int w0 = min(nwords, wv * per), w1 = min(nwords, w0 + per);
    int kn = 0, kf = 0;
    int64_t on = 0, of = 0;
    if (mode) {
        on = ptr[sl] + (NW > 1 ? cntw[(sl * NW + wv) * 2] : 0);
        of = ptr[nslab + 1 + sl] + (NW > 1 ? cntw[(sl * NW + wv) * 2 + 1] : 0);
    }
    for (int w = w0; w < w1; ++w) {
        uint32_t bits = U[w];
        while (bits) {
            int b = __builtin_ctz(bits);
            bits &= bits - 1;
            int a = w * 32 + b;
            Node nd = nodes[a];
            bool in_a = valid && has_nb(mine, nmine, nd.lo, nd.hi);
            if (nd.left < 0) {
                uint64_t m = __ballot(in_a);
                if (m) {
                    if (mode && lane == 0) {
                        out_node[on + kn] = a;
                        out_mask[on + kn] = m;
                    }
                    ++kn;
                }
            } else {
                const int ch[2] = {nd.left, nd.right};
                for (int c = 0; c < 2; ++c) {
                    Node cn = nodes[ch[c]];
                    bool f = in_a && !has_nb(mine, nmine, cn.lo, cn.hi);
                    uint64_t m = __ballot(f);
                    if (!m) continue;
                    if (cn.level >= minlev) {
                        if (mode && lane == 0) {
                            out_node[of + kf] = ch[c];
                            out_mask[of + kf] = m;
                        }
                        ++kf;
                        continue;
                    }
                    // level restriction: a node above the first prunable level
                    // is not pruned; its subtree holds no neighbour of the rows
                    // in m, so they take its descendants on that level as far
                    // nodes and its leaves above that level as near leaves
                    // (depth first, left before right; uniform in the wave)
                    int stk[64];
                    int top = 0;
                    stk[top++] = ch[c];
                    while (top > 0) {
                        const int b = stk[--top];
                        const Node bn = nodes[b];
                        if (bn.level >= minlev) {
                            if (mode && lane == 0) {
                                out_node[of + kf] = b;
                                out_mask[of + kf] = m;
                            }
                            ++kf;
                        } else if (bn.left < 0) {
                            if (mode && lane == 0) {
                                out_node[on + kn] = b;
                                out_mask[on + kn] = m;
                            }
                            ++kn;
                        } else {
                            stk[top++] = bn.right;
                            stk[top++] = bn.left;
                        }
                    }
                }
            }
        }
    }
    if (!mode) {
        if (lane == 0) {
            wcnt[wv] = kn;
            wcnt[NW + wv] = kf;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            int an = 0, af = 0;
            for (int u = 0; u < NW; ++u) {
                if (NW > 1) {
                    cntw[(sl * NW + u) * 2] = an;
                    cntw[(sl * NW + u) * 2 + 1] = af;
                }
                an += wcnt[u];
                af += wcnt[NW + u];
            }
            cnt_near[sl] = an;
            cnt_far[sl] = af;
        }
    }
}

__global__ void k_nbpos_self(const int32_t *__restrict__ perm, const int32_t *__restrict__ iperm,
                             const int32_t *__restrict__ knn_idx, int64_t N, int kappa,
                             int32_t *__restrict__ nb)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    int64_t o = perm[i];
    nb[i * (kappa + 1)] = (int32_t)i;
    for (int t = 0; t < kappa; ++t) nb[i * (kappa + 1) + 1 + t] = iperm[knn_idx[o * kappa + t]];
}

__global__ void k_pair_count(const int32_t *__restrict__ node, const uint64_t *__restrict__ mask,
                             int64_t ne, int64_t n_near, const Node *__restrict__ nodes,
                             const int32_t *__restrict__ skk, unsigned long long *out)
{
    unsigned long long an = 0, af = 0;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < ne;
         e += (int64_t)gridDim.x * blockDim.x) {
        int a = node[e];
        unsigned long long rows = (unsigned long long)__popcll(mask[e]);
        if (e < n_near) an += rows * (unsigned long long)(nodes[a].hi - nodes[a].lo);
        else af += rows * (unsigned long long)skk[a];
    }
    atomicAdd(&out[0], an);
    atomicAdd(&out[1], af);
}

static void run_interactions(askit_handle *h, const Slab *d_slabs, int64_t nslab,
                             const int32_t *nbpos, int nnb, int32_t *&ptr, int32_t *&node,
                             uint64_t *&mask, int64_t &ne_near, int64_t &ne_far,
                             std::vector<void *> &owned, hipStream_t s, bool persistent)
{
    int nn = (int)h->nodes.size();
    size_t shb = sizeof(uint32_t) * ((nn + 31) / 32) + sizeof(int32_t) * 64 * nnb;
    if (shb > 150 * 1024) fail(ASKIT_ERR_UNSUPPORTED, "tree too large for the interaction kernel");
    // few slabs (a batch of new points): four waves share each slab's node scan
    const bool wide = nslab < 2048;
    const void *kfn = wide ? (const void *)k_interactions<4> : (const void *)k_interactions<1>;
    if (shb > 64 * 1024) HIPC(hipFuncSetAttribute(kfn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shb));
    int32_t *cnt, *cntw = nullptr;
    HIPC(ws_alloc((void **)&cnt, sizeof(int32_t) * 2 * (nslab + 1), s));
    if (wide) HIPC(ws_alloc((void **)&cntw, sizeof(int32_t) * 2 * 4 * std::max<int64_t>(nslab, 1), s));
    auto launch = [&](int mode, int32_t *cn, int32_t *cf, const int32_t *pp, int32_t *on, uint64_t *om) {
        if (wide)
            hipLaunchKernelGGL(k_interactions<4>, dim3((unsigned)nslab), dim3(256), shb, s, h->d_nodes, nn,
                               h->leaf_of, d_slabs, nbpos, nnb, mode, cn, cf, pp, nslab, on, om, cntw,
                               h->minlev);
        else
            hipLaunchKernelGGL(k_interactions<1>, dim3((unsigned)nslab), dim3(64), shb, s, h->d_nodes, nn,
                               h->leaf_of, d_slabs, nbpos, nnb, mode, cn, cf, pp, nslab, on, om, cntw,
                               h->minlev);
        HIPC(hipGetLastError());
    };
    launch(0, cnt, cnt + nslab + 1, nullptr, nullptr, nullptr);
    std::vector<int32_t> hc(2 * (nslab + 1));
    HIPC(hipMemcpyAsync(hc.data(), cnt, sizeof(int32_t) * 2 * (nslab + 1), hipMemcpyDeviceToHost, s));
    HIPC(hipStreamSynchronize(s));
    std::vector<int32_t> hp(2 * nslab + 2);
    int64_t acc = 0;
    for (int64_t i = 0; i < nslab; ++i) {
        hp[i] = (int32_t)acc;
        acc += hc[i];
    }
    hp[nslab] = (int32_t)acc;
    ne_near = acc;
    for (int64_t i = 0; i < nslab; ++i) {
        hp[nslab + 1 + i] = (int32_t)acc;
        acc += hc[nslab + 1 + i];
    }
    hp[2 * nslab + 1] = (int32_t)acc;
    ne_far = acc - ne_near;
    if (acc > 0x7fffffff) fail(ASKIT_ERR_UNSUPPORTED, "interaction lists exceed 2^31 entries");
    auto al = [&](size_t b) -> void * {
        void *p;
        if (persistent) p = h->alloc(b, false);
        else {
            HIPC(ws_alloc(&p, std::max<size_t>(b, 16), s));
            owned.push_back(p);
        }
        return p;
    };
    ptr = (int32_t *)al(sizeof(int32_t) * hp.size());
    node = (int32_t *)al(sizeof(int32_t) * std::max<int64_t>(acc, 1));
    mask = (uint64_t *)al(sizeof(uint64_t) * std::max<int64_t>(acc, 1));
    HIPC(hipMemcpyAsync(ptr, hp.data(), sizeof(int32_t) * hp.size(), hipMemcpyHostToDevice, s));
    launch(1, nullptr, nullptr, ptr, node, mask);
    HIPC(ws_free(cnt, s));
    if (cntw) HIPC(ws_free(cntw, s));
}

void build_interactions(askit_handle *h, hipStream_t s)
{
    const int64_t N = h->N;
    const int nnb = h->kappa + 1;
    int32_t *nb;
    HIPC(ws_alloc((void **)&nb, sizeof(int32_t) * N * nnb, s));
    hipLaunchKernelGGL(k_nbpos_self, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, s, h->perm,
                       h->iperm, h->knn_idx, N, h->kappa, nb);
    HIPC(hipGetLastError());
    std::vector<void *> owned;
    run_interactions(h, h->d_slabs, (int64_t)h->slabs.size(), nb, nnb, h->sl_ptr, h->sl_node,
                     h->sl_mask, h->near_entries, h->far_entries, owned, s, true);
    HIPC(ws_free(nb, s));
}

void count_pairs(askit_handle *h, hipStream_t s)
{
    // algorithmic pair counts of one evaluation
    unsigned long long *pc;
    HIPC(ws_alloc((void **)&pc, 16, s));
    HIPC(hipMemsetAsync(pc, 0, 16, s));
    int64_t ne = h->near_entries + h->far_entries;
    if (ne > 0)
        hipLaunchKernelGGL(k_pair_count, dim3(256), dim3(256), 0, s, h->sl_node, h->sl_mask, ne,
                           h->near_entries, h->d_nodes, h->skk, pc);
    unsigned long long hpc[2];
    HIPC(hipMemcpyAsync(hpc, pc, 16, hipMemcpyDeviceToHost, s));
    HIPC(hipStreamSynchronize(s));
    HIPC(ws_free(pc, s));
    h->near_pairs = (int64_t)hpc[0];
    h->far_pairs = (int64_t)hpc[1];
}


// ---- query grouping: sort queries by (leaf of their nearest source, index) so
// that a slab holds spatially close targets (denser masks, small centred norms).
// Sort key of query i: (its segment, the leaf of its nearest source, i); a
// segment is one request of a served batch (seg NULL: one segment).
__global__ void k_qkeys(const int32_t *__restrict__ nb, int64_t M, int kappa,
                        const int32_t *__restrict__ leaf_of, const int32_t *__restrict__ seg, int64_t nn,
                        int64_t M2, uint64_t *__restrict__ key)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= M2) return;
    if (i >= M) {
        key[i] = ~0ull;
        return;
    }
    const uint64_t hi = (uint64_t)(uint32_t)leaf_of[nb[i * kappa]] + (seg ? (uint64_t)seg[i] * (uint64_t)nn : 0ull);
    key[i] = (hi << 32) | (uint64_t)i;
}

__global__ void k_bitonic_step(uint64_t *__restrict__ key, int64_t M2, int64_t j, int64_t k)
{
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= M2 / 2) return;
    int64_t i = 2 * t - (t & (j - 1));
    int64_t q = i + j;
    bool up = (i & k) == 0;
    uint64_t a = key[i], b = key[q];
    if (up ? a > b : a < b) {
        key[i] = b;
        key[q] = a;
    }
}

__global__ void k_qorder(const uint64_t *__restrict__ key, int64_t M, int32_t *__restrict__ order)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < M) order[i] = (int32_t)(key[i] & 0xffffffffull);
}

__global__ void k_gather_i32_rows(const int32_t *__restrict__ src, const int32_t *__restrict__ idx,
                                  int64_t n, int w, int32_t *__restrict__ dst)
{
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t row = t / w;
    if (row >= n) return;
    dst[t] = src[(int64_t)idx[row] * w + (t - row * w)];
}

void sort_u64_pow2(uint64_t *key, int64_t n2, hipStream_t s)
{
    for (int64_t k = 2; k <= n2; k <<= 1)
        for (int64_t j = k >> 1; j > 0; j >>= 1)
            hipLaunchKernelGGL(k_bitonic_step, dim3((unsigned)((n2 / 2 + 255) / 256)), dim3(256), 0, s, key, n2, j,
                               k);
    HIPC(hipGetLastError());
}

void sort_queries(askit_handle *h, const int32_t *nb, int64_t M, int32_t *order, int32_t *nb_sorted,
                  std::vector<void *> &tmp, hipStream_t s, const int32_t *seg)
{
    int64_t M2 = 1;
    while (M2 < M) M2 <<= 1;
    uint64_t *key;
    HIPC(ws_alloc((void **)&key, sizeof(uint64_t) * M2, s));
    tmp.push_back(key);
    hipLaunchKernelGGL(k_qkeys, dim3((unsigned)((M2 + 255) / 256)), dim3(256), 0, s, nb, M, h->kappa,
                       h->leaf_of, seg, (int64_t)h->nodes.size(), M2, key);
    sort_u64_pow2(key, M2, s);
    hipLaunchKernelGGL(k_qorder, dim3((unsigned)((M + 255) / 256)), dim3(256), 0, s, key, M, order);
    int64_t tot = M * h->kappa;
    hipLaunchKernelGGL(k_gather_i32_rows, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, nb,
                       order, M, h->kappa, nb_sorted);
    HIPC(hipGetLastError());
}

void build_query_interactions(askit_handle *h, const int32_t *nb, int64_t M, Slab *&slabs,
                              int32_t *&ptr, int32_t *&node, uint64_t *&mask, int64_t &ne_near,
                              int64_t &ne_far, std::vector<void *> &tmp, hipStream_t s,
                              const std::vector<int64_t> *segs, int64_t &nslab)
{
    // slabs of SLAB consecutive (sorted) queries that never cross a segment;
    // each slab carries its segment in `pad`
    std::vector<Slab> hs;
    int64_t r0 = 0;
    const int64_t nseg = segs ? (int64_t)segs->size() : 1;
    for (int64_t sg = 0; sg < nseg; ++sg) {
        const int64_t len = segs ? (*segs)[sg] : M;
        for (int64_t i = 0; i < len; i += SLAB)
            hs.push_back(Slab{(int32_t)(r0 + i), (int32_t)std::min<int64_t>(SLAB, len - i), -1, (int32_t)sg});
        r0 += len;
    }
    if (r0 != M) fail(ASKIT_ERR_INVALID_ARG, "query segments do not add up to the query count");
    nslab = (int64_t)hs.size();
    Slab *ds;
    HIPC(ws_alloc((void **)&ds, sizeof(Slab) * nslab, s));
    tmp.push_back(ds);
    HIPC(hipMemcpyAsync(ds, hs.data(), sizeof(Slab) * nslab, hipMemcpyHostToDevice, s));
    slabs = ds;
    run_interactions(h, ds, nslab, nb, h->kappa, ptr, node, mask, ne_near, ne_far, tmp, s, false);
}

}  // namespace askit
