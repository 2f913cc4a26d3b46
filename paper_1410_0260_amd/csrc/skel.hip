// Skeletonization (Sec. 2.1, Alg. 3) and skeleton weights (upward pass).
//
// For every non-root node, bottom-up by level: columns C = the node's points
// (leaf) or S_left followed by S_right (internal); rows = the sampled rows
// T_alpha; G = K(T, C) in FP64.  G Pi = Q R by Householder QR with column
// pivoting, one workgroup per node with G resident in device memory
// (column-major, rows contiguous).  Step t pivots on the column with the
// largest residual norm over rows t.. (recomputed after every update, ties
// to the lowest column); the reflector is H = I - beta v v^T with v_t = 1,
// v_i = G[i][t] / (G[t][t] - R_tt), beta = (R_tt - G[t][t]) / R_tt,
// R_tt = -sign(G[t][t]) |x|.  The rank k is the first t with |R_tt| <=
// max(tau, 64 eps) |R_00|, capped by min(s_max, rows, cols).  S = the first
// k pivots, P = R11^{-1} R12 by back substitution.
#include "askit_impl.h"

#include <algorithm>
#include <cmath>

namespace askit {

constexpr double TAU_FLOOR = 64.0 * 2.220446049250313e-16;

__global__ void k_cols(const Node *__restrict__ nodes, const int32_t *__restrict__ ids, int smax,
                       int ncol_max, const int32_t *__restrict__ S, const int32_t *__restrict__ skk,
                       int32_t *__restrict__ colpos, int32_t *__restrict__ ncols)
{
    int q = blockIdx.x, a = ids[q];
    Node nd = nodes[a];
    int32_t *cp = colpos + (int64_t)q * ncol_max;
    int n;
    if (nd.left < 0) {
        n = nd.hi - nd.lo;
        for (int c = threadIdx.x; c < n; c += blockDim.x) cp[c] = nd.lo + c;
    } else {
        int kl = skk[nd.left], kr = skk[nd.right];
        n = kl + kr;
        for (int c = threadIdx.x; c < kl; c += blockDim.x) cp[c] = S[(int64_t)nd.left * smax + c];
        for (int c = threadIdx.x; c < kr; c += blockDim.x) cp[kl + c] = S[(int64_t)nd.right * smax + c];
    }
    if (threadIdx.x == 0) ncols[a] = n;
}

// G[q][c][t] = exp(-D(x_T[t], x_C[c]) / (2 h_c^2)), FP64.  Block per (column, node).
__global__ __launch_bounds__(256) void k_form_G(const float *__restrict__ Xt, int dp, int d,
                                                const int32_t *__restrict__ ids,
                                                const int32_t *__restrict__ T,
                                                const int32_t *__restrict__ T_cnt, int ell,
                                                const int32_t *__restrict__ colpos,
                                                const int32_t *__restrict__ ncols, int ncol_max,
                                                const double *__restrict__ hpos, double h,
                                                double *__restrict__ G)
{
    int c = blockIdx.x, q = blockIdx.y, a = ids[q];
    if (c >= ncols[a]) return;
    int rows = T_cnt[a];
    int32_t cpos = colpos[(int64_t)q * ncol_max + c];
    const float *xc = Xt + (int64_t)cpos * dp;
    double hc = hpos ? hpos[cpos] : h;
    double den = 2.0 * hc * hc;
    double *g = G + ((int64_t)q * ncol_max + c) * ell;
    for (int t = threadIdx.x; t < rows; t += blockDim.x) {
        int32_t tp = T[(int64_t)a * ell + t];
        double D = canon_sqdist(Xt + (int64_t)tp * dp, xc, d);
        g[t] = exp(-D / den);
    }
}

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

constexpr int QR_T = 256;
constexpr int QR_MAXCOL = 2048;
constexpr int QR_MAXROW = 1024;

__global__ __launch_bounds__(QR_T) void k_qrcp(double *__restrict__ Gall, int ell, int ncol_max,
                                               const int32_t *__restrict__ ids,
                                               const int32_t *__restrict__ T_cnt,
                                               const int32_t *__restrict__ ncols, int smax,
                                               double tau, int32_t *__restrict__ colperm,
                                               int32_t *__restrict__ kout)
{
    __shared__ double nrm2[QR_MAXCOL];
    __shared__ int piv[QR_MAXCOL];
    __shared__ double v[QR_MAXROW];
    __shared__ double rd[QR_T / 64];
    __shared__ int ri[QR_T / 64];
    __shared__ double sh_beta;
    const int q = blockIdx.x, a = ids[q];
    const int rows = T_cnt[a], cols = ncols[a];
    const int tid = threadIdx.x, lane = tid % 64, wv = tid / 64;
    double *G = Gall + (int64_t)q * ncol_max * ell;
    for (int c = tid; c < cols; c += QR_T) piv[c] = c;
    for (int c = wv; c < cols; c += QR_T / 64) {
        double s = 0.0;
        for (int i = lane; i < rows; i += 64) s += G[(int64_t)c * ell + i] * G[(int64_t)c * ell + i];
        s = wave_sum(s);
        if (lane == 0) nrm2[c] = s;
    }
    __syncthreads();
    const double teff = tau > TAU_FLOOR ? tau : TAU_FLOOR;
    int kcap = min(smax, min(rows, cols));
    int k = kcap;
    double nrm0 = 0.0;
    for (int t = 0; t < kcap; ++t) {
        // argmax of residual norms over columns t.., ties to the lowest column
        double bv = -1.0;
        int bi = 0x7fffffff;
        for (int c = t + tid; c < cols; c += QR_T) {
            double x = nrm2[c];
            if (x > bv || (x == bv && c < bi)) { bv = x; bi = c; }
        }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            double ov = __shfl_xor(bv, o);
            int oi = __shfl_xor(bi, o);
            if (ov > bv || (ov == bv && oi < bi)) { bv = ov; bi = oi; }
        }
        if (lane == 0) { rd[wv] = bv; ri[wv] = bi; }
        __syncthreads();
        bv = rd[0];
        bi = ri[0];
        for (int w = 1; w < QR_T / 64; ++w)
            if (rd[w] > bv || (rd[w] == bv && ri[w] < bi)) { bv = rd[w]; bi = ri[w]; }
        const double nrm = sqrt(bv);
        bool stop = false;
        if (t == 0) {
            nrm0 = nrm;
            if (!(nrm0 > 0.0)) { k = 0; stop = true; }
        } else if (nrm <= teff * nrm0) {
            k = t;
            stop = true;
        }
        if (stop) break;
        // swap columns t and bi
        if (bi != t) {
            for (int i = tid; i < rows; i += QR_T) {
                double x = G[(int64_t)t * ell + i];
                G[(int64_t)t * ell + i] = G[(int64_t)bi * ell + i];
                G[(int64_t)bi * ell + i] = x;
            }
            if (tid == 0) {
                double x = nrm2[t]; nrm2[t] = nrm2[bi]; nrm2[bi] = x;
                int p = piv[t]; piv[t] = piv[bi]; piv[bi] = p;
            }
        }
        __syncthreads();
        const double x0 = G[(int64_t)t * ell + t];
        const double rtt = x0 >= 0.0 ? -nrm : nrm;
        const double denom = x0 - rtt;
        const double beta = (rtt - x0) / rtt;
        for (int i = t + 1 + tid; i < rows; i += QR_T) v[i] = G[(int64_t)t * ell + i] / denom;
        __syncthreads();
        if (tid == 0) {
            G[(int64_t)t * ell + t] = rtt;
            sh_beta = beta;
        }
        for (int i = t + 1 + tid; i < rows; i += QR_T) G[(int64_t)t * ell + i] = 0.0;
        // apply the reflector to the trailing columns and recompute their norms
        for (int c = t + 1 + wv; c < cols; c += QR_T / 64) {
            double *gc = G + (int64_t)c * ell;
            double s = 0.0;
            for (int i = t + 1 + lane; i < rows; i += 64) s += v[i] * gc[i];
            s = wave_sum(s) + gc[t];
            const double f = beta * s;
            double ns = 0.0;
            for (int i = t + 1 + lane; i < rows; i += 64) {
                double y = gc[i] - f * v[i];
                gc[i] = y;
                ns += y * y;
            }
            ns = wave_sum(ns);
            if (lane == 0) {
                gc[t] -= f;
                nrm2[c] = ns;
            }
        }
        __syncthreads();
    }
    for (int c = tid; c < cols; c += QR_T) colperm[(int64_t)a * ncol_max + c] = piv[c];
    if (tid == 0) kout[a] = k;
}

// P = R11^{-1} R12 in place over R12 (FP64).  Thread per column of R12.
__global__ __launch_bounds__(256) void k_solve(double *__restrict__ Gall, int ell, int ncol_max,
                                               const int32_t *__restrict__ ids,
                                               const int32_t *__restrict__ ncols,
                                               const int32_t *__restrict__ skk)
{
    const int q = blockIdx.y, a = ids[q];
    const int k = skk[a], n = ncols[a];
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n - k) return;
    double *G = Gall + (int64_t)q * ncol_max * ell;
    double *pc = G + (int64_t)(k + c) * ell;        // column k+c: rows 0..k-1 = R12, becomes P
    for (int t = k - 1; t >= 0; --t) {
        double s = pc[t];
        for (int u = t + 1; u < k; ++u) s -= G[(int64_t)u * ell + t] * pc[u];
        pc[t] = s / G[(int64_t)t * ell + t];
    }
}

// S, skeleton coordinates and bandwidth factors, P in FP32 (row stride n-k).
__global__ __launch_bounds__(256) void k_finalize(const double *__restrict__ Gall, int ell,
                                                  int ncol_max, const int32_t *__restrict__ ids,
                                                  const int32_t *__restrict__ colpos,
                                                  const int32_t *__restrict__ ncols,
                                                  const int32_t *__restrict__ skk,
                                                  const int32_t *__restrict__ colperm, int smax,
                                                  const int64_t *__restrict__ pslot,
                                                  const float *__restrict__ Xt, int dp,
                                                  const float *__restrict__ gt,
                                                  int32_t *__restrict__ S, float *__restrict__ P,
                                                  float *__restrict__ Xs, float *__restrict__ gs)
{
    const int q = blockIdx.x, a = ids[q];
    const int k = skk[a], n = ncols[a], nr = n - k;
    const double *G = Gall + (int64_t)q * ncol_max * ell;
    const int32_t *pv = colperm + (int64_t)a * ncol_max;
    const int32_t *cp = colpos + (int64_t)q * ncol_max;
    for (int t = threadIdx.x; t < k; t += blockDim.x) {
        int32_t pos = cp[pv[t]];
        S[(int64_t)a * smax + t] = pos;
        gs[(int64_t)a * smax + t] = gt[pos];
    }
    for (int e = threadIdx.x; e < k * dp; e += blockDim.x) {
        int t = e / dp, j = e % dp;
        Xs[((int64_t)a * smax + t) * dp + j] = Xt[(int64_t)cp[pv[t]] * dp + j];
    }
    float *Pa = P + pslot[a];
    for (int e = threadIdx.x; e < k * nr; e += blockDim.x) {
        int t = e / nr, c = e % nr;
        Pa[e] = (float)G[(int64_t)(k + c) * ell + t];
    }
}

void skeletonize(askit_handle *h, hipStream_t s)
{
    const int nn = (int)h->nodes.size();
    const int ell = h->ell, ncm = h->ncol_max, smax = h->smax;
    if (ncm > QR_MAXCOL || ell > QR_MAXROW)
        fail(ASKIT_ERR_UNSUPPORTED, "ID block larger than 1024 rows x 2048 columns");
    HIPC(hipMemsetAsync(h->skk, 0, sizeof(int32_t) * nn, s));
    HIPC(hipMemsetAsync(h->ncols, 0, sizeof(int32_t) * nn, s));
    if (h->depth == 0) return;
    int maxlev = 0;
    for (auto &lv : h->level_nodes) maxlev = std::max(maxlev, (int)lv.size());
    // batch so that the FP64 blocks stay within ~2 GiB
    const size_t per = (size_t)ncm * ell * sizeof(double);
    int batch = (int)std::max<size_t>(1, std::min<size_t>(maxlev, (size_t)(2ull << 30) / per));
    double *G;
    int32_t *colpos, *d_ids;
    HIPC(hipMallocAsync((void **)&G, per * batch, s));
    HIPC(hipMallocAsync((void **)&colpos, sizeof(int32_t) * (size_t)ncm * batch, s));
    HIPC(hipMallocAsync((void **)&d_ids, sizeof(int32_t) * nn, s));
    const double *hpos = nullptr;
    double *hp_tmp = nullptr;
    if (h->varh) {
        // per tree position bandwidth (FP64) from the per-id array
        HIPC(hipMallocAsync((void **)&hp_tmp, sizeof(double) * h->N, s));
        gather_f64(h->hsrc, h->perm, h->N, hp_tmp, s);
        hpos = hp_tmp;
    }
    std::vector<int32_t> ids;
    hipEvent_t q0, q1;
    HIPC(hipEventCreate(&q0));
    HIPC(hipEventCreate(&q1));
    h->t_qr = 0;
    for (int lev = h->depth; lev >= 1; --lev) {
        const auto &lv = h->level_nodes[lev];
        for (size_t b0 = 0; b0 < lv.size(); b0 += batch) {
            ids.assign(lv.begin() + b0, lv.begin() + std::min(lv.size(), b0 + batch));
            int nb = (int)ids.size();
            HIPC(hipStreamSynchronize(s));
            HIPC(hipMemcpyAsync(d_ids, ids.data(), sizeof(int32_t) * nb, hipMemcpyHostToDevice, s));
            hipLaunchKernelGGL(k_cols, dim3(nb), dim3(256), 0, s, h->d_nodes, d_ids, smax, ncm, h->S,
                               h->skk, colpos, h->ncols);
            hipLaunchKernelGGL(k_form_G, dim3(ncm, nb), dim3(256), 0, s, h->Xt, h->dp, h->d, d_ids,
                               h->T, h->T_cnt, ell, colpos, h->ncols, ncm, hpos, h->prm.bandwidth, G);
            HIPC(hipEventRecord(q0, s));
            hipLaunchKernelGGL(k_qrcp, dim3(nb), dim3(QR_T), 0, s, G, ell, ncm, d_ids, h->T_cnt,
                               h->ncols, smax, h->prm.id_tol, h->colperm, h->skk);
            HIPC(hipEventRecord(q1, s));
            hipLaunchKernelGGL(k_solve, dim3((ncm + 255) / 256, nb), dim3(256), 0, s, G, ell, ncm,
                               d_ids, h->ncols, h->skk);
            hipLaunchKernelGGL(k_finalize, dim3(nb), dim3(256), 0, s, G, ell, ncm, d_ids, colpos,
                               h->ncols, h->skk, h->colperm, smax, h->d_pslot, h->Xt, h->dp, h->gt,
                               h->S, h->P, h->Xs, h->gs);
            HIPC(hipGetLastError());
            HIPC(hipStreamSynchronize(s));
            float ms = 0.f;
            HIPC(hipEventElapsedTime(&ms, q0, q1));
            h->t_qr += ms;
        }
    }
    (void)hipEventDestroy(q0);
    (void)hipEventDestroy(q1);
    HIPC(hipStreamSynchronize(s));
    HIPC(hipFreeAsync(G, s));
    HIPC(hipFreeAsync(colpos, s));
    HIPC(hipFreeAsync(d_ids, s));
    if (hp_tmp) HIPC(hipFreeAsync(hp_tmp, s));
}

// ---------------------------------------------------------------- upward pass
// w~_alpha[t] = Wc[piv t] + sum_c P[t][c] Wc[piv k+c]; Wc = W(X_alpha) at a
// leaf, [w~_left; w~_right] at an internal node.  One wave per (node, t).
__global__ __launch_bounds__(64) void k_upward(const Node *__restrict__ nodes,
                                               const int32_t *__restrict__ ids,
                                               const int32_t *__restrict__ skk,
                                               const int32_t *__restrict__ ncols,
                                               const int32_t *__restrict__ colperm, int ncol_max,
                                               const int64_t *__restrict__ pslot,
                                               const float *__restrict__ P, int smax,
                                               const float *__restrict__ Wt, int R,
                                               float *__restrict__ Wsk)
{
    const int a = ids[blockIdx.x], t = blockIdx.y, lane = threadIdx.x;
    const int k = skk[a];
    if (t >= k) return;
    const Node nd = nodes[a];
    const int n = ncols[a], nr = n - k;
    const int32_t *pv = colperm + (int64_t)a * ncol_max;
    const float *Pt = P + pslot[a] + (int64_t)t * nr;
    const int kl = nd.left >= 0 ? skk[nd.left] : 0;
    auto wc = [&](int c, int r) -> float {
        if (nd.left < 0) return Wt[(int64_t)(nd.lo + c) * R + r];
        return c < kl ? Wsk[((int64_t)nd.left * smax + c) * R + r]
                      : Wsk[((int64_t)nd.right * smax + (c - kl)) * R + r];
    };
    for (int r = 0; r < R; ++r) {
        float acc = 0.0f;
        for (int c = lane; c < nr; c += 64) acc = fmaf(Pt[c], wc(pv[k + c], r), acc);
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
        if (lane == 0) Wsk[((int64_t)a * smax + t) * R + r] = wc(pv[t], r) + acc;
    }
}

void upward(askit_handle *h, hipStream_t s)
{
    const int nn = (int)h->nodes.size();
    if (h->depth == 0) return;
    int32_t *d_ids;
    HIPC(hipMallocAsync((void **)&d_ids, sizeof(int32_t) * nn, s));
    // all level lists packed once, launched bottom-up
    std::vector<int32_t> all;
    std::vector<std::pair<int, int>> seg;
    for (int lev = h->depth; lev >= 1; --lev) {
        seg.push_back({(int)all.size(), (int)h->level_nodes[lev].size()});
        all.insert(all.end(), h->level_nodes[lev].begin(), h->level_nodes[lev].end());
    }
    HIPC(hipMemcpyAsync(d_ids, all.data(), sizeof(int32_t) * all.size(), hipMemcpyHostToDevice, s));
    for (auto &sg : seg) {
        if (sg.second == 0) continue;
        hipLaunchKernelGGL(k_upward, dim3(sg.second, h->smax), dim3(64), 0, s, h->d_nodes,
                           d_ids + sg.first, h->skk, h->ncols, h->colperm, h->ncol_max, h->d_pslot,
                           h->P, h->smax, h->Wt, h->nrhs, h->Wsk);
        HIPC(hipGetLastError());
    }
    HIPC(hipStreamSynchronize(s));
    HIPC(hipFreeAsync(d_ids, s));
}

}  // namespace askit
