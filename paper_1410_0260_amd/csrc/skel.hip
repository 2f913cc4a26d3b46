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
#include <cstdio>
#include <cstdlib>
#include <mutex>

namespace askit {

constexpr double TAU_FLOOR = 64.0 * 2.220446049250313e-16;

__global__ void k_cols(const SkelInst *__restrict__ inst, const int2 *__restrict__ items, int smax, int ncol_max,
                       int32_t *__restrict__ colpos)
{
    const int q = blockIdx.x;
    const int2 it = items[q];
    const SkelInst &I = inst[it.x];
    const int a = it.y;
    const int32_t *S = I.S, *skk = I.skk;
    int32_t *ncols = I.ncols;
    Node nd = I.nodes[a];
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

// G[q][c][t] = exp(-D(x_T[t], x_C[c]) / (2 h_c^2)), FP64.  Block per (node,
// chunk of FG_C columns), FG_R sampled rows per thread (rows t and t +
// blockDim; blockDim = ell / FG_R rounded up to whole waves): the thread holds
// FG_K coordinates of its rows in registers, the chunk's columns are staged
// in LDS as FP64 (every lane reads the same column entry: a broadcast, used
// for FG_R rows), and each of the thread's partial distances adds the
// dimensions in increasing order, so D is the same sequential FP64 sum as
// everywhere else (subtract, square, add; no fused multiply-add).
constexpr int FG_C = 8;           // columns per block
constexpr int FG_K = 16;          // dimensions per stage
constexpr int FG_R = 2;           // sampled rows per thread
constexpr int FG_MAXROW = 1024;

__global__ __launch_bounds__(FG_MAXROW / FG_R) void k_form_G(const SkelInst *__restrict__ inst,
                                                             const int2 *__restrict__ items, int ell,
                                                             const int32_t *__restrict__ colpos, int ncol_max,
                                                             double *__restrict__ G)
{
#pragma clang fp contract(off)
    __shared__ __attribute__((aligned(16))) double sC[FG_K][FG_C];    // [dimension][column]
    __shared__ int32_t sCid[FG_C];
    const int q = blockIdx.y;
    const int2 it = items[q];
    const SkelInst &I = inst[it.x];
    const int a = it.y;
    const float *Xt = I.Xt;
    const int dp = I.dp, d = I.d;
    const double *hpos = I.hpos;
    const double h = I.h;
    const int c0 = blockIdx.x * FG_C;
    const int nc = min(FG_C, I.ncols[a] - c0);
    const int rows = I.T_cnt[a];
    if (nc <= 0 || rows <= 0) return;
    const int t = threadIdx.x, nt = blockDim.x;
    if (t < FG_C) sCid[t] = colpos[(int64_t)q * ncol_max + c0 + min(t, nc - 1)];
    // rows past `rows` repeat the last one and write nothing
    const float *xr[FG_R];
#pragma unroll
    for (int r = 0; r < FG_R; ++r) xr[r] = Xt + (int64_t)I.T[(int64_t)a * ell + min(t + r * nt, rows - 1)] * dp;
    double acc[FG_R][FG_C];
#pragma unroll
    for (int r = 0; r < FG_R; ++r)
#pragma unroll
        for (int c = 0; c < FG_C; ++c) acc[r][c] = 0.0;
    for (int k0 = 0; k0 < d; k0 += FG_K) {
        const int kk = min(FG_K, d - k0);
        // a whole stage: the rows' coordinates first (their loads overlap the
        // staging); rows are 16-byte aligned (dp is a multiple of 16)
        float xv[FG_R][FG_K];
        if (kk == FG_K) {
#pragma unroll
            for (int r = 0; r < FG_R; ++r)
#pragma unroll
                for (int j = 0; j < FG_K; j += 4) {
                    const float4 v = *reinterpret_cast<const float4 *>(xr[r] + k0 + j);
                    xv[r][j] = v.x;
                    xv[r][j + 1] = v.y;
                    xv[r][j + 2] = v.z;
                    xv[r][j + 3] = v.w;
                }
        }
        __syncthreads();                       // sCid written; the previous stage's reads done
        for (int e = t; e < FG_K * FG_C; e += nt) {
            const int j = e / FG_C, c = e % FG_C;
            sC[j][c] = (double)Xt[(int64_t)sCid[c] * dp + min(k0 + j, dp - 1)];
        }
        __syncthreads();
        if (kk == FG_K) {
#pragma unroll
            for (int j = 0; j < FG_K; ++j) {
                double xd[FG_R];
#pragma unroll
                for (int r = 0; r < FG_R; ++r) xd[r] = (double)xv[r][j];
#pragma unroll
                for (int c = 0; c < FG_C; ++c) {
                    const double y = sC[j][c];
#pragma unroll
                    for (int r = 0; r < FG_R; ++r) {
                        const double df = xd[r] - y;
                        acc[r][c] = acc[r][c] + df * df;
                    }
                }
            }
        } else {
            // the last, partial stage (k0 + j < d <= dp)
#pragma unroll 1
            for (int j = 0; j < kk; ++j) {
                double xd[FG_R];
#pragma unroll
                for (int r = 0; r < FG_R; ++r) xd[r] = (double)xr[r][k0 + j];
#pragma unroll
                for (int c = 0; c < FG_C; ++c) {
                    const double y = sC[j][c];
#pragma unroll
                    for (int r = 0; r < FG_R; ++r) {
                        const double df = xd[r] - y;
                        acc[r][c] = acc[r][c] + df * df;
                    }
                }
            }
        }
    }
#pragma unroll
    for (int r = 0; r < FG_R; ++r) {
        const int row = t + r * nt;
        if (row < rows) {
#pragma unroll
            for (int c = 0; c < FG_C; ++c) {
                if (c >= nc) break;
                const double hc = hpos ? hpos[sCid[c]] : h;
                G[((int64_t)q * ncol_max + c0 + c) * ell + row] = exp(-acc[r][c] / (2.0 * hc * hc));
            }
        }
    }
}

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

constexpr int QR_T = 1024;
constexpr int QR_MAXCOL = 2048;
constexpr int QR_MAXROW = 1024;

// Lane l's value from lane l ^ o (o = 8, 4, 2, 1; the partner is always in
// the same group of 16): xor 8 and 4 by a swizzle in the LDS crossbar, xor 2
// and 1 by DPP quad permutes, so no LDS address round trip.
template <int O>
__device__ __forceinline__ double xor_lane(double v)
{
    int lo = __double2loint(v), hi = __double2hiint(v);
    if constexpr (O == 8 || O == 4) {
        constexpr int pat = 0x1f | (O << 10);          // and 31, or 0, xor O
        lo = __builtin_amdgcn_ds_swizzle(lo, pat);
        hi = __builtin_amdgcn_ds_swizzle(hi, pat);
    } else {
        constexpr int ctrl = O == 2 ? 0x4e : 0xb1;     // quad_perm [2,3,0,1] / [1,0,3,2]
        lo = __builtin_amdgcn_mov_dpp(lo, ctrl, 0xf, 0xf, false);
        hi = __builtin_amdgcn_mov_dpp(hi, ctrl, 0xf, 0xf, false);
    }
    return __hiloint2double(hi, lo);
}

// Sum over a group of 16 lanes by the xor butterfly: every lane of the group
// ends with the same value.
__device__ __forceinline__ double group16_sum(double v)
{
    v += xor_lane<8>(v);
    v += xor_lane<4>(v);
    v += xor_lane<2>(v);
    v += xor_lane<1>(v);
    return v;
}

// One block per node.  Every wave works on 4 columns at a time, 16 lanes per
// column, so each wave keeps 4 columns' loads in flight.  RM > 0 (rows <=
// 16 RM): a lane keeps its slice of the column (rows t+1+l16, +16, ...) in
// registers between the reflector's dot product and the update, so a pivot
// step reads and writes every trailing element once; the operations and
// their order are those of RM = 0 (slices re-read from memory).
template <int QT, int RM>
__global__ __launch_bounds__(QT) void k_qrcp(double *__restrict__ Gall, int ell, int ncol_max,
                                               const SkelInst *__restrict__ inst,
                                               const int2 *__restrict__ items, int smax, double tau, int nb)
{
    __shared__ double nrm2[QR_MAXCOL];
    __shared__ int piv[QR_MAXCOL];
    __shared__ double v[QR_MAXROW];
    __shared__ double rd[QT / 64];
    __shared__ int ri[QT / 64];
    constexpr int NW = QT / 64;              // waves
    constexpr int CG = NW * 4;                 // columns in flight per block
    const int tid = threadIdx.x, lane = tid % 64, wv = tid / 64;
    const int g16 = lane >> 4, l16 = lane & 15;
  // nodes q = blockIdx.x, + gridDim.x, ... (launched with one block per node;
  // a smaller grid would bound the factorizations in flight)
  for (int q = blockIdx.x; q < nb; q += gridDim.x) {
    __syncthreads();                           // the previous node is done with the shared arrays
    const int2 it = items[q];
    const SkelInst &I = inst[it.x];
    const int a = it.y;
    const int rows = I.T_cnt[a], cols = I.ncols[a];
    double *G = Gall + (int64_t)q * ncol_max * ell;
    for (int c = tid; c < cols; c += QT) piv[c] = c;
    for (int cb = 0; cb < cols; cb += CG) {
        const int c = cb + wv * 4 + g16;
        double s = 0.0;
        if (c < cols)
            for (int i = l16; i < rows; i += 16) s += G[(int64_t)c * ell + i] * G[(int64_t)c * ell + i];
        s = group16_sum(s);
        if (c < cols && l16 == 0) nrm2[c] = s;
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
        for (int c = t + tid; c < cols; c += QT) {
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
        for (int w = 1; w < NW; ++w)
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
        if (bi != t) {
            for (int i = tid; i < rows; i += QT) {
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
        for (int i = t + 1 + tid; i < rows; i += QT) v[i] = G[(int64_t)t * ell + i] / denom;
        __syncthreads();
        if (tid == 0) G[(int64_t)t * ell + t] = rtt;
        for (int i = t + 1 + tid; i < rows; i += QT) G[(int64_t)t * ell + i] = 0.0;
        // apply the reflector to the trailing columns and recompute their norms
        for (int cb = t + 1; cb < cols; cb += CG) {
            const int c = cb + wv * 4 + g16;
            const bool on = c < cols;
            double *gc = G + (int64_t)(on ? c : t) * ell;
            double s = 0.0;
            double ns = 0.0;
            if constexpr (RM > 0) {
                double xr[RM];
#pragma unroll
                for (int j = 0; j < RM; ++j) {
                    const int i = t + 1 + l16 + 16 * j;
                    xr[j] = (on && i < rows) ? gc[i] : 0.0;
                }
#pragma unroll
                for (int j = 0; j < RM; ++j) {
                    const int i = t + 1 + l16 + 16 * j;
                    if (on && i < rows) s += v[i] * xr[j];
                }
                s = group16_sum(s);
                const double top = on ? gc[t] : 0.0;
                const double f = beta * (s + top);
#pragma unroll
                for (int j = 0; j < RM; ++j) {
                    const int i = t + 1 + l16 + 16 * j;
                    if (on && i < rows) {
                        double y = xr[j] - f * v[i];
                        gc[i] = y;
                        ns += y * y;
                    }
                }
                ns = group16_sum(ns);
                if (on && l16 == 0) {
                    gc[t] = top - f;
                    nrm2[c] = ns;
                }
                continue;
            }
            if (on)
                for (int i = t + 1 + l16; i < rows; i += 16) s += v[i] * gc[i];
            s = group16_sum(s);
            const double top = on ? gc[t] : 0.0;
            const double f = beta * (s + top);
            if (on)
                for (int i = t + 1 + l16; i < rows; i += 16) {
                    double y = gc[i] - f * v[i];
                    gc[i] = y;
                    ns += y * y;
                }
            ns = group16_sum(ns);
            if (on && l16 == 0) {
                gc[t] = top - f;
                nrm2[c] = ns;
            }
        }
        __syncthreads();
    }
    for (int c = tid; c < cols; c += QT) I.colperm[(int64_t)a * I.ncol_max + c] = piv[c];
    if (tid == 0) I.skk[a] = k;
  }
}

// ---------------------------------------------------------------- gang QRCP
// The same factorization with the node's columns held in registers across a
// gang of W workgroups (co-resident by a cooperative launch): column c
// belongs to workgroup c % W, whose 16-lane group (c / W) % 32 keeps it in
// slot (c / W) / 32, lane l16 holding rows l16 + 16 r.  Per pivot step each
// workgroup publishes, in device memory, its best column (largest residual
// norm, ties to the lowest current position) with that column's rows t..,
// and then a sequence number.  Every workgroup waits for the W sequence
// numbers of the step, reads the W candidates, takes the best one as the
// pivot, computes the same reflector from its rows and applies it to its
// own columns.  Column swaps are bookkeeping only: every workgroup keeps
// the same position <-> column maps.  At the end each column is written to
// G at its final position, so the solve and finalize kernels read the same
// layout as after k_qrcp.  Exchanged values are written and read with
// device-coherent (agent-scope) atomic accesses; a wait lasts at most
// `timeout` ticks of the constant-rate clock, past which the kernel sets
// *err and every workgroup returns.  Candidates are double-buffered by step
// parity: a workgroup overwrites a buffer only after every workgroup has
// published the step that followed its use.
constexpr int QG_T = 512;
constexpr double QG_TIMEOUT_S = 10.0;                // wait limit

struct GangSlot {
    double v;
    int32_t pos, col;
    int32_t seq, pad;
};

__device__ __forceinline__ bool qg_better(double v1, int p1, double v2, int p2)
{
    return v1 > v2 || (v1 == v2 && p1 < p2);
}

// TIMING: each workgroup adds the clock cycles of its pivot steps' phases to
// tacc (local argmax, publication, wait for the other members, candidate
// loads, reflector, update of the held columns; then the step count), for
// the ASKIT_QR_TIMING diagnostic.
template <int W, int RM, int CPG, bool TIMING>
__global__ __launch_bounds__(QG_T) void k_qrcp_gang(double *__restrict__ Gall, int ell, int ncol_max,
                                                     const SkelInst *__restrict__ inst,
                                                     const int2 *__restrict__ items, int smax, double tau,
                                                     int nb, GangSlot *__restrict__ slots,
                                                     double *__restrict__ sdata, int32_t *__restrict__ err,
                                                     uint64_t timeout, unsigned long long *__restrict__ tacc)
{
    constexpr int RMAX = 16 * RM;
    __shared__ int piv[QR_MAXCOL];            // position -> column
    __shared__ int posof[QR_MAXCOL];          // column -> position
    __shared__ double cd[W][RMAX];            // the W candidates' rows
    __shared__ double svr[RMAX];              // the reflector's rows below t
    __shared__ double cv[W];
    __shared__ int cp[W], cc[W];
    __shared__ double rdv[QG_T / 64];
    __shared__ int rdp[QG_T / 64], rdc[QG_T / 64];
    __shared__ int s_fail;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int grp = tid >> 4, l16 = tid & 15;
    // workgroups are dealt to the 8 XCDs round robin (id mod 8): the members
    // of a gang are ids 8 apart, so a gang stays on one XCD, where its
    // exchanges take about a fifth of the time they take across XCDs (the
    // protocol itself does not depend on the placement)
    const int ngang = gridDim.x / W;
    const int gang = (int)(blockIdx.x / (8 * W)) * 8 + (int)(blockIdx.x % 8), w = (int)(blockIdx.x / 8) % W;
    int32_t gs = 0;                           // steps published by this gang
    unsigned long long tph[7] = {0, 0, 0, 0, 0, 0, 0};
    // an earlier gang of this skeletonization timed out: nothing to do (the
    // flag was set before this launch began, so every workgroup sees it)
    if (__hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return;
    if (tid == 0) s_fail = 0;
    for (int q = gang; q < nb; q += ngang) {
        __syncthreads();
        const int2 it = items[q];
        const SkelInst &I = inst[it.x];
        const int a = it.y;
        const int rows = I.T_cnt[a], cols = I.ncols[a];
        double *G = Gall + (int64_t)q * ncol_max * ell;
        for (int c = tid; c < cols; c += QG_T) {
            piv[c] = c;
            posof[c] = c;
        }
        double x[CPG][RM];
        double nv[CPG];
        bool act[CPG];
#pragma unroll
        for (int j = 0; j < CPG; ++j) {
            const int c = w + W * (grp + 32 * j);
            act[j] = c < cols;
            double sq = 0.0;
#pragma unroll
            for (int r = 0; r < RM; ++r) {
                const int i = l16 + 16 * r;
                x[j][r] = (act[j] && i < rows) ? G[(int64_t)c * ell + i] : 0.0;
                if (i < rows) sq += x[j][r] * x[j][r];
            }
            nv[j] = group16_sum(sq);
        }
        __syncthreads();
        const double teff = tau > TAU_FLOOR ? tau : TAU_FLOOR;
        const int kcap = min(smax, min(rows, cols));
        int k = kcap;
        double nrm0 = 0.0;
        for (int t = 0; t < kcap; ++t) {
            unsigned long long c0 = 0, c1 = 0, c2 = 0, c3 = 0, c4 = 0, c5 = 0;
            if constexpr (TIMING) c0 = clock64();
            // this workgroup's best active column
            double bv = -1.0;
            int bp = 0x7fffffff, bc = -1;
#pragma unroll
            for (int j = 0; j < CPG; ++j) {
                if (!act[j]) continue;
                const int c = w + W * (grp + 32 * j);
                const int pc = posof[c];
                if (qg_better(nv[j], pc, bv, bp)) { bv = nv[j]; bp = pc; bc = c; }
            }
#pragma unroll
            for (int o = 32; o >= 16; o >>= 1) {
                const double ov = __shfl_xor(bv, o);
                const int op = __shfl_xor(bp, o), oc = __shfl_xor(bc, o);
                if (qg_better(ov, op, bv, bp)) { bv = ov; bp = op; bc = oc; }
            }
            if (lane == 0) { rdv[wv] = bv; rdp[wv] = bp; rdc[wv] = bc; }
            __syncthreads();
            if constexpr (TIMING) c1 = clock64();
            ++gs;
            const int par = gs & 1;
            GangSlot *sl = slots + ((int64_t)gang * 2 + par) * W;
            double *sd = sdata + ((int64_t)gang * 2 + par) * W * RMAX;   // RMAX rows per member
            // every thread reduces the waves' candidates (same order, same
            // result), so no barrier is needed before the rows are published
            bv = rdv[0];
            bp = rdp[0];
            bc = rdc[0];
            for (int u = 1; u < QG_T / 64; ++u)
                if (qg_better(rdv[u], rdp[u], bv, bp)) { bv = rdv[u]; bp = rdp[u]; bc = rdc[u]; }
            if (tid == 0) {
                __hip_atomic_store(&sl[w].v, bv, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                __hip_atomic_store(&sl[w].pos, bp, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                __hip_atomic_store(&sl[w].col, bc, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
            {
                const int lbc = bc;
                if (lbc >= 0 && grp == (lbc / W) % 32) {
                    const int jb = (lbc / W) / 32;
                    double *dst = sd + (int64_t)w * RMAX;
                    // whole slices from the one holding row t (a uniform test;
                    // rows < t and >= rows are written too and never read)
#pragma unroll
                    for (int j = 0; j < CPG; ++j) {
                        if (j != jb) continue;
#pragma unroll
                        for (int r = 0; r < RM; ++r)
                            if (r >= (t >> 4))
                                __hip_atomic_store(&dst[l16 + 16 * r], x[j][r], __ATOMIC_RELAXED,
                                                   __HIP_MEMORY_SCOPE_AGENT);
                    }
                }
            }
            // Publication order.  The members of a gang run on one XCD and
            // exchange through agent-scope atomics, which bypass the
            // non-coherent caches.  Every wave waits until its stores are
            // complete (vmcnt reaches 0: acknowledged by the memory system),
            // the block barrier orders that before thread 0's store of the
            // sequence number; the signal fences stop the compiler from moving
            // the stores across.  (Agent-scope release/acquire fences give the
            // same order through a write-back of the L2 and a cache invalidate
            // per pivot step; measured, they made the QR 2.5x slower.)
            __atomic_signal_fence(__ATOMIC_SEQ_CST);
            asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
            __syncthreads();
            __atomic_signal_fence(__ATOMIC_SEQ_CST);
            if (tid == 0) __hip_atomic_store(&sl[w].seq, gs, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if constexpr (TIMING) c2 = clock64();
            // every wave waits for the W candidates of this step itself (its
            // lanes < W poll), then loads its share: the loads of a lane are
            // issued only after its wave saw all W sequence numbers
            if (lane < W) {
                const uint64_t t0 = wall_clock64();
                while (__hip_atomic_load(&sl[lane].seq, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != gs) {
                    if (wall_clock64() - t0 > timeout) {
                        atomicExch(err, 1);
                        s_fail = 1;
                        break;
                    }
                    __builtin_amdgcn_s_sleep(1);
                }
            }
            __builtin_amdgcn_wave_barrier();
            if constexpr (TIMING) c3 = clock64();
            // the loads below are issued after the poll in program order (the
            // hardware issues a wave's loads in order; the fence keeps the
            // compiler from hoisting them above the loop)
            __atomic_signal_fence(__ATOMIC_SEQ_CST);
            // the headers and every candidate's rows t.. in one round of loads
            // (a workgroup without a candidate left stale rows: not used)
            if (tid < W) {
                cv[tid] = __hip_atomic_load(&sl[tid].v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                cp[tid] = __hip_atomic_load(&sl[tid].pos, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                cc[tid] = __hip_atomic_load(&sl[tid].col, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
            for (int e = tid; e < W * (rows - t); e += QG_T) {
                const int u = e / (rows - t), i = t + e % (rows - t);
                cd[u][i] = __hip_atomic_load(&sd[(int64_t)u * RMAX + i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
            __syncthreads();
            if (s_fail) return;
            if constexpr (TIMING) c4 = clock64();
            double gv = -1.0;
            int gp = 0x7fffffff, pc = -1, pw = 0;
#pragma unroll
            for (int u = 0; u < W; ++u)
                if (cc[u] >= 0 && qg_better(cv[u], cp[u], gv, gp)) { gv = cv[u]; gp = cp[u]; pc = cc[u]; pw = u; }
            if (pc < 0) { k = t; break; }              // no active column with a finite norm
            const double nrm = sqrt(gv);
            if (t == 0) {
                nrm0 = nrm;
                if (!(nrm0 > 0.0)) { k = 0; break; }
            } else if (nrm <= teff * nrm0) {
                k = t;
                break;
            }
            // swap positions t and posof[pc] (read again only after the
            // barrier that follows the reflector rows below)
            if (tid == 0) {
                const int ct = piv[t], pp = posof[pc];
                piv[t] = pc;
                piv[pp] = ct;
                posof[ct] = pp;
                posof[pc] = t;
            }
            // the reflector, computed alike in every workgroup
            const double *vs = cd[pw];
            const double x0 = vs[t];
            const double rtt = x0 >= 0.0 ? -nrm : nrm;
            const double denom = x0 - rtt;
            const double beta = (rtt - x0) / rtt;
            const int rt = t / 16, lt = t % 16;
            if (pw == w && grp == (pc / W) % 32) {
                const int jp = (pc / W) / 32;
#pragma unroll
                for (int j = 0; j < CPG; ++j) {
                    if (j != jp) continue;
#pragma unroll
                    for (int r = 0; r < RM; ++r) {
                        if (r > rt) {
                            x[j][r] = 0.0;             // rows past `rows` hold zeros already
                        } else if (r == rt) {
                            if (l16 > lt) x[j][r] = 0.0;
                            else if (l16 == lt) x[j][r] = rtt;
                        }
                    }
                    act[j] = false;
                }
            }
            for (int i = tid; i < RMAX; i += QG_T) svr[i] = (i > t && i < rows) ? vs[i] / denom : 0.0;
            __syncthreads();
            double vr[RM];
#pragma unroll
            for (int r = 0; r < RM; ++r) vr[r] = svr[l16 + 16 * r];
            if constexpr (TIMING) c5 = clock64();
            const int src = (lane & ~15) | lt;
            const bool lane_after = l16 > lt, lane_at = l16 == lt;
#pragma unroll
            for (int j = 0; j < CPG; ++j) {
                if (!act[j]) continue;                 // group-uniform
                // vr is zero outside rows (t, rows): the dot product needs no
                // row test
                double sdot = 0.0, top = 0.0;
#pragma unroll
                for (int r = 0; r < RM; ++r) {
                    sdot += vr[r] * x[j][r];
                    if (r == rt) top = x[j][r];
                }
                sdot = group16_sum(sdot);
                top = __shfl(top, src);
                const double f = beta * (sdot + top);
                double ns = 0.0;
                // slices after rt change whole (their rows past `rows` hold
                // zeros with zero reflector entries and stay zero), slice rt
                // changes its rows > t and row t becomes R(t, c), slices
                // before it keep their R rows: uniform tests per slice and
                // one lane test, instead of a row test per element
#pragma unroll
                for (int r = 0; r < RM; ++r) {
                    const double y = x[j][r] - f * vr[r];
                    if (r > rt) {
                        x[j][r] = y;
                        ns += y * y;
                    } else if (r == rt) {
                        if (lane_after) {
                            x[j][r] = y;
                            ns += y * y;
                        } else if (lane_at) {
                            x[j][r] = top - f;
                        }
                    }
                }
                nv[j] = group16_sum(ns);
            }
            if constexpr (TIMING) {
                const unsigned long long c6 = clock64();
                tph[0] += c1 - c0;
                tph[1] += c2 - c1;
                tph[2] += c3 - c2;
                tph[3] += c4 - c3;
                tph[4] += c5 - c4;
                tph[5] += c6 - c5;
                tph[6] += 1;
            }
        }
        // every column to its final position
        __syncthreads();
#pragma unroll
        for (int j = 0; j < CPG; ++j) {
            const int c = w + W * (grp + 32 * j);
            if (c < cols) {
                const int pos = posof[c];
#pragma unroll
                for (int r = 0; r < RM; ++r) {
                    const int i = l16 + 16 * r;
                    if (i < rows) G[(int64_t)pos * ell + i] = x[j][r];
                }
            }
        }
        if (w == 0) {
            for (int c = tid; c < cols; c += QG_T) I.colperm[(int64_t)a * I.ncol_max + c] = piv[c];
            if (tid == 0) I.skk[a] = k;
        }
    }
    if constexpr (TIMING) {
        if (tid == 0)
            for (int i = 0; i < 7; ++i) atomicAdd(&tacc[i], tph[i]);
    }
}

// P = R11^{-1} R12 in place over R12 (FP64).  Block per (node, chunk of SV_C
// columns of R12): the chunk is held in LDS and solved right-looking: for
// t = k-1 .. 0, P[t] = R12'[t] / R_tt, then R12'[u] -= R_ut P[t] for u < t.
constexpr int SV_T = 256;
constexpr int SV_C = 16;

__global__ __launch_bounds__(SV_T) void k_solve(double *__restrict__ Gall, int ell, int ncol_max,
                                                const SkelInst *__restrict__ inst,
                                                const int2 *__restrict__ items)
{
    extern __shared__ double sP[];             // k x SV_C
    const int q = blockIdx.y;
    const int2 it = items[q];
    const int a = it.y;
    const int k = inst[it.x].skk[a], n = inst[it.x].ncols[a];
    const int c0 = blockIdx.x * SV_C;
    const int cw = min(SV_C, n - k - c0);
    if (cw <= 0 || k == 0) return;
    double *G = Gall + (int64_t)q * ncol_max * ell;
    for (int e = threadIdx.x; e < k * SV_C; e += SV_T) {
        int c = e / k, t = e % k;
        sP[t * SV_C + c] = c < cw ? G[(int64_t)(k + c0 + c) * ell + t] : 0.0;
    }
    __syncthreads();
    for (int t = k - 1; t >= 0; --t) {
        const double rtt = G[(int64_t)t * ell + t];
        if (threadIdx.x < SV_C) sP[t * SV_C + threadIdx.x] /= rtt;
        __syncthreads();
        const double *rcol = G + (int64_t)t * ell;     // R[u][t], u < t
        for (int e = threadIdx.x; e < t * SV_C; e += SV_T) {
            int u = e / SV_C, c = e % SV_C;
            sP[u * SV_C + c] -= rcol[u] * sP[t * SV_C + c];
        }
        __syncthreads();
    }
    for (int e = threadIdx.x; e < k * SV_C; e += SV_T) {
        int c = e / k, t = e % k;
        if (c < cw) G[(int64_t)(k + c0 + c) * ell + t] = sP[t * SV_C + c];
    }
}

// S, skeleton coordinates and bandwidth factors, P in FP32 (row stride n-k).
// The same solve for k <= 256, register-blocked: a block takes 32 columns
// of R12, each column spread over 8 lanes that hold rows j, j + 8, ... in
// registers.  R's columns are staged in LDS 8 at a time, so a block
// synchronises twice per 8 rows instead of twice per row; row t's value is
// divided by R_tt by the lane that holds it and broadcast to the column's
// lanes.  The updates of every element come in the same order as above
// (t = k-1 down to the row + 1).
constexpr int SR_L = 8;       // lanes per column
constexpr int SR_R = 32;      // rows per lane (k <= 256)
constexpr int SR_C = 32;      // columns per block

__global__ __launch_bounds__(256) void k_solve_reg(double *__restrict__ Gall, int ell, int ncol_max,
                                                   const SkelInst *__restrict__ inst,
                                                   const int2 *__restrict__ items)
{
    __shared__ double sR[SR_L * SR_L * SR_R];       // 8 columns of R, rows 0 .. 255
    const int q = blockIdx.y;
    const int2 it = items[q];
    const int a = it.y;
    const int k = inst[it.x].skk[a], m = inst[it.x].ncols[a] - k;
    const int c0 = blockIdx.x * SR_C;
    if (k == 0 || c0 >= m) return;
    const int tid = threadIdx.x, lane = tid % 64;
    const int col = tid / SR_L, j = tid % SR_L, base = lane & ~(SR_L - 1);
    const bool cok = c0 + col < m;
    double *G = Gall + (int64_t)q * ncol_max * ell;
    double *pc = G + (int64_t)(k + c0 + (cok ? col : 0)) * ell;
    // loads are unconditional (indices clamped inside the block) so that they
    // are all in flight at once; entries outside R are replaced by zeros
    double P[SR_R];
#pragma unroll
    for (int i = 0; i < SR_R; ++i) {
        const int u = SR_L * i + j;
        const double v = pc[min(u, ell - 1)];
        P[i] = (cok && u < k) ? v : 0.0;
    }
    // R's columns 8 ib .. 8 ib + 7: loaded into registers one group ahead
    // (their loads are in flight while the previous group is solved), then
    // stored to LDS
    static_assert((SR_L * SR_L * SR_R) % 256 == 0, "the staging loop covers the block exactly");
    constexpr int SV = SR_L * SR_L * SR_R / 256;
    auto load_group = [&](int ib, double (&v)[SV]) {
#pragma unroll
        for (int r = 0; r < SV; ++r) {
            const int e = tid + 256 * r;
            const int cc = e / (SR_L * SR_R), u = e % (SR_L * SR_R), t = SR_L * ib + cc;
            v[r] = G[(int64_t)min(t, k - 1) * ell + min(u, ell - 1)];
        }
    };
    const int ibt = (k - 1) / SR_L;              // the last group holding a column of R11
    double v[SV];
    load_group(ibt, v);
#pragma clang loop unroll(full)
    for (int ib = SR_R - 1; ib >= 0; --ib) {
        if (ib > ibt) continue;
        __syncthreads();
#pragma unroll
        for (int r = 0; r < SV; ++r) {
            const int e = tid + 256 * r;
            const int cc = e / (SR_L * SR_R), u = e % (SR_L * SR_R), t = SR_L * ib + cc;
            sR[e] = (t < k && u <= t) ? v[r] : 0.0;
        }
        __syncthreads();
        if (ib > 0) load_group(ib - 1, v);
        for (int jj = SR_L - 1; jj >= 0; --jj) {
            const int t = SR_L * ib + jj;
            if (t >= k) continue;
            const double *rc = sR + jj * (SR_L * SR_R);      // column t of R
            const double pt = __shfl(P[ib], base + jj) / rc[t];
            if (j == jj) P[ib] = pt;
#pragma clang loop unroll(full)
            for (int i = 0; i < ib; ++i) P[i] -= rc[SR_L * i + j] * pt;
            if (j < jj) P[ib] -= rc[SR_L * ib + j] * pt;
        }
    }
#pragma unroll
    for (int i = 0; i < SR_R; ++i) {
        const int u = SR_L * i + j;
        if (cok && u < k) pc[u] = P[i];
    }
}

__global__ __launch_bounds__(256) void k_finalize(const double *__restrict__ Gall, int ell,
                                                  int ncol_max, const SkelInst *__restrict__ inst,
                                                  const int2 *__restrict__ items,
                                                  const int32_t *__restrict__ colpos, int smax)
{
    const int q = blockIdx.x;
    const int2 it = items[q];
    const SkelInst &I = inst[it.x];
    const int a = it.y;
    const int dp = I.dp;
    const float *Xt = I.Xt, *gt = I.gt;
    int32_t *S = I.S;
    float *Xs = I.Xs, *gs = I.gs;
    const int k = I.skk[a], n = I.ncols[a], nr = n - k;
    const double *G = Gall + (int64_t)q * ncol_max * ell;
    const int32_t *pv = I.colperm + (int64_t)a * I.ncol_max;
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
    // P (row t, column c) = R12 solution (G column k + c, row t) in FP32,
    // through 64 x 64 tiles in LDS: reads run down G's columns and writes
    // along P's rows (both contiguous); loads are unconditional (indices
    // clamped inside the block) so that all of a tile's are in flight at once
    __shared__ float tP[64][65];
    float *Pa = I.P + I.pslot[a];
    const int l64 = threadIdx.x & 63, w4 = threadIdx.x >> 6;
    for (int t0 = 0; t0 < k; t0 += 64)
        for (int c0 = 0; c0 < nr; c0 += 64) {
            const int tr = min(t0 + l64, k - 1);
            float v[16];
#pragma unroll
            for (int i = 0; i < 16; ++i) {
                const int c = min(c0 + w4 + 4 * i, nr - 1);
                v[i] = (float)G[(int64_t)(k + c) * ell + tr];
            }
#pragma unroll
            for (int i = 0; i < 16; ++i) tP[w4 + 4 * i][l64] = v[i];
            __syncthreads();
#pragma unroll
            for (int i = 0; i < 16; ++i) {
                const int t = t0 + w4 + 4 * i, c = c0 + l64;
                if (t < k && c < nr) Pa[(int64_t)t * nr + c] = tP[l64][w4 + 4 * i];
            }
            __syncthreads();
        }
}

// Scratch of the gang factorization: per gang two rounds of W candidate
// slots and candidate columns (ell rows each); one error flag.
constexpr int QG_GMAX = 256;
struct GangScratch {
    GangSlot *slots = nullptr;
    double *sdata = nullptr;
    int32_t *err = nullptr;
    unsigned long long *tacc = nullptr;     // ASKIT_QR_TIMING: phase cycle sums, else NULL
};

// Clears n exchange slots, and the error flag when err is given (once per
// skeletonization: the flag then stays set once any gang timed out).
__global__ void k_gang_reset(GangSlot *__restrict__ slots, int n, int32_t *__restrict__ err)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) {
        slots[i].seq = 0;
        slots[i].col = -1;
    }
    if (i == 0 && err) *err = 0;
}

// Gang launches are serialized across host threads: each needs all of its
// workgroups resident at once, which a cooperative launch guarantees for
// one kernel at a time.
static std::mutex g_gang_mu;

template <int W, int RM, int CPG, bool TIMING>
static bool qr_gang_launch1(double *G, int ell, int ncm, const SkelInst *inst, const int2 *items, int smax,
                            double tau, int nb, const GangScratch &gs, uint64_t timeout, hipStream_t s)
{
    int dev = 0, ncu = 0, per = 0;
    HIPC(hipGetDevice(&dev));
    HIPC(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
    HIPC(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_qrcp_gang<W, RM, CPG, TIMING>, QG_T, 0));
    // a multiple of 8 gangs (one set per XCD); gangs past the last node idle
    const int fit = std::min(QG_GMAX, per * ncu / W) / 8 * 8;
    const int ngang = std::min(fit, (nb + 7) / 8 * 8);
    if (ngang < 8) return false;
    const int nslot = ngang * 2 * W;
    hipLaunchKernelGGL(k_gang_reset, dim3((unsigned)((nslot + 255) / 256)), dim3(256), 0, s, gs.slots, nslot,
                       (int32_t *)nullptr);
    HIPC(hipGetLastError());
    GangSlot *slots = gs.slots;
    double *sdata = gs.sdata;
    int32_t *err = gs.err;
    unsigned long long *tacc = gs.tacc;
    void *args[] = {&G, &ell, &ncm, (void *)&inst, (void *)&items, &smax, &tau, &nb, &slots, &sdata, &err, &timeout,
                    &tacc};
    HIPC(hipLaunchCooperativeKernel((const void *)k_qrcp_gang<W, RM, CPG, TIMING>, dim3((unsigned)(ngang * W)),
                                    dim3(QG_T), args, 0, s));
    return true;
}

template <int W, int RM, int CPG>
static bool qr_gang_launch(double *G, int ell, int ncm, const SkelInst *inst, const int2 *items, int smax,
                           double tau, int nb, const GangScratch &gs, uint64_t timeout, hipStream_t s)
{
    return gs.tacc ? qr_gang_launch1<W, RM, CPG, true>(G, ell, ncm, inst, items, smax, tau, nb, gs, timeout, s)
                   : qr_gang_launch1<W, RM, CPG, false>(G, ell, ncm, inst, items, smax, tau, nb, gs, timeout, s);
}

void skeletonize(askit_handle *h, hipStream_t s)
{
    std::vector<askit_handle *> one{h};
    skeletonize_multi(one, s);
}

// The ID of every node of every given handle (Alg. 3 with the sampled rows of
// Eq. e:sk_targets), level by level from the deepest: one launch of each
// kernel per level (in batches that bound the FP64 blocks) over the nodes of
// that level in all handles, each node reading its handle's arrays from an
// instance table.  The handles share ell, s_max and the ID tolerance.  Every
// node sees the same operations as when its handle is skeletonized alone.
void skeletonize_multi(const std::vector<askit_handle *> &hs, hipStream_t s)
{
    if (hs.empty()) return;
    const askit_handle *h0 = hs[0];
    const int ell = h0->ell, smax = h0->smax;
    const double tau = h0->prm.id_tol;
    int ncm = 0, maxdepth = 0;
    for (auto *h : hs) {
        if (h->ell != ell || h->smax != smax || h->prm.id_tol != tau)
            fail(ASKIT_ERR_INVALID_ARG, "fused skeletonization needs one ell, s_max and tolerance");
        ncm = std::max(ncm, h->ncol_max);
        maxdepth = std::max(maxdepth, h->depth);
    }
    if (ncm > QR_MAXCOL || ell > QR_MAXROW || ell > FG_MAXROW)
        fail(ASKIT_ERR_UNSUPPORTED, "ID block larger than 1024 rows x 2048 columns");
    for (auto *h : hs) {
        HIPC(hipMemsetAsync(h->skk, 0, sizeof(int32_t) * h->nodes.size(), s));
        HIPC(hipMemsetAsync(h->ncols, 0, sizeof(int32_t) * h->nodes.size(), s));
        h->t_qr = 0;
    }
    if (maxdepth == 0) return;
    std::vector<void *> tmp;
    struct Free {
        std::vector<void *> &t;
        hipStream_t s;
        ~Free()
        {
            (void)hipStreamSynchronize(s);
            for (void *p : t) (void)ws_free(p, s);
        }
    } fr{tmp, s};
    auto ta = [&](size_t b) {
        void *p;
        HIPC(ws_alloc(&p, std::max<size_t>(b, 16), s));
        tmp.push_back(p);
        return p;
    };
    // the instance table
    std::vector<SkelInst> hin(hs.size());
    for (size_t i = 0; i < hs.size(); ++i) {
        askit_handle *h = hs[i];
        SkelInst &I = hin[i];
        I.nodes = h->d_nodes;
        I.Xt = h->Xt;
        I.gt = h->gt;
        I.T = h->T;
        I.T_cnt = h->T_cnt;
        I.S = h->S;
        I.skk = h->skk;
        I.ncols = h->ncols;
        I.colperm = h->colperm;
        I.pslot = h->d_pslot;
        I.P = h->P;
        I.Xs = h->Xs;
        I.gs = h->gs;
        I.h = h->prm.bandwidth;
        I.hpos = nullptr;
        I.dp = h->dp;
        I.d = h->d;
        I.ncol_max = h->ncol_max;
        if (h->varh) {
            // per tree position bandwidth (FP64) from the per-id array
            double *hp = (double *)ta(sizeof(double) * h->N);
            gather_f64(h->hsrc, h->perm, h->N, hp, s);
            I.hpos = hp;
        }
    }
    SkelInst *d_inst = (SkelInst *)ta(sizeof(SkelInst) * hs.size());
    HIPC(hipMemcpyAsync(d_inst, hin.data(), sizeof(SkelInst) * hs.size(), hipMemcpyHostToDevice, s));
    // batch so that the FP64 blocks stay within ~4 GiB (one batch per level
    // up to 3,800 nodes of 512 columns x 276 rows)
    int64_t maxlev = 0;
    for (int lev = 1; lev <= maxdepth; ++lev) {
        int64_t c = 0;
        for (auto *h : hs)
            if (lev <= h->depth) c += (int64_t)h->level_nodes[lev].size();
        maxlev = std::max(maxlev, c);
    }
    const size_t per = (size_t)ncm * ell * sizeof(double);
    const int batch = (int)std::max<size_t>(1, std::min<size_t>((size_t)maxlev, (size_t)(4ull << 30) / per));
    double *G = (double *)ta(per * batch);
    int32_t *colpos = (int32_t *)ta(sizeof(int32_t) * (size_t)ncm * batch);
    const size_t sv_lds = sizeof(double) * (size_t)std::min(smax, ell) * SV_C;
    if (sv_lds > 64 * 1024)
        HIPC(hipFuncSetAttribute((const void *)k_solve, hipFuncAttributeMaxDynamicSharedMemorySize,
                                 (int)sv_lds));
    // gang factorization: needs cooperative launches, at most 512 columns
    // (the registers of 4 x 32 x 4 slots) and 288 rows (18 per lane)
    int coop = 0, clk_khz = 0;
    {
        int dev = 0;
        HIPC(hipGetDevice(&dev));
        HIPC(hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, dev));
        HIPC(hipDeviceGetAttribute(&clk_khz, hipDeviceAttributeWallClockRate, dev));
    }
    // (by default the nodes of large point sets only, as each handle alone
    // would: a node takes the same form of the QR alone and fused).
    // ASKIT_QR_GANG=1 uses it at any size, 0 never.
    const char *genv = std::getenv("ASKIT_QR_GANG");
    const int gmode = genv ? std::atoi(genv) : -1;
    const bool can_gang = coop && clk_khz > 0 && ncm <= 512 && ell <= 16 * 18 && gmode != 0;
    auto gang_node = [&](const askit_handle *h) { return can_gang && (gmode == 1 || h->N >= (1 << 18)); };
    bool use_gang = false;
    for (auto *h : hs) use_gang = use_gang || gang_node(h);
    const uint64_t g_timeout = (uint64_t)((double)clk_khz * 1000.0 * QG_TIMEOUT_S);
    GangScratch gsc;
    if (use_gang) {
        gsc.slots = (GangSlot *)ta(sizeof(GangSlot) * QG_GMAX * 2 * 8);
        gsc.sdata = (double *)ta(sizeof(double) * QG_GMAX * 2 * 8 * 16 * 18);
        gsc.err = (int32_t *)ta(sizeof(int32_t));
        // ASKIT_QR_TIMING=1: per gang launch, the mean clock cycles of a pivot
        // step's phases on stderr (a diagnostic; off by default)
        const char *tenv = std::getenv("ASKIT_QR_TIMING");
        if (tenv && std::atoi(tenv) == 1) gsc.tacc = (unsigned long long *)ta(sizeof(unsigned long long) * 8);
    }
    // every level's batches of nodes (those that take the gang form first),
    // uploaded at once: the levels then follow each other on the stream with
    // no host wait between them (the gang diagnostic waits per level)
    struct Batch {
        int lev, off, nb, ng;
    };
    std::vector<Batch> bat;
    std::vector<int2> items;
    for (int lev = maxdepth; lev >= 1; --lev) {
        std::vector<int2> all;
        for (int pass = 0; pass < 2; ++pass)
            for (size_t i = 0; i < hs.size(); ++i)
                if (lev <= hs[i]->depth && gang_node(hs[i]) == (pass == 0))
                    for (int a : hs[i]->level_nodes[lev]) all.push_back(int2{(int)i, a});
        for (size_t b0 = 0; b0 < all.size(); b0 += batch) {
            const int nb = (int)std::min<size_t>(batch, all.size() - b0);
            int ng = 0;
            while (ng < nb && gang_node(hs[all[b0 + ng].x])) ++ng;
            bat.push_back(Batch{lev, (int)items.size(), nb, ng});
            items.insert(items.end(), all.begin() + b0, all.begin() + b0 + nb);
        }
    }
    int2 *d_items_all = (int2 *)ta(sizeof(int2) * std::max<size_t>(items.size(), 1));
    if (!items.empty())
        HIPC(hipMemcpyAsync(d_items_all, items.data(), sizeof(int2) * items.size(), hipMemcpyHostToDevice, s));
    // gang launches of other threads wait for this whole pass (a gang needs
    // its workgroups co-resident)
    std::unique_lock<std::mutex> glk(g_gang_mu, std::defer_lock);
    if (use_gang) {
        glk.lock();
        hipLaunchKernelGGL(k_gang_reset, dim3(1), dim3(64), 0, s, gsc.slots, 0, gsc.err);
        HIPC(hipGetLastError());
    }
    std::vector<hipEvent_t> qev;                // brackets of each batch's factorization (timing only)
    struct QevFree {
        std::vector<hipEvent_t> &v;
        ~QevFree()
        {
            for (hipEvent_t e : v) (void)hipEventDestroy(e);
        }
    } qevf{qev};
    bool any_gang = false;
    for (const Batch &bt : bat) {
        const int nb = bt.nb, ng = bt.ng, lev = bt.lev;
        int2 *d_items = d_items_all + bt.off;
        hipLaunchKernelGGL(k_cols, dim3(nb), dim3(256), 0, s, d_inst, d_items, smax, ncm, colpos);
        {
            dim3 gg((ncm + FG_C - 1) / FG_C, nb), gb(((ell + FG_R - 1) / FG_R + 63) / 64 * 64);
            hipLaunchKernelGGL(k_form_G, gg, gb, 0, s, d_inst, d_items, ell, colpos, ncm, G);
            HIPC(hipGetLastError());
        }
        qev.resize(qev.size() + 2);
        HIPC(hipEventCreate(&qev[qev.size() - 2]));
        HIPC(hipEventCreate(&qev.back()));
        HIPC(hipEventRecord(qev[qev.size() - 2], s));
        // every level: the node's columns in registers across a gang of
        // workgroups (4 per node from 64 nodes on, else 8), as many gangs
        // as fit at once, each taking nodes in turn; one workgroup per
        // node streaming G when the gang cannot run (no cooperative
        // launch, more than 512 columns or 288 rows)
        bool gang = false;
        if (use_gang && ng > 0) {
            if (gsc.tacc) HIPC(hipMemsetAsync(gsc.tacc, 0, sizeof(unsigned long long) * 8, s));
            if (ell <= 16 * 8)
                gang = ng >= 64 ? qr_gang_launch<4, 8, 4>(G, ell, ncm, d_inst, d_items, smax, tau, ng, gsc,
                                                         g_timeout, s)
                                : qr_gang_launch<8, 8, 2>(G, ell, ncm, d_inst, d_items, smax, tau, ng, gsc,
                                                         g_timeout, s);
            else
                gang = ng >= 64 ? qr_gang_launch<4, 18, 4>(G, ell, ncm, d_inst, d_items, smax, tau, ng, gsc,
                                                          g_timeout, s)
                                : qr_gang_launch<8, 18, 2>(G, ell, ncm, d_inst, d_items, smax, tau, ng, gsc,
                                                          g_timeout, s);
        }
        any_gang = any_gang || gang;
        // the rest (all items when the gang did not run), streaming G
        const int q0i = gang ? ng : 0, nrest = nb - q0i;
        double *Gr = G + (int64_t)q0i * ncm * ell;
        const int2 *ir = d_items + q0i;
        if (nrest == 0) {
        } else if (ell <= 16 * 8)
            hipLaunchKernelGGL((k_qrcp<512, 8>), dim3((unsigned)nrest), dim3(512), 0, s, Gr, ell, ncm, d_inst,
                               ir, smax, tau, nrest);
        else if (ell <= 16 * 18)
            hipLaunchKernelGGL((k_qrcp<512, 18>), dim3((unsigned)nrest), dim3(512), 0, s, Gr, ell, ncm,
                               d_inst, ir, smax, tau, nrest);
        else
            hipLaunchKernelGGL((k_qrcp<QR_T, 0>), dim3((unsigned)nrest), dim3(QR_T), 0, s, Gr, ell, ncm,
                               d_inst, ir, smax, tau, nrest);
        HIPC(hipEventRecord(qev.back(), s));
        if (smax <= SR_L * SR_R)
            hipLaunchKernelGGL(k_solve_reg, dim3((ncm + SR_C - 1) / SR_C, nb), dim3(256), 0, s, G, ell, ncm,
                               d_inst, d_items);
        else
            hipLaunchKernelGGL(k_solve, dim3((ncm + SV_C - 1) / SV_C, nb), dim3(SV_T), sv_lds, s, G, ell,
                               ncm, d_inst, d_items);
        hipLaunchKernelGGL(k_finalize, dim3(nb), dim3(256), 0, s, G, ell, ncm, d_inst, d_items, colpos, smax);
        HIPC(hipGetLastError());
        if (gang && gsc.tacc) {
            HIPC(hipStreamSynchronize(s));
            unsigned long long tc[8];
            HIPC(hipMemcpy(tc, gsc.tacc, sizeof(tc), hipMemcpyDeviceToHost));
            const double st = tc[6] ? (double)tc[6] : 1.0;
            std::fprintf(stderr,
                         "[askit qr timing] level %d: %d nodes, %llu workgroup pivot steps; cycles per step: "
                         "argmax %.0f, publish %.0f, wait %.0f, load %.0f, reflector %.0f, update %.0f\n",
                         lev, ng, tc[6], tc[0] / st, tc[1] / st, tc[2] / st, tc[3] / st, tc[4] / st, tc[5] / st);
        }
    }
    HIPC(hipStreamSynchronize(s));
    if (any_gang) {
        // the flag stays set once any gang exchange timed out
        int32_t herr = 0;
        HIPC(hipMemcpy(&herr, gsc.err, sizeof(int32_t), hipMemcpyDeviceToHost));
        if (herr) fail(ASKIT_ERR_DEVICE, "QR gang exchange timed out (workgroups not co-resident)");
    }
    if (glk.owns_lock()) glk.unlock();
    double t_qr = 0.0;
    for (size_t e = 0; e < qev.size(); e += 2) {
        float ms = 0.f;
        HIPC(hipEventElapsedTime(&ms, qev[e], qev[e + 1]));
        t_qr += ms;
    }
    for (auto *h : hs) h->t_qr = t_qr;
}

// ---------------------------------------------------------------- upward pass
// w~_alpha[t] = Wc[piv t] + sum_c P[t][c] Wc[piv k+c]; Wc = W(X_alpha) at a
// leaf, [w~_left; w~_right] at an internal node.  One wave per (node, t).
// Skeleton weights of row t of node a, columns [r0, r1): w~_t = w(S_t) +
// sum_c P_tc w(R_c) (Alg. 3, the far field by skeletonization).  Each
// column's sum runs over c = lane, lane + 64, ... as an fma chain per lane,
// then a xor butterfly across the wave (every lane ends with the same total);
// the columns are taken RT at a time so that their weight loads are in flight
// together.  A column's arithmetic does not depend on RT, on the column range
// or on the number of columns.
template <int RT>
__device__ __forceinline__ void upward_row(const Node &nd, int a, int t, int k, int nr, int kl,
                                           const int32_t *__restrict__ pv, const float *__restrict__ Pt,
                                           const float *__restrict__ Wt, float *__restrict__ Wsk, int smax, int R,
                                           int r0, int r1)
{
    const int lane = threadIdx.x;
    // row of column c of the node's block: its own points at a leaf, else the
    // children's skeleton rows (left first)
    auto wrow = [&](int c) -> const float * {
        if (nd.left < 0) return Wt + (int64_t)(nd.lo + c) * R;
        return c < kl ? Wsk + ((int64_t)nd.left * smax + c) * R
                      : Wsk + ((int64_t)nd.right * smax + (c - kl)) * R;
    };
    const float *w0 = wrow(pv[t]);
    for (int rt = r0; rt < r1; rt += RT) {
        float acc[RT];
#pragma unroll
        for (int j = 0; j < RT; ++j) acc[j] = 0.0f;
#pragma unroll 2
        for (int c = lane; c < nr; c += 64) {
            const float pc = Pt[c];
            const float *wr = wrow(pv[k + c]);
            float wv[RT];
#pragma unroll
            for (int j = 0; j < RT; ++j) wv[j] = wr[min(rt + j, r1 - 1)];   // clamped: unconditional loads
#pragma unroll
            for (int j = 0; j < RT; ++j) acc[j] = fmaf(pc, wv[j], acc[j]);
        }
#pragma unroll
        for (int j = 0; j < RT; ++j) {
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) acc[j] += __shfl_xor(acc[j], o);
        }
        float v = acc[0];
#pragma unroll
        for (int j = 1; j < RT; ++j) v = lane == j ? acc[j] : v;
        if (lane < RT && rt + lane < r1) Wsk[((int64_t)a * smax + t) * R + rt + lane] = w0[rt + lane] + v;
    }
}

template <int RT>
__global__ __launch_bounds__(64) void k_upward(const Node *__restrict__ nodes,
                                               const int32_t *__restrict__ ids,
                                               const int32_t *__restrict__ skk,
                                               const int32_t *__restrict__ ncols,
                                               const int32_t *__restrict__ colperm, int ncol_max,
                                               const int64_t *__restrict__ pslot,
                                               const float *__restrict__ P, int smax,
                                               const float *__restrict__ Wt, int R,
                                               float *__restrict__ Wsk, int r0, int r1)
{
    const int a = ids[blockIdx.x], t = blockIdx.y;
    const int k = skk[a];
    if (t >= k) return;
    const Node nd = nodes[a];
    const int nr = ncols[a] - k;
    const int kl = nd.left >= 0 ? skk[nd.left] : 0;
    upward_row<RT>(nd, a, t, k, nr, kl, colperm + (int64_t)a * ncol_max, P + pslot[a] + (int64_t)t * nr, Wt, Wsk,
                   smax, R, r0, r1);
}

// The same rows of skeleton weights for many columns: one workgroup per
// (node, UP_TT skeleton rows).  For each tile of RT columns the node's
// non-skeleton weight rows are staged in LDS once, then the four waves take
// the skeleton rows in turn.  Every column's arithmetic is that of
// upward_row (fma chain over c = lane, lane + 64, ..., xor butterfly,
// w(S_t) added last), so both forms give the same bits.
constexpr int UP_TT = 64;

template <int RT>
__device__ __forceinline__ void upward_block(const Node &nd, int a, int k, int nr, int kl,
                                             const int32_t *__restrict__ pv, const float *__restrict__ Pa,
                                             const float *__restrict__ Wt, float *__restrict__ Wsk, int smax,
                                             int R, int r0, int r1, int t0, int32_t *sPv, float *sW)
{
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    auto wrow = [&](int c) -> const float * {
        if (nd.left < 0) return Wt + (int64_t)(nd.lo + c) * R;
        return c < kl ? Wsk + ((int64_t)nd.left * smax + c) * R
                      : Wsk + ((int64_t)nd.right * smax + (c - kl)) * R;
    };
    for (int c = tid; c < nr; c += 256) sPv[c] = pv[k + c];
    const int tn = min(UP_TT, k - t0);
    const int ne = nr * RT;
    for (int rt = r0; rt < r1; rt += RT) {
        __syncthreads();
        // rows c of the block, columns rt .. rt + RT (clamped: unconditional loads, four in flight)
        for (int e0 = tid; e0 < ne; e0 += 256 * 4) {
            float v[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int e = min(e0 + 256 * u, ne - 1);
                v[u] = wrow(sPv[e / RT])[min(rt + e % RT, r1 - 1)];
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int e = e0 + 256 * u;
                if (e < ne) sW[(e / RT) * (RT + 1) + e % RT] = v[u];
            }
        }
        __syncthreads();
        for (int tt = wv; tt < tn; tt += 4) {
            const int t = t0 + tt;
            const float *Pt = Pa + (int64_t)t * nr;
            float acc[RT];
#pragma unroll
            for (int j = 0; j < RT; ++j) acc[j] = 0.0f;
#pragma unroll 2
            for (int c = lane; c < nr; c += 64) {
                const float pc = Pt[c];
                const float *wr = sW + c * (RT + 1);
#pragma unroll
                for (int j = 0; j < RT; ++j) acc[j] = fmaf(pc, wr[j], acc[j]);
            }
#pragma unroll
            for (int j = 0; j < RT; ++j) {
#pragma unroll
                for (int o = 32; o > 0; o >>= 1) acc[j] += __shfl_xor(acc[j], o);
            }
            float v = acc[0];
#pragma unroll
            for (int j = 1; j < RT; ++j) v = lane == j ? acc[j] : v;
            if (lane < RT && rt + lane < r1)
                Wsk[((int64_t)a * smax + t) * R + rt + lane] = wrow(pv[t])[rt + lane] + v;
        }
    }
}

template <int RT>
__global__ __launch_bounds__(256) void k_upward_blk(const Node *__restrict__ nodes,
                                                    const int32_t *__restrict__ ids,
                                                    const int32_t *__restrict__ skk,
                                                    const int32_t *__restrict__ ncols,
                                                    const int32_t *__restrict__ colperm, int ncol_max,
                                                    const int64_t *__restrict__ pslot,
                                                    const float *__restrict__ P, int smax,
                                                    const float *__restrict__ Wt, int R,
                                                    float *__restrict__ Wsk, int r0, int r1)
{
    extern __shared__ float usm[];
    const int a = ids[blockIdx.x], t0 = blockIdx.y * UP_TT;
    const int k = skk[a];
    if (t0 >= k) return;
    const Node nd = nodes[a];
    const int nr = ncols[a] - k;
    const int kl = nd.left >= 0 ? skk[nd.left] : 0;
    upward_block<RT>(nd, a, k, nr, kl, colperm + (int64_t)a * ncol_max, P + pslot[a], Wt, Wsk, smax, R, r0, r1,
                     t0, (int32_t *)usm, usm + ncol_max);
}

// columns per tile of the upward pass for a range of nc columns
static int upward_tile(int nc) { return nc >= 16 ? 16 : (nc >= 4 ? 4 : 1); }

// LDS of the block form for RT columns and blocks of up to ncol_max columns
static size_t upward_lds(int RT, int ncol_max) { return sizeof(float) * (size_t)ncol_max * (RT + 2); }
constexpr size_t UP_LDS_MAX = 64 * 1024;

void prepare_upward(askit_handle *h)
{
    std::vector<int32_t> all;
    h->up_seg.clear();
    for (int lev = h->depth; lev >= 1; --lev) {
        h->up_seg.push_back({(int)all.size(), (int)h->level_nodes[lev].size()});
        all.insert(all.end(), h->level_nodes[lev].begin(), h->level_nodes[lev].end());
    }
    h->up_ids = (int32_t *)h->alloc(sizeof(int32_t) * std::max<size_t>(all.size(), 1), false);
    if (!all.empty())
        HIPC(hipMemcpy(h->up_ids, all.data(), sizeof(int32_t) * all.size(), hipMemcpyHostToDevice));
}

void upward(askit_handle *h, const WeightSet &ws, hipStream_t s, int r0, int r1)
{
    if (r1 < 0) r1 = ws.R;
    for (auto &sg : h->up_seg) {
        if (sg.second == 0) continue;
        const int rt = upward_tile(r1 - r0);
        const size_t lds = upward_lds(rt, h->ncol_max);
        const dim3 gb(sg.second, (h->smax + UP_TT - 1) / UP_TT), bb(256);
        const dim3 g(sg.second, h->smax), b(64);
        if (rt == 16 && lds <= UP_LDS_MAX)
            hipLaunchKernelGGL(k_upward_blk<16>, gb, bb, lds, s, h->d_nodes, h->up_ids + sg.first, h->skk,
                               h->ncols, h->colperm, h->ncol_max, h->d_pslot, h->P, h->smax, ws.Wt, ws.R, ws.Wsk,
                               r0, r1);
        else if (rt == 4 && lds <= UP_LDS_MAX)
            hipLaunchKernelGGL(k_upward_blk<4>, gb, bb, lds, s, h->d_nodes, h->up_ids + sg.first, h->skk,
                               h->ncols, h->colperm, h->ncol_max, h->d_pslot, h->P, h->smax, ws.Wt, ws.R, ws.Wsk,
                               r0, r1);
        else if (rt == 16)
            hipLaunchKernelGGL(k_upward<16>, g, b, 0, s, h->d_nodes, h->up_ids + sg.first, h->skk, h->ncols,
                               h->colperm, h->ncol_max, h->d_pslot, h->P, h->smax, ws.Wt, ws.R, ws.Wsk, r0, r1);
        else if (rt == 4)
            hipLaunchKernelGGL(k_upward<4>, g, b, 0, s, h->d_nodes, h->up_ids + sg.first, h->skk, h->ncols,
                               h->colperm, h->ncol_max, h->d_pslot, h->P, h->smax, ws.Wt, ws.R, ws.Wsk, r0, r1);
        else
            hipLaunchKernelGGL(k_upward<1>, g, b, 0, s, h->d_nodes, h->up_ids + sg.first, h->skk, h->ncols,
                               h->colperm, h->ncol_max, h->d_pslot, h->P, h->smax, ws.Wt, ws.R, ws.Wsk, r0, r1);
        HIPC(hipGetLastError());
    }
}

// Batched upward pass: the same computation as k_upward, one wave per
// ((instance, node), t) with the instance's tables and weight offsets.
template <int RT>
__global__ __launch_bounds__(64) void k_upward_multi(const UpInst *__restrict__ inst,
                                                     const int2 *__restrict__ items, int R,
                                                     const float *__restrict__ Wt_all,
                                                     float *__restrict__ Wsk_all)
{
    const int2 it = items[blockIdx.x];
    const UpInst &I = inst[it.x];
    const int a = it.y, t = blockIdx.y;
    const int k = I.skk[a];
    if (t >= k) return;
    const Node nd = I.nodes[a];
    const int nr = I.ncols[a] - k;
    const int kl = nd.left >= 0 ? I.skk[nd.left] : 0;
    upward_row<RT>(nd, a, t, k, nr, kl, I.colperm + (int64_t)a * I.ncol_max, I.P + I.pslot[a] + (int64_t)t * nr,
                   Wt_all + I.wt_off * R, Wsk_all + I.wsk_off * R, I.smax, R, 0, R);
}

void upward_batch(const UpInst *inst, const int2 *items, const std::vector<std::pair<int64_t, int64_t>> &levels,
                  int smax, const float *Wt, float *Wsk, int R, hipStream_t s)
{
    for (const auto &lv : levels) {
        if (lv.second == 0) continue;
        const dim3 g((unsigned)lv.second, (unsigned)smax), b(64);
        switch (upward_tile(R)) {
        case 16:
            hipLaunchKernelGGL(k_upward_multi<16>, g, b, 0, s, inst, items + lv.first, R, Wt, Wsk);
            break;
        case 4:
            hipLaunchKernelGGL(k_upward_multi<4>, g, b, 0, s, inst, items + lv.first, R, Wt, Wsk);
            break;
        default:
            hipLaunchKernelGGL(k_upward_multi<1>, g, b, 0, s, inst, items + lv.first, R, Wt, Wsk);
        }
        HIPC(hipGetLastError());
    }
}

}  // namespace askit
