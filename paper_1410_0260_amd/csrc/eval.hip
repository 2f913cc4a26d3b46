// Downward pass (Alg. 4) over the slab interaction lists.
//
// One workgroup per slab of up to 64 targets.  For every near entry (a leaf:
// its points and weights) and far entry (a pruned node: its skeleton points
// and skeleton weights), sources are taken in tiles of 64:
//   r^2 = |x - c|^2 + |y - c|^2 - 2 (x - c).(y - c),  c = the slab's first
//   target (centring keeps the cancellation small),
// with the 64 x 64 dot products on MFMA (v_mfma_f32_32x32x2_f32, each wave a
// 32 x 32 quadrant, operands staged through LDS in 64-dimension chunks), then
// K = exp2(g_j r^2), g_j = -log2(e) / (2 h_j^2), and u_i += K_ij w_j for
// the rows i whose bit is set in the entry's mask.  Every slab owns its
// output rows, so the sums are deterministic (no atomics).
#include "askit_impl.h"

#include <algorithm>

namespace askit {

typedef __attribute__((ext_vector_type(16))) float f32x16;
typedef __attribute__((ext_vector_type(8))) __bf16 bf16x8;

// Round-to-nearest-even FP32 -> bf16 (finite inputs).
__device__ __forceinline__ uint32_t ev_f2bf(float x)
{
    uint32_t u = __float_as_uint(x);
    u += 0x7fffu + ((u >> 16) & 1u);
    return u >> 16;
}
__device__ __forceinline__ float ev_bf2f(uint32_t b) { return __uint_as_float(b << 16); }

constexpr int EV_T = 256;
constexpr int EV_KC = 64;              // dimensions per LDS chunk
constexpr int EV_LD = EV_KC + 4;       // padded LDS row (floats)
constexpr int EV_RB = 8;               // largest right-hand-side block per pass
constexpr int EV_LH = EV_KC + 8;       // padded LDS row of the bf16 operands (elements)

struct EvalParams {
    const float *Y;            // targets (rows of stride dp)
    const Slab *slabs;
    const int32_t *ptr, *node;
    const uint64_t *mask;
    const int32_t *outmap;
    float *U;
    int64_t ldu;
    int64_t nslab;
    const Node *nodes;
    const float *Xt, *gt, *Wt;   // near sources (tree order)
    const float *Xs, *gs, *Wsk;  // far sources (skeletons)
    const int32_t *skk;
    int smax, dp, R, r0, rb;
    // batched form: per-instance tables (slab.pad = instance), optional work queue
    const EvalInst *inst;
    const int32_t *order;      // persistent mode: item -> slab (cost order)
    int32_t *queue;            // persistent mode: next item (zeroed before the launch)
    int persistent;
};

// BF: distance products as bf16 hi/lo split (hi*hi + hi*lo + lo*hi) on
// v_mfma_f32_32x32x16_bf16 with FP32 accumulation and an FP64 final combine of
// |x|^2 + |y|^2 - 2 x.y; otherwise FP32 products on v_mfma_f32_32x32x2_f32.
template <int RB, bool BF, bool MULTI>
__global__ __launch_bounds__(EV_T) void k_eval(EvalParams p)
{
    __shared__ __attribute__((aligned(16))) float sA[BF ? 16 : 64 * EV_LD];
    __shared__ __attribute__((aligned(16))) float sB[BF ? 16 : 64 * EV_LD];
    __shared__ __attribute__((aligned(16))) uint16_t sAh[BF ? 64 * EV_LH : 8], sAl[BF ? 64 * EV_LH : 8];
    __shared__ __attribute__((aligned(16))) uint16_t sBh[BF ? 64 * EV_LH : 8], sBl[BF ? 64 * EV_LH : 8];
    __shared__ float sC[1024 + 64];      // centre (dp <= 1024)
    __shared__ float sAn[64], sBn[64], sBg[64], sBw[64 * RB];
    __shared__ float sRed[2][64 * RB];

    const int tid = threadIdx.x, lane = tid % 64, wv = tid / 64;
    const int half = lane >> 5, l32 = lane & 31;
    const int rq = 32 * (wv >> 1), cq = 32 * (wv & 1);
    __shared__ int64_t sItem;

  auto process = [&](const int64_t slab) {
    const Slab sb = p.slabs[slab];
    const Node *nodes = p.nodes;
    const float *Y = p.Y, *Xt = p.Xt, *gt = p.gt, *Xs = p.Xs, *gs = p.gs, *Wt = p.Wt, *Wsk = p.Wsk;
    const int32_t *skk = p.skk, *outmap = p.outmap;
    int smax = p.smax, dp = p.dp;
    if constexpr (MULTI) {
        const EvalInst &I = p.inst[sb.pad];
        nodes = I.nodes;
        Y = I.Y;
        Xt = I.Xt;
        gt = I.gt;
        Xs = I.Xs;
        gs = I.gs;
        skk = I.skk;
        outmap = I.outmap;
        smax = I.smax;
        dp = I.dp;
        Wt = p.Wt + I.wt_off * p.R;
        Wsk = p.Wsk + I.wsk_off * p.R;
    }
    const float *Yb = Y + (int64_t)sb.row0 * dp;
    const int nchunk = (dp + EV_KC - 1) / EV_KC;

    for (int k = tid; k < dp; k += EV_T) sC[k] = Yb[k];
    __syncthreads();

    // load one 64 x EV_KC chunk of rows (centred) into dst; row r valid when r < nrow
    // src row r at base + r * dp; returns the per-row partial squared norms in nrm
    auto load_chunk = [&](float *dst, uint16_t *dh, uint16_t *dl, const float *base, int nrow, int k0,
                          float *nrm, bool accum) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            int idx = tid + EV_T * u;
            int row = idx >> 4, qd = (idx & 15) * 4;
            float4 v = {0.f, 0.f, 0.f, 0.f};
            int kk = k0 + qd;
            if (row < nrow && kk < dp) {
                float4 x = *reinterpret_cast<const float4 *>(base + (int64_t)row * dp + kk);
                v.x = x.x - sC[kk];
                v.y = x.y - sC[kk + 1];
                v.z = x.z - sC[kk + 2];
                v.w = x.w - sC[kk + 3];
            }
            if constexpr (BF) {
                uint32_t h0 = ev_f2bf(v.x), h1 = ev_f2bf(v.y), h2 = ev_f2bf(v.z), h3 = ev_f2bf(v.w);
                uint32_t l0 = ev_f2bf(v.x - ev_bf2f(h0)), l1 = ev_f2bf(v.y - ev_bf2f(h1));
                uint32_t l2 = ev_f2bf(v.z - ev_bf2f(h2)), l3 = ev_f2bf(v.w - ev_bf2f(h3));
                *reinterpret_cast<uint2 *>(dh + row * EV_LH + qd) = uint2{h0 | (h1 << 16), h2 | (h3 << 16)};
                *reinterpret_cast<uint2 *>(dl + row * EV_LH + qd) = uint2{l0 | (l1 << 16), l2 | (l3 << 16)};
            } else {
                *reinterpret_cast<float4 *>(dst + row * EV_LD + qd) = v;
            }
            if (nrm) {
                float s = v.x * v.x + v.y * v.y + v.z * v.z + v.w * v.w;
#pragma unroll
                for (int o = 1; o < 16; o <<= 1) s += __shfl_xor(s, o);
                if ((idx & 15) == 0) nrm[row] = accum ? nrm[row] + s : s;
            }
        }
    };

    // target norms (all chunks); the target chunk stays resident when dp <= EV_KC
    for (int ch = 0; ch < nchunk; ++ch) {
        load_chunk(sA, sAh, sAl, Yb, sb.nrows, ch * EV_KC, sAn, ch > 0);
        __syncthreads();
    }

    float accu[16][RB];
#pragma unroll
    for (int r = 0; r < 16; ++r)
#pragma unroll
        for (int j = 0; j < RB; ++j) accu[r][j] = 0.0f;

    const int e_near0 = p.ptr[slab], e_near1 = p.ptr[slab + 1];
    const int e_far0 = p.ptr[p.nslab + 1 + slab], e_far1 = p.ptr[p.nslab + 2 + slab];
    const int ne = (e_near1 - e_near0) + (e_far1 - e_far0);
    for (int e = 0; e < ne; ++e) {
        const bool near = e < e_near1 - e_near0;
        const int eid = near ? e_near0 + e : e_far0 + (e - (e_near1 - e_near0));
        const int a = p.node[eid];
        const uint64_t msk = p.mask[eid];
        const float *src, *g, *w;
        int ns;
        if (near) {
            const Node nd = nodes[a];
            ns = nd.hi - nd.lo;
            src = Xt + (int64_t)nd.lo * dp;
            g = gt + nd.lo;
            w = Wt + (int64_t)nd.lo * p.R;
        } else {
            ns = skk[a];
            src = Xs + (int64_t)a * smax * dp;
            g = gs + (int64_t)a * smax;
            w = Wsk + (int64_t)a * smax * p.R;
        }
        float mb[16];
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            int row = rq + 8 * (r / 4) + 4 * half + (r % 4);
            mb[r] = (float)((msk >> row) & 1ull);
        }
        for (int s0 = 0; s0 < ns; s0 += 64) {
            const int nt = min(64, ns - s0);
            f32x16 acc = {};
            for (int ch = 0; ch < nchunk; ++ch) {
                __syncthreads();
                if (nchunk > 1) load_chunk(sA, sAh, sAl, Yb, sb.nrows, ch * EV_KC, nullptr, false);
                load_chunk(sB, sBh, sBl, src + (int64_t)s0 * dp, nt, ch * EV_KC, sBn, ch > 0);
                if (ch == 0 && tid < 64) {
                    bool ok = tid < nt;
                    sBg[tid] = ok ? g[s0 + tid] : 0.0f;
#pragma unroll
                    for (int j = 0; j < RB; ++j)
                        sBw[tid * RB + j] = (ok && j < p.rb) ? w[(int64_t)(s0 + tid) * p.R + p.r0 + j] : 0.0f;
                }
                __syncthreads();
                const int kc = min(EV_KC, dp - ch * EV_KC);
                if constexpr (BF) {
                    const uint16_t *ph = sAh + (rq + l32) * EV_LH + 8 * half;
                    const uint16_t *pl = sAl + (rq + l32) * EV_LH + 8 * half;
                    const uint16_t *qh = sBh + (cq + l32) * EV_LH + 8 * half;
                    const uint16_t *ql = sBl + (cq + l32) * EV_LH + 8 * half;
                    for (int k16 = 0; k16 < kc; k16 += 16) {
                        bf16x8 ah = __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4 *>(ph + k16));
                        bf16x8 al = __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4 *>(pl + k16));
                        bf16x8 bh = __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4 *>(qh + k16));
                        bf16x8 bl = __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4 *>(ql + k16));
                        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bh, acc, 0, 0, 0);
                        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bl, acc, 0, 0, 0);
                        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al, bh, acc, 0, 0, 0);
                    }
                } else {
                    const float *pa = sA + (rq + l32) * EV_LD + 4 * half;
                    const float *pb = sB + (cq + l32) * EV_LD + 4 * half;
                    for (int g8 = 0; g8 < kc; g8 += 8) {
                        float4 a4 = *reinterpret_cast<const float4 *>(pa + g8);
                        float4 b4 = *reinterpret_cast<const float4 *>(pb + g8);
                        acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a4.x, b4.x, acc, 0, 0, 0);
                        acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a4.y, b4.y, acc, 0, 0, 0);
                        acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a4.z, b4.z, acc, 0, 0, 0);
                        acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a4.w, b4.w, acc, 0, 0, 0);
                    }
                }
            }
            const int col = cq + l32;
            const float bn = sBn[col], bg = sBg[col];
            float bw[RB];
#pragma unroll
            for (int j = 0; j < RB; ++j) bw[j] = sBw[col * RB + j];
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int row = rq + 8 * (r / 4) + 4 * half + (r % 4);
                float r2;
                if constexpr (BF)
                    r2 = (float)fmax((double)sAn[row] + (double)bn - 2.0 * (double)acc[r], 0.0);
                else
                    r2 = fmaxf(sAn[row] + bn - 2.0f * acc[r], 0.0f);
                float kv = exp2f(bg * r2) * mb[r];
#pragma unroll
                for (int j = 0; j < RB; ++j) accu[r][j] = fmaf(kv, bw[j], accu[r][j]);
            }
        }
    }
    // reduce over the 32 columns held by the lanes of each half, then over the two
    // waves that share the same rows
#pragma unroll
    for (int r = 0; r < 16; ++r)
#pragma unroll
        for (int j = 0; j < RB; ++j) {
            float v = accu[r][j];
#pragma unroll
            for (int o = 1; o < 32; o <<= 1) v += __shfl_xor(v, o);
            accu[r][j] = v;
        }
    __syncthreads();
    if (l32 == 0) {
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int row = rq + 8 * (r / 4) + 4 * half + (r % 4);
#pragma unroll
            for (int j = 0; j < RB; ++j) sRed[wv & 1][row * RB + j] = accu[r][j];
        }
    }
    __syncthreads();
    for (int e = tid; e < sb.nrows * p.rb; e += EV_T) {
        int row = e / p.rb, j = e % p.rb;
        float v = sRed[0][row * RB + j] + sRed[1][row * RB + j];
        int64_t orow = outmap ? outmap[sb.row0 + row] : (int64_t)sb.row0 + row;
        p.U[orow * p.ldu + p.r0 + j] = v;
    }
  };

    if (!MULTI || !p.persistent) {
        process(blockIdx.x);
        return;
    }
    // persistent: take slabs from the queue (largest first) until it is empty
    for (;;) {
        __syncthreads();            // the previous item is done with the shared buffers
        if (tid == 0) sItem = atomicAdd(p.queue, 1);
        __syncthreads();
        const int64_t item = sItem;
        if (item >= p.nslab) break;
        process(p.order ? (int64_t)p.order[item] : item);
    }
}

void evaluate(askit_handle *h, const WeightSet &ws, const EvalArgs &a, hipStream_t s)
{
    if (h->dp > 1024) fail(ASKIT_ERR_UNSUPPORTED, "dimension above 1024 is not supported");
    EvalParams p;
    p.Y = a.Y;
    p.slabs = a.slabs;
    p.ptr = a.ptr;
    p.node = a.node;
    p.mask = a.mask;
    p.outmap = a.outmap;
    p.U = a.U;
    p.ldu = a.ldu;
    p.nslab = a.nslab;
    p.nodes = h->d_nodes;
    p.Xt = h->Xt;
    p.gt = h->gt;
    p.Wt = ws.Wt;
    p.Xs = h->Xs;
    p.gs = h->gs;
    p.Wsk = ws.Wsk;
    p.skk = h->skk;
    p.smax = h->smax;
    p.dp = h->dp;
    p.R = ws.R;
    p.inst = nullptr;
    p.order = nullptr;
    p.queue = nullptr;
    p.persistent = 0;
    if (a.nslab == 0) return;
    const bool bf = h->prm.precision == ASKIT_PREC_BF16X3;
    for (int r0 = 0; r0 < ws.R; r0 += EV_RB) {
        p.r0 = r0;
        p.rb = std::min(EV_RB, ws.R - r0);
        dim3 g((unsigned)a.nslab), b(EV_T);
        if (p.rb == 1) {
            if (bf) hipLaunchKernelGGL((k_eval<1, true, false>), g, b, 0, s, p);
            else hipLaunchKernelGGL((k_eval<1, false, false>), g, b, 0, s, p);
        } else if (p.rb <= 4) {
            if (bf) hipLaunchKernelGGL((k_eval<4, true, false>), g, b, 0, s, p);
            else hipLaunchKernelGGL((k_eval<4, false, false>), g, b, 0, s, p);
        } else {
            if (bf) hipLaunchKernelGGL((k_eval<EV_RB, true, false>), g, b, 0, s, p);
            else hipLaunchKernelGGL((k_eval<EV_RB, false, false>), g, b, 0, s, p);
        }
        HIPC(hipGetLastError());
    }
}

__global__ void k_zero_i32(int32_t *__restrict__ p, int n)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0;
}

void evaluate_batch(const BatchEvalArgs &b, hipStream_t s)
{
    if (b.nslab == 0) return;
    EvalParams p{};
    p.slabs = b.slabs;
    p.ptr = b.ptr;
    p.node = b.node;
    p.mask = b.mask;
    p.nslab = b.nslab;
    p.U = b.U;
    p.ldu = b.ldu;
    p.Wt = b.Wt;
    p.Wsk = b.Wsk;
    p.R = b.R;
    p.inst = b.inst;
    p.order = b.order;
    p.persistent = b.persistent > 0;
    const int passes = (b.R + EV_RB - 1) / EV_RB;
    if (p.persistent) {
        // counters are cleared by a kernel, not a memset node, so that the
        // sequence can be captured in a graph and replayed
        hipLaunchKernelGGL(k_zero_i32, dim3(1), dim3(64), 0, s, b.queue, passes);
        HIPC(hipGetLastError());
    }
    for (int r0 = 0, pass = 0; r0 < b.R; r0 += EV_RB, ++pass) {
        p.r0 = r0;
        p.rb = std::min(EV_RB, b.R - r0);
        p.queue = b.queue ? b.queue + pass : nullptr;
        dim3 g((unsigned)(p.persistent ? std::min<int64_t>(b.persistent, b.nslab) : b.nslab)), blk(EV_T);
        if (p.rb == 1) {
            if (b.bf) hipLaunchKernelGGL((k_eval<1, true, true>), g, blk, 0, s, p);
            else hipLaunchKernelGGL((k_eval<1, false, true>), g, blk, 0, s, p);
        } else if (p.rb <= 4) {
            if (b.bf) hipLaunchKernelGGL((k_eval<4, true, true>), g, blk, 0, s, p);
            else hipLaunchKernelGGL((k_eval<4, false, true>), g, blk, 0, s, p);
        } else {
            if (b.bf) hipLaunchKernelGGL((k_eval<EV_RB, true, true>), g, blk, 0, s, p);
            else hipLaunchKernelGGL((k_eval<EV_RB, false, true>), g, blk, 0, s, p);
        }
        HIPC(hipGetLastError());
    }
}

}  // namespace askit
