// Downward pass (Alg. 4) as sums over (target, source node) pairs.
//
// Work item: a chunk of up to 64 targets that all use one source node
// (near: a leaf's points and weights; far: a pruned node's skeleton points
// and skeleton weights).  Sources are taken in tiles of 64:
//   r^2 = |x - c|^2 + |y - c|^2 - 2 (x - c).(y - c),  c = the chunk's first
//   target: the rounding error of r^2 is a few ulps of |x - c|^2 + |y - c|^2,
//   small where the kernel is not (a skeleton can span distant clusters, so
//   a point of the source node would not do),
// with the 64 x 64 products on MFMA, sources as the rows and targets as the
// columns (v_mfma_f32_32x32x2_f32, or the bf16 hi/lo split on
// v_mfma_f32_32x32x16_bf16 with an FP64 final combine), each wave one
// 32 x 32 quadrant, operands staged through LDS in 64-dimension chunks; then
// K = exp2(g_j r^2), g_j = -log2(e) / (2 h_j^2), and the contraction with
// the tile's weights: for up to 4 right-hand sides on the vector units, for
// more as a second MFMA with the weights as the A operand (the kernel tile,
// which the first MFMA left with targets along the lanes and sources along
// the registers, is exactly the B operand layout), 32 or 64 columns per
// pass.  Each pair's sum goes to its own slot; a second kernel adds a
// target's slots in order, so the result is deterministic (no atomics).
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
constexpr int EV_LH = EV_KC + 8;       // padded LDS row of the bf16 operands (elements)

struct ChunkParams {
    const Chunk *chunks;
    int64_t nchunk;
    const int32_t *tpos, *tslot;
    // single problem (MULTI = false)
    const Node *nodes;
    const float *Y, *Xt, *gt, *Xs, *gs;
    const int32_t *skk;
    int smax, dp;
    // batch (MULTI = true)
    const EvalInst *inst;
    int32_t *queue;
    int persistent;
    // weights and output
    const float *Wt, *Wsk;     // single: the problem's; batch: shared buffers (instance offsets)
    float *part;
    int R, r0, rb;             // columns [r0, r0 + rb) in this pass
};

// CM: columns per pass and contraction: 1 or 4 on the vector units, 32 or 64 on MFMA.
template <int CM, bool BF, bool MULTI>
__global__ __launch_bounds__(EV_T) void k_eval_chunks(ChunkParams p)
{
    constexpr bool MC = CM >= 32;
    constexpr int NACC = MC ? CM / 32 : 1;
    __shared__ __attribute__((aligned(16))) float sT[BF ? 16 : 64 * EV_LD];
    __shared__ __attribute__((aligned(16))) float sS[BF ? 16 : 64 * EV_LD];
    __shared__ __attribute__((aligned(16))) uint16_t sTh[BF ? 64 * EV_LH : 8], sTl[BF ? 64 * EV_LH : 8];
    __shared__ __attribute__((aligned(16))) uint16_t sSh[BF ? 64 * EV_LH : 8], sSl[BF ? 64 * EV_LH : 8];
    __shared__ float sC[1024];                 // centre (dp <= 1024)
    __shared__ float sTn[64], sSn[64], sSg[64];
    __shared__ float sW[64 * CM];               // weights of the source tile
    __shared__ float sRed[MC ? 64 * CM : 2 * 64 * CM];
    __shared__ int sRow[64], sSlot[64];
    __shared__ int64_t sItem;

    const int tid = threadIdx.x, lane = tid % 64, wv = tid / 64;
    const int half = lane >> 5, l32 = lane & 31;
    const int sq = 32 * (wv >> 1), tq = 32 * (wv & 1);   // source rows / target columns of this wave

  auto process = [&](const int64_t ci) {
    const Chunk ch = p.chunks[ci];
    const int kind = ch.kind & 1;
    const Node *nodes = p.nodes;
    const float *Y = p.Y, *Xt = p.Xt, *gt = p.gt, *Xs = p.Xs, *gs = p.gs, *Wt = p.Wt, *Wsk = p.Wsk;
    const int32_t *skk = p.skk;
    int smax = p.smax, dp = p.dp;
    if constexpr (MULTI) {
        const EvalInst &I = p.inst[ch.kind >> 1];
        nodes = I.nodes;
        Y = I.Y;
        Xt = I.Xt;
        gt = I.gt;
        Xs = I.Xs;
        gs = I.gs;
        skk = I.skk;
        smax = I.smax;
        dp = I.dp;
        Wt = p.Wt + I.wt_off * p.R;
        Wsk = p.Wsk + I.wsk_off * p.R;
    }
    const int a = ch.node, nt = ch.count;
    const float *src, *g, *w;
    int ns;
    if (kind == 0) {
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
    const int nchunk = (dp + EV_KC - 1) / EV_KC;
    if (tid < 64) {
        sRow[tid] = tid < nt ? p.tpos[ch.first + tid] : -1;
        sSlot[tid] = tid < nt ? p.tslot[ch.first + tid] : -1;
    }
    __syncthreads();
    {
        // centre: the chunk's first target (the targets of a chunk are close to
        // one another; sources far from them have negligible kernel values)
        const float *c0 = Y + (int64_t)sRow[0] * dp;
        for (int k = tid; k < dp; k += EV_T) sC[k] = c0[k];
    }
    __syncthreads();

    // one 64 x EV_KC chunk of (centred) rows into LDS; rows given by `row(r)`
    // (negative: padding); per-row partial squared norms into nrm
    // (get(u, rp, kk) gives the row's coordinates kk..kk+3: a load, or a
    // register filled ahead of time)
    auto put_chunk = [&](float *dst, uint16_t *dh, uint16_t *dl, auto row_ptr, int k0, float *nrm, bool accum,
                         auto get) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            int idx = tid + EV_T * u;
            int row = idx >> 4, qd = (idx & 15) * 4;
            float4 v = {0.f, 0.f, 0.f, 0.f};
            int kk = k0 + qd;
            const float *rp = row_ptr(row);
            if (rp && kk < dp) {
                float4 x = get(u, rp, kk);
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
                float s2 = v.x * v.x + v.y * v.y + v.z * v.z + v.w * v.w;
#pragma unroll
                for (int o = 1; o < 16; o <<= 1) s2 += __shfl_xor(s2, o);
                if ((idx & 15) == 0) nrm[row] = accum ? nrm[row] + s2 : s2;
            }
        }
    };
    auto load_chunk = [&](float *dst, uint16_t *dh, uint16_t *dl, auto row_ptr, int k0, float *nrm, bool accum) {
        put_chunk(dst, dh, dl, row_ptr, k0, nrm, accum,
                  [](int, const float *rp, int kk) { return *reinterpret_cast<const float4 *>(rp + kk); });
    };
    auto trow = [&](int r) -> const float * { return sRow[r] >= 0 ? Y + (int64_t)sRow[r] * dp : nullptr; };

    // target norms (all dimension chunks); the target chunk stays resident when dp <= EV_KC
    for (int c = 0; c < nchunk; ++c) {
        load_chunk(sT, sTh, sTl, trow, c * EV_KC, sTn, c > 0);
        __syncthreads();
    }

    f32x16 uacc[NACC];
    float vacc[MC ? 1 : CM];
#pragma unroll
    for (int q = 0; q < NACC; ++q) uacc[q] = f32x16{};
#pragma unroll
    for (int j = 0; j < (MC ? 1 : CM); ++j) vacc[j] = 0.0f;

    // one dimension chunk (dp <= 64): the next source block's rows, factors
    // and weights are loaded into registers while the current one is on the
    // MFMA (indices kept valid for rows past the node's end; those values
    // are not used)
    const bool pf = nchunk == 1;
    constexpr int NWP = 64 * CM >= EV_T ? 64 * CM / EV_T : 1;
    float4 px[4];
    float pg = 0.0f, pw[NWP];
    auto fetch = [&](int s1) {
        const int n1 = min(64, ns - s1);
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int idx = tid + EV_T * u, row = idx >> 4, qd = (idx & 15) * 4;
            px[u] = *reinterpret_cast<const float4 *>(src + (int64_t)(s1 + (row < n1 ? row : 0)) * dp +
                                                       (qd < dp ? qd : 0));
        }
        pg = g[s1 + (tid < n1 ? tid : 0)];
#pragma unroll
        for (int u = 0; u < NWP; ++u) {
            const int e = tid + EV_T * u, r = e / CM, j = e % CM;
            const bool in = e < 64 * CM && r < n1 && j < p.rb;
            pw[u] = w[in ? (int64_t)(s1 + r) * p.R + p.r0 + j : (int64_t)s1 * p.R + p.r0];
        }
    };
    if (pf) fetch(0);
    for (int s0 = 0; s0 < ns; s0 += 64) {
        const int nsrc = min(64, ns - s0);
        auto srow = [&](int r) -> const float * { return r < nsrc ? src + (int64_t)(s0 + r) * dp : nullptr; };
        f32x16 acc = {};
        for (int c = 0; c < nchunk; ++c) {
            __syncthreads();
            if (pf) {
                put_chunk(sS, sSh, sSl, srow, 0, sSn, false, [&](int u, const float *, int) { return px[u]; });
                if (tid < 64) sSg[tid] = tid < nsrc ? pg : 0.0f;
#pragma unroll
                for (int u = 0; u < NWP; ++u) {
                    const int e = tid + EV_T * u, r = e / CM, j = e % CM;
                    if (e < 64 * CM) sW[e] = (r < nsrc && j < p.rb) ? pw[u] : 0.0f;
                }
                __syncthreads();
                if (s0 + 64 < ns) fetch(s0 + 64);
            } else {
            if (nchunk > 1) load_chunk(sT, sTh, sTl, trow, c * EV_KC, nullptr, false);
            load_chunk(sS, sSh, sSl, srow, c * EV_KC, sSn, c > 0);
            if (c == 0) {
                if (tid < 64) sSg[tid] = tid < nsrc ? g[s0 + tid] : 0.0f;
                if constexpr (64 * CM >= EV_T) {
                    // unconditional loads (indices clamped to the tile's first
                    // entry), all in flight, then masked
                    constexpr int NW = 64 * CM / EV_T;
                    float wv_[NW];
#pragma unroll
                    for (int u = 0; u < NW; ++u) {
                        const int e = tid + EV_T * u, r = e / CM, j = e % CM;
                        const bool in = r < nsrc && j < p.rb;
                        wv_[u] = w[in ? (int64_t)(s0 + r) * p.R + p.r0 + j : (int64_t)s0 * p.R + p.r0];
                    }
#pragma unroll
                    for (int u = 0; u < NW; ++u) asm volatile("" : "+v"(wv_[u]));
#pragma unroll
                    for (int u = 0; u < NW; ++u) {
                        const int e = tid + EV_T * u, r = e / CM, j = e % CM;
                        sW[e] = (r < nsrc && j < p.rb) ? wv_[u] : 0.0f;
                    }
                } else {
                    for (int e = tid; e < 64 * CM; e += EV_T) {
                        const int r = e / CM, j = e % CM;
                        sW[e] = (r < nsrc && j < p.rb) ? w[(int64_t)(s0 + r) * p.R + p.r0 + j] : 0.0f;
                    }
                }
            }
            __syncthreads();
            }
            const int kc = min(EV_KC, dp - c * EV_KC);
            if constexpr (BF) {
                const uint16_t *ph = sSh + (sq + l32) * EV_LH + 8 * half;
                const uint16_t *pl = sSl + (sq + l32) * EV_LH + 8 * half;
                const uint16_t *qh = sTh + (tq + l32) * EV_LH + 8 * half;
                const uint16_t *ql = sTl + (tq + l32) * EV_LH + 8 * half;
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
                const float *pa = sS + (sq + l32) * EV_LD + 4 * half;
                const float *pb = sT + (tq + l32) * EV_LD + 4 * half;
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
        // kernel values: lane = target tq + l32, register r = source sq + 8(r/4) + 4 half + r%4
        const float tn = sTn[tq + l32];
        float kv[16];
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int sr = sq + 8 * (r / 4) + 4 * half + (r % 4);
            float r2;
            if constexpr (BF)
                r2 = (float)fmax((double)sSn[sr] + (double)tn - 2.0 * (double)acc[r], 0.0);
            else
                r2 = fmaxf(sSn[sr] + tn - 2.0f * acc[r], 0.0f);
            // the hardware 2^x (v_exp_f32): the exponent is <= 0 and values
            // below 2^-126 (flushed) are far below any sum's rounding
            kv[r] = __builtin_amdgcn_exp2f(sSg[sr] * r2);
        }
        if constexpr (MC) {
            // U^T (columns x targets) += W^T (columns x sources) K (sources x targets), two sources per step
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int sr = sq + 8 * (r / 4) + 4 * half + (r % 4);
#pragma unroll
                for (int q = 0; q < NACC; ++q)
                    uacc[q] = __builtin_amdgcn_mfma_f32_32x32x2f32(sW[sr * CM + 32 * q + l32], kv[r], uacc[q], 0,
                                                                   0, 0);
            }
        } else {
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int sr = sq + 8 * (r / 4) + 4 * half + (r % 4);
#pragma unroll
                for (int j = 0; j < CM; ++j) vacc[j] = fmaf(kv[r], sW[sr * CM + j], vacc[j]);
            }
        }
    }

    // combine the two waves that share the target columns, then write each
    // target's partial sum into its slot
    __syncthreads();
    if constexpr (MC) {
        if (sq == 0) {
#pragma unroll
            for (int q = 0; q < NACC; ++q)
#pragma unroll
                for (int r = 0; r < 16; ++r) {
                    const int col = 32 * q + 8 * (r / 4) + 4 * half + (r % 4);
                    sRed[col * 64 + tq + l32] = uacc[q][r];
                }
        }
        __syncthreads();
        if (sq == 32) {
            const int t = tq + l32;
            const int slot = sSlot[t];
#pragma unroll
            for (int q = 0; q < NACC; ++q)
#pragma unroll
                for (int r = 0; r < 16; ++r) {
                    const int col = 32 * q + 8 * (r / 4) + 4 * half + (r % 4);
                    if (t < nt && col < p.rb)
                        p.part[(int64_t)slot * p.R + p.r0 + col] = sRed[col * 64 + t] + uacc[q][r];
                }
        }
    } else {
#pragma unroll
        for (int j = 0; j < CM; ++j) vacc[j] += __shfl_xor(vacc[j], 32);   // the two source halves
        if (half == 0) {
#pragma unroll
            for (int j = 0; j < CM; ++j) sRed[((sq >> 5) * 64 + tq + l32) * CM + j] = vacc[j];
        }
        __syncthreads();
        for (int e = tid; e < 64 * CM; e += EV_T) {
            const int t = e / CM, j = e % CM;
            if (t < nt && j < p.rb)
                p.part[(int64_t)sSlot[t] * p.R + p.r0 + j] = sRed[t * CM + j] + sRed[(64 + t) * CM + j];
        }
    }
  };

    if (!MULTI || !p.persistent) {
        process(blockIdx.x);
        return;
    }
    // persistent: take chunks from the queue until it is empty
    for (;;) {
        __syncthreads();            // the previous item is done with the shared buffers
        if (tid == 0) sItem = atomicAdd(p.queue, 1);
        __syncthreads();
        const int64_t item = sItem;
        if (item >= p.nchunk) break;
        process(item);
    }
}

// u[i, r] = sum of target i's slots, in slot order.  Its near slots come
// first, so the running sum after them is the near-field part of u (the
// direct sums over the near leaves alone), written to Unear when given.
// Columns [r0, r0 + rb) of part (row stride R) into U's columns [0, rb).
__global__ void k_sum_slots(const int32_t *__restrict__ sbase, int64_t ntarget, const float *__restrict__ part,
                            int R, const int32_t *__restrict__ outmap, float *__restrict__ U, int64_t ldu,
                            const int32_t *__restrict__ snear, float *__restrict__ Unear, int64_t ldun, int r0,
                            int rb)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t i = t / rb;
    if (i >= ntarget) return;
    const int j = (int)(t - i * rb), r = r0 + j;
    const int64_t o = outmap ? outmap[i] : i;
    float u = 0.0f;
    int sl = sbase[i];
    if (Unear) {
        for (; sl < snear[i]; ++sl) u += part[(int64_t)sl * R + r];
        Unear[o * ldun + j] = u;
    }
    for (; sl < sbase[i + 1]; ++sl) u += part[(int64_t)sl * R + r];
    U[o * ldu + j] = u;
}

__global__ void k_zero_i32(int32_t *__restrict__ p, int n)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0;
}

template <bool MULTI>
static void launch_passes(ChunkParams p, bool bf, int R, int64_t grid, int32_t *queue, hipStream_t s, int c0 = 0,
                          int plan = 0)
{
    // passes over columns [c0, R): plan 0 (wide) of 64, 32, 4 or 1 columns,
    // plan 1 (narrow) of 32 or 1.  A column sees the same arithmetic in
    // either (MFMA for a remainder above 4 columns, the vector units below;
    // the 32 and 64 forms, and the 1 and 4 forms, treat each column alike)
    for (int r0 = c0; r0 < R;) {
        const int left = R - r0;
        const int cm = plan == 1 ? (left > 4 ? 32 : 1) : (left > 32 ? 64 : left > 4 ? 32 : left > 1 ? 4 : 1);
        p.r0 = r0;
        p.rb = std::min(cm, left);
        p.queue = queue;
        if (MULTI && p.persistent) {
            hipLaunchKernelGGL(k_zero_i32, dim3(1), dim3(64), 0, s, queue, 1);
            HIPC(hipGetLastError());
        }
        dim3 g((unsigned)grid), b(EV_T);
#define EV_LAUNCH(CMV)                                                                             \
    if (bf) hipLaunchKernelGGL((k_eval_chunks<CMV, true, MULTI>), g, b, 0, s, p);                 \
    else hipLaunchKernelGGL((k_eval_chunks<CMV, false, MULTI>), g, b, 0, s, p);
        if (cm == 1) { EV_LAUNCH(1) }
        else if (cm == 4) { EV_LAUNCH(4) }
        else if (cm == 32) { EV_LAUNCH(32) }
        else { EV_LAUNCH(64) }
#undef EV_LAUNCH
        HIPC(hipGetLastError());
        r0 += p.rb;
    }
}

void evaluate(const askit_handle *h, const WeightSet &ws, const float *Y, const PairLists &L,
              const int32_t *outmap, float *U, int64_t ldu, float *part, hipStream_t s, float *Unear,
              int64_t ldun)
{
    if (h->dp > 1024) fail(ASKIT_ERR_UNSUPPORTED, "dimension above 1024 is not supported");
    if (L.ntarget == 0) return;
    if (L.nchunk > 0) {
        ChunkParams p{};
        p.chunks = L.chunks;
        p.nchunk = L.nchunk;
        p.tpos = L.tpos;
        p.tslot = L.tslot;
        p.nodes = h->d_nodes;
        p.Y = Y;
        p.Xt = h->Xt;
        p.gt = h->gt;
        p.Xs = h->Xs;
        p.gs = h->gs;
        p.skk = h->skk;
        p.smax = h->smax;
        p.dp = h->dp;
        p.Wt = ws.Wt;
        p.Wsk = ws.Wsk;
        p.part = part;
        p.R = ws.R;
        launch_passes<false>(p, h->prm.precision == ASKIT_PREC_BF16X3, ws.R, L.nchunk, nullptr, s);
    }
    const int64_t tot = L.ntarget * ws.R;
    hipLaunchKernelGGL(k_sum_slots, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, L.sbase, L.ntarget, part,
                       ws.R, outmap, U, ldu, L.snear, Unear, ldun, 0, ws.R);
    HIPC(hipGetLastError());
}

void evaluate_chunk_range(const askit_handle *h, const WeightSet &ws, const PairLists &L, int64_t ch0, int64_t ch1,
                          int c0, int c1, float *part, hipStream_t s)
{
    if (h->dp > 1024) fail(ASKIT_ERR_UNSUPPORTED, "dimension above 1024 is not supported");
    ch1 = std::min(ch1, L.nchunk);
    if (ch1 <= ch0 || c1 <= c0) return;
    ChunkParams p{};
    p.chunks = L.chunks + ch0;
    p.nchunk = ch1 - ch0;
    p.tpos = L.tpos;
    p.tslot = L.tslot;
    p.nodes = h->d_nodes;
    p.Y = h->Xt;
    p.Xt = h->Xt;
    p.gt = h->gt;
    p.Xs = h->Xs;
    p.gs = h->gs;
    p.skk = h->skk;
    p.smax = h->smax;
    p.dp = h->dp;
    p.Wt = ws.Wt;
    p.Wsk = ws.Wsk;
    p.part = part;
    p.R = ws.R;
    launch_passes<false>(p, h->prm.precision == ASKIT_PREC_BF16X3, c1, ch1 - ch0, nullptr, s, c0);
}

void sum_slot_cols(const askit_handle *h, const PairLists &L, const float *part, int R, int c0, int rb,
                   const int32_t *outmap, float *U, int64_t ldu, hipStream_t s)
{
    const int64_t tot = L.ntarget * rb;
    hipLaunchKernelGGL(k_sum_slots, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, L.sbase, L.ntarget, part,
                       R, outmap, U, ldu, (const int32_t *)nullptr, (float *)nullptr, (int64_t)0, c0, rb);
    HIPC(hipGetLastError());
}

void evaluate_batch(const BatchEvalArgs &b, hipStream_t s)
{
    if (b.rows == 0) return;
    if (b.nchunk > 0) {
        ChunkParams p{};
        p.chunks = b.chunks;
        p.nchunk = b.nchunk;
        p.tpos = b.tpos;
        p.tslot = b.tslot;
        p.inst = b.inst;
        p.persistent = b.persistent > 0;
        p.Wt = b.Wt;
        p.Wsk = b.Wsk;
        p.part = b.part;
        p.R = b.R;
        const int64_t grid = p.persistent ? std::min<int64_t>(b.persistent, b.nchunk) : b.nchunk;
        launch_passes<true>(p, b.bf, b.R, grid, b.queue, s, 0, b.plan);
    }
    const int64_t tot = b.rows * b.R;
    hipLaunchKernelGGL(k_sum_slots, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, b.sbase, b.rows, b.part,
                       b.R, b.outrow, b.U, b.ldu, (const int32_t *)nullptr, (float *)nullptr, (int64_t)0, 0, b.R);
    HIPC(hipGetLastError());
}

}  // namespace askit
