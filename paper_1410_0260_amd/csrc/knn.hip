// Exact kappa-nearest neighbours on gfx950.
//
// The neighbour lists are defined exactly: the kappa smallest (D, j), D the
// canonical FP64 squared distance, j the point id (self excluded for the
// point set).  They are found in three steps:
//   1. k_knn_cand: approximate squared distances |q|^2 + |x|^2 - 2 q.x with
//      the dot product as bf16 hi/lo split products (hi*hi + hi*lo + lo*hi)
//      on MFMA 32x32x16 with FP32 accumulation; each query row keeps its 64
//      smallest approximate distances in a wave-wide sorted list.
//   2. k_knn_refine: exact FP64 distances of the 64 candidates, sorted by
//      (D, j); the row is certified when the kappa-th exact distance is
//      below (64th approximate distance - E), E a bound on the
//      approximation error, so no point outside the candidates can enter.
//   3. k_knn_exact: full FP64 scan for the rows that are not certified.
#include "askit_impl.h"

namespace askit {

typedef __attribute__((ext_vector_type(8))) __bf16 bf16x8;
typedef __attribute__((ext_vector_type(16))) float f32x16;

constexpr int KB_M = 128;     // query rows per block (32 per wave)
constexpr int KB_N = 64;      // reference points per tile
constexpr int KCB = 32;       // survivor buffer per row

struct ListEntry {
    float d;
    int i;
    float thr;
};

__device__ __forceinline__ bool lt_fi(float d1, int i1, float d2, int i2)
{
    return d1 < d2 || (d1 == d2 && i1 < i2);
}

// Sort (d, i) ascending across the 64 lanes of a wave.
__device__ __forceinline__ void wave_sort64(float &d, int &i, int lane)
{
#pragma unroll
    for (int k = 2; k <= 64; k <<= 1) {
#pragma unroll
        for (int j = k >> 1; j > 0; j >>= 1) {
            float od = __shfl_xor(d, j);
            int oi = __shfl_xor(i, j);
            bool up = (lane & k) == 0;
            bool lower = (lane & j) == 0;
            bool take = (lower == up) ? lt_fi(od, oi, d, i) : lt_fi(d, i, od, oi);
            if (take) { d = od; i = oi; }
        }
    }
}

// Merge a row's survivor buffer (cnt entries in LDS) into its sorted list
// (one entry per lane); returns the lane's new entry and the 64th distance.
__device__ __noinline__ ListEntry merge_list(float ld, int li, const float *bd, const int *bi,
                                             int cnt, int lane)
{
    float d = lane < cnt ? bd[lane] : INFINITY;
    int i = lane < cnt ? bi[lane] : 0x7fffffff;
    wave_sort64(d, i, lane);
    float rd = __shfl(d, 63 - lane);
    int ri = __shfl(i, 63 - lane);
    if (lt_fi(rd, ri, ld, li)) { ld = rd; li = ri; }
#pragma unroll
    for (int j = 32; j > 0; j >>= 1) {
        float od = __shfl_xor(ld, j);
        int oi = __shfl_xor(li, j);
        bool lower = (lane & j) == 0;
        bool take = lower ? lt_fi(od, oi, ld, li) : lt_fi(ld, li, od, oi);
        if (take) { ld = od; li = oi; }
    }
    ListEntry e;
    e.d = ld;
    e.i = li;
    e.thr = __shfl(ld, 63);
    return e;
}

__device__ __forceinline__ bf16x8 ld_bf8(const uint16_t *p)
{
    uint4 v = *reinterpret_cast<const uint4 *>(p);
    return __builtin_bit_cast(bf16x8, v);
}

// KS = dp / 16 MFMA k-steps; the query fragments stay in registers.
template <int KS>
__global__ __launch_bounds__(256) void k_knn_cand(const uint16_t *__restrict__ Qh,
                                                  const uint16_t *__restrict__ Ql,
                                                  const float *__restrict__ Qn, int64_t M,
                                                  const uint16_t *__restrict__ Xh,
                                                  const uint16_t *__restrict__ Xl,
                                                  const float *__restrict__ Xn, int64_t N,
                                                  int excl, int32_t *__restrict__ cand,
                                                  float *__restrict__ thr_out)
{
    constexpr int DP = KS * 16;
    constexpr int LDB = DP + 8;                      // padded LDS row (bf16 elements)
    __shared__ __attribute__((aligned(16))) uint16_t sBh[KB_N * LDB];
    __shared__ __attribute__((aligned(16))) uint16_t sBl[KB_N * LDB];
    __shared__ float sBn[KB_N];
    __shared__ float sbd[KB_M * KCB];
    __shared__ int sbi[KB_M * KCB];

    const int tid = threadIdx.x, lane = tid % WAVE, wv = tid / WAVE;
    const int half = lane >> 5, l32 = lane & 31;
    const int64_t q0 = (int64_t)blockIdx.x * KB_M + wv * 32;

    // query fragments and norms
    bf16x8 ah[KS], al[KS];
    {
        int64_t row = q0 + l32;
        bool ok = row < M;
#pragma unroll
        for (int s = 0; s < KS; ++s) {
            if (ok) {
                ah[s] = ld_bf8(Qh + row * DP + 16 * s + 8 * half);
                al[s] = ld_bf8(Ql + row * DP + 16 * s + 8 * half);
            } else {
                ah[s] = bf16x8{};
                al[s] = bf16x8{};
            }
        }
    }
    float qn[16], thrv[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        int64_t row = q0 + 8 * (r / 4) + 4 * half + (r % 4);
        qn[r] = row < M ? Qn[row] : 0.0f;
        thrv[r] = INFINITY;
    }
    float list_d[32];
    int list_i[32], cnt[32];
#pragma unroll
    for (int R = 0; R < 32; ++R) {
        list_d[R] = INFINITY;
        list_i[R] = 0x7fffffff;
        cnt[R] = 0;
    }
    float *bd = sbd + wv * 32 * KCB;
    int *bi = sbi + wv * 32 * KCB;

    const int64_t ntiles = (N + KB_N - 1) / KB_N;
    constexpr int CHUNKS = KB_N * DP / 8;            // 16-byte chunks per operand tile
    constexpr int PER = (CHUNKS + 255) / 256;
    uint4 rh[PER], rl[PER];
    float rn = 0.0f;
    auto load_tile = [&](int64_t t) {
#pragma unroll
        for (int u = 0; u < PER; ++u) {
            int c = tid + 256 * u;
            int row = c / (DP / 8), off = (c % (DP / 8)) * 8;
            int64_t g = t * KB_N + row;
            if (c < CHUNKS && g < N) {
                rh[u] = *reinterpret_cast<const uint4 *>(Xh + g * DP + off);
                rl[u] = *reinterpret_cast<const uint4 *>(Xl + g * DP + off);
            } else {
                rh[u] = uint4{0, 0, 0, 0};
                rl[u] = uint4{0, 0, 0, 0};
            }
        }
        int64_t g = t * KB_N + tid;
        rn = (tid < KB_N && g < N) ? Xn[g] : 0.0f;
    };
    auto store_tile = [&]() {
#pragma unroll
        for (int u = 0; u < PER; ++u) {
            int c = tid + 256 * u;
            if (c < CHUNKS) {
                int row = c / (DP / 8), off = (c % (DP / 8)) * 8;
                *reinterpret_cast<uint4 *>(sBh + row * LDB + off) = rh[u];
                *reinterpret_cast<uint4 *>(sBl + row * LDB + off) = rl[u];
            }
        }
        if (tid < KB_N) sBn[tid] = rn;
    };

    load_tile(0);
    store_tile();
    __syncthreads();
    for (int64_t t = 0; t < ntiles; ++t) {
        if (t + 1 < ntiles) load_tile(t + 1);
        f32x16 acc0 = {}, acc1 = {};
#pragma unroll
        for (int s = 0; s < KS; ++s) {
            bf16x8 bh0 = ld_bf8(sBh + l32 * LDB + 16 * s + 8 * half);
            bf16x8 bl0 = ld_bf8(sBl + l32 * LDB + 16 * s + 8 * half);
            bf16x8 bh1 = ld_bf8(sBh + (32 + l32) * LDB + 16 * s + 8 * half);
            bf16x8 bl1 = ld_bf8(sBl + (32 + l32) * LDB + 16 * s + 8 * half);
            acc0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[s], bh0, acc0, 0, 0, 0);
            acc1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[s], bh1, acc1, 0, 0, 0);
            acc0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[s], bl0, acc0, 0, 0, 0);
            acc1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[s], bl1, acc1, 0, 0, 0);
            acc0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al[s], bh0, acc0, 0, 0, 0);
            acc1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al[s], bh1, acc1, 0, 0, 0);
        }
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            const int64_t colg = t * KB_N + 32 * c + l32;
            const float ny = sBn[32 * c + l32];
            const bool colok = colg < N;
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int64_t qrow = q0 + 8 * (r / 4) + 4 * half + (r % 4);
                float a = c == 0 ? acc0[r] : acc1[r];
                float dv = qn[r] + ny - 2.0f * a;
                if (!colok || (excl && colg == qrow)) dv = INFINITY;
                bool pred = dv < thrv[r];
                uint64_t mask = __ballot(pred);
                if (mask == 0) continue;
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    const int R = 8 * (r / 4) + (r % 4) + 4 * h;
                    uint32_t mh = (uint32_t)(mask >> (32 * h));
                    if (mh == 0) continue;
                    int nnew = __popc(mh);
                    if (cnt[R] + nnew > KCB) {
                        ListEntry e = merge_list(list_d[R], list_i[R], bd + R * KCB, bi + R * KCB,
                                                 cnt[R], lane);
                        list_d[R] = e.d;
                        list_i[R] = e.i;
                        cnt[R] = 0;
                        if (half == h) thrv[r] = e.thr;
                        pred = dv < thrv[r];
                        mh = (uint32_t)(__ballot(pred) >> (32 * h));
                        nnew = __popc(mh);
                    }
                    if (half == h && pred) {
                        int pos = cnt[R] + __popc(mh & ((1u << l32) - 1u));
                        bd[R * KCB + pos] = dv;
                        bi[R * KCB + pos] = (int)colg;
                    }
                    cnt[R] += nnew;
                }
            }
        }
        __syncthreads();
        if (t + 1 < ntiles) {
            store_tile();
            __syncthreads();
        }
    }
    // final merge and output
#pragma unroll
    for (int R = 0; R < 32; ++R) {
        float th = list_d[R];
        if (cnt[R] > 0) {
            ListEntry e = merge_list(list_d[R], list_i[R], bd + R * KCB, bi + R * KCB, cnt[R], lane);
            list_d[R] = e.d;
            list_i[R] = e.i;
        }
        th = __shfl(list_d[R], 63);
        int64_t row = q0 + R;
        if (row < M) {
            cand[row * KNN_CAND + lane] = list_i[R] == 0x7fffffff ? -1 : list_i[R];
            if (lane == 0) thr_out[row] = th;
        }
    }
}

// Generic variant for dp > 128: query fragments re-read from memory per tile.
__global__ __launch_bounds__(256) void k_knn_cand_wide(const uint16_t *__restrict__ Qh,
                                                       const uint16_t *__restrict__ Ql,
                                                       const float *__restrict__ Qn, int64_t M,
                                                       const uint16_t *__restrict__ Xh,
                                                       const uint16_t *__restrict__ Xl,
                                                       const float *__restrict__ Xn, int64_t N,
                                                       int dp, int excl, int32_t *__restrict__ cand,
                                                       float *__restrict__ thr_out)
{
    constexpr int KC = 128;                          // dims per LDS chunk
    constexpr int LDB = KC + 8;
    __shared__ __attribute__((aligned(16))) uint16_t sBh[KB_N * LDB];
    __shared__ __attribute__((aligned(16))) uint16_t sBl[KB_N * LDB];
    __shared__ float sBn[KB_N];
    __shared__ float sbd[KB_M * KCB];
    __shared__ int sbi[KB_M * KCB];

    const int tid = threadIdx.x, lane = tid % WAVE, wv = tid / WAVE;
    const int half = lane >> 5, l32 = lane & 31;
    const int64_t q0 = (int64_t)blockIdx.x * KB_M + wv * 32;
    const int64_t arow = q0 + l32;
    const bool aok = arow < M;

    float qn[16], thrv[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        int64_t row = q0 + 8 * (r / 4) + 4 * half + (r % 4);
        qn[r] = row < M ? Qn[row] : 0.0f;
        thrv[r] = INFINITY;
    }
    float list_d[32];
    int list_i[32], cnt[32];
#pragma unroll
    for (int R = 0; R < 32; ++R) {
        list_d[R] = INFINITY;
        list_i[R] = 0x7fffffff;
        cnt[R] = 0;
    }
    float *bd = sbd + wv * 32 * KCB;
    int *bi = sbi + wv * 32 * KCB;
    const int64_t ntiles = (N + KB_N - 1) / KB_N;

    for (int64_t t = 0; t < ntiles; ++t) {
        f32x16 acc0 = {}, acc1 = {};
        for (int k0 = 0; k0 < dp; k0 += KC) {
            const int kc = min(KC, dp - k0);
            __syncthreads();
            for (int c = tid; c < KB_N * (KC / 8); c += 256) {
                int row = c / (KC / 8), off = (c % (KC / 8)) * 8;
                int64_t g = t * KB_N + row;
                uint4 vh = {0, 0, 0, 0}, vl = {0, 0, 0, 0};
                if (g < N && off < kc) {
                    vh = *reinterpret_cast<const uint4 *>(Xh + g * dp + k0 + off);
                    vl = *reinterpret_cast<const uint4 *>(Xl + g * dp + k0 + off);
                }
                *reinterpret_cast<uint4 *>(sBh + row * LDB + off) = vh;
                *reinterpret_cast<uint4 *>(sBl + row * LDB + off) = vl;
            }
            if (k0 == 0 && tid < KB_N) {
                int64_t g = t * KB_N + tid;
                sBn[tid] = g < N ? Xn[g] : 0.0f;
            }
            __syncthreads();
            for (int s = 0; s < kc / 16; ++s) {
                bf16x8 qa = aok ? ld_bf8(Qh + arow * dp + k0 + 16 * s + 8 * half) : bf16x8{};
                bf16x8 qb = aok ? ld_bf8(Ql + arow * dp + k0 + 16 * s + 8 * half) : bf16x8{};
                bf16x8 bh0 = ld_bf8(sBh + l32 * LDB + 16 * s + 8 * half);
                bf16x8 bl0 = ld_bf8(sBl + l32 * LDB + 16 * s + 8 * half);
                bf16x8 bh1 = ld_bf8(sBh + (32 + l32) * LDB + 16 * s + 8 * half);
                bf16x8 bl1 = ld_bf8(sBl + (32 + l32) * LDB + 16 * s + 8 * half);
                acc0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(qa, bh0, acc0, 0, 0, 0);
                acc1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(qa, bh1, acc1, 0, 0, 0);
                acc0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(qa, bl0, acc0, 0, 0, 0);
                acc1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(qa, bl1, acc1, 0, 0, 0);
                acc0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(qb, bh0, acc0, 0, 0, 0);
                acc1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(qb, bh1, acc1, 0, 0, 0);
            }
        }
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            const int64_t colg = t * KB_N + 32 * c + l32;
            const float ny = sBn[32 * c + l32];
            const bool colok = colg < N;
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int64_t qrow = q0 + 8 * (r / 4) + 4 * half + (r % 4);
                float a = c == 0 ? acc0[r] : acc1[r];
                float dv = qn[r] + ny - 2.0f * a;
                if (!colok || (excl && colg == qrow)) dv = INFINITY;
                bool pred = dv < thrv[r];
                uint64_t mask = __ballot(pred);
                if (mask == 0) continue;
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    const int R = 8 * (r / 4) + (r % 4) + 4 * h;
                    uint32_t mh = (uint32_t)(mask >> (32 * h));
                    if (mh == 0) continue;
                    int nnew = __popc(mh);
                    if (cnt[R] + nnew > KCB) {
                        ListEntry e = merge_list(list_d[R], list_i[R], bd + R * KCB, bi + R * KCB,
                                                 cnt[R], lane);
                        list_d[R] = e.d;
                        list_i[R] = e.i;
                        cnt[R] = 0;
                        if (half == h) thrv[r] = e.thr;
                        pred = dv < thrv[r];
                        mh = (uint32_t)(__ballot(pred) >> (32 * h));
                        nnew = __popc(mh);
                    }
                    if (half == h && pred) {
                        int pos = cnt[R] + __popc(mh & ((1u << l32) - 1u));
                        bd[R * KCB + pos] = dv;
                        bi[R * KCB + pos] = (int)colg;
                    }
                    cnt[R] += nnew;
                }
            }
        }
    }
#pragma unroll
    for (int R = 0; R < 32; ++R) {
        if (cnt[R] > 0) {
            ListEntry e = merge_list(list_d[R], list_i[R], bd + R * KCB, bi + R * KCB, cnt[R], lane);
            list_d[R] = e.d;
            list_i[R] = e.i;
        }
        float th = __shfl(list_d[R], 63);
        int64_t row = q0 + R;
        if (row < M) {
            cand[row * KNN_CAND + lane] = list_i[R] == 0x7fffffff ? -1 : list_i[R];
            if (lane == 0) thr_out[row] = th;
        }
    }
}

void knn_candidates(const uint16_t *Qh, const uint16_t *Ql, const float *Qn, int64_t M,
                    const uint16_t *Xh, const uint16_t *Xl, const float *Xn, int64_t N, int dp,
                    bool exclude_self, int32_t *cand, float *thr, hipStream_t s)
{
    dim3 grid((unsigned)((M + KB_M - 1) / KB_M)), block(256);
    int ex = exclude_self ? 1 : 0;
    switch (dp) {
    case 16: hipLaunchKernelGGL(k_knn_cand<1>, grid, block, 0, s, Qh, Ql, Qn, M, Xh, Xl, Xn, N, ex, cand, thr); break;
    case 32: hipLaunchKernelGGL(k_knn_cand<2>, grid, block, 0, s, Qh, Ql, Qn, M, Xh, Xl, Xn, N, ex, cand, thr); break;
    case 48: hipLaunchKernelGGL(k_knn_cand<3>, grid, block, 0, s, Qh, Ql, Qn, M, Xh, Xl, Xn, N, ex, cand, thr); break;
    case 64: hipLaunchKernelGGL(k_knn_cand<4>, grid, block, 0, s, Qh, Ql, Qn, M, Xh, Xl, Xn, N, ex, cand, thr); break;
    case 80: hipLaunchKernelGGL(k_knn_cand<5>, grid, block, 0, s, Qh, Ql, Qn, M, Xh, Xl, Xn, N, ex, cand, thr); break;
    case 96: hipLaunchKernelGGL(k_knn_cand<6>, grid, block, 0, s, Qh, Ql, Qn, M, Xh, Xl, Xn, N, ex, cand, thr); break;
    case 112: hipLaunchKernelGGL(k_knn_cand<7>, grid, block, 0, s, Qh, Ql, Qn, M, Xh, Xl, Xn, N, ex, cand, thr); break;
    case 128: hipLaunchKernelGGL(k_knn_cand<8>, grid, block, 0, s, Qh, Ql, Qn, M, Xh, Xl, Xn, N, ex, cand, thr); break;
    default:
        hipLaunchKernelGGL(k_knn_cand_wide, grid, block, 0, s, Qh, Ql, Qn, M, Xh, Xl, Xn, N, dp, ex,
                           cand, thr);
    }
    HIPC(hipGetLastError());
}

// ---------------------------------------------------------------- refine
__device__ __forceinline__ bool lt_di(double d1, int i1, double d2, int i2)
{
    return d1 < d2 || (d1 == d2 && i1 < i2);
}

// One wave per query row: exact distances of the 64 candidates, sorted by
// (D, id); kappa first kept; certificate against the approximate threshold.
__global__ __launch_bounds__(256) void k_knn_refine(const float *__restrict__ Q, int64_t M,
                                                    const float *__restrict__ X, int64_t N, int d,
                                                    int dp, int kappa,
                                                    const int32_t *__restrict__ cand,
                                                    const float *__restrict__ thr,
                                                    const float *__restrict__ Qn, double maxnorm,
                                                    double gamma, int32_t *__restrict__ idx,
                                                    double *__restrict__ dist,
                                                    int32_t *__restrict__ bad_rows,
                                                    int32_t *__restrict__ bad_count)
{
    int64_t row = (int64_t)blockIdx.x * 4 + threadIdx.x / WAVE;
    int lane = threadIdx.x % WAVE;
    if (row >= M) return;
    int j = cand[row * KNN_CAND + lane];
    double D = INFINITY;
    if (j >= 0 && j < N) D = canon_sqdist(Q + row * dp, X + (int64_t)j * dp, d);
    else j = 0x7fffffff;
#pragma unroll
    for (int k = 2; k <= 64; k <<= 1) {
#pragma unroll
        for (int s = k >> 1; s > 0; s >>= 1) {
            double od = __shfl_xor(D, s);
            int oj = __shfl_xor(j, s);
            bool up = (lane & k) == 0;
            bool lower = (lane & s) == 0;
            bool take = (lower == up) ? lt_di(od, oj, D, j) : lt_di(D, j, od, oj);
            if (take) { D = od; j = oj; }
        }
    }
    if (lane < kappa) {
        idx[row * kappa + lane] = j;
        dist[row * kappa + lane] = D;
    }
    double Dk = __shfl(D, kappa - 1);
    double th = (double)thr[row];
    double E = gamma * ((double)Qn[row] + maxnorm);
    bool ok = isinf(th) || (Dk < th - E);
    if (!ok && lane == 0) {
        int p = atomicAdd(bad_count, 1);
        bad_rows[p] = (int32_t)row;
    }
}

void knn_refine(const float *Q, int64_t M, const float *X, int64_t N, int d, int dp, int kappa,
                const int32_t *cand, const float *thr, const float *Qn, float maxnorm,
                bool exclude_self, int32_t *idx, double *dist, int32_t *bad_rows,
                int32_t *bad_count, hipStream_t s)
{
    (void)exclude_self;
    // |approx - exact| <= g (|q|^2 + |x|^2) with g = 3.1 2^-16 (hi/lo split) +
    // (4 dp + 4) 2^-24 (FP32 accumulation, norms, final combine); doubled.
    double g = 2.0 * (3.1 * ldexp(1.0, -16) + (4.0 * dp + 4.0) * ldexp(1.0, -24));
    hipLaunchKernelGGL(k_knn_refine, dim3((unsigned)((M + 3) / 4)), dim3(256), 0, s, Q, M, X, N, d,
                       dp, kappa, cand, thr, Qn, (double)maxnorm * (1.0 + 1e-5), g, idx, dist,
                       bad_rows, bad_count);
    HIPC(hipGetLastError());
}

// ---------------------------------------------------------------- exact fallback
// One block per row: every thread keeps a sorted top-kappa of a strided slice
// of the points, then the lists are merged pairwise.
constexpr int KX_T = 128;
constexpr int KX_K = 64;     // largest kappa supported by the fallback

__global__ __launch_bounds__(KX_T) void k_knn_exact(const float *__restrict__ Qb,
                                                    const float *__restrict__ X, int64_t N, int d,
                                                    int dp, int kappa, int excl,
                                                    const int32_t *__restrict__ rows,
                                                    int32_t *__restrict__ idx,
                                                    double *__restrict__ dist)
{
    extern __shared__ unsigned char smem[];
    double *ld = reinterpret_cast<double *>(smem);
    int *li = reinterpret_cast<int *>(ld + KX_T * kappa);
    int tid = threadIdx.x;
    int64_t row = rows[blockIdx.x];
    const float *q = Qb + row * dp;
    double *md = ld + tid * kappa;
    int *mi = li + tid * kappa;
    for (int t = 0; t < kappa; ++t) {
        md[t] = INFINITY;
        mi[t] = 0x7fffffff;
    }
    for (int64_t j = tid; j < N; j += KX_T) {
        if (excl && j == row) continue;
        double D = canon_sqdist(q, X + j * dp, d);
        if (!lt_di(D, (int)j, md[kappa - 1], mi[kappa - 1])) continue;
        int p = kappa - 1;
        while (p > 0 && lt_di(D, (int)j, md[p - 1], mi[p - 1])) {
            md[p] = md[p - 1];
            mi[p] = mi[p - 1];
            --p;
        }
        md[p] = D;
        mi[p] = (int)j;
    }
    __syncthreads();
    for (int st = 1; st < KX_T; st <<= 1) {
        if (tid % (2 * st) == 0) {
            double *bd2 = ld + (tid + st) * kappa;
            int *bi2 = li + (tid + st) * kappa;
            double tdd[KX_K];
            int tii[KX_K];
            int a = 0, b = 0;
            for (int t = 0; t < kappa; ++t) {
                if (lt_di(md[a], mi[a], bd2[b], bi2[b])) { tdd[t] = md[a]; tii[t] = mi[a]; ++a; }
                else { tdd[t] = bd2[b]; tii[t] = bi2[b]; ++b; }
            }
            for (int t = 0; t < kappa; ++t) {
                md[t] = tdd[t];
                mi[t] = tii[t];
            }
        }
        __syncthreads();
    }
    if (tid < kappa) {
        idx[row * kappa + tid] = li[tid];
        dist[row * kappa + tid] = ld[tid];
    }
}

void knn_exact_rows(const float *Q, const float *X, int64_t N, int d, int dp, int kappa,
                    bool exclude_self, const int32_t *rows, int nrows, int32_t *idx, double *dist,
                    hipStream_t s)
{
    if (nrows <= 0) return;
    if (kappa > KX_K) fail(ASKIT_ERR_UNSUPPORTED, "kappa above 64 is not supported");
    size_t sh = (size_t)KX_T * kappa * (sizeof(double) + sizeof(int));
    hipLaunchKernelGGL(k_knn_exact, dim3(nrows), dim3(KX_T), sh, s, Q, X, N, d, dp, kappa,
                       exclude_self ? 1 : 0, rows, idx, dist);
    HIPC(hipGetLastError());
}

}  // namespace askit
