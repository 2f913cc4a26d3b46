// Exact kappa-nearest neighbours on gfx950.
//
// The neighbour lists are defined exactly: the kappa smallest (D, j), D the
// canonical FP64 squared distance, j the point id (self excluded for the
// point set).  They are found in three steps:
//   1. k_knn_cand: approximate squared distances |q|^2 + |x|^2 - 2 q.x with
//      the dot product as bf16 hi/lo split products (hi*hi + hi*lo + lo*hi)
//      on MFMA 32x32x16 with FP32 accumulation; each query row keeps its 64
//      smallest approximate distances in a wave-wide sorted list.
//   2. k_knn_refine: exact FP64 distances of the candidates, sorted by
//      (D, j); the row is certified when the kappa-th exact distance is
//      below (the threshold - E), E a bound on the approximation error and
//      every point outside the candidates at or above the threshold in
//      approximate distance, so none of them can enter.
//   The threshold filter (k_knn_filter + k_knn_select) keeps nsel <= 64
//   candidates per row (knn_nsel: a margin above kappa) with the nsel-th
//   approximate distance as threshold; the list sweeps keep 64.
//   3. k_knn_exact: full FP64 scan for the rows that are not certified.
#include "askit_impl.h"

#include <algorithm>
#include <cstdlib>
#include <type_traits>

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

#define QMAPPED false
#define QROW(q) (q)

// Survivor handling for one (column half c, register r) of the 32 x 64 tile
// held by a wave: values below the row's threshold are appended to the row's
// LDS buffer; a full buffer is first merged into the row's sorted list.
#define KNN_SURVIVORS(ACC, C, R)                                                                   \
    {                                                                                              \
        const int64_t colg = tbase + 32 * (C) + l32;                                               \
        const float dv = ACC[R];                                                                   \
        bool pred = dv < thrv[R];                                                                  \
        uint64_t mask = __ballot(pred);                                                            \
        if (mask) {                                                                                \
            _Pragma("unroll") for (int h = 0; h < 2; ++h)                                          \
            {                                                                                      \
                const int RR = 8 * ((R) / 4) + ((R) % 4) + 4 * h;                                  \
                uint32_t mh = (uint32_t)(mask >> (32 * h));                                        \
                if (mh == 0) continue;                                                             \
                int nnew = __popc(mh);                                                             \
                if (cnt[RR] + nnew > KCB) {                                                        \
                    ListEntry e = merge_list(list_d[RR], list_i[RR], bd + RR * KCB, bi + RR * KCB, \
                                             cnt[RR], lane);                                       \
                    list_d[RR] = e.d;                                                              \
                    list_i[RR] = e.i;                                                              \
                    cnt[RR] = 0;                                                                   \
                    if (half == h) thrv[R] = e.thr;                                                \
                    pred = dv < thrv[R];                                                           \
                    mh = (uint32_t)(__ballot(pred) >> (32 * h));                                   \
                    nnew = __popc(mh);                                                             \
                }                                                                                  \
                if (half == h && pred) {                                                           \
                    int pos = cnt[RR] + __popc(mh & ((1u << l32) - 1u));                           \
                    bd[RR * KCB + pos] = dv;                                                       \
                    bi[RR * KCB + pos] = (int)colg;                                                \
                }                                                                                  \
                cnt[RR] += nnew;                                                                   \
            }                                                                                      \
        }                                                                                          \
    }

// Approximate squared distances of one tile (from ACC0/ACC1 into the local
// arrays dA/dB, norms of the tile's points in NB): sets `any` when a value of
// the wave is below its row's threshold.  Only the last tile (ragged) and the tile holding the
// wave's own rows (self exclusion) need per-element checks.
#define KNN_DISTANCES(ACC0, ACC1, NB)                                                              \
    bool any = false;                                                                              \
    float dA[16], dB[16];                                                                          \
    {                                                                                              \
        const float ny0 = (NB)[l32], ny1 = (NB)[32 + l32];                                         \
        const int edge = __builtin_amdgcn_readfirstlane(                                           \
            (int)((tbase + KB_N > N) || (excl && (QMAPPED || (tbase < q0 + 32 && q0 < tbase + KB_N))))); \
        if (edge) {                                                                                \
            _Pragma("unroll") for (int r = 0; r < 16; ++r)                                         \
            {                                                                                      \
                float d0 = fmaf(-2.0f, ACC0[r], qn[r] + ny0);                                      \
                float d1 = fmaf(-2.0f, ACC1[r], qn[r] + ny1);                                      \
                const int64_t qrow = QROW(q0 + 8 * (r / 4) + 4 * half + (r % 4));                  \
                const int64_t c0 = tbase + l32, c1 = tbase + 32 + l32;                             \
                if (c0 >= N || (excl && c0 == qrow)) d0 = INFINITY;                                \
                if (c1 >= N || (excl && c1 == qrow)) d1 = INFINITY;                                \
                dA[r] = d0;                                                                        \
                dB[r] = d1;                                                                        \
                any |= (d0 < thrv[r]) | (d1 < thrv[r]);                                            \
            }                                                                                      \
        } else {                                                                                   \
            _Pragma("unroll") for (int r = 0; r < 16; ++r)                                         \
            {                                                                                      \
                float d0 = fmaf(-2.0f, ACC0[r], qn[r] + ny0);                                      \
                float d1 = fmaf(-2.0f, ACC1[r], qn[r] + ny1);                                      \
                dA[r] = d0;                                                                        \
                dB[r] = d1;                                                                        \
                any |= (d0 < thrv[r]) | (d1 < thrv[r]);                                            \
            }                                                                                      \
        }                                                                                          \
    }

// Tile loads (global -> registers stage st) and stores (stage st -> LDS buffer b).
#define KNN_TILE_IO()                                                                              \
    auto load_tile = [&](int st, int64_t tt) {                                                     \
        _Pragma("unroll") for (int u = 0; u < PER; ++u)                                            \
        {                                                                                          \
            int c = tid + 256 * u;                                                                 \
            int row = c / (DP / 8), off = (c % (DP / 8)) * 8;                                      \
            int64_t g = tt * KB_N + row;                                                           \
            if (c < CHUNKS && g < N) {                                                             \
                rh[st][u] = *reinterpret_cast<const uint4 *>(Xh + g * DP + off);                   \
                rl[st][u] = *reinterpret_cast<const uint4 *>(Xl + g * DP + off);                   \
            } else {                                                                               \
                rh[st][u] = uint4{0, 0, 0, 0};                                                     \
                rl[st][u] = uint4{0, 0, 0, 0};                                                     \
            }                                                                                      \
        }                                                                                          \
        int64_t g = tt * KB_N + tid;                                                               \
        rn[st] = (tid < KB_N && g < N) ? Xn[g] : 0.0f;                                             \
    };                                                                                             \
    auto store_tile = [&](int st, int b) {                                                         \
        _Pragma("unroll") for (int u = 0; u < PER; ++u)                                            \
        {                                                                                          \
            int c = tid + 256 * u;                                                                 \
            if (c < CHUNKS) {                                                                      \
                int row = c / (DP / 8), off = (c % (DP / 8)) * 8;                                  \
                *reinterpret_cast<uint4 *>(&sBh[b * TB + row * LDB + off]) = rh[st][u];            \
                *reinterpret_cast<uint4 *>(&sBl[b * TB + row * LDB + off]) = rl[st][u];            \
            }                                                                                      \
        }                                                                                          \
        if (tid < KB_N) sBn[b * KB_N + tid] = rn[st];                                              \
    };

// KS = dp / 16 MFMA k-steps; the query fragments stay in registers.  Three
// LDS buffers and two accumulator sets software-pipeline the sweep: while
// the distances of tile t are checked on the VALU, the MFMAs of tile t+1 run,
// and the points of tile t+2 (loaded one iteration earlier) go to LDS.  With
// start_local the sweep starts at the tile holding the block's own rows and
// wraps around: on tree-ordered points the first tiles hold each row's
// neighbourhood, so the lists fill at once and later tiles rarely add
// candidates.
// qpos (optional): query row q is row qpos[q] of Qh/Ql/Qn and of the outputs
// (self exclusion and the sweep start use that row); M counts mapped rows.
template <int KS>
__global__ __launch_bounds__(256) void k_knn_cand(const uint16_t *__restrict__ Qh,
                                                  const uint16_t *__restrict__ Ql,
                                                  const float *__restrict__ Qn, int64_t M,
                                                  const uint16_t *__restrict__ Xh,
                                                  const uint16_t *__restrict__ Xl,
                                                  const float *__restrict__ Xn, int64_t N,
                                                  int excl, int start_local, int win_tiles,
                                                  const int32_t *__restrict__ qpos,
                                                  int32_t *__restrict__ cand,
                                                  float *__restrict__ thr_out,
                                                  float *__restrict__ cand_d)
{
    constexpr int DP = KS * 16;
    constexpr int LDB = DP + 8;                      // padded LDS row (bf16 elements)
    constexpr int TB = KB_N * LDB;                   // one operand tile
    __shared__ __attribute__((aligned(16))) uint16_t sBh[3 * TB];
    __shared__ __attribute__((aligned(16))) uint16_t sBl[3 * TB];
    __shared__ float sBn[3 * KB_N];
    __shared__ float sbd[KB_M * KCB];
    __shared__ int sbi[KB_M * KCB];

    const int tid = threadIdx.x, lane = tid % WAVE;
    const int wv = __builtin_amdgcn_readfirstlane(tid / WAVE);
    const int half = lane >> 5, l32 = lane & 31;
    const int64_t q0 = (int64_t)blockIdx.x * KB_M + wv * 32;
    auto qmap = [&](int64_t q) -> int64_t { return qpos ? (int64_t)qpos[q] : q; };

    bf16x8 ah[KS], al[KS];
    {
        int64_t row = q0 + l32;
        bool ok = row < M;
        int64_t src = ok ? qmap(row) : 0;
#pragma unroll
        for (int s = 0; s < KS; ++s) {
            if (ok) {
                ah[s] = ld_bf8(Qh + src * DP + 16 * s + 8 * half);
                al[s] = ld_bf8(Ql + src * DP + 16 * s + 8 * half);
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
        qn[r] = row < M ? Qn[qmap(row)] : 0.0f;
        // segment sweeps start from the row's known bound (thr_out on entry)
        thrv[r] = (cand_d && row < M) ? thr_out[qmap(row)] : INFINITY;
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

    const int64_t ntiles_all = (N + KB_N - 1) / KB_N;
    // win_tiles > 0: sweep only the win_tiles tiles around the block's own rows
    // (tree order), which gives every row an upper bound of its 64th distance
    const int64_t qfirst = qmap(min((int64_t)blockIdx.x * KB_M, M - 1));
    int64_t t0 = start_local ? (qfirst / KB_N) % ntiles_all : 0;
    int64_t ntiles = ntiles_all;
    if (win_tiles > 0 && win_tiles < ntiles_all) {
        ntiles = win_tiles;
        int64_t c = (int64_t)blockIdx.x * KB_M / KB_N + (KB_M / KB_N) / 2 - win_tiles / 2;
        t0 = c < 0 ? 0 : (c + win_tiles > ntiles_all ? ntiles_all - win_tiles : c);
    }
    // cand_d != NULL: segment blockIdx.y of gridDim.y contiguous tile ranges;
    // the lists and their distances go to (segment, row) slots for a merge
    if (cand_d) {
        const int64_t per = (ntiles_all + gridDim.y - 1) / gridDim.y;
        t0 = (int64_t)blockIdx.y * per;
        ntiles = t0 < ntiles_all ? min(per, ntiles_all - t0) : 0;
    }
    if (ntiles == 0) {
        // empty segment: empty lists
        for (int R = 0; R < 32; ++R) {
            const int64_t row = q0 + R;
            if (row < M) {
                const int64_t o = ((int64_t)blockIdx.y * M + row) * KNN_CAND + lane;
                cand[o] = -1;
                cand_d[o] = INFINITY;
            }
        }
        return;
    }
    constexpr int CHUNKS = KB_N * DP / 8;            // 16-byte chunks per operand tile
    constexpr int PER = (CHUNKS + 255) / 256;
    uint4 rh[2][PER], rl[2][PER];
    float rn[2] = {0.0f, 0.0f};
    auto tile_of = [&](int64_t t) {
        int64_t tt = t0 + t;
        return tt >= ntiles_all ? tt - ntiles_all : tt;
    };
    KNN_TILE_IO();
    auto mfma_tile = [&](int b, f32x16 &acc0, f32x16 &acc1) {
        const uint16_t *ph = sBh + b * TB, *pl = sBl + b * TB;
        acc0 = f32x16{};
        acc1 = f32x16{};
#pragma unroll
        for (int s = 0; s < KS; ++s) {
            bf16x8 bh0 = ld_bf8(ph + l32 * LDB + 16 * s + 8 * half);
            bf16x8 bl0 = ld_bf8(pl + l32 * LDB + 16 * s + 8 * half);
            bf16x8 bh1 = ld_bf8(ph + (32 + l32) * LDB + 16 * s + 8 * half);
            bf16x8 bl1 = ld_bf8(pl + (32 + l32) * LDB + 16 * s + 8 * half);
            acc0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[s], bh0, acc0, 0, 0, 0);
            acc1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[s], bh1, acc1, 0, 0, 0);
            acc0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[s], bl0, acc0, 0, 0, 0);
            acc1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[s], bl1, acc1, 0, 0, 0);
            acc0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al[s], bh0, acc0, 0, 0, 0);
            acc1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al[s], bh1, acc1, 0, 0, 0);
        }
    };

    // prologue: tiles 0 and 1 in LDS buffers 0 and 1, tile 2 in register stage 0
    load_tile(0, tile_of(0));
    store_tile(0, 0);
    if (ntiles > 1) {
        load_tile(1, tile_of(1));
        store_tile(1, 1);
    }
    if (ntiles > 2) load_tile(0, tile_of(2));
    __syncthreads();
    f32x16 accA0, accA1, accB0, accB1;
    mfma_tile(0, accA0, accA1);

    // iteration t: the accumulators of tile t are ready (CUR selects the set);
    // MFMAs of tile t+1 read LDS buffer (t+1)%3; register stage t%2 holds tile
    // t+2, stored to buffer (t+2)%3; loads of tile t+3 go to stage (t+1)%2
#undef QMAPPED
#undef QROW
#define QMAPPED (qpos != nullptr)
#define QROW(q) ((q) < M ? qmap(q) : (int64_t)-1)
    auto iter = [&](auto CUR, int64_t t, f32x16 &c0, f32x16 &c1, f32x16 &n0, f32x16 &n1) {
        constexpr int st = decltype(CUR)::value;
        const int64_t tbase = tile_of(t) * KB_N;
        if (t + 3 < ntiles) load_tile(st ^ 1, tile_of(t + 3));
        if (t + 1 < ntiles) mfma_tile((int)((t + 1) % 3), n0, n1);
        KNN_DISTANCES(c0, c1, sBn + (t % 3) * KB_N);
        if (__ballot(any)) {
#pragma unroll
            for (int r = 0; r < 16; ++r) KNN_SURVIVORS(dA, 0, r);
#pragma unroll
            for (int r = 0; r < 16; ++r) KNN_SURVIVORS(dB, 1, r);
        }
        if (t + 2 < ntiles) store_tile(st, (int)((t + 2) % 3));
        __syncthreads();
    };
    for (int64_t t = 0; t < ntiles; t += 2) {
        iter(std::integral_constant<int, 0>{}, t, accA0, accA1, accB0, accB1);
        if (t + 1 < ntiles) iter(std::integral_constant<int, 1>{}, t + 1, accB0, accB1, accA0, accA1);
    }
    // final merge and output
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
            if (cand_d) {
                const int64_t o = ((int64_t)blockIdx.y * M + row) * KNN_CAND + lane;
                cand[o] = list_i[R] == 0x7fffffff ? -1 : list_i[R];
                cand_d[o] = list_d[R];
            } else {
                int64_t orow = qmap(row);
                cand[orow * KNN_CAND + lane] = list_i[R] == 0x7fffffff ? -1 : list_i[R];
                if (lane == 0) thr_out[orow] = th;
            }
        }
    }
#undef QMAPPED
#undef QROW
#define QMAPPED false
#define QROW(q) (q)
}

// Per row (one wave): the 64 smallest of the rows' segment lists; output
// through the row map (candidates and the 64th distance as threshold).
__global__ __launch_bounds__(256) void k_knn_merge_seg(int64_t M, int nseg, const int32_t *__restrict__ qpos,
                                                       const int32_t *__restrict__ si, const float *__restrict__ sd,
                                                       int32_t *__restrict__ cand, float *__restrict__ thr)
{
    const int64_t r = (int64_t)blockIdx.x * 4 + threadIdx.x / WAVE;
    const int lane = threadIdx.x % WAVE;
    if (r >= M) return;
    float ld = INFINITY;
    int li = 0x7fffffff;
    for (int g = 0; g < nseg; ++g) {
        const int64_t o = ((int64_t)g * M + r) * KNN_CAND;
        ListEntry e = merge_list(ld, li, sd + o, si + o, KNN_CAND, lane);
        ld = e.d;
        li = e.i;
    }
    const int64_t orow = qpos ? (int64_t)qpos[r] : r;
    cand[orow * KNN_CAND + lane] = (li == 0x7fffffff || li < 0) ? -1 : li;
    const float th = __shfl(ld, 63);
    if (lane == 0) thr[orow] = th;
}

// Generic variant for dp > 128: query fragments re-read from memory per tile,
// reference tiles staged in LDS in chunks of 128 dimensions.
__global__ __launch_bounds__(256) void k_knn_cand_wide(const uint16_t *__restrict__ Qh,
                                                       const uint16_t *__restrict__ Ql,
                                                       const float *__restrict__ Qn, int64_t M,
                                                       const uint16_t *__restrict__ Xh,
                                                       const uint16_t *__restrict__ Xl,
                                                       const float *__restrict__ Xn, int64_t N,
                                                       int dp, int excl, int start_local,
                                                       int32_t *__restrict__ cand,
                                                       float *__restrict__ thr_out)
{
    constexpr int KC = 128;                          // dims per LDS chunk
    constexpr int LDB = KC + 8;
    __shared__ __attribute__((aligned(16))) uint16_t sBh[1][KB_N * LDB];
    __shared__ __attribute__((aligned(16))) uint16_t sBl[1][KB_N * LDB];
    __shared__ float sBn[1][KB_N];
    __shared__ float sbd[KB_M * KCB];
    __shared__ int sbi[KB_M * KCB];
    const int cur = 0;

    const int tid = threadIdx.x, lane = tid % WAVE;
    const int wv = __builtin_amdgcn_readfirstlane(tid / WAVE);
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
    const int64_t t0 = start_local ? ((int64_t)blockIdx.x * KB_M / KB_N) % ntiles : 0;

    for (int64_t t = 0; t < ntiles; ++t) {
        int64_t tt = t0 + t;
        if (tt >= ntiles) tt -= ntiles;
        const int64_t tbase = tt * KB_N;
        f32x16 acc0 = {}, acc1 = {};
        for (int k0 = 0; k0 < dp; k0 += KC) {
            const int kc = min(KC, dp - k0);
            __syncthreads();
            for (int c = tid; c < KB_N * (KC / 8); c += 256) {
                int row = c / (KC / 8), off = (c % (KC / 8)) * 8;
                int64_t g = tbase + row;
                uint4 vh = {0, 0, 0, 0}, vl = {0, 0, 0, 0};
                if (g < N && off < kc) {
                    vh = *reinterpret_cast<const uint4 *>(Xh + g * dp + k0 + off);
                    vl = *reinterpret_cast<const uint4 *>(Xl + g * dp + k0 + off);
                }
                *reinterpret_cast<uint4 *>(&sBh[0][row * LDB + off]) = vh;
                *reinterpret_cast<uint4 *>(&sBl[0][row * LDB + off]) = vl;
            }
            if (k0 == 0 && tid < KB_N) {
                int64_t g = tbase + tid;
                sBn[0][tid] = g < N ? Xn[g] : 0.0f;
            }
            __syncthreads();
            for (int s = 0; s < kc / 16; ++s) {
                bf16x8 qa = aok ? ld_bf8(Qh + arow * dp + k0 + 16 * s + 8 * half) : bf16x8{};
                bf16x8 qb = aok ? ld_bf8(Ql + arow * dp + k0 + 16 * s + 8 * half) : bf16x8{};
                bf16x8 bh0 = ld_bf8(&sBh[0][l32 * LDB + 16 * s + 8 * half]);
                bf16x8 bl0 = ld_bf8(&sBl[0][l32 * LDB + 16 * s + 8 * half]);
                bf16x8 bh1 = ld_bf8(&sBh[0][(32 + l32) * LDB + 16 * s + 8 * half]);
                bf16x8 bl1 = ld_bf8(&sBl[0][(32 + l32) * LDB + 16 * s + 8 * half]);
                acc0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(qa, bh0, acc0, 0, 0, 0);
                acc1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(qa, bh1, acc1, 0, 0, 0);
                acc0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(qa, bl0, acc0, 0, 0, 0);
                acc1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(qa, bl1, acc1, 0, 0, 0);
                acc0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(qb, bh0, acc0, 0, 0, 0);
                acc1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(qb, bh1, acc1, 0, 0, 0);
            }
        }
        KNN_DISTANCES(acc0, acc1, sBn[0]);
        if (__ballot(any)) {
#pragma unroll
            for (int r = 0; r < 16; ++r) KNN_SURVIVORS(dA, 0, r);
#pragma unroll
            for (int r = 0; r < 16; ++r) KNN_SURVIVORS(dB, 1, r);
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


// Filter sweep: every reference point whose approximate squared distance to
// query row i is at most T_i (an upper bound of the row's 64th smallest
// approximate distance, from the window pass, slightly widened) is appended
// to the row's segment of `out` (capacity cap; count in ocnt).  Same MFMA
// arithmetic and pipelining as k_knn_cand, without per-row lists.
// SYM (the point set against itself, all rows in one launch): the block of
// rows [128 b, 128 b + 128) sweeps only the tiles from its own onwards, and a
// distance of a later tile's point j to row i is also offered to row j
// (appended to j's segment when it is at most T_j), so every unordered pair
// is computed once.  Survivors are then in no particular order, and a row
// may keep fewer than 64 of the window's points (their distances can come
// from the transposed product, rounded differently); the selection and its
// certificate allow both.
template <int KS, bool SYM>
__global__ __launch_bounds__(256, 2) void k_knn_filter(const uint16_t *__restrict__ Qh,
                                                       const uint16_t *__restrict__ Ql,
                                                       const float *__restrict__ Qn, int64_t M,
                                                       const uint16_t *__restrict__ Xh,
                                                       const uint16_t *__restrict__ Xl,
                                                       const float *__restrict__ Xn, int64_t N,
                                                       int excl, int64_t row0,
                                                       const float *__restrict__ Tin,
                                                       int cap, int32_t *__restrict__ ocnt,
                                                       uint2 *__restrict__ oe, int win_tiles,
                                                       const int32_t *__restrict__ tlist,
                                                       const int64_t *__restrict__ toff,
                                                       const int4 *__restrict__ items)
{
    constexpr int DP = KS * 16;
    constexpr int LDB = DP + 8;
    constexpr int TB = KB_N * LDB;
    __shared__ __attribute__((aligned(16))) uint16_t sBh[3 * TB];
    __shared__ __attribute__((aligned(16))) uint16_t sBl[3 * TB];
    __shared__ float sBn[3 * KB_N];
    __shared__ float sBt[SYM ? 3 * KB_N : 1];       // SYM: thresholds of the tile's points
    __shared__ int sTile[3];                          // tile held by each buffer

    const int tid = threadIdx.x, lane = tid % WAVE;
    const int wv = __builtin_amdgcn_readfirstlane(tid / WAVE);
    const int half = lane >> 5, l32 = lane & 31;
    // listed sweep: workgroup i takes the piece items[i] = (row block, first
    // list position, tile count) of a block's tile list
    const int4 item = tlist ? items[blockIdx.x] : int4{(int)blockIdx.x, 0, 0, 0};
    const int64_t bx = item.x;
    const int64_t q0 = bx * KB_M + wv * 32;     // local row (output segments)

    bf16x8 ah[KS], al[KS];
    {
        int64_t row = q0 + l32;
        bool ok = row < M;
#pragma unroll
        for (int s = 0; s < KS; ++s) {
            if (ok) {
                ah[s] = ld_bf8(Qh + (row0 + row) * DP + 16 * s + 8 * half);
                al[s] = ld_bf8(Ql + (row0 + row) * DP + 16 * s + 8 * half);
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
        qn[r] = row < M ? Qn[row0 + row] : 0.0f;
        thrv[r] = row < M ? Tin[row0 + row] : -INFINITY;
    }
    // 32-bit row indices (M < 2^31) keep the survivor path's state small
    const uint32_t qbase = (uint32_t)q0 + 4u * (uint32_t)half;
    const int64_t ntiles_all = (N + KB_N - 1) / KB_N;
    const int64_t tself = ((row0 + bx * KB_M) / KB_N) % ntiles_all;   // the block's own tile
    int64_t ntiles = SYM ? ntiles_all - tself : ntiles_all;
    int64_t t0 = tself;
    if (!SYM && win_tiles > 0 && win_tiles < ntiles_all) {
        // the win_tiles tiles centred on the block's rows (the window pass's range)
        ntiles = win_tiles;
        const int64_t c = (row0 + (int64_t)blockIdx.x * KB_M) / KB_N + (KB_M / KB_N) / 2 - win_tiles / 2;
        t0 = c < 0 ? 0 : (c + win_tiles > ntiles_all ? ntiles_all - win_tiles : c);
    }
    if (!SYM && gridDim.y > 1) {
        // column segment blockIdx.y of gridDim.y contiguous tile ranges (the
        // segments of a row append to the same output segment)
        const int64_t per = (ntiles_all + gridDim.y - 1) / gridDim.y;
        t0 = (int64_t)blockIdx.y * per;
        ntiles = t0 < ntiles_all ? min(per, ntiles_all - t0) : 0;
    }
    // tile lists: only the tiles that may hold a survivor (SYM: the block's
    // own two first), in increasing order; this workgroup's piece of them
    const int32_t *tl = nullptr;
    if (tlist) {
        tl = tlist + toff[bx] + item.y;
        ntiles = item.z;
    }
    if (ntiles <= 0) return;
    // tile counts fit 32 bits (N < 2^31 points)
    const int nt32 = (int)ntiles, t032 = (int)t0, nta32 = (int)ntiles_all;
    constexpr int CHUNKS = KB_N * DP / 8;
    constexpr int PER = (CHUNKS + 255) / 256;
    uint4 rh[1][PER], rl[1][PER];
    float rn[1] = {0.0f};
    // entry of list position t: the tile, and in bits 27-30 the waves that
    // sweep it (all four without lists)
    // with lists: 64 entries per register (one per lane), the next 64 loaded
    // a full chunk ahead; entries are read with a uniform lane index, so the
    // next tile's address never waits on a list load
    int lcur = 0, lnxt = 0;
    if (tl) {
        lcur = lane < nt32 ? tl[lane] : 0;
        lnxt = 64 + lane < nt32 ? tl[64 + lane] : 0;
    }
    auto tile_of = [&](int t) -> int {
        if (tl) {
            // positions are asked for in order 0, 1, 2, ...
            if ((t & 63) == 0 && t > 0) {
                lcur = lnxt;
                lnxt = t + 64 + lane < nt32 ? tl[t + 64 + lane] : 0;
            }
            return __builtin_amdgcn_readlane(lcur, t & 63);
        }
        const int tt = t032 + t;
        return (tt >= nta32 ? tt - nta32 : tt) | (15 << 27);
    };
    auto wave_on = [&](int ent) -> bool { return (ent >> (27 + wv)) & 1; };
    KNN_TILE_IO();
    float rt = -INFINITY;
    auto load_thr = [&](int64_t tt) {
        if constexpr (SYM) {
            const int64_t g = tt * KB_N + tid;
            rt = (tid < KB_N && g < N) ? Tin[g] : -INFINITY;
        }
    };
    auto store_thr = [&](int b) {
        if constexpr (SYM) {
            if (tid < KB_N) sBt[b * KB_N + tid] = rt;
        }
    };
    auto mfma_tile = [&](int b, f32x16 &acc0, f32x16 &acc1) {
        const uint16_t *ph = sBh + b * TB, *pl = sBl + b * TB;
        acc0 = f32x16{};
        acc1 = f32x16{};
#pragma unroll
        for (int s = 0; s < KS; ++s) {
            bf16x8 bh0 = ld_bf8(ph + l32 * LDB + 16 * s + 8 * half);
            bf16x8 bl0 = ld_bf8(pl + l32 * LDB + 16 * s + 8 * half);
            bf16x8 bh1 = ld_bf8(ph + (32 + l32) * LDB + 16 * s + 8 * half);
            bf16x8 bl1 = ld_bf8(pl + (32 + l32) * LDB + 16 * s + 8 * half);
            acc0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[s], bh0, acc0, 0, 0, 0);
            acc1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[s], bh1, acc1, 0, 0, 0);
            acc0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[s], bl0, acc0, 0, 0, 0);
            acc1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[s], bl1, acc1, 0, 0, 0);
            acc0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al[s], bh0, acc0, 0, 0, 0);
            acc1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al[s], bh1, acc1, 0, 0, 0);
        }
    };
    int tnext = tile_of(0);                 // entry of the next load (kept in a register)
    load_tile(0, tnext & 0x7ffffff);
    load_thr(tnext & 0x7ffffff);
    store_tile(0, 0);
    store_thr(0);
    if (tid == 0) sTile[0] = tnext;
    if (ntiles > 1) {
        tnext = tile_of(1);
        load_tile(0, tnext & 0x7ffffff);
        load_thr(tnext & 0x7ffffff);
        store_tile(0, 1);
        store_thr(1);
        if (tid == 0) sTile[1] = tnext;
    }
    __syncthreads();
    f32x16 accA0, accA1, accB0, accB1;
    if (wave_on(sTile[0])) mfma_tile(0, accA0, accA1);
    // iteration t: accumulators of tile t ready; MFMAs of tile t+1 read buffer
    // (t+1)%3; the points of tile t+2 are loaded and stored to buffer (t+2)%3
    auto iter = [&](auto CUR, int t, f32x16 &c0, f32x16 &c1, f32x16 &n0, f32x16 &n1) {
        const int ent = sTile[t % 3];
        const int tbase = (ent & 0x7ffffff) * KB_N;
        const bool on = wave_on(ent);
        if (t + 2 < nt32) {
            tnext = tile_of(t + 2);
            load_tile(0, tnext & 0x7ffffff);
            load_thr(tnext & 0x7ffffff);
        }
        if (t + 1 < nt32 && wave_on(sTile[(t + 1) % 3])) mfma_tile((t + 1) % 3, n0, n1);
        // <= keeps the window's own 64 points (same arithmetic as the window pass)
        const float *nb = sBn + (t % 3) * KB_N;
        const float ny0 = nb[l32], ny1 = nb[32 + l32];
        // the 32 distances of the lane, computed once for both tests
        float dv[32];
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            dv[r] = fmaf(-2.0f, c0[r], qn[r] + ny0);
            dv[16 + r] = fmaf(-2.0f, c1[r], qn[r] + ny1);
        }
        bool any = false;
        if (on) {
#pragma unroll
            for (int r = 0; r < 16; ++r) any |= (dv[r] <= thrv[r]) | (dv[16 + r] <= thrv[r]);
        }
        if (__ballot(any)) {
            const uint32_t cA = (uint32_t)tbase + (uint32_t)l32, cB = cA + 32u;
            const uint32_t n32 = (uint32_t)N;
            const uint32_t below = (1u << l32) - 1u;
            // an opaque copy of the rows' base: otherwise the compiler hoists
            // the 16 rows' 64-bit segment offsets out of the sweep loop, spills
            // them, and every append waits on a scratch reload
            uint32_t qb = qbase;
            asm volatile("" : "+v"(qb));
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                // the 32 lanes of a half-wave hold the same row: one counter
                // update per row and half-wave, lanes write at their prefix
                const uint32_t qrow = qb + (uint32_t)(8 * (r / 4) + (r % 4));
                const float dA = dv[r];
                const float dB = dv[16 + r];
                const bool pA = dA <= thrv[r] && cA < n32 && !(excl && cA == qrow + (uint32_t)row0);
                const bool pB = dB <= thrv[r] && cB < n32 && !(excl && cB == qrow + (uint32_t)row0);
                const uint64_t bA = __ballot(pA), bB = __ballot(pB);
                const uint32_t hA = (uint32_t)(bA >> (32 * half)), hB = (uint32_t)(bB >> (32 * half));
                if ((hA | hB) == 0u) continue;
                const int lead = 32 * half + __ffs(hA | hB) - 1;
                uint32_t p0 = 0;
                if (lane == lead) p0 = (uint32_t)atomicAdd(&ocnt[qrow], __popc(hA) + __popc(hB));
                p0 = (uint32_t)__shfl((int)p0, lead);
                if (pA) {
                    const uint32_t p = p0 + __popc(hA & below);
                    if (p < (uint32_t)cap) {
                        oe[(size_t)qrow * (uint32_t)cap + p] = make_uint2(__float_as_uint(dA), cA);
                    }
                }
                if (pB) {
                    const uint32_t p = p0 + __popc(hA) + __popc(hB & below);
                    if (p < (uint32_t)cap) {
                        oe[(size_t)qrow * (uint32_t)cap + p] = make_uint2(__float_as_uint(dB), cB);
                    }
                }
            }
        }
        if constexpr (SYM) {
            // tiles after the block's own two: offer each distance to the tile's point too
            if ((ent & 0x7ffffff) >= tself + 2 && on) {
                const float *tb = sBt + (t % 3) * KB_N;
                const float tA = tb[l32], tB = tb[32 + l32];
                bool anyc = false;
#pragma unroll
                for (int r = 0; r < 16; ++r) anyc |= (dv[r] <= tA) | (dv[16 + r] <= tB);
                if (__ballot(anyc)) {
                    const uint32_t cA = (uint32_t)tbase + (uint32_t)l32, cB = cA + 32u;
                    const uint32_t m32 = (uint32_t)M;
#pragma unroll
                    for (int r = 0; r < 16; ++r) {
                        const uint32_t qrow = qbase + (uint32_t)(8 * (r / 4) + (r % 4));
                        if (qrow >= m32) continue;
                        const float dA = dv[r];
                        const float dB = dv[16 + r];
                        if (dA <= tA) {
                            uint32_t p = (uint32_t)atomicAdd(&ocnt[cA], 1);
                            if (p < (uint32_t)cap) {
                                oe[(size_t)cA * (uint32_t)cap + p] = make_uint2(__float_as_uint(dA), qrow);
                            }
                        }
                        if (dB <= tB) {
                            uint32_t p = (uint32_t)atomicAdd(&ocnt[cB], 1);
                            if (p < (uint32_t)cap) {
                                oe[(size_t)cB * (uint32_t)cap + p] = make_uint2(__float_as_uint(dB), qrow);
                            }
                        }
                    }
                }
            }
        }
        if (t + 2 < nt32) {
            store_tile(0, (t + 2) % 3);
            store_thr((t + 2) % 3);
            if (tid == 0) sTile[(t + 2) % 3] = tnext;
        }
        __syncthreads();
    };
    for (int t = 0; t < nt32; t += 2) {
        iter(std::integral_constant<int, 0>{}, t, accA0, accA1, accB0, accB1);
        if (t + 1 < nt32) iter(std::integral_constant<int, 1>{}, t + 1, accB0, accB1, accA0, accA1);
    }
}

// Per row (one wave): the nsel smallest (approximate distance, position) of
// the filter's output, as candidates + the certificate threshold.  Rows whose
// segment overflowed are listed for the retry sweep (when bad_count is given).
// The nsel-th smallest distance is found by a radix selection on an
// order-preserving image of the FP32 values (four 8-bit digits, a histogram
// per wave in LDS); the candidates are every stored entry below it and, among
// those equal to it, the ones with the smallest positions.  Candidates are
// written in no particular order (the certificate re-sorts them exactly).
constexpr int SEL_Q = 16;                  // stored entries per lane (cap <= 1024)

__device__ __forceinline__ uint32_t f2key(float f)
{
    const uint32_t u = __float_as_uint(f);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

__device__ __forceinline__ float key2f(uint32_t k)
{
    return __uint_as_float((k & 0x80000000u) ? (k & 0x7fffffffu) : ~k);
}

__global__ __launch_bounds__(256) void k_knn_select(int64_t M, int64_t row0, int cap, int nsel,
                                                    const int32_t *__restrict__ ocnt,
                                                    const uint2 *__restrict__ oe,
                                                    int32_t *__restrict__ cand,
                                                    float *__restrict__ thr,
                                                    int32_t *__restrict__ bad_rows,
                                                    int32_t *__restrict__ bad_count)
{
    __shared__ int hist[4][256];
    const int wv = threadIdx.x / WAVE, lane = threadIdx.x % WAVE;
    int64_t lrow = (int64_t)blockIdx.x * 4 + wv;
    if (lrow >= M) return;
    const int64_t row = row0 + lrow;
    const int n = ocnt[lrow];
    const float tin = thr[row];          // the filter threshold: every point left out is above it
    if (n > cap && lane == 0 && bad_count) {
        int p = atomicAdd(bad_count, 1);
        bad_rows[p] = (int32_t)row;
    }
    const int nk = min(n, cap);
    const uint2 *re = oe + lrow * cap;          // (distance bits, id) per stored entry
    int32_t *co = cand + row * KNN_CAND;
    if (nk <= nsel) {
        // every stored entry is a candidate
        co[lane] = lane < nk ? (int32_t)re[lane].y : -1;
        float m = -INFINITY;
        if (nk == nsel) {
            m = lane < nk ? __uint_as_float(re[lane].x) : -INFINITY;
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) m = fmaxf(m, __shfl_xor(m, o));
        }
        if (lane == 0) thr[row] = n > cap ? m + fabsf(m) * 1e-5f + 1e-30f : (n >= nsel ? m : tin);
        return;
    }
    // keys and ids of the stored entries; the loads are unconditional (index
    // clamped to the last entry) so that all of them are in flight at once
    // the stored distances, loaded unconditionally (index clamped to the last
    // entry) and pinned by an empty asm so that the loads are not sunk into
    // per-entry branches: all of them are in flight at once
    float kv[SEL_Q];
#pragma unroll
    for (int q = 0; q < SEL_Q; ++q) kv[q] = __uint_as_float(re[min(lane + WAVE * q, nk - 1)].x);
#pragma unroll
    for (int q = 0; q < SEL_Q; ++q) asm volatile("" : "+v"(kv[q]));
    uint32_t key[SEL_Q];
#pragma unroll
    for (int q = 0; q < SEL_Q; ++q) key[q] = lane + WAVE * q < nk ? f2key(kv[q]) : 0xffffffffu;
    // the nsel-th smallest key, one 8-bit digit at a time
    uint32_t prefix = 0, pmask = 0;
    int kk = nsel;                       // rank sought among the keys matching prefix
    int *hw = hist[wv];
#pragma unroll 1
    for (int shift = 24; shift >= 0; shift -= 8) {
#pragma unroll
        for (int u = 0; u < 4; ++u) hw[lane * 4 + u] = 0;
        __builtin_amdgcn_wave_barrier();
#pragma unroll
        for (int q = 0; q < SEL_Q; ++q)
            if (lane + WAVE * q < nk && (key[q] & pmask) == prefix) atomicAdd(&hw[(key[q] >> shift) & 255u], 1);
        __builtin_amdgcn_wave_barrier();
        int c[4], c4 = 0;
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            c[u] = hw[lane * 4 + u];
            c4 += c[u];
        }
        int inc = c4;                    // inclusive scan over lanes (bins in order)
#pragma unroll
        for (int o = 1; o < WAVE; o <<= 1) {
            const int y = __shfl_up(inc, o);
            if (lane >= o) inc += y;
        }
        const int ex = inc - c4;
        const uint64_t hit = __ballot(ex < kk && inc >= kk);
        const int L = __ffsll((long long)hit) - 1;
        int bin = 0, below = ex;
        if (lane == L) {
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                if (below + c[u] >= kk) { bin = lane * 4 + u; break; }
                below += c[u];
            }
        }
        bin = __shfl(bin, L);
        below = __shfl(below, L);
        kk -= below;
        prefix |= (uint32_t)bin << shift;
        pmask |= 255u << shift;
        __builtin_amdgcn_wave_barrier();
    }
    const uint32_t K = prefix;           // kk of the keys equal to K complete the nsel
    // the winners' entry positions go to a per-wave list in LDS (the
    // histogram's space), then each lane loads one id: entries below K (nsel
    // - kk of them), then the kk equal ones with the smallest positions;
    // lanes from nsel on hold no candidate
    int *slot = hw;
    int base = 0;
#pragma unroll
    for (int q = 0; q < SEL_Q; ++q) {
        const bool pr = key[q] < K;
        const uint64_t bm = __ballot(pr);
        if (pr) slot[base + __popcll(bm & ((1ull << lane) - 1ull))] = lane + WAVE * q;
        base += __popcll(bm);
    }
    int nslot = base;
    int neq = 0;
#pragma unroll
    for (int q = 0; q < SEL_Q; ++q) neq += __popcll(__ballot(key[q] == K));
    if (neq == kk) {
#pragma unroll
        for (int q = 0; q < SEL_Q; ++q) {
            const bool pr = key[q] == K;
            const uint64_t bm = __ballot(pr);
            if (pr) slot[base + __popcll(bm & ((1ull << lane) - 1ull))] = lane + WAVE * q;
            base += __popcll(bm);
        }
        nslot = base;
    } else {
        // ties at the 64th distance: the kk smallest ids among them
        int last = -1;
        for (int take = 0; take < kk; ++take) {
            int mi = 0x7fffffff;
#pragma unroll
            for (int q = 0; q < SEL_Q; ++q) {
                const int e = lane + WAVE * q;
                if (key[q] == K && e < nk) {
                    const int p = (int)re[e].y;
                    if (p > last && p < mi) mi = p;
                }
            }
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) mi = min(mi, __shfl_xor(mi, o));
            if (lane == 0) co[base + take] = mi;
            last = mi;
        }
    }
    __builtin_amdgcn_wave_barrier();
    if (lane < nslot) co[lane] = (int32_t)re[slot[lane]].y;
    else if (lane >= nsel) co[lane] = -1;
    // bound for the points outside the candidates: the nsel-th survivor.  A
    // row whose segment overflowed is swept again; the nsel-th of its stored
    // survivors (real distances, so at least its nsel-th smallest), widened as
    // the window threshold, starts that sweep.
    const float th = key2f(K);
    if (lane == 0) thr[row] = n > cap ? th + fabsf(th) * 1e-5f + 1e-30f : th;
}

template <int KS>
static void launch_cand(dim3 g, dim3 b, hipStream_t s, const uint16_t *Qh, const uint16_t *Ql,
                        const float *Qn, int64_t M, const uint16_t *Xh, const uint16_t *Xl,
                        const float *Xn, int64_t N, int ex, int sl, int win, const int32_t *qpos,
                        int32_t *cand, float *thr, float *cand_d = nullptr)
{
    hipLaunchKernelGGL(k_knn_cand<KS>, g, b, 0, s, Qh, Ql, Qn, M, Xh, Xl, Xn, N, ex, sl, win, qpos, cand,
                       thr, cand_d);
}

template <int KS>
static void launch_filter(dim3 g, dim3 b, hipStream_t s, const uint16_t *Qh, const uint16_t *Ql,
                          const float *Qn, int64_t M, const uint16_t *Xh, const uint16_t *Xl,
                          const float *Xn, int64_t N, int ex, int64_t row0, const float *T, int cap,
                          int32_t *ocnt, uint2 *oe, bool sym, int win = 0,
                          const int32_t *tlist = nullptr, const int64_t *toff = nullptr,
                          const int4 *items = nullptr)
{
    if (sym)
        hipLaunchKernelGGL((k_knn_filter<KS, true>), g, b, 0, s, Qh, Ql, Qn, M, Xh, Xl, Xn, N, ex, row0, T, cap,
                           ocnt, oe, 0, tlist, toff, items);
    else
        hipLaunchKernelGGL((k_knn_filter<KS, false>), g, b, 0, s, Qh, Ql, Qn, M, Xh, Xl, Xn, N, ex, row0, T,
                           cap, ocnt, oe, win, tlist, toff, items);
}

__global__ void k_fill_f32(float *__restrict__ p, int64_t n, float v)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

__global__ void k_widen(float *__restrict__ T, int64_t M)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < M) {
        float t = T[i];
        T[i] = t + fabsf(t) * 1e-5f + 1e-30f;
    }
}

#define KNN_DISPATCH(FN, ...)                                                                      \
    switch (dp) {                                                                                  \
    case 16: FN<1>(__VA_ARGS__); break;                                                            \
    case 32: FN<2>(__VA_ARGS__); break;                                                            \
    case 48: FN<3>(__VA_ARGS__); break;                                                            \
    case 64: FN<4>(__VA_ARGS__); break;                                                            \
    case 80: FN<5>(__VA_ARGS__); break;                                                            \
    case 96: FN<6>(__VA_ARGS__); break;                                                            \
    case 112: FN<7>(__VA_ARGS__); break;                                                           \
    default: FN<8>(__VA_ARGS__); break;                                                            \
    }

// List sweep of every point for rows [0, M) (through qpos when given): with
// few row blocks the point range is split in segments so that about 2048
// workgroups share the sweep, and the segment lists are merged per row.  With
// seeded, thr holds each row's known bound on entry (segments only).
template <int KS>
static void list_sweep(hipStream_t s, const uint16_t *Qh, const uint16_t *Ql, const float *Qn, int64_t M,
                       const uint16_t *Xh, const uint16_t *Xl, const float *Xn, int64_t N, int ex, int sl,
                       const int32_t *qpos, bool seeded, int32_t *cand, float *thr)
{
    const int64_t ntiles = (N + KB_N - 1) / KB_N;
    const int rb = (int)((M + KB_M - 1) / KB_M);
    const int nseg = (int)std::max<int64_t>(1, std::min<int64_t>({32, 2048 / rb, ntiles / 16}));
    if (nseg == 1) {
        launch_cand<KS>(dim3((unsigned)rb), dim3(256), s, Qh, Ql, Qn, M, Xh, Xl, Xn, N, ex, sl, 0, qpos, cand,
                        thr);
    } else {
        int32_t *si;
        float *sd;
        HIPC(ws_alloc((void **)&si, sizeof(int32_t) * nseg * M * KNN_CAND, s));
        HIPC(ws_alloc((void **)&sd, sizeof(float) * nseg * M * KNN_CAND, s));
        if (!seeded) {
            // unseeded: every row starts from +inf (the rows are the identity map)
            hipLaunchKernelGGL(k_fill_f32, dim3((unsigned)((M + 255) / 256)), dim3(256), 0, s, thr, M, INFINITY);
        }
        launch_cand<KS>(dim3((unsigned)rb, (unsigned)nseg), dim3(256), s, Qh, Ql, Qn, M, Xh, Xl, Xn, N, ex, 0, 0,
                        qpos, si, thr, sd);
        hipLaunchKernelGGL(k_knn_merge_seg, dim3((unsigned)((M + 3) / 4)), dim3(256), 0, s, M, nseg, qpos, si, sd,
                           cand, thr);
        HIPC(ws_free(si, s));
        HIPC(ws_free(sd, s));
    }
    HIPC(hipGetLastError());
}

// Column segments of a filter launch over rows [0, m): enough workgroups to
// fill the chip when the row blocks alone do not.
static int filter_segments(int64_t m, int64_t ntiles)
{
    const int64_t rb = (m + KB_M - 1) / KB_M;
    return (int)std::max<int64_t>(1, std::min<int64_t>({64, 2048 / rb, ntiles / 16}));
}

constexpr int KNN_WIN = 64;                 // window tiles (4096 points)
constexpr int KNN_CAP = 1024;               // filter output per row
constexpr int64_t KNN_CHUNK = 1 << 20;      // query rows per filter pass (bounds the buffers)

// Filter output buffers of up to `rows` rows.
struct FilterBufs {
    int32_t *ocnt = nullptr;
    uint2 *oe = nullptr;                      // (distance bits, id) per slot, KNN_CAP slots per row
    int nsel = KNN_CAND;                      // candidates the selection keeps per row
};

// Threshold filter of rows [0, M) against a reference set, in passes of
// `chunk` rows, each followed by the selection (cand, thr of every row; rows
// whose output overflowed appended to over[1..], count over[0], when over is
// given).  win > 0: only the win tiles around each row block; sym: the
// triangular sweep.  ev collects HIP events around each filter launch.
static void filter_select(int dp, hipStream_t s, const uint16_t *Qh, const uint16_t *Ql, const float *Qn,
                          int64_t M, const uint16_t *Xh, const uint16_t *Xl, const float *Xn, int64_t N, int ex,
                          int64_t chunk, float *thr, const FilterBufs &B, int32_t *cand, int32_t *over, bool sym,
                          int win, std::vector<hipEvent_t> *ev, const int32_t *tlist = nullptr,
                          const int64_t *toff = nullptr, const int4 *items = nullptr, int64_t nitems = 0)
{
    const int64_t ntl = (N + KB_N - 1) / KB_N;
    for (int64_t r0 = 0; r0 < M; r0 += chunk) {
        const int64_t m = std::min<int64_t>(chunk, M - r0);
        dim3 g((unsigned)((m + KB_M - 1) / KB_M), (unsigned)((sym || win > 0) ? 1 : filter_segments(m, ntl)));
        if (tlist) g = dim3((unsigned)nitems);             // one workgroup per list piece
        HIPC(hipMemsetAsync(B.ocnt, 0, sizeof(int32_t) * m, s));
        if (ev) {
            ev->resize(ev->size() + 2);
            HIPC(hipEventCreate(&(*ev)[ev->size() - 2]));
            HIPC(hipEventCreate(&ev->back()));
            HIPC(hipEventRecord((*ev)[ev->size() - 2], s));
        }
        if (!tlist || nitems > 0)
            KNN_DISPATCH(launch_filter, g, dim3(256), s, Qh, Ql, Qn, m, Xh, Xl, Xn, N, ex, r0, thr, KNN_CAP, B.ocnt,
                         B.oe, sym, win, tlist, toff, items);
        if (ev) HIPC(hipEventRecord(ev->back(), s));
        hipLaunchKernelGGL(k_knn_select, dim3((unsigned)((m + 3) / 4)), dim3(256), 0, s, m, r0, KNN_CAP, B.nsel,
                           B.ocnt, B.oe, cand, thr, over ? over + 1 : nullptr, over);
        HIPC(hipGetLastError());
    }
}

static void widen(float *thr, int64_t M, hipStream_t s)
{
    hipLaunchKernelGGL(k_widen, dim3((unsigned)((M + 255) / 256)), dim3(256), 0, s, thr, M);
    HIPC(hipGetLastError());
}

// Thresholds from the nested strided samples for rows [0, M): every point of
// the coarsest sample (at most KNN_CAP) passes the filter at +inf; at each
// level the nsel-th smallest survivor bounds the row's nsel-th smallest
// distance over the whole set (an upper bound: those are real points), and the
// next, 8 times denser, level (a superset) keeps at least those nsel at that
// bound -- about 8 nsel points.  Each step only lowers a valid bound (a row
// with fewer than nsel survivors keeps its threshold).  seeded: thr already
// holds valid bounds to start from, else every row starts at +inf.  The
// sample passes' candidate lists (in cand) are scratch; thr leaves widened.
// No self exclusion: a row that is itself a sample point may count itself.
static void sample_thresholds(int dp, hipStream_t s, const uint16_t *Qh, const uint16_t *Ql, const float *Qn,
                              int64_t M, const KnnSample &S, int64_t chunk, float *thr, const FilterBufs &B,
                              int32_t *cand, bool seeded = false)
{
    if (!seeded)
        hipLaunchKernelGGL(k_fill_f32, dim3((unsigned)((M + 255) / 256)), dim3(256), 0, s, thr, M, INFINITY);
    for (int lv = 0; lv < S.levels; ++lv) {
        filter_select(dp, s, Qh, Ql, Qn, M, S.h[lv], S.l[lv], S.n[lv], S.rows[lv], 0, chunk, thr, B, cand,
                      nullptr, false, 0, nullptr);
        widen(thr, M, s);
    }
}

// Retry rows of the point set against itself (tree positions rows[0, n)),
// filtered through compact copies: the compact candidates go back to their
// rows with the row itself removed (the compact pass cannot exclude it; every
// other point left out stays at or above the threshold, so the certificate
// holds).  Rows that overflow again get an unseeded list sweep (thr = +inf:
// the stored 64th may count the row itself).
__global__ __launch_bounds__(256) void k_scatter_retry(int64_t n, const int32_t *__restrict__ rows,
                                                       const int32_t *__restrict__ cc, const float *__restrict__ tc,
                                                       const int32_t *__restrict__ ocnt, int cap,
                                                       int32_t *__restrict__ cand, float *__restrict__ thr,
                                                       int32_t *__restrict__ over_rows,
                                                       int32_t *__restrict__ over_count)
{
    const int64_t i = (int64_t)blockIdx.x * 4 + threadIdx.x / WAVE;
    const int lane = threadIdx.x % WAVE;
    if (i >= n) return;
    const int64_t row = rows[i];
    const int c = cc[i * KNN_CAND + lane];
    cand[row * KNN_CAND + lane] = c == row ? -1 : c;
    if (lane == 0) {
        if (ocnt[i] > cap) {
            over_rows[atomicAdd(over_count, 1)] = (int32_t)row;
            thr[row] = INFINITY;
        } else {
            thr[row] = tc[i];
        }
    }
}

__global__ void k_gather_qrows(const int32_t *__restrict__ rows, int64_t n, int dp,
                               const uint16_t *__restrict__ Qh, const uint16_t *__restrict__ Ql,
                               const float *__restrict__ Qn, const float *__restrict__ tb,
                               uint16_t *__restrict__ Bh, uint16_t *__restrict__ Bl, float *__restrict__ Bn,
                               float *__restrict__ Bt);

// ---------------------------------------------------------------- tile skipping
// In the symmetric sweep a (row group, tile) pair can be skipped when no pair
// of its points can pass either threshold test: with c and r a centre and a
// radius of a set of points (every point within r of c), every distance
// between a row of group a and a point of tile b is at least
// L = |c_a - c_b| - r_a - r_b, and an approximate squared distance differs
// from the exact one by at most E = g (|q|^2 + |x|^2) (the certificate's
// bound).  The pair is skipped when L > 0 and L^2 exceeds (the largest
// threshold of the group's rows and of the tile's points + the largest E) by
// a relative margin of 1e-6 -- then no survivor is lost and the filter output
// is exactly the full sweep's.  Row groups are the 32 rows of one wave; a
// block's tile list keeps the tiles that any of its four waves needs, with a
// 4-bit mask of those waves in bits 27-30 of the entry.  Centres are FP32
// copies of the FP64 means; radii are FP64 distances to those copies,
// enlarged by 1e-9 relative, and centre distances are shrunk by 1e-9
// relative.  ASKIT_KNN_NO_SKIP=1 in the environment sweeps every pair (the
// same output, for comparison).
constexpr int TL_TILE_BITS = 27;
constexpr int64_t KNN_PIECE = 2048;         // tiles per work item of the listed sweep
constexpr int32_t TL_TILE_MASK = (1 << TL_TILE_BITS) - 1;

struct TileGeom {
    double r;        // radius around c
    float tmax;      // largest row threshold of the points
    float nmax;      // largest FP32 squared norm of the points
};

// Geometry of consecutive groups of G points (G <= 64), one wave per group.
template <int G>
__global__ __launch_bounds__(64) void k_tile_geom(const float *__restrict__ Xf, int dp, int d, int64_t N,
                                                  const float *__restrict__ thr, const float *__restrict__ Xn,
                                                  float *__restrict__ cen, TileGeom *__restrict__ geo)
{
#pragma clang fp contract(off)
    // per 64 coordinates: the group's rows with one coalesced row load per
    // point (lane = coordinate); the centre is their FP64 sum in point order
    // over n, rounded to FP32; the rows then pass through LDS so that each
    // lane (point) forms its squared distance to that FP32 centre in FP64
    __shared__ float rows[G * 65];
    __shared__ float cs[64];
    const int64_t t = blockIdx.x;
    const int lane = threadIdx.x;
    const int64_t p0 = t * G;
    const int n = (int)min<int64_t>(G, N - p0);
    double r2 = 0.0;
    for (int k0 = 0; k0 < d; k0 += 64) {
        const int kc = min(k0 + lane, dp - 1);
        float x[G];
#pragma unroll
        for (int i = 0; i < G; ++i) x[i] = Xf[(p0 + min(i, n - 1)) * dp + kc];
        double v = 0.0;
#pragma unroll
        for (int i = 0; i < G; ++i)
            if (i < n) v += (double)x[i];
        const float c = (float)(v / (double)n);
        if (k0 + lane < d) cen[t * dp + k0 + lane] = c;
        cs[lane] = c;
#pragma unroll
        for (int i = 0; i < G; ++i) rows[i * 65 + lane] = x[i];
        __syncthreads();
        if (lane < n) {
            const int kn = min(64, d - k0);
            for (int j = 0; j < kn; ++j) {
                const double u = (double)rows[lane * 65 + j] - (double)cs[j];
                r2 += u * u;
            }
        }
        __syncthreads();
    }
    float tm = -INFINITY, nm = 0.0f;
    if (lane < n) {
        tm = thr ? thr[p0 + lane] : -INFINITY;
        nm = Xn[p0 + lane];
    } else {
        r2 = 0.0;
    }
    for (int o = 32; o > 0; o >>= 1) {
        r2 = fmax(r2, __shfl_xor(r2, o));
        tm = fmaxf(tm, __shfl_xor(tm, o));
        nm = fmaxf(nm, __shfl_xor(nm, o));
    }
    if (lane == 0) geo[t] = TileGeom{sqrt(r2) * (1.0 + 1e-9) + 1e-30, tm, nm};
}

// Row blocks b = TM_B q .. TM_B q + TM_B - 1 per workgroup q (row groups 4b ..
// 4b + 3 each), so that each tile's centre read serves 4 TM_B groups.  A
// block's mask words cover the tiles from tA(b) on (sym: 2b rounded down to a
// multiple of 64, the same for the TM_B blocks of a workgroup; else 0): bit
// (t - tA) of word w (w = the wave) is set when that wave must sweep tile t.
// sym: tiles before the block's own two are never set, its own two always
// are.  cnt[b] += tiles any wave needs, wcnt[b] += (wave, tile) sweeps (both
// start at zero).  The tiles are split in ranges of `span` (a multiple of
// 256) over gridDim.y, so that a sweep of few rows still fills the device.
// Without sym the tiles' own thresholds play no part (only the rows take
// survivors).
constexpr int TM_B = 4;
static_assert(64 % (2 * TM_B) == 0, "the blocks of a workgroup share their first mask word");

__device__ __forceinline__ int64_t tile_mask_base(int64_t b, int sym) { return sym ? (2 * b) & ~(int64_t)63 : 0; }

__global__ __launch_bounds__(256) void k_tile_mask(const float *__restrict__ cen_g, const TileGeom *__restrict__ geo_g,
                                                   int64_t ngroups, int64_t nblk, const float *__restrict__ cen_t,
                                                   const TileGeom *__restrict__ geo_t, int dp, int d,
                                                   int64_t ntiles, double g, int sym, int64_t span,
                                                   const int64_t *__restrict__ moff,
                                                   uint64_t *__restrict__ mask, int64_t *__restrict__ cnt,
                                                   int64_t *__restrict__ wcnt)
{
    constexpr int NG = 4 * TM_B;
    __shared__ __attribute__((aligned(16))) float ca[NG][128];
    __shared__ TileGeom sg[NG];
    __shared__ int wsum[TM_B][4], wwsum[TM_B][4];
    const int64_t b0 = (int64_t)blockIdx.x * TM_B, g0 = 4 * b0;
    const int nb = (int)min<int64_t>(TM_B, nblk - b0);
    const int ng = (int)min<int64_t>(NG, ngroups - g0);
    const int64_t tA = tile_mask_base(b0, sym);
    for (int e = threadIdx.x; e < NG * d; e += 256) {
        const int w = e / d, k = e % d;
        ca[w][k] = cen_g[(g0 + min(w, ng - 1)) * dp + k];
    }
    if (threadIdx.x < NG) sg[threadIdx.x] = geo_g[g0 + min((int)threadIdx.x, ng - 1)];
    __syncthreads();
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    int64_t total[TM_B], wtotal[TM_B];
#pragma unroll
    for (int i = 0; i < TM_B; ++i) total[i] = wtotal[i] = 0;
    const int64_t tbeg = tA + (int64_t)blockIdx.y * span, tend = min(ntiles, tbeg + span);
    for (int64_t base = tbeg; base < tend; base += 256) {
        const int64_t t = base + threadIdx.x;
        // squared centre distances to the NG groups in FP32, four coordinates
        // per load (rows are 16-byte aligned), each group's sum in coordinate
        // order
        float sw[NG];
#pragma unroll
        for (int w = 0; w < NG; ++w) sw[w] = 0.0f;
        const TileGeom gt = geo_t[min(t, ntiles - 1)];
        const float *ct = cen_t + min(t, ntiles - 1) * dp;
        int k = 0;
        for (; k + 4 <= d; k += 4) {
            const float4 c = *reinterpret_cast<const float4 *>(ct + k);
#pragma unroll
            for (int w = 0; w < NG; ++w) {
                const float4 q = *reinterpret_cast<const float4 *>(&ca[w][k]);
                float u = q.x - c.x;
                sw[w] = fmaf(u, u, sw[w]);
                u = q.y - c.y;
                sw[w] = fmaf(u, u, sw[w]);
                u = q.z - c.z;
                sw[w] = fmaf(u, u, sw[w]);
                u = q.w - c.w;
                sw[w] = fmaf(u, u, sw[w]);
            }
        }
        for (; k < d; ++k) {
            const float c = ct[k];
#pragma unroll
            for (int w = 0; w < NG; ++w) {
                const float u = ca[w][k] - c;
                sw[w] = fmaf(u, u, sw[w]);
            }
        }
        const int64_t wd = (base - tA) / 64 + wv;
#pragma unroll
        for (int i = 0; i < TM_B; ++i) {
            const int64_t b = b0 + i;
            const int64_t t0 = sym ? 2 * b : 0;
            const int nown = sym ? (int)min<int64_t>(2, ntiles - t0) : 0;
            const int ngb = (int)min<int64_t>(4, ngroups - 4 * b);
            uint64_t any = 0;
            int nw = 0;
#pragma unroll
            for (int w = 0; w < 4; ++w) {
                const int gi = 4 * i + w;
                bool keep = false;
                if (i < nb && w < ngb && t < ntiles && t >= t0) {
                    if (t < t0 + nown) {
                        keep = true;
                    } else {
                        // the test shrinks the centre distance by a relative
                        // 1e-5, above the FP32 rounding bound (d + 2) 2^-24
                        // for d <= 128
                        const TileGeom gr = sg[gi];
                        const double L = sqrt((double)sw[gi]) * (1.0 - 1e-5) - gr.r - gt.r;
                        const double bound = ((double)(sym ? fmaxf(gr.tmax, gt.tmax) : gr.tmax) +
                                              g * ((double)gr.nmax + (double)gt.nmax)) * (1.0 + 1e-6);
                        keep = !(L > 0.0 && L * L > bound);
                    }
                }
                const uint64_t bits = __ballot(keep);
                any |= bits;
                nw += __popcll(bits);
                if (i < nb && lane == 0 && tA + 64 * wd < ntiles) mask[(moff[b] + wd) * 4 + w] = bits;
            }
            if (lane == 0) {
                wsum[i][wv] = __popcll(any);
                wwsum[i][wv] = nw;
            }
        }
        __syncthreads();
#pragma unroll
        for (int i = 0; i < TM_B; ++i) {
            total[i] += wsum[i][0] + wsum[i][1] + wsum[i][2] + wsum[i][3];
            wtotal[i] += wwsum[i][0] + wwsum[i][1] + wwsum[i][2] + wwsum[i][3];
        }
        __syncthreads();
    }
    if (threadIdx.x < nb) {
#pragma unroll
        for (int i = 0; i < TM_B; ++i)
            if (i == (int)threadIdx.x) {
                atomicAdd((unsigned long long *)&cnt[b0 + i], (unsigned long long)total[i]);
                atomicAdd((unsigned long long *)&wcnt[b0 + i], (unsigned long long)wtotal[i]);
            }
    }
}

// Expands each block's masks into its list of entries (increasing tile
// order): tile | (wave mask << 27).
__global__ __launch_bounds__(64) void k_tile_list(const uint64_t *__restrict__ mask, const int64_t *__restrict__ moff,
                                                  int64_t ntiles, int sym, const int64_t *__restrict__ toff,
                                                  int32_t *__restrict__ tlist)
{
    const int64_t b = blockIdx.x, t0 = tile_mask_base(b, sym);
    const int64_t nw = (ntiles - t0 + 63) / 64;
    int64_t o = toff[b];
    const int lane = threadIdx.x;
    for (int64_t w = 0; w < nw; ++w) {
        const uint64_t *m = mask + (moff[b] + w) * 4;
        const uint64_t m0 = m[0], m1 = m[1], m2 = m[2], m3 = m[3], any = m0 | m1 | m2 | m3;
        if ((any >> lane) & 1ull) {
            const int32_t nib = (int32_t)(((m0 >> lane) & 1ull) | (((m1 >> lane) & 1ull) << 1) |
                                          (((m2 >> lane) & 1ull) << 2) | (((m3 >> lane) & 1ull) << 3));
            tlist[o + __popcll(any & ((1ull << lane) - 1ull))] = (int32_t)(t0 + 64 * w + lane) | (nib << TL_TILE_BITS);
        }
        o += __popcll(any);
    }
}

// Builds the tile lists of a sweep of M rows (FP32 coordinates Xr, stride
// dp, thresholds thr_r, FP32 norms Xn_r) over N points (Xp, thr_p, Xn_p):
// sym, the symmetric sweep of the point set against itself (rows = points),
// or the rows against every tile.  Returns false (no lists) when they do not
// apply.  Allocations go to tmp.
static bool build_tile_lists(const float *Xr, const float *thr_r, const float *Xn_r, int64_t M, const float *Xp,
                             const float *thr_p, const float *Xn_p, int64_t N, int dp, int d, bool sym,
                             int32_t *&tlist, int64_t *&toff, int64_t &kept, int64_t &kept_waves, int4 *&items,
                             int64_t &nitems, std::vector<void *> &tmp, hipStream_t s)
{
    static_assert(KB_M == 2 * KB_N && KB_M == 4 * 32, "a row block is two tiles and four waves of 32 rows");
    const int64_t ntiles = (N + KB_N - 1) / KB_N, nblk = (M + KB_M - 1) / KB_M, ngroups = (M + 31) / 32;
    if (!Xr || !Xp || M <= 0 || d > 128 || ntiles > TL_TILE_MASK) return false;
    auto ta = [&](size_t b) {
        void *p;
        HIPC(ws_alloc(&p, std::max<size_t>(b, 16), s));
        tmp.push_back(p);
        return p;
    };
    std::vector<int64_t> hmoff(nblk + 1);
    int64_t words = 0;
    for (int64_t b = 0; b < nblk; ++b) {
        hmoff[b] = words;
        words += (ntiles - (sym ? (2 * b) & ~(int64_t)63 : 0) + 63) / 64;
    }
    hmoff[nblk] = words;
    float *cen_t = (float *)ta(sizeof(float) * ntiles * dp);
    TileGeom *geo_t = (TileGeom *)ta(sizeof(TileGeom) * ntiles);
    float *cen_g = (float *)ta(sizeof(float) * ngroups * dp);
    TileGeom *geo_g = (TileGeom *)ta(sizeof(TileGeom) * ngroups);
    int64_t *moff = (int64_t *)ta(sizeof(int64_t) * (nblk + 1));
    uint64_t *mask = (uint64_t *)ta(sizeof(uint64_t) * words * 4);
    int64_t *cnt = (int64_t *)ta(sizeof(int64_t) * nblk);
    int64_t *wcnt = (int64_t *)ta(sizeof(int64_t) * nblk);
    toff = (int64_t *)ta(sizeof(int64_t) * (nblk + 1));
    HIPC(hipMemcpyAsync(moff, hmoff.data(), sizeof(int64_t) * (nblk + 1), hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(k_tile_geom<64>, dim3((unsigned)ntiles), dim3(64), 0, s, Xp, dp, d, N, thr_p, Xn_p, cen_t,
                       geo_t);
    hipLaunchKernelGGL(k_tile_geom<32>, dim3((unsigned)ngroups), dim3(64), 0, s, Xr, dp, d, M, thr_r, Xn_r, cen_g,
                       geo_g);
    const double g = 2.0 * (3.1 * ldexp(1.0, -16) + (4.0 * dp + 8.0) * ldexp(1.0, -24));
    // about 1024 workgroups or more: few row blocks split the tiles
    const int64_t nwg = (nblk + TM_B - 1) / TM_B, nchunk = (ntiles + 255) / 256;
    const int64_t nsplit = sym ? 1 : std::max<int64_t>(1, std::min<int64_t>(nchunk, 1024 / nwg));
    const int64_t span = (nchunk + nsplit - 1) / nsplit * 256;
    HIPC(hipMemsetAsync(cnt, 0, sizeof(int64_t) * nblk, s));
    HIPC(hipMemsetAsync(wcnt, 0, sizeof(int64_t) * nblk, s));
    hipLaunchKernelGGL(k_tile_mask, dim3((unsigned)nwg, (unsigned)nsplit), dim3(256), 0, s, cen_g, geo_g, ngroups,
                       nblk, cen_t, geo_t, dp, d, ntiles, g, sym ? 1 : 0, span, moff, mask, cnt, wcnt);
    HIPC(hipGetLastError());
    std::vector<int64_t> hc(nblk), ho(nblk + 1), hw(nblk);
    HIPC(hipMemcpyAsync(hc.data(), cnt, sizeof(int64_t) * nblk, hipMemcpyDeviceToHost, s));
    HIPC(hipMemcpyAsync(hw.data(), wcnt, sizeof(int64_t) * nblk, hipMemcpyDeviceToHost, s));
    HIPC(hipStreamSynchronize(s));
    kept_waves = 0;
    for (int64_t b = 0; b < nblk; ++b) kept_waves += hw[b];
    ho[0] = 0;
    for (int64_t b = 0; b < nblk; ++b) ho[b + 1] = ho[b] + hc[b];
    kept = ho[nblk];
    // Work items: the lists vary by more than 10x between row blocks (dense
    // regions keep many tiles), so each list is cut into pieces of at most
    // KNN_PIECE tiles and the pieces are launched longest first: the
    // workgroups that start last are the short ones, and no single list sets
    // the sweep's length.  A sweep of few rows takes shorter pieces (about
    // 2048 of them in all), so that it still fills the device.
    const int64_t piece = sym ? KNN_PIECE : std::max<int64_t>(64, std::min<int64_t>(KNN_PIECE, kept / 2048 + 1));
    std::vector<int4> hi;
    for (int64_t b = 0; b < nblk; ++b) {
        const int64_t c = hc[b];
        const int64_t np = (c + piece - 1) / piece;
        for (int64_t q = 0; q < np; ++q) {
            const int64_t a0 = c * q / np, a1 = c * (q + 1) / np;
            hi.push_back(int4{(int)b, (int)a0, (int)(a1 - a0), 0});
        }
    }
    std::stable_sort(hi.begin(), hi.end(), [](const int4 &x, const int4 &y) { return x.z > y.z; });
    nitems = (int64_t)hi.size();
    items = (int4 *)ta(sizeof(int4) * std::max<int64_t>(nitems, 1));
    if (nitems > 0) HIPC(hipMemcpyAsync(items, hi.data(), sizeof(int4) * nitems, hipMemcpyHostToDevice, s));
    tlist = (int32_t *)ta(sizeof(int32_t) * std::max<int64_t>(kept, 1));
    HIPC(hipMemcpyAsync(toff, ho.data(), sizeof(int64_t) * (nblk + 1), hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(k_tile_list, dim3((unsigned)nblk), dim3(64), 0, s, mask, moff, ntiles, sym ? 1 : 0, toff,
                       tlist);
    HIPC(hipGetLastError());
    HIPC(hipStreamSynchronize(s));          // the host tables are released on return
    return true;
}

void knn_candidates(const uint16_t *Qh, const uint16_t *Ql, const float *Qn, int64_t M,
                    const uint16_t *Xh, const uint16_t *Xl, const float *Xn, int64_t N, int dp,
                    bool exclude_self, bool start_local, int32_t *cand, float *thr,
                    int32_t *bad_rows, int32_t *bad_count, hipStream_t s, float *t_filter_ms,
                    int *n_filter, int *n_retry, const KnnSample *samp, std::vector<int32_t> *retry_rows,
                    const float *Xf, int d, int64_t *tiles_swept, int nsel)
{
    if (retry_rows) retry_rows->clear();
    if (tiles_swept) *tiles_swept = -1;
    if (t_filter_ms) *t_filter_ms = 0.f;
    if (n_filter) *n_filter = 0;
    if (n_retry) *n_retry = 0;
    if (M <= 0) return;
    dim3 grid((unsigned)((M + KB_M - 1) / KB_M)), block(256);
    int ex = exclude_self ? 1 : 0, sl = start_local ? 1 : 0;
    const int64_t ntiles = (N + KB_N - 1) / KB_N;
    if (dp > 128) {
        hipLaunchKernelGGL(k_knn_cand_wide, grid, block, 0, s, Qh, Ql, Qn, M, Xh, Xl, Xn, N, dp, ex, sl,
                           cand, thr);
        HIPC(hipGetLastError());
        return;
    }
    const bool have_samp = samp && samp->levels > 0 && ntiles > 4 * KNN_WIN;
    // new points against the set: thresholds from the strided samples
    const bool sampled = !exclude_self && !start_local && have_samp;
    if (!sampled && (!start_local || ntiles <= 4 * KNN_WIN)) {
        KNN_DISPATCH(list_sweep, s, Qh, Ql, Qn, M, Xh, Xl, Xn, N, ex, sl, (const int32_t *)nullptr, false, cand,
                     thr);
        return;
    }
    // the point set against itself with every row's segment in one buffer:
    // one triangular sweep (each unordered pair once); else row chunks
    const bool sym = exclude_self && Qh == Xh && M == N && (double)N * KNN_CAP * 8.0 <= 48.0 * (1ull << 30);
    const int64_t chunk = sym ? M : KNN_CHUNK;
    const int64_t mc = std::min<int64_t>(M, chunk);
    FilterBufs B;
    B.nsel = std::max(1, std::min(nsel, KNN_CAND));
    int32_t *retry, *over;
    HIPC(ws_alloc((void **)&B.ocnt, sizeof(int32_t) * mc, s));
    HIPC(ws_alloc((void **)&B.oe, sizeof(uint2) * mc * KNN_CAP, s));
    HIPC(ws_alloc((void **)&retry, sizeof(int32_t) * (M + 1), s));
    HIPC(ws_alloc((void **)&over, sizeof(int32_t) * (M + 1), s));
    HIPC(hipMemsetAsync(retry, 0, sizeof(int32_t), s));
    HIPC(hipMemsetAsync(over, 0, sizeof(int32_t), s));
    if (sampled) {
        sample_thresholds(dp, s, Qh, Ql, Qn, M, *samp, chunk, thr, B, cand);
    } else {
        // window threshold: thr = nsel-th approximate distance among the 4096
        // tree-order neighbours of the row's block, in three steps with the
        // same arithmetic: the nsel-th of the 4 tiles around the block's rows
        // (its own two and one on each side; every point passes at +inf)
        // bounds it; the threshold filter over the window at that bound keeps
        // every closer point (so at least those nsel); their nsel-th is the
        // exact window value (or a bound, when more than the capacity survive)
        hipLaunchKernelGGL(k_fill_f32, dim3((unsigned)((M + 255) / 256)), dim3(256), 0, s, thr, M, INFINITY);
        filter_select(dp, s, Qh, Ql, Qn, M, Xh, Xl, Xn, N, ex, chunk, thr, B, cand, nullptr, false, 4, nullptr);
        widen(thr, M, s);
        filter_select(dp, s, Qh, Ql, Qn, M, Xh, Xl, Xn, N, ex, chunk, thr, B, cand, nullptr, false, KNN_WIN,
                      nullptr);
        widen(thr, M, s);
    }
    // symmetric sweep: only the (row block, tile) pairs whose bounding balls
    // come within the thresholds
    std::vector<void *> ttmp;
    int32_t *tlist = nullptr;
    int64_t *toff = nullptr, kept = 0, kept_waves = 0, nitems = 0;
    int4 *items = nullptr;
    if (sym && !std::getenv("ASKIT_KNN_NO_SKIP") &&
        build_tile_lists(Xf, thr, Xn, N, Xf, thr, Xn, N, dp, d, true, tlist, toff, kept, kept_waves, items, nitems,
                         ttmp, s)) {
        if (tiles_swept) *tiles_swept = kept_waves;
    } else {
        tlist = nullptr;
        toff = nullptr;
        items = nullptr;
    }
    std::vector<hipEvent_t> ev;             // brackets of each filter launch (timing only)
    filter_select(dp, s, Qh, Ql, Qn, M, Xh, Xl, Xn, N, ex, chunk, thr, B, cand, retry, sym, 0,
                  t_filter_ms ? &ev : nullptr, tlist, toff, items, nitems);
    int32_t nretry = 0;
    HIPC(hipMemcpyAsync(&nretry, retry, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    HIPC(hipStreamSynchronize(s));
    if (t_filter_ms) {
        float tot = 0.f;
        for (size_t e = 0; e < ev.size(); e += 2) {
            float ms = 0.f;
            HIPC(hipEventElapsedTime(&ms, ev[e], ev[e + 1]));
            tot += ms;
        }
        for (hipEvent_t e : ev) (void)hipEventDestroy(e);
        *t_filter_ms = tot;
        if (n_filter) *n_filter = (int)(ev.size() / 2);
    }
    if (n_retry) *n_retry = nretry;
    if (retry_rows && nretry > 0) {
        retry_rows->resize(nretry);
        HIPC(hipMemcpyAsync(retry_rows->data(), retry + 1, sizeof(int32_t) * nretry, hipMemcpyDeviceToHost, s));
        HIPC(hipStreamSynchronize(s));
    }
    // rows whose output overflowed (their window bound was far above their
    // 64th distance)
    const int32_t *list = retry + 1;
    int32_t nlist = nretry;
    if (nretry > 0 && nretry <= mc && exclude_self && have_samp && Qh == Xh) {
        // the point set against itself: the sampled thresholds on compact
        // copies of the rows, then the filter over all points (one pass: the
        // rows fit the filter buffers)
        const int64_t n = nretry;
        uint16_t *Bh, *Bl;
        float *Bn, *tc;
        int32_t *cc;
        HIPC(ws_alloc((void **)&Bh, sizeof(uint16_t) * n * dp, s));
        HIPC(ws_alloc((void **)&Bl, sizeof(uint16_t) * n * dp, s));
        HIPC(ws_alloc((void **)&Bn, sizeof(float) * n, s));
        HIPC(ws_alloc((void **)&tc, sizeof(float) * n, s));
        HIPC(ws_alloc((void **)&cc, sizeof(int32_t) * n * KNN_CAND, s));
        // the rows in sweep (tree) order, so that the 32 rows of a wave lie
        // close together and their bounding balls skip most tiles
        {
            std::vector<int32_t> hl(n);
            HIPC(hipMemcpyAsync(hl.data(), retry + 1, sizeof(int32_t) * n, hipMemcpyDeviceToHost, s));
            HIPC(hipStreamSynchronize(s));
            std::sort(hl.begin(), hl.end());
            HIPC(hipMemcpyAsync(retry + 1, hl.data(), sizeof(int32_t) * n, hipMemcpyHostToDevice, s));
            HIPC(hipStreamSynchronize(s));
        }
        hipLaunchKernelGGL(k_gather_qrows, dim3((unsigned)n), dim3(128), 0, s, list, n, dp, Qh, Ql, Qn, thr, Bh, Bl,
                           Bn, tc);
        // seeded with the bound the selection left (the nsel-th of the
        // row's stored survivors, real points, widened)
        sample_thresholds(dp, s, Bh, Bl, Bn, n, *samp, n, tc, B, cc, true);
        // the filter over every point, only on the tiles the rows' sampled
        // thresholds can reach (the same survivors as the full sweep)
        std::vector<void *> rtmp;
        int32_t *rl = nullptr;
        int64_t *ro = nullptr, rkept = 0, rkw = 0, rni = 0;
        int4 *ri = nullptr;
        bool rlists = false;
        if (Xf && !std::getenv("ASKIT_KNN_NO_SKIP")) {
            float *Bf;
            HIPC(ws_alloc((void **)&Bf, sizeof(float) * n * dp, s));
            rtmp.push_back(Bf);
            gather_rows(Xf, list, n, dp, Bf, s);
            rlists = build_tile_lists(Bf, tc, Bn, n, Xf, nullptr, Xn, N, dp, d, false, rl, ro, rkept, rkw, ri, rni,
                                      rtmp, s);
        }
        filter_select(dp, s, Bh, Bl, Bn, n, Xh, Xl, Xn, N, 0, n, tc, B, cc, nullptr, false, 0, nullptr,
                      rlists ? rl : nullptr, rlists ? ro : nullptr, rlists ? ri : nullptr, rni);
        hipLaunchKernelGGL(k_scatter_retry, dim3((unsigned)((n + 3) / 4)), dim3(256), 0, s, n, list, cc, tc,
                           B.ocnt, KNN_CAP, cand, thr, over + 1, over);
        HIPC(hipGetLastError());
        HIPC(hipMemcpyAsync(&nlist, over, sizeof(int32_t), hipMemcpyDeviceToHost, s));
        HIPC(hipStreamSynchronize(s));
        list = over + 1;
        HIPC(ws_free(Bh, s));
        HIPC(ws_free(Bl, s));
        HIPC(ws_free(Bn, s));
        HIPC(ws_free(tc, s));
        HIPC(ws_free(cc, s));
        for (void *q : rtmp) HIPC(ws_free(q, s));
    }
    // the rest: list sweep over every point on the compacted rows, seeded with
    // the bound the selection left
    if (nlist > 0)
        KNN_DISPATCH(list_sweep, s, Qh, Ql, Qn, (int64_t)nlist, Xh, Xl, Xn, N, ex, sl, list, true, cand, thr);
    HIPC(ws_free(B.ocnt, s));
    HIPC(ws_free(B.oe, s));
    HIPC(ws_free(retry, s));
    HIPC(ws_free(over, s));
    for (void *p : ttmp) HIPC(ws_free(p, s));
    (void)bad_rows;
    (void)bad_count;
}

__global__ void k_stride_rows(const uint16_t *__restrict__ h, const uint16_t *__restrict__ l,
                              const float *__restrict__ n, int dp, int stride, int64_t rows,
                              uint16_t *__restrict__ oh, uint16_t *__restrict__ ol, float *__restrict__ on)
{
    const int cpr = dp / 8;                  // 16-byte chunks per row
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= rows * cpr) return;
    const int64_t r = i / cpr, c = i % cpr, src = r * stride;
    *reinterpret_cast<uint4 *>(oh + r * dp + 8 * c) = *reinterpret_cast<const uint4 *>(h + src * dp + 8 * c);
    *reinterpret_cast<uint4 *>(ol + r * dp + 8 * c) = *reinterpret_cast<const uint4 *>(l + src * dp + 8 * c);
    if (c == 0) on[r] = n[src];
}

void knn_build_sample(askit_handle *h, hipStream_t s)
{
    h->ksamp = KnnSample{};
    const int64_t N = h->N;
    const int dp = h->dp;
    if (dp > 128 || (N + KB_N - 1) / KB_N <= 4 * KNN_WIN) return;
    // coarsest stride 8^L: the fewest levels whose coarsest sample fits the
    // filter output (every point of it passes the first filter)
    int L = 1;
    int64_t st = 8;
    while ((N + st - 1) / st > KNN_CAP) {
        st *= 8;
        ++L;
    }
    if (L > KnnSample::MAXL) return;
    // one allocation for every level (rows of 2 dp bf16 values and one float)
    int64_t total = 0;
    for (int64_t t = st; t >= 8; t /= 8) total += (N + t - 1) / t;
    char *base = (char *)h->alloc((size_t)total * (4 * dp + 4) + 256 * 3 * L, false);
    auto take = [&](size_t b) {
        char *p = base;
        base += (b + 255) / 256 * 256;
        return p;
    };
    for (int lv = 0; lv < L; ++lv, st /= 8) {
        const int64_t rows = (N + st - 1) / st;              // positions st * r < N
        h->ksamp.h[lv] = (uint16_t *)take(sizeof(uint16_t) * rows * dp);
        h->ksamp.l[lv] = (uint16_t *)take(sizeof(uint16_t) * rows * dp);
        h->ksamp.n[lv] = (float *)take(sizeof(float) * rows);
        h->ksamp.rows[lv] = rows;
        const int64_t nthr = rows * (dp / 8);
        hipLaunchKernelGGL(k_stride_rows, dim3((unsigned)((nthr + 255) / 256)), dim3(256), 0, s, h->Xh, h->Xl,
                           h->Xn, dp, (int)st, rows, h->ksamp.h[lv], h->ksamp.l[lv], h->ksamp.n[lv]);
        HIPC(hipGetLastError());
    }
    h->ksamp.levels = L;
}

// ---------------------------------------------------------------- refine
__device__ __forceinline__ bool lt_di(double d1, int i1, double d2, int i2)
{
    return d1 < d2 || (d1 == d2 && i1 < i2);
}

// One wave per query row: exact distances of the 64 candidates (reference
// positions), sorted by (D, point id) with id = idmap[position]; the kappa
// first are written as point ids to output row rowmap[row] (identity when
// NULL); certificate against the approximate threshold.
// D(a, b) = sum_k (a_k - b_k)^2 in FP64, k increasing, no fused multiply-add
// (the canonical distance), for rows padded to dp (a multiple of 16): 64
// coordinates are loaded at a time, unconditionally (indices kept inside the
// padded row), before the chain runs over them.
__device__ __forceinline__ double canon_sqdist_rows(const float *__restrict__ a, const float *__restrict__ b, int d,
                                                    int dp)
{
#pragma clang fp contract(off)
    double s = 0.0;
    for (int k0 = 0; k0 < d; k0 += 64) {
        float4 xa[16], xb[16];
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            const int k = min(k0 + 4 * i, dp - 4);
            xa[i] = *reinterpret_cast<const float4 *>(a + k);
            xb[i] = *reinterpret_cast<const float4 *>(b + k);
        }
        const int kn = min(64, d - k0);
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            const float pa[4] = {xa[i].x, xa[i].y, xa[i].z, xa[i].w};
            const float pb[4] = {xb[i].x, xb[i].y, xb[i].z, xb[i].w};
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                if (4 * i + u < kn) {
                    const double t = (double)pa[u] - (double)pb[u];
                    s += t * t;
                }
            }
        }
    }
    return s;
}

__global__ __launch_bounds__(256) void k_knn_refine(const float *__restrict__ Q, int64_t M,
                                                    const float *__restrict__ X, int64_t N, int d,
                                                    int dp, int kappa,
                                                    const int32_t *__restrict__ cand,
                                                    const float *__restrict__ thr,
                                                    const float *__restrict__ Qn, double maxnorm,
                                                    double gamma, const int32_t *__restrict__ idmap,
                                                    const int32_t *__restrict__ rowmap,
                                                    int32_t *__restrict__ idx,
                                                    double *__restrict__ dist,
                                                    int32_t *__restrict__ bad_rows,
                                                    int32_t *__restrict__ bad_count,
                                                    float *__restrict__ tbound)
{
    // the row is the same for the whole wave (made explicit, so that the
    // query row's coordinates come through scalar loads)
    const int64_t row = __builtin_amdgcn_readfirstlane((int)(blockIdx.x * 4 + threadIdx.x / WAVE));
    int lane = threadIdx.x % WAVE;
    if (row >= M) return;
    int j = cand[row * KNN_CAND + lane];
    const bool valid = j >= 0 && j < N;
    // canonical distance of every lane's candidate (empty slots read row 0
    // and are dropped), 64 coordinates of loads in flight at a time
    const double Dc = canon_sqdist_rows(Q + row * dp, X + (int64_t)(valid ? j : 0) * dp, d, dp);
    double D = INFINITY;
    if (valid) {
        D = Dc;
        j = idmap[j];
    } else {
        j = 0x7fffffff;
    }
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
    const int64_t orow = rowmap ? rowmap[row] : row;
    if (lane < kappa) {
        idx[orow * kappa + lane] = j;
        dist[orow * kappa + lane] = D;
    }
    double Dk = __shfl(D, kappa - 1);
    double th = (double)thr[row];
    double E = gamma * ((double)Qn[row] + maxnorm);
    bool ok = isinf(th) || (Dk < th - E);
    if (!ok && lane == 0) {
        int p = atomicAdd(bad_count, 1);
        bad_rows[p] = (int32_t)row;
        // every true neighbour has an approximate distance <= Dk + E: the
        // threshold of the filtered fallback, rounded up to FP32
        const double b = Dk + E;
        float f = (float)b;
        if ((double)f < b) f = __uint_as_float(__float_as_uint(f) + 1u);   // next float up (b >= 0)
        tbound[row] = f;
    }
}

void knn_refine(const float *Q, int64_t M, const float *X, int64_t N, int d, int dp, int kappa,
                const int32_t *cand, const float *thr, const float *Qn, float maxnorm,
                const int32_t *idmap, const int32_t *rowmap, int32_t *idx, double *dist,
                int32_t *bad_rows, int32_t *bad_count, float *tbound, hipStream_t s)
{
    // |approx - exact| <= g (|q|^2 + |x|^2) with g = 3.1 2^-16 (hi/lo split) +
    // (4 dp + 8) 2^-24 (FP32 accumulation, norms, final combine); doubled.
    double g = 2.0 * (3.1 * ldexp(1.0, -16) + (4.0 * dp + 8.0) * ldexp(1.0, -24));
    hipLaunchKernelGGL(k_knn_refine, dim3((unsigned)((M + 3) / 4)), dim3(256), 0, s, Q, M, X, N, d,
                       dp, kappa, cand, thr, Qn, (double)maxnorm * (1.0 + 1e-5), g, idmap, rowmap, idx,
                       dist, bad_rows, bad_count, tbound);
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
                                                    const int32_t *__restrict__ idmap,
                                                    const int32_t *__restrict__ rowmap,
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
        const int id = idmap[j];
        if (!lt_di(D, id, md[kappa - 1], mi[kappa - 1])) continue;
        int p = kappa - 1;
        while (p > 0 && lt_di(D, id, md[p - 1], mi[p - 1])) {
            md[p] = md[p - 1];
            mi[p] = mi[p - 1];
            --p;
        }
        md[p] = D;
        mi[p] = id;
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
        const int64_t orow = rowmap ? rowmap[row] : row;
        idx[orow * kappa + tid] = li[tid];
        dist[orow * kappa + tid] = ld[tid];
    }
}

void knn_exact_rows(const float *Q, const float *X, int64_t N, int d, int dp, int kappa,
                    bool exclude_self, const int32_t *rows, int nrows, const int32_t *idmap,
                    const int32_t *rowmap, int32_t *idx, double *dist, hipStream_t s)
{
    if (nrows <= 0) return;
    if (kappa > KX_K) fail(ASKIT_ERR_UNSUPPORTED, "kappa above 64 is not supported");
    size_t sh = (size_t)KX_T * kappa * (sizeof(double) + sizeof(int));
    hipLaunchKernelGGL(k_knn_exact, dim3(nrows), dim3(KX_T), sh, s, Q, X, N, d, dp, kappa,
                       exclude_self ? 1 : 0, rows, idmap, rowmap, idx, dist);
    HIPC(hipGetLastError());
}

// ---------------------------------------------------------------- filtered fallback
// Threshold sweep for rows wider than 128 dimensions (dimension chunks of
// 128 through LDS, as k_knn_cand_wide): every point whose approximate
// distance to row i is at most T_i is appended to the row's segment.
__global__ __launch_bounds__(256) void k_knn_filter_wide(const uint16_t *__restrict__ Qh,
                                                         const uint16_t *__restrict__ Ql,
                                                         const float *__restrict__ Qn, int64_t M,
                                                         const uint16_t *__restrict__ Xh,
                                                         const uint16_t *__restrict__ Xl,
                                                         const float *__restrict__ Xn, int64_t N, int dp,
                                                         const float *__restrict__ Tin, int cap,
                                                         int32_t *__restrict__ ocnt, uint2 *__restrict__ oe)
{
    constexpr int KC = 128;
    constexpr int LDB = KC + 8;
    __shared__ __attribute__((aligned(16))) uint16_t sBh[KB_N * LDB];
    __shared__ __attribute__((aligned(16))) uint16_t sBl[KB_N * LDB];
    __shared__ float sBn[KB_N];
    const int tid = threadIdx.x, lane = tid % WAVE;
    const int wv = __builtin_amdgcn_readfirstlane(tid / WAVE);
    const int half = lane >> 5, l32 = lane & 31;
    const int64_t q0 = (int64_t)blockIdx.x * KB_M + wv * 32;
    const int64_t arow = q0 + l32;
    const bool aok = arow < M;
    float qn[16], thrv[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        int64_t row = q0 + 8 * (r / 4) + 4 * half + (r % 4);
        qn[r] = row < M ? Qn[row] : 0.0f;
        thrv[r] = row < M ? Tin[row] : -INFINITY;
    }
    const int64_t ntiles = (N + KB_N - 1) / KB_N;
    for (int64_t t = 0; t < ntiles; ++t) {
        const int64_t tbase = t * KB_N;
        f32x16 acc0 = {}, acc1 = {};
        for (int k0 = 0; k0 < dp; k0 += KC) {
            const int kc = min(KC, dp - k0);
            __syncthreads();
            for (int c = tid; c < KB_N * (KC / 8); c += 256) {
                int row = c / (KC / 8), off = (c % (KC / 8)) * 8;
                int64_t g = tbase + row;
                uint4 vh = {0, 0, 0, 0}, vl = {0, 0, 0, 0};
                if (g < N && off < kc) {
                    vh = *reinterpret_cast<const uint4 *>(Xh + g * dp + k0 + off);
                    vl = *reinterpret_cast<const uint4 *>(Xl + g * dp + k0 + off);
                }
                *reinterpret_cast<uint4 *>(&sBh[row * LDB + off]) = vh;
                *reinterpret_cast<uint4 *>(&sBl[row * LDB + off]) = vl;
            }
            if (k0 == 0 && tid < KB_N) {
                int64_t g = tbase + tid;
                sBn[tid] = g < N ? Xn[g] : 0.0f;
            }
            __syncthreads();
            for (int s = 0; s < kc / 16; ++s) {
                bf16x8 qa = aok ? ld_bf8(Qh + arow * dp + k0 + 16 * s + 8 * half) : bf16x8{};
                bf16x8 qb = aok ? ld_bf8(Ql + arow * dp + k0 + 16 * s + 8 * half) : bf16x8{};
                bf16x8 bh0 = ld_bf8(&sBh[l32 * LDB + 16 * s + 8 * half]);
                bf16x8 bl0 = ld_bf8(&sBl[l32 * LDB + 16 * s + 8 * half]);
                bf16x8 bh1 = ld_bf8(&sBh[(32 + l32) * LDB + 16 * s + 8 * half]);
                bf16x8 bl1 = ld_bf8(&sBl[(32 + l32) * LDB + 16 * s + 8 * half]);
                acc0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(qa, bh0, acc0, 0, 0, 0);
                acc1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(qa, bh1, acc1, 0, 0, 0);
                acc0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(qa, bl0, acc0, 0, 0, 0);
                acc1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(qa, bl1, acc1, 0, 0, 0);
                acc0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(qb, bh0, acc0, 0, 0, 0);
                acc1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(qb, bh1, acc1, 0, 0, 0);
            }
        }
        const float ny0 = sBn[l32], ny1 = sBn[32 + l32];
        const int64_t cA = tbase + l32, cB = cA + 32;
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int64_t qrow = q0 + 8 * (r / 4) + 4 * half + (r % 4);
            const float dA = fmaf(-2.0f, acc0[r], qn[r] + ny0);
            const float dB = fmaf(-2.0f, acc1[r], qn[r] + ny1);
            if (dA <= thrv[r] && cA < N) {
                int p = atomicAdd(&ocnt[qrow], 1);
                if (p < cap) oe[qrow * cap + p] = make_uint2(__float_as_uint(dA), (uint32_t)cA);
            }
            if (dB <= thrv[r] && cB < N) {
                int p = atomicAdd(&ocnt[qrow], 1);
                if (p < cap) oe[qrow * cap + p] = make_uint2(__float_as_uint(dB), (uint32_t)cB);
            }
        }
    }
}

__global__ void k_gather_qrows(const int32_t *__restrict__ rows, int64_t n, int dp,
                               const uint16_t *__restrict__ Qh, const uint16_t *__restrict__ Ql,
                               const float *__restrict__ Qn, const float *__restrict__ tb,
                               uint16_t *__restrict__ Bh, uint16_t *__restrict__ Bl, float *__restrict__ Bn,
                               float *__restrict__ Bt)
{
    const int64_t i = blockIdx.x;
    const int64_t r = rows[i];
    for (int k = threadIdx.x; k < dp; k += blockDim.x) {
        Bh[i * dp + k] = Qh[r * dp + k];
        Bl[i * dp + k] = Ql[r * dp + k];
    }
    if (threadIdx.x == 0) {
        Bn[i] = Qn[r];
        Bt[i] = tb[r];
    }
}

// One wave per fallback row: exact FP64 distances of the row's survivors,
// the kappa smallest (D, id) kept in a sorted 64-entry list (chunks of 64
// sorted, then merged by a bitonic half-cleaner); rows whose survivors did
// not fit are listed for the full scan.
__global__ __launch_bounds__(256) void k_knn_rerank(const int32_t *__restrict__ rows, int64_t n,
                                                    const float *__restrict__ Q, const float *__restrict__ X,
                                                    int d, int dp, int kappa, int excl, int cap,
                                                    const int32_t *__restrict__ ocnt,
                                                    const uint2 *__restrict__ oe,
                                                    const int32_t *__restrict__ idmap,
                                                    const int32_t *__restrict__ rowmap,
                                                    int32_t *__restrict__ idx, double *__restrict__ dist,
                                                    int32_t *__restrict__ over_rows,
                                                    int32_t *__restrict__ over_count)
{
    const int64_t i = (int64_t)blockIdx.x * 4 + threadIdx.x / WAVE;
    const int lane = threadIdx.x % WAVE;
    if (i >= n) return;
    const int64_t row = rows[i];
    const int cnt = ocnt[i];
    if (cnt > cap) {
        if (lane == 0) over_rows[atomicAdd(over_count, 1)] = (int32_t)row;
        return;
    }
    double bD = INFINITY;
    int bj = 0x7fffffff;
    for (int c0 = 0; c0 < cnt; c0 += 64) {
        double D = INFINITY;
        int j = 0x7fffffff;
        if (c0 + lane < cnt) {
            const int pos = (int)oe[i * cap + c0 + lane].y;
            if (!(excl && pos == row)) {
                D = canon_sqdist(Q + row * dp, X + (int64_t)pos * dp, d);
                j = idmap ? idmap[pos] : pos;
            }
        }
        // sort the chunk ascending
#pragma unroll
        for (int k = 2; k <= 64; k <<= 1) {
#pragma unroll
            for (int st = k >> 1; st > 0; st >>= 1) {
                double oD = __shfl_xor(D, st);
                int oj = __shfl_xor(j, st);
                bool up = (lane & k) == 0;
                bool lower = (lane & st) == 0;
                bool take = (lower == up) ? lt_di(oD, oj, D, j) : lt_di(D, j, oD, oj);
                if (take) { D = oD; j = oj; }
            }
        }
        // merge with the kept list: min against the reversed chunk, then clean
        double rD = __shfl(D, 63 - lane);
        int rj = __shfl(j, 63 - lane);
        if (lt_di(rD, rj, bD, bj)) { bD = rD; bj = rj; }
#pragma unroll
        for (int st = 32; st > 0; st >>= 1) {
            double oD = __shfl_xor(bD, st);
            int oj = __shfl_xor(bj, st);
            bool lower = (lane & st) == 0;
            bool take = lower ? lt_di(oD, oj, bD, bj) : lt_di(bD, bj, oD, oj);
            if (take) { bD = oD; bj = oj; }
        }
    }
    if (lane < kappa) {
        const int64_t orow = rowmap ? rowmap[row] : row;
        idx[orow * kappa + lane] = bj;
        dist[orow * kappa + lane] = bD;
    }
}

void knn_fallback(const float *Q, const uint16_t *Qh, const uint16_t *Ql, const float *Qn, const float *X,
                  const uint16_t *Xh, const uint16_t *Xl, const float *Xn, int64_t N, int d, int dp, int kappa,
                  bool exclude_self, const int32_t *rows, int nrows, const float *tbound, const int32_t *idmap,
                  const int32_t *rowmap, int32_t *idx, double *dist, hipStream_t s)
{
    if (nrows <= 0) return;
    constexpr int FCAP = 2048;
    std::vector<void *> tmp;
    auto ta = [&](size_t b) {
        void *p;
        HIPC(ws_alloc(&p, std::max<size_t>(b, 16), s));
        tmp.push_back(p);
        return p;
    };
    const int64_t n = nrows;
    uint16_t *Bh = (uint16_t *)ta(sizeof(uint16_t) * n * dp), *Bl = (uint16_t *)ta(sizeof(uint16_t) * n * dp);
    float *Bn = (float *)ta(sizeof(float) * n), *Bt = (float *)ta(sizeof(float) * n);
    int32_t *ocnt = (int32_t *)ta(sizeof(int32_t) * n);
    uint2 *oe = (uint2 *)ta(sizeof(uint2) * n * FCAP);
    int32_t *over = (int32_t *)ta(sizeof(int32_t) * (n + 1));
    hipLaunchKernelGGL(k_gather_qrows, dim3((unsigned)n), dim3(128), 0, s, rows, n, dp, Qh, Ql, Qn, tbound, Bh, Bl,
                       Bn, Bt);
    HIPC(hipMemsetAsync(ocnt, 0, sizeof(int32_t) * n, s));
    HIPC(hipMemsetAsync(over, 0, sizeof(int32_t), s));
    dim3 g((unsigned)((n + KB_M - 1) / KB_M)), block(256);
    if (dp > 128) {
        hipLaunchKernelGGL(k_knn_filter_wide, g, block, 0, s, Bh, Bl, Bn, n, Xh, Xl, Xn, N, dp, Bt, FCAP, ocnt,
                           oe);
    } else {
        // few rows: the points are split into column segments, one workgroup
        // each, appending to the rows' common outputs
        g.y = (unsigned)filter_segments(n, (N + KB_N - 1) / KB_N);
        KNN_DISPATCH(launch_filter, g, block, s, Bh, Bl, Bn, n, Xh, Xl, Xn, N, 0, 0, Bt, FCAP, ocnt, oe,
                     false);
    }
    HIPC(hipGetLastError());
    hipLaunchKernelGGL(k_knn_rerank, dim3((unsigned)((n + 3) / 4)), dim3(256), 0, s, rows, n, Q, X, d, dp, kappa,
                       exclude_self ? 1 : 0, FCAP, ocnt, oe, idmap, rowmap, idx, dist, over + 1, over);
    HIPC(hipGetLastError());
    int32_t nover = 0;
    HIPC(hipMemcpyAsync(&nover, over, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    HIPC(hipStreamSynchronize(s));
    knn_exact_rows(Q, X, N, d, dp, kappa, exclude_self, over + 1, nover, idmap, rowmap, idx, dist, s);
    for (void *p : tmp) HIPC(ws_free(p, s));
}

}  // namespace askit
