// Median-split binary tree on the GPU (Sec. 2.2, Fig. "The tree").
//
// A node with n > m points is split by: centre c (mean), x_l = the point
// farthest from c, x_r = the point farthest from x_l, projection p_i =
// (x_i - x_l).(x_r - x_l), and a median split: the ceil(n/2) smallest
// (p_i, i) go left, the rest right, each child keeping its points in the
// parent's order (which is increasing point id, by induction from the root).
// All values that decide the split are FP64 and computed in a fixed order,
// so the permutation is reproducible bit for bit:
//   - c: blocks of 64 consecutive points summed by pairwise halving within
//     a wave (lane t adds lane t+32, then t+16, ..., t+1), block sums added
//     in block order, divided by n;
//   - distances and projections: sums over increasing k without FMA;
//   - argmax ties go to the smaller point id;
//   - the median is found by an 8-pass radix select on an order-preserving
//     64-bit image of p, ties resolved by position (= point id order).
// The tree shape depends only on N and m, so every level's node ranges are
// known on the host before the level runs.
#include "askit_impl.h"

#include <algorithm>

namespace askit {

struct Split {
    int32_t lo, n;
};

struct BestD {
    double d;
    int32_t id;
    int32_t pad;
};

__device__ __forceinline__ bool better(double d1, int i1, double d2, int i2)
{
    return d1 > d2 || (d1 == d2 && i1 < i2);
}

// Coordinate sums of each 64-point block of a split (points in the split's
// order, those past its end counting as zero): lane k holds coordinate k of
// the block's points (one coalesced row load per point) and reduces them by
// pairwise halving, v_i + v_(i+o) for o = 32, 16, ..., 1, in registers.
__global__ __launch_bounds__(64) void k_block_sums(const float *__restrict__ X, int dp, int d,
                                                   const int32_t *__restrict__ perm,
                                                   const Split *__restrict__ sp, int maxblk,
                                                   double *__restrict__ bsum)
{
    const int b = blockIdx.x, q = blockIdx.y, lane = threadIdx.x;
    const Split s = sp[q];
    if (b * 64 >= s.n) return;
    const int np = min(64, s.n - b * 64);
    // rows past the end read a valid row and count as zero
    const int myid = perm[s.lo + b * 64 + (lane < np ? lane : 0)];
    double *out = bsum + ((int64_t)q * maxblk + b) * d;
    for (int k0 = 0; k0 < d; k0 += 64) {
        const int k = k0 + lane;
        const bool kin = k < d;
        // unconditional loads (the index clamped inside the padded row) keep
        // all 64 in flight; lanes past d are masked afterwards
        const int kc = min(k, dp - 1);
        float x[64];
#pragma unroll
        for (int i = 0; i < 64; ++i) {
            const int id = __builtin_amdgcn_readlane(myid, i);
            x[i] = X[(int64_t)id * dp + kc];
        }
        double v[64];
#pragma unroll
        for (int i = 0; i < 64; ++i) v[i] = (i < np && kin) ? (double)x[i] : 0.0;
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1)
#pragma unroll
            for (int i = 0; i < o; ++i) v[i] = v[i] + v[i + o];
        if (kin) out[k] = v[0];
    }
}

__global__ void k_centroid(const double *__restrict__ bsum, const Split *__restrict__ sp, int maxblk,
                           int d, double *__restrict__ cen)
{
    int q = blockIdx.x;
    Split s = sp[q];
    int nb = (s.n + 63) / 64;
    for (int k = threadIdx.x; k < d; k += blockDim.x) {
        const double *bs = bsum + (int64_t)q * maxblk * d + k;
        double acc = 0.0;
        int b = 0;
        // sixteen loads in flight, added in block order
        for (; b + 16 <= nb; b += 16) {
            double v[16];
#pragma unroll
            for (int u = 0; u < 16; ++u) v[u] = bs[(int64_t)(b + u) * d];
#pragma unroll
            for (int u = 0; u < 16; ++u) acc += v[u];
        }
        for (; b < nb; ++b) acc += bs[(int64_t)b * d];
        cen[(int64_t)q * d + k] = acc / (double)s.n;
    }
}

// Rows of 64 points staged through LDS: lane k loads coordinate k of each
// point (one coalesced row per instruction), so that lane i can then read
// point i's coordinates in increasing k.  Row stride 65 words: the transposed
// reads fall in distinct banks.
constexpr int TR_PAD = 65;

__device__ __forceinline__ void stage_rows(const float *__restrict__ X, int dp, int myid, int k0,
                                           float *rows)
{
    const int lane = threadIdx.x;
    // unconditional loads (index clamped inside the padded row: all 64 in
    // flight); coordinates past d are never read back
    const int kc = min(k0 + lane, dp - 1);
    float x[64];
#pragma unroll
    for (int i = 0; i < 64; ++i) {
        const int id = __builtin_amdgcn_readlane(myid, i);
        x[i] = X[(int64_t)id * dp + kc];
    }
#pragma unroll
    for (int i = 0; i < 64; ++i) rows[i * TR_PAD + lane] = x[i];
}

// Farthest point of each split from a reference, per 64-point chunk: the
// largest canonical distance D (ties to the smaller id).  mode 0: D(x, the
// split's centre) (FP64 centre); mode 1: D(x, x_ref[q]).
__global__ __launch_bounds__(64) void k_far_partial(const float *__restrict__ X, int dp, int d,
                                                    const int32_t *__restrict__ perm,
                                                    const Split *__restrict__ sp,
                                                    const double *__restrict__ cen,
                                                    const int32_t *__restrict__ ref, int mode,
                                                    int nchunk, BestD *__restrict__ part)
{
#pragma clang fp contract(off)
    __shared__ float rows[64 * TR_PAD];
    __shared__ double rv[64];
    const int c = blockIdx.x, q = blockIdx.y, lane = threadIdx.x;
    const Split s = sp[q];
    if (c * 64 >= s.n) return;
    const int np = min(64, s.n - c * 64);
    const int myid = perm[s.lo + c * 64 + (lane < np ? lane : 0)];
    const float *xr = mode == 0 ? nullptr : X + (int64_t)ref[q] * dp;
    double D = 0.0;
    for (int k0 = 0; k0 < d; k0 += 64) {
        const int k = k0 + lane;
        rv[lane] = k < d ? (mode == 0 ? cen[(int64_t)q * d + k] : (double)xr[k]) : 0.0;
        stage_rows(X, dp, myid, k0, rows);
        __syncthreads();
        const int kn = min(64, d - k0);
        for (int j = 0; j < kn; ++j) {
            const double t = (double)rows[lane * TR_PAD + j] - rv[j];
            D += t * t;
        }
        __syncthreads();
    }
    double bd = lane < np ? D : -1.0;
    int bi = lane < np ? myid : 0x7fffffff;
    for (int o = 32; o > 0; o >>= 1) {
        const double od = __shfl_xor(bd, o);
        const int oi = __shfl_xor(bi, o);
        if (better(od, oi, bd, bi)) { bd = od; bi = oi; }
    }
    if (lane == 0) part[(int64_t)q * nchunk + c] = BestD{bd, bi, 0};
}

__global__ void k_far_final(const BestD *__restrict__ part, const Split *__restrict__ sp, int nchunk,
                            int32_t *__restrict__ out)
{
    int q = blockIdx.x, lane = threadIdx.x;
    int nc = (sp[q].n + 63) / 64;
    double bd = -1.0;
    int bi = 0x7fffffff;
    for (int c = lane; c < nc; c += 64) {
        BestD b = part[(int64_t)q * nchunk + c];
        if (better(b.d, b.id, bd, bi)) { bd = b.d; bi = b.id; }
    }
    for (int o = 32; o > 0; o >>= 1) {
        double od = __shfl_xor(bd, o);
        int oi = __shfl_xor(bi, o);
        if (better(od, oi, bd, bi)) { bd = od; bi = oi; }
    }
    if (lane == 0) out[q] = bi;
}

// Split key of every point: p = (x - x_l) . (x_r - x_l) in FP64, k increasing,
// per 64-point chunk (rows staged as above).
__global__ __launch_bounds__(64) void k_project(const float *__restrict__ X, int dp, int d,
                                                const int32_t *__restrict__ perm,
                                                const Split *__restrict__ sp, const int32_t *__restrict__ L,
                                                const int32_t *__restrict__ Rr, uint64_t *__restrict__ key)
{
#pragma clang fp contract(off)
    __shared__ float rows[64 * TR_PAD];
    __shared__ double lv[64], bv[64];
    const int c = blockIdx.x, q = blockIdx.y, lane = threadIdx.x;
    const Split s = sp[q];
    if (c * 64 >= s.n) return;
    const int np = min(64, s.n - c * 64);
    const int myid = perm[s.lo + c * 64 + (lane < np ? lane : 0)];
    const float *xl = X + (int64_t)L[q] * dp;
    const float *xr = X + (int64_t)Rr[q] * dp;
    double acc = 0.0;
    for (int k0 = 0; k0 < d; k0 += 64) {
        const int k = k0 + lane;
        if (k < d) {
            lv[lane] = (double)xl[k];
            bv[lane] = (double)xr[k] - (double)xl[k];
        }
        stage_rows(X, dp, myid, k0, rows);
        __syncthreads();
        const int kn = min(64, d - k0);
        for (int j = 0; j < kn; ++j) {
            const double a = (double)rows[lane * TR_PAD + j] - lv[j];
            acc += a * bv[j];
        }
        __syncthreads();
    }
    if (lane < np) key[s.lo + c * 64 + lane] = dkey(acc);
}

// Radix select state per split: prefix of the pivot key, remaining rank.
struct Sel {
    uint64_t prefix;
    int64_t krem;
};

__global__ __launch_bounds__(256) void k_radix_hist(const uint64_t *__restrict__ key,
                                                    const Split *__restrict__ sp,
                                                    const Sel *__restrict__ sel, int shift,
                                                    uint32_t *__restrict__ hist)
{
    __shared__ uint32_t lh[256];
    int c = blockIdx.x, q = blockIdx.y, tid = threadIdx.x;
    Split s = sp[q];
    lh[tid] = 0;
    __syncthreads();
    uint64_t hm = shift >= 56 ? 0ull : (~0ull << (shift + 8));
    uint64_t pre = sel[q].prefix;
    for (int i = c * 1024 + tid; i < min(s.n, (c + 1) * 1024); i += 256) {
        uint64_t k = key[s.lo + i];
        if (((k ^ pre) & hm) == 0) atomicAdd(&lh[(k >> shift) & 255u], 1u);
    }
    __syncthreads();
    if (lh[tid]) atomicAdd(&hist[q * 256 + tid], lh[tid]);
}

// The digit of each split's median key, one wave per split: the 256 bins'
// counts, an exclusive prefix across the wave, and the first bin whose
// cumulative count passes the remaining rank; the histogram is cleared.
__global__ __launch_bounds__(64) void k_radix_pick(uint32_t *__restrict__ hist, Sel *__restrict__ sel, int nsp,
                                                   int shift)
{
    const int q = blockIdx.x, lane = threadIdx.x;
    if (q >= nsp) return;
    uint4 *hq = reinterpret_cast<uint4 *>(hist + (int64_t)q * 256);
    const uint4 c4 = hq[lane];                    // bins 4 lane .. 4 lane + 3
    const uint32_t cs[4] = {c4.x, c4.y, c4.z, c4.w};
    const uint32_t tot = cs[0] + cs[1] + cs[2] + cs[3];
    uint32_t inc = tot;
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t v = __shfl_up(inc, o);
        if (lane >= o) inc += v;
    }
    Sel st = sel[q];
    int64_t cum = (int64_t)(inc - tot);
    int dg = -1;
    int below = 0;
    for (int j = 0; j < 4; ++j) {
        if (dg < 0 && cum + cs[j] > st.krem) {
            dg = 4 * lane + j;
            below = (int)cum;
        }
        cum += cs[j];
    }
    const unsigned long long hit = __ballot(dg >= 0);
    if (hit) {
        const int src = __ffsll(hit) - 1;
        st.prefix |= (uint64_t)__shfl(dg, src) << shift;
        st.krem -= __shfl(below, src);
    }
    hq[lane] = make_uint4(0u, 0u, 0u, 0u);
    if (lane == 0) sel[q] = st;
}

struct PartCnt {
    int32_t less, eq;
};

// Block-wide exclusive prefix of two flags; returns totals in *tl, *te.
__device__ __forceinline__ void block_scan2(int fl, int fe, int &pl, int &pe, int &tl, int &te)
{
    __shared__ int wl[4], we[4];
    int tid = threadIdx.x, lane = tid % 64, w = tid / 64;
    uint64_t bl = __ballot(fl), be = __ballot(fe);
    uint64_t lt = lane ? (~0ull >> (64 - lane)) : 0ull;
    int il = __popcll(bl & lt), ie = __popcll(be & lt);
    if (lane == 0) {
        wl[w] = __popcll(bl);
        we[w] = __popcll(be);
    }
    __syncthreads();
    int ol = 0, oe = 0;
    tl = 0;
    te = 0;
    for (int v = 0; v < 4; ++v) {
        if (v < w) { ol += wl[v]; oe += we[v]; }
        tl += wl[v];
        te += we[v];
    }
    pl = ol + il;
    pe = oe + ie;
    __syncthreads();
}

__global__ __launch_bounds__(256) void k_part_count(const uint64_t *__restrict__ key,
                                                    const Split *__restrict__ sp,
                                                    const Sel *__restrict__ sel, int nchunk,
                                                    PartCnt *__restrict__ cnt)
{
    int c = blockIdx.x, q = blockIdx.y, tid = threadIdx.x;
    Split s = sp[q];
    int i = c * 256 + tid;
    uint64_t pv = sel[q].prefix;
    int fl = 0, fe = 0;
    if (i < s.n) {
        uint64_t k = key[s.lo + i];
        fl = k < pv;
        fe = k == pv;
    }
    int pl, pe, tl, te;
    block_scan2(fl, fe, pl, pe, tl, te);
    if (tid == 0) cnt[(int64_t)q * nchunk + c] = PartCnt{tl, te};
}

// Exclusive prefix of the chunks' (less, equal) counts of each split, one
// wave per split, 64 chunks at a time.
__global__ __launch_bounds__(64) void k_part_scan(PartCnt *__restrict__ cnt, const Split *__restrict__ sp, int nsp,
                                                  int nchunk)
{
    const int q = blockIdx.x, lane = threadIdx.x;
    if (q >= nsp) return;
    const int nc = (sp[q].n + 255) / 256;
    PartCnt *cq = cnt + (int64_t)q * nchunk;
    int al = 0, ae = 0;
    for (int c0 = 0; c0 < nc; c0 += 64) {
        const int c = c0 + lane;
        const PartCnt v = c < nc ? cq[c] : PartCnt{0, 0};
        int il = v.less, ie = v.eq;
        for (int o = 1; o < 64; o <<= 1) {
            const int a = __shfl_up(il, o), b = __shfl_up(ie, o);
            if (lane >= o) {
                il += a;
                ie += b;
            }
        }
        if (c < nc) cq[c] = PartCnt{al + il - v.less, ae + ie - v.eq};
        al += __shfl(il, 63);
        ae += __shfl(ie, 63);
    }
}

__global__ __launch_bounds__(256) void k_part_scatter(const uint64_t *__restrict__ key,
                                                      const int32_t *__restrict__ perm,
                                                      const Split *__restrict__ sp,
                                                      const Sel *__restrict__ sel, int nchunk,
                                                      const PartCnt *__restrict__ cnt,
                                                      int32_t *__restrict__ out)
{
    int c = blockIdx.x, q = blockIdx.y, tid = threadIdx.x;
    Split s = sp[q];
    int i = c * 256 + tid;
    uint64_t pv = sel[q].prefix;
    int64_t take = sel[q].krem + 1;
    int fl = 0, fe = 0;
    uint64_t k = 0;
    if (i < s.n) {
        k = key[s.lo + i];
        fl = k < pv;
        fe = k == pv;
    }
    int pl, pe, tl, te;
    block_scan2(fl, fe, pl, pe, tl, te);
    if (i >= s.n) return;
    PartCnt base = cnt[(int64_t)q * nchunk + c];
    int64_t lb = base.less + pl, eb = base.eq + pe;
    int64_t gb = i - lb - eb;
    int64_t nl = (s.n + 1) / 2;
    int64_t dst;
    if (fl) dst = lb + min(eb, take);
    else if (fe) dst = eb < take ? lb + eb : nl + gb + (eb - take);
    else dst = nl + gb + max((int64_t)0, eb - take);
    if (dst >= 0 && dst < s.n) out[s.lo + dst] = perm[s.lo + i];
}

__global__ void k_iota(int32_t *p, int64_t n)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = (int32_t)i;
}

__global__ void k_invert(const int32_t *__restrict__ p, int64_t n, int32_t *__restrict__ ip)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) ip[p[i]] = (int32_t)i;
}

// Median split of every node of a level by its keys: the ceil(n/2) smallest
// (key, position) go left, each side keeps the parent's order (radix select of
// the median key in 8 passes of 8 bits, then a stable partition).  perm is
// updated in place through pout; sel must hold (0, ceil(n/2) - 1) per split and
// hist must be zero.
static void median_split(const uint64_t *key, const Split *d_sp, int nsp, int maxn, Sel *sel, uint32_t *hist,
                         PartCnt *pc, int32_t *perm, int32_t *pout, int64_t N, hipStream_t s)
{
    const int nchunk = (maxn + 255) / 256;
    const int hchunk = (maxn + 1023) / 1024;
    for (int pass = 0; pass < 8; ++pass) {
        int shift = 56 - 8 * pass;
        hipLaunchKernelGGL(k_radix_hist, dim3(hchunk, nsp), dim3(256), 0, s, key, d_sp, sel, shift, hist);
        hipLaunchKernelGGL(k_radix_pick, dim3(nsp), dim3(64), 0, s, hist, sel, nsp, shift);
    }
    hipLaunchKernelGGL(k_part_count, dim3(nchunk, nsp), dim3(256), 0, s, key, d_sp, sel, nchunk, pc);
    hipLaunchKernelGGL(k_part_scan, dim3(nsp), dim3(64), 0, s, pc, d_sp, nsp, nchunk);
    HIPC(hipMemcpyAsync(pout, perm, sizeof(int32_t) * N, hipMemcpyDeviceToDevice, s));
    hipLaunchKernelGGL(k_part_scatter, dim3(nchunk, nsp), dim3(256), 0, s, key, perm, d_sp, sel, nchunk, pc,
                       pout);
    HIPC(hipGetLastError());
    HIPC(hipMemcpyAsync(perm, pout, sizeof(int32_t) * N, hipMemcpyDeviceToDevice, s));
}

// Splits every node of each level (host split tables, one vector per level,
// top-down) by the tree rule, permuting perm in place.  Every level's table
// is uploaded once; the levels then run back to back on the stream.
static void run_split_levels(const askit_handle *h, int32_t *perm, const std::vector<std::vector<Split>> &levels,
                             hipStream_t s)
{
    const int64_t N = h->N;
    const int d = h->d, dp = h->dp;
    std::vector<Split> all_sp;
    std::vector<Sel> all_sel;
    std::vector<size_t> off;
    std::vector<int> lmaxn;
    int64_t maxsp = 1, blk_total = 1, part_total = 1, pc_total = 1;
    for (const auto &lv : levels) {
        off.push_back(all_sp.size());
        int maxn = 0;
        for (const Split &sp : lv) {
            all_sp.push_back(sp);
            all_sel.push_back(Sel{0ull, (int64_t)((sp.n + 1) / 2 - 1)});
            maxn = std::max(maxn, (int)sp.n);
        }
        lmaxn.push_back(maxn);
        const int64_t nsp = (int64_t)lv.size();
        maxsp = std::max(maxsp, nsp);
        blk_total = std::max(blk_total, nsp * ((maxn + 63) / 64));
        part_total = std::max(part_total, nsp * ((maxn + 63) / 64));
        pc_total = std::max(pc_total, nsp * ((maxn + 255) / 256));
    }
    if (all_sp.empty()) return;
    std::vector<void *> tmp;
    struct Guard {
        std::vector<void *> &t;
        hipStream_t s;
        ~Guard() { for (void *p : t) (void)ws_free(p, s); }
    } guard{tmp, s};
    auto talloc = [&](size_t b) {
        void *p;
        HIPC(ws_alloc(&p, std::max<size_t>(b, 16), s));
        tmp.push_back(p);
        return p;
    };
    Split *d_sp = (Split *)talloc(sizeof(Split) * all_sp.size());
    Sel *sel = (Sel *)talloc(sizeof(Sel) * all_sel.size());
    double *bsum = (double *)talloc(sizeof(double) * blk_total * d + 64);
    double *cen = (double *)talloc(sizeof(double) * maxsp * d);
    BestD *part = (BestD *)talloc(sizeof(BestD) * part_total);
    int32_t *L = (int32_t *)talloc(sizeof(int32_t) * maxsp);
    int32_t *Rr = (int32_t *)talloc(sizeof(int32_t) * maxsp);
    uint64_t *key = (uint64_t *)talloc(sizeof(uint64_t) * N);
    uint32_t *hist = (uint32_t *)talloc(sizeof(uint32_t) * 256 * maxsp);
    PartCnt *pc = (PartCnt *)talloc(sizeof(PartCnt) * pc_total);
    int32_t *pout = (int32_t *)talloc(sizeof(int32_t) * N);
    HIPC(hipMemsetAsync(hist, 0, sizeof(uint32_t) * 256 * maxsp, s));
    HIPC(hipMemcpyAsync(d_sp, all_sp.data(), sizeof(Split) * all_sp.size(), hipMemcpyHostToDevice, s));
    HIPC(hipMemcpyAsync(sel, all_sel.data(), sizeof(Sel) * all_sel.size(), hipMemcpyHostToDevice, s));
    HIPC(hipStreamSynchronize(s));              // the host tables are released on return

    for (size_t l = 0; l < levels.size(); ++l) {
        const int nsp = (int)levels[l].size();
        if (nsp == 0) continue;
        const Split *lsp = d_sp + off[l];
        Sel *lsel = sel + off[l];
        const int maxn = lmaxn[l];
        const int maxblk = (maxn + 63) / 64;
        const int nch = (maxn + 63) / 64;
        hipLaunchKernelGGL(k_block_sums, dim3(maxblk, nsp), dim3(64), 0, s, h->Xo, dp, d, perm, lsp, maxblk,
                           bsum);
        hipLaunchKernelGGL(k_centroid, dim3(nsp), dim3(std::min(256, round_up(d, 64))), 0, s, bsum, lsp, maxblk,
                           d, cen);
        hipLaunchKernelGGL(k_far_partial, dim3(nch, nsp), dim3(64), 0, s, h->Xo, dp, d, perm, lsp, cen,
                           (const int32_t *)nullptr, 0, nch, part);
        hipLaunchKernelGGL(k_far_final, dim3(nsp), dim3(64), 0, s, part, lsp, nch, L);
        hipLaunchKernelGGL(k_far_partial, dim3(nch, nsp), dim3(64), 0, s, h->Xo, dp, d, perm, lsp, cen, L, 1,
                           nch, part);
        hipLaunchKernelGGL(k_far_final, dim3(nsp), dim3(64), 0, s, part, lsp, nch, Rr);
        hipLaunchKernelGGL(k_project, dim3(nch, nsp), dim3(64), 0, s, h->Xo, dp, d, perm, lsp, L, Rr, key);
        median_split(key, lsp, nsp, maxn, lsel, hist, pc, perm, pout, N, s);
    }
}

void build_tree(askit_handle *h, hipStream_t s)
{
    const int64_t N = h->N;
    unsigned nb = (unsigned)((N + 255) / 256);
    hipLaunchKernelGGL(k_iota, dim3(nb), dim3(256), 0, s, h->perm, N);
    HIPC(hipGetLastError());
    std::vector<std::vector<Split>> levels;
    for (const auto &lv : h->level_nodes) {
        levels.emplace_back();
        for (int a : lv) {
            const Node &nd = h->nodes[a];
            if (nd.left >= 0) levels.back().push_back(Split{nd.lo, nd.hi - nd.lo});
        }
    }
    run_split_levels(h, h->perm, levels, s);
    hipLaunchKernelGGL(k_invert, dim3(nb), dim3(256), 0, s, h->perm, N, h->iperm);
    HIPC(hipGetLastError());
}

// Finer order of the points for the neighbour search: the tree's leaves split
// further by the same rule until every cell holds at most mfine points.  It
// refines the tree order (each leaf keeps its range), so cells of consecutive
// positions are spatially compact: the sweep's tiles and row blocks then have
// small bounding balls and far pairs of them are skipped.  Only the search
// uses it (its results are point ids and exact distances).
void build_fine_order(const askit_handle *h, int mfine, int32_t *perm_f, hipStream_t s)
{
    HIPC(hipMemcpyAsync(perm_f, h->perm, sizeof(int32_t) * h->N, hipMemcpyDeviceToDevice, s));
    std::vector<std::vector<Split>> levels;
    std::vector<Split> cur;
    for (int a : h->leaves) {
        const Node &nd = h->nodes[a];
        if (nd.hi - nd.lo > mfine) cur.push_back(Split{nd.lo, nd.hi - nd.lo});
    }
    while (!cur.empty()) {
        levels.push_back(cur);
        std::vector<Split> nxt;
        for (const Split &sp : cur) {
            const int32_t nl = (sp.n + 1) / 2;
            if (nl > mfine) nxt.push_back(Split{sp.lo, nl});
            if (sp.n - nl > mfine) nxt.push_back(Split{sp.lo + nl, sp.n - nl});
        }
        cur.swap(nxt);
    }
    run_split_levels(h, perm_f, levels, s);
}

// ---------------------------------------------------------------- pruning diagnostic
// Nodes visited by the traversal of Alg. 4 per target under the neighbour rule
// (Eq. e:prune) and under distance pruning (prune alpha when the target lies
// outside the ball around the node's centroid that holds all its points), the
// comparison of Table t:prune.  Centroids use the tree's blocked summation
// over each node's points (increasing id); the ball test compares squared
// distances, D(x, c) > R^2, with R^2 = max D(x_j, c) over the node.
__global__ __launch_bounds__(256) void k_node_r2(const float *__restrict__ X, int dp, int d,
                                                 const int32_t *__restrict__ perm, const Split *__restrict__ sp,
                                                 const int32_t *__restrict__ ids, const double *__restrict__ cen,
                                                 double *__restrict__ r2)
{
    __shared__ double sm[256];
    const int q = blockIdx.x;
    const Split s = sp[q];
    const int a = ids[q];
    double m = 0.0;
    for (int i = threadIdx.x; i < s.n; i += 256)
        m = fmax(m, canon_sqdist_c(X + (int64_t)perm[s.lo + i] * dp, cen + (int64_t)q * d, d));
    sm[threadIdx.x] = m;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) sm[threadIdx.x] = fmax(sm[threadIdx.x], sm[threadIdx.x + o]);
        __syncthreads();
    }
    if (threadIdx.x == 0) r2[a] = sm[0];
}

__global__ void k_scatter_cen(const double *__restrict__ cen_q, const int32_t *__restrict__ ids, int nq, int d,
                              double *__restrict__ cen)
{
    const int q = blockIdx.x;
    if (q >= nq) return;
    for (int k = threadIdx.x; k < d; k += blockDim.x) cen[(int64_t)ids[q] * d + k] = cen_q[(int64_t)q * d + k];
}

__global__ __launch_bounds__(128) void k_prune_visits(const float *__restrict__ X, int dp, int d, int64_t N,
                                                      const Node *__restrict__ nodes, const int32_t *__restrict__ iperm,
                                                      const int32_t *__restrict__ knn_idx, int kappa,
                                                      const double *__restrict__ cen, const double *__restrict__ r2,
                                                      int32_t *__restrict__ vk, int32_t *__restrict__ vd)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    int32_t nb[65];
    nb[0] = iperm[i];
    for (int t = 0; t < kappa; ++t) nb[1 + t] = iperm[knn_idx[i * kappa + t]];
    const int nnb = kappa + 1;
    const float *x = X + i * dp;
    int32_t stk[128];
    for (int rule = 0; rule < 2; ++rule) {
        int top = 0, v = 0;
        stk[top++] = 0;
        while (top > 0) {
            const int a = stk[--top];
            const Node nd = nodes[a];
            ++v;
            bool prune;
            if (rule == 0) {
                bool has = false;
                for (int q = 0; q < nnb; ++q) has |= nb[q] >= nd.lo && nb[q] < nd.hi;
                prune = !has;
            } else {
                prune = canon_sqdist_c(x, cen + (int64_t)a * d, d) > r2[a];
            }
            if (prune || nd.left < 0) continue;
            stk[top++] = nd.right;
            stk[top++] = nd.left;
        }
        (rule == 0 ? vk : vd)[i] = v;
    }
}

void prune_visits(const askit_handle *h, int32_t *vk, int32_t *vd, hipStream_t s)
{
    const int d = h->d, dp = h->dp;
    const int64_t nn = (int64_t)h->nodes.size();
    std::vector<void *> tmp;
    struct Guard {
        std::vector<void *> &t;
        hipStream_t s;
        ~Guard() { for (void *p : t) (void)ws_free(p, s); }
    } guard{tmp, s};
    auto ta = [&](size_t b) {
        void *p;
        HIPC(ws_alloc(&p, std::max<size_t>(b, 16), s));
        tmp.push_back(p);
        return p;
    };
    int64_t maxq = 1;
    for (auto &lv : h->level_nodes) maxq = std::max<int64_t>(maxq, (int64_t)lv.size());
    const int64_t blk_total = (h->N + 63) / 64 + 2 * maxq;
    Split *d_sp = (Split *)ta(sizeof(Split) * maxq);
    int32_t *d_ids = (int32_t *)ta(sizeof(int32_t) * maxq);
    double *bsum = (double *)ta(sizeof(double) * blk_total * d + 64);
    double *cen_q = (double *)ta(sizeof(double) * maxq * d);
    double *cen = (double *)ta(sizeof(double) * nn * d);
    double *r2 = (double *)ta(sizeof(double) * nn);
    std::vector<Split> hsp;
    std::vector<int32_t> hids;
    for (const auto &lv : h->level_nodes) {
        hsp.clear();
        hids.clear();
        int maxn = 0;
        for (int a : lv) {
            const Node &nd = h->nodes[a];
            hsp.push_back(Split{nd.lo, nd.hi - nd.lo});
            hids.push_back(a);
            maxn = std::max(maxn, nd.hi - nd.lo);
        }
        const int nq = (int)hsp.size();
        if (nq == 0) continue;
        HIPC(hipMemcpyAsync(d_sp, hsp.data(), sizeof(Split) * nq, hipMemcpyHostToDevice, s));
        HIPC(hipMemcpyAsync(d_ids, hids.data(), sizeof(int32_t) * nq, hipMemcpyHostToDevice, s));
        const int maxblk = (maxn + 63) / 64;
        hipLaunchKernelGGL(k_block_sums, dim3(maxblk, nq), dim3(64), 0, s, h->Xo, dp, d, h->perm, d_sp, maxblk, bsum);
        hipLaunchKernelGGL(k_centroid, dim3(nq), dim3(std::min(256, round_up(d, 64))), 0, s, bsum, d_sp, maxblk, d,
                           cen_q);
        hipLaunchKernelGGL(k_node_r2, dim3(nq), dim3(256), 0, s, h->Xo, dp, d, h->perm, d_sp, d_ids, cen_q, r2);
        hipLaunchKernelGGL(k_scatter_cen, dim3(nq), dim3(64), 0, s, cen_q, d_ids, nq, d, cen);
        HIPC(hipGetLastError());
        HIPC(hipStreamSynchronize(s));          // host tables are reused by the next level
    }
    hipLaunchKernelGGL(k_prune_visits, dim3((unsigned)((h->N + 127) / 128)), dim3(128), 0, s, h->Xo, dp, d, h->N,
                       h->d_nodes, h->iperm, h->knn_idx, h->kappa, cen, r2, vk, vd);
    HIPC(hipGetLastError());
    HIPC(hipStreamSynchronize(s));
}

// ---------------------------------------------------------------- approximate neighbours
// Greedy search with random projection trees (Sec. 2.2, "Computing nearest
// neighbors"): each iteration builds a tree whose nodes split at the median of
// the points' projections on a random direction, gives every point the
// candidates of its leaf by exhaustive search, keeps each point's kappa best
// (distance, id) pairs seen so far, and discards the tree.
//
// Direction of a node: coordinate k has sign -1 when bit (k mod 64) of output
// floor(k / 64) of a SplitMix64 stream (Steele, Lea, Flood 2014) is set, +1
// otherwise.  The stream state starts at seed XOR (key * golden), key =
// ((iteration + 1) << 53) XOR (level << 48) XOR path; output t =
// mix(state + (t + 1) * golden).  The projection sum_k sign_k x_k is added in
// FP64 in increasing k, so the splits (median by (projection, position), as
// the tree rule) are reproducible bit for bit.
namespace {

constexpr uint64_t RP_GOLDEN = 0x9E3779B97F4A7C15ull;

__device__ __forceinline__ uint64_t rp_out(uint64_t base, uint64_t t)
{
    uint64_t z = base + (t + 1) * RP_GOLDEN;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

}  // namespace

__global__ void k_rp_project(const float *__restrict__ X, int dp, int d, const int32_t *__restrict__ perm,
                             const Split *__restrict__ sp, const uint64_t *__restrict__ sbase,
                             uint64_t *__restrict__ key)
{
#pragma clang fp contract(off)
    const int c = blockIdx.x, q = blockIdx.y;
    const Split s = sp[q];
    const int i = c * 256 + threadIdx.x;
    if (i >= s.n) return;
    const float *x = X + (int64_t)perm[s.lo + i] * dp;
    const uint64_t base = sbase[q];
    double acc = 0.0;
    uint64_t z = 0;
    for (int k = 0; k < d; ++k) {
        if ((k & 63) == 0) z = rp_out(base, (uint64_t)(k >> 6));
        const double v = (double)x[k];
        acc = ((z >> (k & 63)) & 1ull) ? acc - v : acc + v;
    }
    key[s.lo + i] = dkey(acc);
}

__global__ void k_rp_init(int32_t *__restrict__ idx, double *__restrict__ dist, int64_t n)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    idx[t] = -1;
    dist[t] = __longlong_as_double(0x7ff0000000000000ll);   // +inf: empty slot
}

// One workgroup per leaf; each thread merges the other points of the leaf
// into one point's list (canonical FP64 distances, order (distance, id)).
__global__ __launch_bounds__(256) void k_rp_leaf_search(const float *__restrict__ X, int dp, int d,
                                                        const int32_t *__restrict__ perm,
                                                        const Split *__restrict__ leaves, int kappa,
                                                        int32_t *__restrict__ idx, double *__restrict__ dist)
{
    const Split lf = leaves[blockIdx.x];
    for (int ii = threadIdx.x; ii < lf.n; ii += blockDim.x) {
        const int32_t i = perm[lf.lo + ii];
        int32_t li[64];
        double ld[64];
        for (int t = 0; t < kappa; ++t) {
            li[t] = idx[(int64_t)i * kappa + t];
            ld[t] = dist[(int64_t)i * kappa + t];
        }
        const float *xi = X + (int64_t)i * dp;
        for (int jj = 0; jj < lf.n; ++jj) {
            if (jj == ii) continue;
            const int32_t j = perm[lf.lo + jj];
            const double D = canon_sqdist(xi, X + (int64_t)j * dp, d);
            const double wd = ld[kappa - 1];
            if (!(D < wd || (D == wd && j < li[kappa - 1]))) continue;
            bool dup = false;
            for (int t = 0; t < kappa; ++t) dup |= li[t] == j;
            if (dup) continue;
            int q = kappa - 1;
            while (q > 0 && (ld[q - 1] > D || (ld[q - 1] == D && li[q - 1] > j))) {
                ld[q] = ld[q - 1];
                li[q] = li[q - 1];
                --q;
            }
            ld[q] = D;
            li[q] = j;
        }
        for (int t = 0; t < kappa; ++t) {
            idx[(int64_t)i * kappa + t] = li[t];
            dist[(int64_t)i * kappa + t] = ld[t];
        }
    }
}

void rp_knn(const float *Xo, int64_t N, int d, int dp, int kappa, int leaf, int iters, uint64_t seed,
            int32_t *idx, double *dist, hipStream_t s)
{
    // tree shape (depends on N and the leaf size only), breadth first
    struct RpNode {
        int32_t lo, n, level;
        int64_t path;
    };
    std::vector<RpNode> nodes{RpNode{0, (int32_t)N, 0, 0}};
    for (size_t a = 0; a < nodes.size(); ++a) {
        const RpNode nd = nodes[a];
        if (nd.n <= leaf) continue;
        const int32_t nl = (nd.n + 1) / 2;
        nodes.push_back(RpNode{nd.lo, nl, nd.level + 1, nd.path << 1});
        nodes.push_back(RpNode{nd.lo + nl, nd.n - nl, nd.level + 1, (nd.path << 1) | 1});
    }
    int depth = 0, minleaf = (int)N;
    for (auto &nd : nodes) depth = std::max(depth, (int)nd.level);
    std::vector<std::vector<int>> lev(depth + 1);
    std::vector<Split> hleaves;
    for (size_t a = 0; a < nodes.size(); ++a) {
        lev[nodes[a].level].push_back((int)a);
        if (nodes[a].n <= leaf) {
            hleaves.push_back(Split{nodes[a].lo, nodes[a].n});
            minleaf = std::min(minleaf, (int)nodes[a].n);
        }
    }
    if (minleaf - 1 < kappa)
        fail(ASKIT_ERR_INVALID_ARG, "leaf size too small: every leaf must hold more than kappa points");
    std::vector<void *> tmp;
    struct Guard {
        std::vector<void *> &t;
        hipStream_t s;
        ~Guard() { for (void *p : t) (void)ws_free(p, s); }
    } guard{tmp, s};
    auto ta = [&](size_t b) {
        void *p;
        HIPC(ws_alloc(&p, std::max<size_t>(b, 16), s));
        tmp.push_back(p);
        return p;
    };
    int64_t maxsp = 1;
    for (auto &l : lev) maxsp = std::max<int64_t>(maxsp, (int64_t)l.size());
    int64_t chunk_total = (N + 255) / 256 + 2 * maxsp;
    int32_t *perm = (int32_t *)ta(sizeof(int32_t) * N);
    int32_t *pout = (int32_t *)ta(sizeof(int32_t) * N);
    uint64_t *key = (uint64_t *)ta(sizeof(uint64_t) * N);
    Split *d_sp = (Split *)ta(sizeof(Split) * maxsp);
    uint64_t *d_base = (uint64_t *)ta(sizeof(uint64_t) * maxsp);
    Sel *sel = (Sel *)ta(sizeof(Sel) * maxsp);
    uint32_t *hist = (uint32_t *)ta(sizeof(uint32_t) * 256 * maxsp);
    PartCnt *pc = (PartCnt *)ta(sizeof(PartCnt) * chunk_total);
    Split *d_leaves = (Split *)ta(sizeof(Split) * hleaves.size());
    HIPC(hipMemsetAsync(hist, 0, sizeof(uint32_t) * 256 * maxsp, s));
    HIPC(hipMemcpyAsync(d_leaves, hleaves.data(), sizeof(Split) * hleaves.size(), hipMemcpyHostToDevice, s));
    const int64_t tot = N * kappa;
    hipLaunchKernelGGL(k_rp_init, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, idx, dist, tot);
    HIPC(hipGetLastError());
    const unsigned nb = (unsigned)((N + 255) / 256);
    std::vector<Split> hsp;
    std::vector<Sel> hsel;
    std::vector<uint64_t> hbase;
    for (int it = 0; it < iters; ++it) {
        hipLaunchKernelGGL(k_iota, dim3(nb), dim3(256), 0, s, perm, N);
        for (int l = 0; l <= depth; ++l) {
            hsp.clear();
            hsel.clear();
            hbase.clear();
            int maxn = 0;
            for (int a : lev[l]) {
                const RpNode &nd = nodes[a];
                if (nd.n <= leaf) continue;
                hsp.push_back(Split{nd.lo, nd.n});
                hsel.push_back(Sel{0ull, (int64_t)((nd.n + 1) / 2 - 1)});
                const uint64_t k = ((uint64_t)(it + 1) << 53) ^ ((uint64_t)nd.level << 48) ^ (uint64_t)nd.path;
                hbase.push_back(seed ^ (k * RP_GOLDEN));
                maxn = std::max(maxn, (int)nd.n);
            }
            const int nsp = (int)hsp.size();
            if (nsp == 0) continue;
            HIPC(hipMemcpyAsync(d_sp, hsp.data(), sizeof(Split) * nsp, hipMemcpyHostToDevice, s));
            HIPC(hipMemcpyAsync(sel, hsel.data(), sizeof(Sel) * nsp, hipMemcpyHostToDevice, s));
            HIPC(hipMemcpyAsync(d_base, hbase.data(), sizeof(uint64_t) * nsp, hipMemcpyHostToDevice, s));
            hipLaunchKernelGGL(k_rp_project, dim3((maxn + 255) / 256, nsp), dim3(256), 0, s, Xo, dp, d, perm, d_sp,
                               d_base, key);
            median_split(key, d_sp, nsp, maxn, sel, hist, pc, perm, pout, N, s);
            HIPC(hipStreamSynchronize(s));   // the host split tables are reused by the next level
        }
        hipLaunchKernelGGL(k_rp_leaf_search, dim3((unsigned)hleaves.size()), dim3(256), 0, s, Xo, dp, d, perm,
                           d_leaves, kappa, idx, dist);
        HIPC(hipGetLastError());
    }
    HIPC(hipStreamSynchronize(s));
}

}  // namespace askit
