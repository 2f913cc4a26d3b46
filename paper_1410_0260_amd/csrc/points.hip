// Point-array preparation: strided copy with zero padding, bf16 hi/lo split
// with FP32 norms, and row gathers.
#include "askit_impl.h"

#include <cstring>

namespace askit {

__global__ void k_pack_points(const float *__restrict__ X, int64_t N, int d, int64_t ldx, int dp,
                              float *__restrict__ out, int32_t *bad)
{
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t row = t / dp;
    int k = (int)(t - row * dp);
    if (row >= N) return;
    float v = 0.0f;
    if (k < d) {
        v = X[row * ldx + k];
        if (!isfinite(v)) atomicOr(bad, 1);
    }
    out[row * dp + k] = v;
}

void pack_points(const float *X, int64_t N, int d, int64_t ldx, int dp, float *out, int32_t *bad,
                 hipStream_t s)
{
    int64_t total = N * dp;
    hipLaunchKernelGGL(k_pack_points, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, X, N,
                       d, ldx, dp, out, bad);
    HIPC(hipGetLastError());
}

// Round-to-nearest-even FP32 -> bf16 (finite inputs).
__device__ __forceinline__ uint16_t f2bf(float x)
{
    uint32_t u = __float_as_uint(x);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

// x = hi + lo + e with hi = bf16(x), lo = bf16(x - hi): |e| <= 2^-16 |x|.
// One wave per row, lane k holding x_k (64 coordinates at a time); nrm = the
// FP32 sum of squares s = fma(x_k, x_k, s) in increasing k, which every lane
// forms from the broadcast coordinates (rows are padded to 16 coordinates).
__global__ __launch_bounds__(256) void k_split_bf16(const float *__restrict__ X, int64_t N, int dp,
                                                    uint16_t *__restrict__ hi, uint16_t *__restrict__ lo,
                                                    float *__restrict__ nrm)
{
    const int64_t row = (int64_t)blockIdx.x * (blockDim.x / WAVE) + threadIdx.x / WAVE;
    const int lane = threadIdx.x % WAVE;
    if (row >= N) return;
    const float *x = X + row * dp;
    float s = 0.0f;
    for (int k0 = 0; k0 < dp; k0 += WAVE) {
        const int k = k0 + lane;
        const float xv = x[min(k, dp - 1)];             // unconditional load
        const float v = k < dp ? xv : 0.0f;
        if (k < dp) {
            const uint16_t h = f2bf(v);
            hi[row * dp + k] = h;
            lo[row * dp + k] = f2bf(v - bf2f(h));
        }
        const int vi = __float_as_int(v);
        if (k0 + WAVE <= dp) {
#pragma unroll
            for (int j = 0; j < WAVE; ++j) {
                const float xj = __int_as_float(__builtin_amdgcn_readlane(vi, j));
                s = fmaf(xj, xj, s);
            }
        } else {
#pragma unroll
            for (int j = 0; j < WAVE; j += 16) {
                if (j >= dp - k0) break;
#pragma unroll
                for (int u = 0; u < 16; ++u) {
                    const float xj = __int_as_float(__builtin_amdgcn_readlane(vi, j + u));
                    s = fmaf(xj, xj, s);
                }
            }
        }
    }
    if (lane == 0) nrm[row] = s;
}

void split_bf16(const float *X, int64_t N, int dp, uint16_t *hi, uint16_t *lo, float *nrm,
                hipStream_t s)
{
    if (dp % 16 != 0) fail(ASKIT_ERR_UNSUPPORTED, "point rows must be padded to a multiple of 16 coordinates");
    hipLaunchKernelGGL(k_split_bf16, dim3((unsigned)((N + 3) / 4)), dim3(256), 0, s, X, N, dp, hi,
                       lo, nrm);
    HIPC(hipGetLastError());
}

// dst row r = src row idx[r], four coordinates per thread (rows are padded
// to a multiple of 16 coordinates, so 16-byte aligned).
__global__ void k_gather_rows(const float *__restrict__ src, const int32_t *__restrict__ idx,
                              int64_t n, int dp, float *__restrict__ dst)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int q = dp / 4;
    const int64_t row = t / q;
    if (row >= n) return;
    const int k = (int)(t - row * q) * 4;
    *reinterpret_cast<float4 *>(dst + row * dp + k) =
        *reinterpret_cast<const float4 *>(src + (int64_t)idx[row] * dp + k);
}

void gather_rows(const float *src, const int32_t *idx, int64_t n, int dp, float *dst, hipStream_t s)
{
    if (dp % 16 != 0) fail(ASKIT_ERR_UNSUPPORTED, "point rows must be padded to a multiple of 16 coordinates");
    const int64_t total = n * (dp / 4);
    if (total == 0) return;
    hipLaunchKernelGGL(k_gather_rows, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, src,
                       idx, n, dp, dst);
    HIPC(hipGetLastError());
}

// Largest entry of a non-negative FP32 array (bit pattern order = value order).
__global__ void k_max_norm(const float *__restrict__ v, int64_t n, unsigned *out)
{
    unsigned best = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        best = max(best, __float_as_uint(v[i]));
    for (int o = 32; o > 0; o >>= 1) best = max(best, (unsigned)__shfl_xor((int)best, o));
    if ((threadIdx.x % WAVE) == 0) atomicMax(out, best);
}

float max_norm(const float *nrm, int64_t N, hipStream_t s)
{
    unsigned *d;
    HIPC(ws_alloc((void **)&d, sizeof(unsigned), s));
    HIPC(hipMemsetAsync(d, 0, sizeof(unsigned), s));
    hipLaunchKernelGGL(k_max_norm, dim3(256), dim3(256), 0, s, nrm, N, d);
    HIPC(hipGetLastError());
    unsigned hbits = 0;
    HIPC(hipMemcpyAsync(&hbits, d, sizeof(unsigned), hipMemcpyDeviceToHost, s));
    HIPC(hipStreamSynchronize(s));
    HIPC(ws_free(d, s));
    float f;
    std::memcpy(&f, &hbits, 4);
    return f;
}

}  // namespace askit
