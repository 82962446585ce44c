// Kernels of the message-passing initialiser: a learned proposal of restart
// points over the clause-variable incidence graph (3 rounds of messages,
// hidden width H, BF16 matrix-core products with FP32 accumulation).
//
//  * k_gemm: C = op(A) op(B) on the matrix cores (gfx950's
//    v_mfma_f32_32x32x16 bf16, 16 reduction terms per instruction): one
//    wave per 32x32 tile of C, operands read as FP32 (two 16-byte loads per
//    lane where the reduction dimension is contiguous and aligned) and
//    rounded to bfloat16 (round to nearest even) in registers, FP32
//    accumulators; optional split of the reduction dimension into fixed
//    slices (summed in a fixed order afterwards), bias + ReLU epilogue.
//  * k_gather: per-row weighted sums over the incidence (both directions),
//    used for the messages and for their transposes in the backward pass.
//  * head (tanh of a dot product), loss, column sums, Adam, proposals.
#include "mpnn_internal.h"

namespace ffsat {

typedef short __attribute__((ext_vector_type(8))) s16x8_t;
typedef __bf16 __attribute__((ext_vector_type(8))) bf16x8_t;
typedef float __attribute__((ext_vector_type(16))) f32x16_t;

__device__ __forceinline__ short to_bf16(float f)
{
    unsigned u = __float_as_uint(f);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (short)(u >> 16);
}

// The 8 values of a lane's share of one 16-term block: p[0..7] when the
// block lies inside [.., lim) and contiguous rows may be read as two
// aligned 16-byte loads (vec), else element by element with stride st,
// zero past lim.
__device__ __forceinline__ s16x8_t load8_bf16(const float *p, size_t st, int k, int lim, bool ok, bool vec)
{
    float v[8];
    if (ok && vec && k + 8 <= lim) {
        const float4 x0 = *reinterpret_cast<const float4 *>(p);
        const float4 x1 = *reinterpret_cast<const float4 *>(p + 4);
        v[0] = x0.x; v[1] = x0.y; v[2] = x0.z; v[3] = x0.w;
        v[4] = x1.x; v[5] = x1.y; v[6] = x1.z; v[7] = x1.w;
    } else {
#pragma unroll
        for (int q = 0; q < 8; ++q) v[q] = (ok && k + q < lim) ? p[(size_t)q * st] : 0.f;
    }
    s16x8_t r;
#pragma unroll
    for (int q = 0; q < 8; ++q) r[q] = to_bf16(v[q]);
    return r;
}

// C[M][N] (ldc) = sum over k in this block's slice of opA[i][k] * opB[k][j]
//   opA[i][k] = TA ? A[k*lda + i] : A[i*lda + k]
//   opB[k][j] = TB ? B[j*ldb + k] : B[k*ldb + j]
// EPI 0: C (+ slice * slice_stride) = acc; EPI 1: C = relu(acc + bias[j]).
// One 32x32x16 instruction per 16 reduction terms: lane l supplies the 8
// terms k0 + 8*(l/32) + v (v = 0..7) of row l % 32 of opA and of column
// l % 32 of opB (the same k for both operands, so the sum covers the block
// whatever order the unit takes them in), and holds
// D[8*(q/4) + 4*(l/32) + q%4][l % 32], q = 0..15.  vec_a / vec_b: the
// contiguous operand (opA rows for !TA, opB columns for TB) may be read as
// 16-byte loads (base 16-byte aligned, leading dimension a multiple of 4;
// slices and blocks start at multiples of 16).
template <bool TA, bool TB, int EPI>
__global__ __launch_bounds__(64) void k_gemm(int M, int N, int K, const float *__restrict__ A, int lda,
                                             const float *__restrict__ B, int ldb, float *C, int ldc,
                                             const float *__restrict__ bias, int kslice, size_t slice_stride,
                                             int vec_a, int vec_b)
{
    const int l = threadIdx.x;
    const int i0 = blockIdx.x * 32, j0 = blockIdx.y * 32;
    const int kb = blockIdx.z * kslice;
    const int ke = min(K, kb + kslice);
    const int ai = i0 + (l & 31);
    const int bj = j0 + (l & 31);
    const int kh = 8 * (l >> 5);
    const bool aok = ai < M, bok = bj < N;
    f32x16_t acc;
#pragma unroll
    for (int q = 0; q < 16; ++q) acc[q] = 0.f;
    for (int k0 = kb; k0 < ke; k0 += 16) {
        const int k = k0 + kh;
        const s16x8_t a = TA ? load8_bf16(A + (size_t)k * lda + ai, (size_t)lda, k, ke, aok, false)
                             : load8_bf16(A + (size_t)ai * lda + k, 1, k, ke, aok, vec_a != 0);
        const s16x8_t b = TB ? load8_bf16(B + (size_t)bj * ldb + k, 1, k, ke, bok, vec_b != 0)
                             : load8_bf16(B + (size_t)k * ldb + bj, (size_t)ldb, k, ke, bok, false);
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8_t, a), __builtin_bit_cast(bf16x8_t, b),
                                                      acc, 0, 0, 0);
    }
    const int j = j0 + (l & 31);
    if (j >= N) return;
#pragma unroll
    for (int q = 0; q < 16; ++q) {
        const int i = i0 + 8 * (q >> 2) + 4 * (l >> 5) + (q & 3);
        if (i >= M) continue;
        if constexpr (EPI == 0) {
            C[blockIdx.z * slice_stride + (size_t)i * ldc + j] = acc[q];
        } else {
            const float y = acc[q] + bias[j];
            C[(size_t)i * ldc + j] = y > 0.f ? y : 0.f;
        }
    }
}

// Reduction terms per slice when K is split `splits` ways: whole 16-term
// blocks of the matrix-core instruction.
static int gemm_kslice(int K, int splits)
{
    splits = splits < 1 ? 1 : splits;
    const int kslice = (K + splits - 1) / splits;
    return std::max(16, ((kslice + 15) / 16) * 16);
}

int gemm_slices(int K, int splits)
{
    const int kslice = gemm_kslice(K, splits);
    return std::max(1, (K + kslice - 1) / kslice);
}

hipError_t gemm(bool ta, bool tb, int epi, int M, int N, int K, const float *A, int lda, const float *B, int ldb,
                float *C, int ldc, const float *bias, int splits, size_t slice_stride, hipStream_t s)
{
    if (M <= 0 || N <= 0) return hipSuccess;
    int kslice = gemm_kslice(K, splits);
    splits = gemm_slices(K, splits);
    dim3 grid((M + 31) / 32, (N + 31) / 32, epi == 0 ? splits : 1);
    if (epi == 1) kslice = ((K + 15) / 16) * 16;
    const int vec_a = !ta && ((uintptr_t)A % 16 == 0) && lda % 4 == 0;
    const int vec_b = tb && ((uintptr_t)B % 16 == 0) && ldb % 4 == 0;
#define LAUNCH(TA, TB, E)                                                                                   \
    hipLaunchKernelGGL((k_gemm<TA, TB, E>), grid, dim3(64), 0, s, M, N, K, A, lda, B, ldb, C, ldc, bias, kslice, \
                       slice_stride, vec_a, vec_b)
    if (epi == 0) {
        if (!ta && !tb) LAUNCH(false, false, 0);
        else if (!ta && tb) LAUNCH(false, true, 0);
        else if (ta && !tb) LAUNCH(true, false, 0);
        else LAUNCH(true, true, 0);
    } else {
        if (ta || tb) return hipErrorInvalidValue;
        LAUNCH(false, false, 1);
    }
#undef LAUNCH
    return hipGetLastError();
}

// out[i] = sum_{s < S} part[s * stride + i]  (fixed order), optionally added to out
__global__ void k_sum_slices(int64_t len, int S, const float *__restrict__ part, size_t stride, float *out, int add)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= len) return;
    float acc = 0.f;
    for (int s = 0; s < S; ++s) acc += part[(size_t)s * stride + i];
    out[i] = add ? out[i] + acc : acc;
}

hipError_t sum_slices(int64_t len, int S, const float *part, size_t stride, float *out, bool add, hipStream_t s)
{
    if (len <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_sum_slices, dim3((unsigned)((len + 255) / 256)), dim3(256), 0, s, len, S, part, stride, out,
                       add ? 1 : 0);
    return hipGetLastError();
}

// Weighted incidence sums, one wave per destination row, lanes over the H
// features.  Row r owns edges e = row_ptr[r] .. row_ptr[r+1]; the edge's slot
// is edges[e] (or e itself when edges is null); its source row is
// src_of[slot], its weight w[slot], its sign from the literal lit[slot].
//  mode 0 (messages):  dst[r][dpos + f] = sum over positive edges of w * src[src][f]
//                      dst[r][dneg + f] = sum over negative edges  (written)
//                      and, with hcopy, dst[r][f] = hcopy[r][f] (the row's own state)
//  mode 1 (transposes): dst[r][f] += sum_e w * src[src][(pos ? spos : sneg) + f]
// The metadata of up to 64 edges is loaded lane-parallel (one edge per lane)
// and broadcast with readlane, so that the feature loads of consecutive
// edges do not wait on each other's index loads; the terms are added in edge
// order.
__global__ __launch_bounds__(256) void k_gather(int rows, int H, const int32_t *__restrict__ row_ptr,
                                                const int32_t *__restrict__ edges, const int32_t *__restrict__ src_of,
                                                const int32_t *__restrict__ lit, const float *__restrict__ w,
                                                const float *__restrict__ src, int sstride, int spos, int sneg,
                                                float *dst, int dstride, int dpos, int dneg, int mode,
                                                const float *__restrict__ hcopy)
{
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int r = blockIdx.x * (blockDim.x >> 6) + wave;
    if (r >= rows) return;
    const int lane = threadIdx.x & 63;
    const int e0 = row_ptr[r], e1 = row_ptr[r + 1];
    for (int f0 = 0; f0 < H; f0 += 64) {
        const int f = f0 + lane;
        const bool fin = f < H;
        const int fc = fin ? f : 0;
        float ap = 0.f, an = 0.f;
        for (int eb = e0; eb < e1; eb += 64) {
            const int e = eb + lane;
            int so = 0, pos = 1;
            float we = 0.f;
            if (e < e1) {
                const int slot = edges ? edges[e] : e;
                pos = lit[slot] >= 0 ? 1 : 0;
                // element offset of the feature row this edge reads
                so = src_of[slot] * sstride + (mode == 0 ? spos : (pos ? spos : sneg));
                we = w[slot];
            }
            const int cnt = min(64, e1 - eb);
            int q = 0;
            for (; q + 4 <= cnt; q += 4) {
                float v[4], wq[4];
                int pq[4];
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    const int o = __builtin_amdgcn_readlane(so, q + t);
                    pq[t] = __builtin_amdgcn_readlane(pos, q + t);
                    wq[t] = __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, we), q + t));
                    v[t] = src[(size_t)o + fc];
                }
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    if (mode == 0) {
                        if (pq[t]) ap += wq[t] * v[t];
                        else an += wq[t] * v[t];
                    } else {
                        ap += wq[t] * v[t];
                    }
                }
            }
            for (; q < cnt; ++q) {
                const int o = __builtin_amdgcn_readlane(so, q);
                const int pq = __builtin_amdgcn_readlane(pos, q);
                const float wq = __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, we), q));
                const float v = src[(size_t)o + fc];
                if (mode == 0) {
                    if (pq) ap += wq * v;
                    else an += wq * v;
                } else {
                    ap += wq * v;
                }
            }
        }
        if (!fin) continue;
        if (mode == 0) {
            dst[(size_t)r * dstride + dpos + f] = ap;
            dst[(size_t)r * dstride + dneg + f] = an;
            if (hcopy) dst[(size_t)r * dstride + f] = hcopy[(size_t)r * H + f];
        } else {
            dst[(size_t)r * dstride + f] += ap;
        }
    }
}

hipError_t gather(int rows, int H, const int32_t *row_ptr, const int32_t *edges, const int32_t *src_of,
                  const int32_t *lit, const float *w, const float *src, int sstride, int spos, int sneg, float *dst,
                  int dstride, int dpos, int dneg, int mode, hipStream_t s, const float *hcopy)
{
    if (rows <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_gather, dim3((unsigned)((rows + 3) / 4)), dim3(256), 0, s, rows, H, row_ptr, edges, src_of,
                       lit, w, src, sstride, spos, sneg, dst, dstride, dpos, dneg, mode, hcopy);
    return hipGetLastError();
}

// dZ = dH * (Y > 0), in place on dH; also copies the first H columns of a
// dX buffer into dH when dx is given (dH = dx[:, :H] * (Y > 0)).
__global__ void k_relu_back(int64_t total, int H, float *dH, const float *__restrict__ Y,
                            const float *__restrict__ dx, int dxstride)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= total) return;
    float g = dH[i];
    if (dx) {
        const int64_t r = i / H;
        g = dx[(size_t)r * dxstride + (i - r * H)];
    }
    dH[i] = Y[i] > 0.f ? g : 0.f;
}

hipError_t relu_back(int rows, int H, float *dH, const float *Y, const float *dx, int dxstride, hipStream_t s)
{
    const int64_t total = (int64_t)rows * H;
    if (total <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_relu_back, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, total, H, dH, Y, dx,
                       dxstride);
    return hipGetLastError();
}

// column sums of a rows x H matrix over fixed row slices: part[slice][f]
__global__ void k_colsum_part(int rows, int H, const float *__restrict__ X, int rows_per_slice, float *part)
{
    const int f = blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= H) return;
    const int r0 = blockIdx.y * rows_per_slice, r1 = min(rows, r0 + rows_per_slice);
    float acc = 0.f;
    for (int r = r0; r < r1; ++r) acc += X[(size_t)r * H + f];
    part[(size_t)blockIdx.y * H + f] = acc;
}

hipError_t colsum(int rows, int H, const float *X, float *part, int max_slices, float *out, hipStream_t s)
{
    int slices = std::max(1, std::min(max_slices, (rows + 255) / 256));
    const int rps = (rows + slices - 1) / slices;
    slices = std::max(1, (rows + rps - 1) / rps);
    hipLaunchKernelGGL(k_colsum_part, dim3((unsigned)((H + 63) / 64), (unsigned)slices), dim3(64), 0, s, rows, H, X,
                       rps, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return sum_slices(H, slices, part, (size_t)H, out, false, s);
}

// head: z_v = h_v . wo + bo, mu_v = tanh(z_v); one wave per variable
__global__ __launch_bounds__(256) void k_head(int n, int H, const float *__restrict__ hv, const float *__restrict__ wo,
                                              const float *__restrict__ bo, float *mu)
{
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int v = blockIdx.x * (blockDim.x >> 6) + wave;
    if (v >= n) return;
    const int lane = threadIdx.x & 63;
    float acc = 0.f;
    for (int f = lane; f < H; f += 64) acc += hv[(size_t)v * H + f] * wo[f];
#pragma unroll
    for (int d = 32; d > 0; d >>= 1) acc += __shfl_xor(acc, d, 64);
    if (lane == 0) mu[v] = tanhf(acc + bo[0]);
}

hipError_t head(int n, int H, const float *hv, const float *wo, const float *bo, float *mu, hipStream_t s)
{
    hipLaunchKernelGGL(k_head, dim3((unsigned)((n + 3) / 4)), dim3(256), 0, s, n, H, hv, wo, bo, mu);
    return hipGetLastError();
}

// head backward and loss: dz_v = 2 (mu - t) / n * (1 - mu^2), dH_v = dz_v wo,
// loss terms (mu - t)^2 / n and dz into per-variable buffers.
__global__ void k_head_back(int n, int H, const float *__restrict__ mu, const float *__restrict__ t,
                            const float *__restrict__ wo, float *dz, float *lterm, float *dH)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)n * H) return;
    const int v = (int)(i / H);
    const int f = (int)(i - (int64_t)v * H);
    const float d = mu[v] - t[v];
    const float g = 2.f * d / (float)n * (1.f - mu[v] * mu[v]);
    dH[i] = g * wo[f];
    if (f == 0) {
        dz[v] = g;
        lterm[v] = d * d / (float)n;
    }
}

hipError_t head_back(int n, int H, const float *mu, const float *t, const float *wo, float *dz, float *lterm,
                     float *dH, hipStream_t s)
{
    const int64_t total = (int64_t)n * H;
    hipLaunchKernelGGL(k_head_back, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, n, H, mu, t, wo, dz,
                       lterm, dH);
    return hipGetLastError();
}

// dwo[f] = sum_v dz_v h_v[f] over fixed variable slices (partials)
__global__ void k_dwo_part(int n, int H, const float *__restrict__ dz, const float *__restrict__ hv, int per,
                           float *part)
{
    const int f = blockIdx.x * blockDim.x + threadIdx.x;
    if (f > H) return;
    const int v0 = blockIdx.y * per, v1 = min(n, v0 + per);
    float acc = 0.f;
    for (int v = v0; v < v1; ++v) acc += dz[v] * (f < H ? hv[(size_t)v * H + f] : 1.f);
    part[(size_t)blockIdx.y * (H + 1) + f] = acc;
}

hipError_t dwo(int n, int H, const float *dz, const float *hv, float *part, int max_slices, float *out,
               hipStream_t s)
{
    int slices = std::max(1, std::min(max_slices, (n + 255) / 256));
    const int per = (n + slices - 1) / slices;
    slices = std::max(1, (n + per - 1) / per);
    hipLaunchKernelGGL(k_dwo_part, dim3((unsigned)((H + 1 + 63) / 64), (unsigned)slices), dim3(64), 0, s, n, H, dz,
                       hv, per, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return sum_slices(H + 1, slices, part, (size_t)(H + 1), out, false, s);
}

// Adam (Kingma & Ba 2015) on FP32 master weights; step t starts at 1.
__global__ void k_adam(int64_t P, float *w, const float *__restrict__ g, float *m1, float *m2, float lr, float b1,
                       float b2, float eps, float c1, float c2)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= P) return;
    const float gi = g[i];
    const float a = b1 * m1[i] + (1.f - b1) * gi;
    const float b = b2 * m2[i] + (1.f - b2) * gi * gi;
    m1[i] = a;
    m2[i] = b;
    w[i] -= lr * (a / c1) / (sqrtf(b / c2) + eps);
}

hipError_t adam(int64_t P, float *w, const float *g, float *m1, float *m2, float lr, float b1, float b2, float eps,
                int step, hipStream_t s)
{
    const float c1 = 1.f - powf(b1, (float)step), c2 = 1.f - powf(b2, (float)step);
    hipLaunchKernelGGL(k_adam, dim3((unsigned)((P + 255) / 256)), dim3(256), 0, s, P, w, g, m1, m2, lr, b1, b2, eps, c1,
                       c2);
    return hipGetLastError();
}

__device__ __forceinline__ uint64_t splitmix64_m(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

// x[v][b] = clip(mu_v + sigma u, -1, 1) for b < nl, else u; u uniform in
// [-1, 1) from SplitMix64 of seed + (i+1) * golden gamma, i = v*B + b.
__global__ void k_propose(int64_t total, int B, int nl, const float *__restrict__ mu, float sigma, uint64_t seed,
                          float *x)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= total) return;
    const int b = (int)(i % B);
    const int64_t v = i / B;
    const uint64_t r = splitmix64_m(seed + (uint64_t)(i + 1) * 0x9e3779b97f4a7c15ull);
    const float u = (float)(r >> 40) * (2.0f / 16777216.0f) - 1.0f;
    if (b < nl) x[i] = fminf(fmaxf(mu[v] + sigma * u, -1.f), 1.f);
    else x[i] = u;
}

hipError_t propose(int64_t total, int B, int nl, const float *mu, float sigma, uint64_t seed, float *x, hipStream_t s)
{
    hipLaunchKernelGGL(k_propose, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, total, B, nl, mu, sigma, seed,
                       x);
    return hipGetLastError();
}

}  // namespace ffsat

namespace ffsat {

__global__ void k_fill_f32(int64_t n, float *p, float v)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

hipError_t fill_f32(int64_t n, float *p, float v, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_f32, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, p, v);
    return hipGetLastError();
}

// dst[r][f] = X[r][f] for f < H (first H columns of a rows x xstride matrix)
__global__ void k_take_cols(int64_t total, int H, const float *__restrict__ X, int xstride, float *dst)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= total) return;
    const int64_t r = i / H;
    dst[i] = X[(size_t)r * xstride + (i - r * H)];
}

hipError_t take_cols(int rows, int H, const float *X, int xstride, float *dst, hipStream_t s)
{
    const int64_t total = (int64_t)rows * H;
    if (total <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_take_cols, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, total, H, X, xstride, dst);
    return hipGetLastError();
}

}  // namespace ffsat
