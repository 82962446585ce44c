// Reductions and the per-round kernels around the evaluation:
//  * segmented reduction of per-literal slots into the gradient over the
//    variable-major transpose (fixed order, deterministic), optionally
//    fused with the projected step (App. A.3, Alg. 5: clip to [-1,1]);
//  * two-level deterministic sum of objective partials (Def. 3), the second
//    level over 16 waves per block of 64 restarts;
//  * projected step; rounding of the variables (Alg. 1); adaptive weights
//    (Prop. 3); weight gradient; small utilities.  The exact constraint
//    check runs inside the evaluation kernels.
#include <algorithm>

#include "internal.h"

namespace ffsat {

static constexpr int RED_BLOCK = 256;
static constexpr int F_ROWS_PER_SPLIT = 64;

int f_splits(int rows) { return (rows + F_ROWS_PER_SPLIT - 1) / F_ROWS_PER_SPLIT; }

// Grid: x = variable (uniform per block, so the transpose is read with
// scalar loads) then one block column per split of objective rows; y =
// restart chunk of RED_BLOCK.
template <typename IO, bool STEP>
__global__ __launch_bounds__(RED_BLOCK) void k_reduce(ReduceArgs<IO> a, int n_grad)
{
    const int bx = blockIdx.x;
    const int b = blockIdx.y * RED_BLOCK + threadIdx.x;
    if (b >= a.B) return;
    if (a.skip != nullptr && *a.skip == 0) return;
    const int B = a.B;
    if (bx < n_grad) {
        const int v = bx;
        const int e0 = a.vptr[v], e1 = a.vptr[v + 1];
        double acc = 0.0;
        int e = e0;
        // independent loads first, then the additions in slot order
        for (; e + 8 <= e1; e += 8) {
            IO sv[8];
#pragma unroll
            for (int q = 0; q < 8; ++q) sv[q] = a.slot[(size_t)a.vslot[e + q] * B + b];
#pragma unroll
            for (int q = 0; q < 8; ++q) acc += (double)sv[q];
        }
        for (; e < e1; ++e) acc += (double)a.slot[(size_t)a.vslot[e] * B + b];
        const size_t idx = (size_t)v * B + b;
        if constexpr (STEP) {
            // same rounding as evaluating the gradient, then the step (step
            // size from device memory when given: one captured graph serves
            // every step size)
            const float g = (float)acc;
            const float eta = a.eta_dev != nullptr ? *a.eta_dev : a.eta;
            const float y = __builtin_fmaf(-eta, g, a.x_step[idx]);
            a.x_step[idx] = fminf(fmaxf(y, -1.0f), 1.0f);
        } else {
            a.grad[idx] = (IO)acc;
        }
    } else {
        // level 1 of the objective / count sums: one split of F_ROWS_PER_SPLIT rows
        const int split = bx - n_grad;
        const int r0 = split * F_ROWS_PER_SPLIT;
        const int r1 = min(a.rows, r0 + F_ROWS_PER_SPLIT);
        if (a.F != nullptr) {
            double acc = 0.0;
#pragma unroll 8
            for (int r = r0; r < r1; ++r) acc += (double)a.fpart[(size_t)r * B + b];
            a.ftmp[(size_t)split * B + b] = (IO)acc;
        }
        if (a.n_sat != nullptr) {
            int acc = 0;
#pragma unroll 8
            for (int r = r0; r < r1; ++r) acc += a.cpart[(size_t)r * B + b];
            a.ctmp[(size_t)split * B + b] = acc;
        }
    }
}

// Level 2: a block per 64 restarts (lane = restart); its FSUM_WAVES waves
// each add a contiguous share of the splits in order, then wave 0 adds the
// waves' partials in wave order (a fixed order: deterministic).
static constexpr int FSUM_WAVES = 16;
template <typename IO>
__global__ __launch_bounds__(64 * FSUM_WAVES) void k_fsum2(ReduceArgs<IO> a, int splits)
{
    __shared__ double fp[FSUM_WAVES][64];
    __shared__ int cp[FSUM_WAVES][64];
    const int lane = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int b = blockIdx.x * 64 + lane;
    if (a.skip != nullptr && *a.skip == 0) return;   // uniform: the whole block leaves
    const bool ok = b < a.B;
    const int s0 = (int)(((int64_t)splits * w) / FSUM_WAVES), s1 = (int)(((int64_t)splits * (w + 1)) / FSUM_WAVES);
    double facc = 0.0;
    int cacc = 0;
    if (ok) {
        if (a.F != nullptr) {
#pragma unroll 8
            for (int q = s0; q < s1; ++q) facc += (double)a.ftmp[(size_t)q * a.B + b];
        }
        if (a.n_sat != nullptr) {
#pragma unroll 8
            for (int q = s0; q < s1; ++q) cacc += a.ctmp[(size_t)q * a.B + b];
        }
    }
    fp[w][lane] = facc;
    cp[w][lane] = cacc;
    __syncthreads();
    if (w != 0 || !ok) return;
    double f = 0.0;
    int c = 0;
#pragma unroll
    for (int q = 0; q < FSUM_WAVES; ++q) {
        f += fp[q][lane];
        c += cp[q][lane];
    }
    if (a.F != nullptr) a.F[b] = (IO)f;
    if (a.n_sat != nullptr) a.n_sat[b] = a.m - c;
}

// parts: 1 = gradient (and step) with level 1 of the sums, 2 = level 2 of
// the sums, 3 = both in order.
template <typename IO, bool STEP>
static hipError_t reduce_impl(const ReduceArgs<IO> &a, hipStream_t s, int parts = 3)
{
    const bool want_g = STEP ? (a.x_step != nullptr) : (a.grad != nullptr);
    const int n_grad = want_g ? a.n : 0;
    const bool rows = a.F != nullptr || a.n_sat != nullptr;
    const int splits = rows ? f_splits(a.rows) : 0;
    const int nbb = (a.B + RED_BLOCK - 1) / RED_BLOCK;
    if ((parts & 1) && n_grad + splits > 0) {
        hipLaunchKernelGGL((k_reduce<IO, STEP>), dim3((unsigned)(n_grad + splits), (unsigned)nbb), dim3(RED_BLOCK),
                           0, s, a, n_grad);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    if ((parts & 2) && rows) {
        hipLaunchKernelGGL((k_fsum2<IO>), dim3((a.B + 63) / 64), dim3(64 * FSUM_WAVES), 0, s, a, splits);
        return hipGetLastError();
    }
    return hipSuccess;
}

hipError_t launch_reduce_f32(const ReduceArgs<float> &r, hipStream_t s)
{
    if (r.x_step) return reduce_impl<float, true>(r, s);
    return reduce_impl<float, false>(r, s);
}

hipError_t launch_reduce_f64(const ReduceArgs<double> &r, hipStream_t s)
{
    return reduce_impl<double, false>(r, s);
}

hipError_t launch_reduce_part_f32(const ReduceArgs<float> &r, int parts, hipStream_t s)
{
    if (r.x_step) return reduce_impl<float, true>(r, s, parts);
    return reduce_impl<float, false>(r, s, parts);
}

// ---------------------------------------------------------------- projected step

__global__ void k_step_f32(int64_t total, int B, float *x, const float *g, const float *eta_b,
                           float eta)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= total) return;
    const float e = eta_b ? eta_b[i % B] : eta;
    const float y = __builtin_fmaf(-e, g[i], x[i]);
    x[i] = fminf(fmaxf(y, -1.0f), 1.0f);
}

__global__ void k_step_f64(int64_t total, int B, double *x, const double *g, const double *eta_b,
                           double eta)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= total) return;
    const double e = eta_b ? eta_b[i % B] : eta;
    const double y = __builtin_fma(-e, g[i], x[i]);
    x[i] = fmin(fmax(y, -1.0), 1.0);
}

hipError_t launch_step_f32(int64_t total, int B, float *x, const float *g, const float *eta_b,
                           float eta, hipStream_t s)
{
    if (total <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_step_f32, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, total, B,
                       x, g, eta_b, eta);
    return hipGetLastError();
}

hipError_t launch_step_f64(int64_t total, int B, double *x, const double *g,
                           const double *eta_b, double eta, hipStream_t s)
{
    if (total <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_step_f64, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, total, B,
                       x, g, eta_b, eta);
    return hipGetLastError();
}

// ---------------------------------------------------------------- rounding

template <typename IO>
__global__ void k_assign_bits(int n, int B, const IO *__restrict__ x, uint32_t *bits)
{
    const int wn = (n + 31) / 32;
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)wn * B) return;
    const int word = (int)(idx / B);
    const int b = (int)(idx - (int64_t)word * B);
    uint32_t w = 0;
    for (int q = 0; q < 32; ++q) {
        const int v = word * 32 + q;
        if (v >= n) break;
        if (x[(size_t)v * B + b] < IO(0)) w |= 1u << q;
    }
    bits[(size_t)b * wn + word] = w;
}

__global__ void k_fill_i32(int32_t *p, int64_t n, int32_t v)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

__global__ void k_set_f32x2(float *p, float a, float b)
{
    if (threadIdx.x == 0) {
        p[0] = a;
        p[1] = b;
    }
}

hipError_t launch_set_f32x2(float *p, float a, float b, hipStream_t s)
{
    hipLaunchKernelGGL(k_set_f32x2, dim3(1), dim3(64), 0, s, p, a, b);
    return hipGetLastError();
}

hipError_t launch_fill_i32(int32_t *p, int64_t n, int32_t v, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_i32, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, n, v);
    return hipGetLastError();
}

template <typename IO>
static hipError_t assign_impl(int n, int B, const IO *x, uint32_t *bits, hipStream_t s)
{
    const int64_t tot = (int64_t)((n + 31) / 32) * B;
    hipLaunchKernelGGL((k_assign_bits<IO>), dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, n, B, x, bits);
    return hipGetLastError();
}

hipError_t launch_assign_bits_f32(int n, int B, const float *x, uint32_t *bits, hipStream_t s)
{
    return assign_impl<float>(n, B, x, bits, s);
}
hipError_t launch_assign_bits_f64(int n, int B, const double *x, uint32_t *bits, hipStream_t s)
{
    return assign_impl<double>(n, B, x, bits, s);
}

// ---------------------------------------------------------------- adaptive weights

// ERWA (Prop. 3): w_c <- (1 - alpha) w_c + alpha U_c / max_c' U_c'.
// Up to ERWA_ONE_BLOCK constraints one launch: every 1024-thread block
// computes the maximum (eight loads in flight per thread, wave reductions)
// and updates its slice; beyond that, per-block partial maxima first, then
// every block of the update reduces the (at most 1024) partials itself.
constexpr int ERWA_ONE_BLOCK = 1 << 16;

__device__ __forceinline__ int32_t strided_max(int m, const int32_t *__restrict__ U, int begin, int stride)
{
    int32_t mx = 0;
    int c = begin;
    for (; c + 7 * stride < m; c += 8 * stride) {
        int32_t q[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) q[u] = U[c + u * stride];
#pragma unroll
        for (int u = 0; u < 8; ++u) mx = max(mx, q[u]);
    }
    for (; c < m; c += stride) mx = max(mx, U[c]);
    return mx;
}

// every block finds the maximum itself (1024 threads, eight loads in
// flight each), then updates its own 1024 weights
__global__ __launch_bounds__(1024) void k_erwa_one(int m, const int32_t *__restrict__ U, float *w, float alpha,
                                                   const float *__restrict__ alpha_dev)
{
    __shared__ int32_t red[16];
    if (alpha_dev != nullptr) alpha = *alpha_dev;
    const int32_t umax = block_max_1024(strided_max(m, U, threadIdx.x, 1024), red);
    const float inv = umax > 0 ? 1.0f / (float)umax : 0.0f;
    const int c = blockIdx.x * 1024 + threadIdx.x;
    if (c < m) w[c] = erwa_weight(w[c], U[c], umax, inv, alpha);
}

__global__ __launch_bounds__(1024) void k_umax_part(int m, const int32_t *__restrict__ U, int32_t *part)
{
    __shared__ int32_t red[16];
    const int32_t v = block_max_1024(strided_max(m, U, blockIdx.x * 1024 + threadIdx.x, gridDim.x * 1024), red);
    if (threadIdx.x == 0) part[blockIdx.x] = v;
}

__global__ __launch_bounds__(1024) void k_erwa_apply(int m, int nparts, const int32_t *__restrict__ part,
                                                     const int32_t *__restrict__ U, float *w, float alpha,
                                                     const float *__restrict__ alpha_dev)
{
    __shared__ int32_t red[16];
    if (alpha_dev != nullptr) alpha = *alpha_dev;
    const int32_t umax = block_max_1024((int)threadIdx.x < nparts ? part[threadIdx.x] : 0, red);
    const float inv = umax > 0 ? 1.0f / (float)umax : 0.0f;
    for (int c = blockIdx.x * 1024 + threadIdx.x; c < m; c += gridDim.x * 1024)
        w[c] = erwa_weight(w[c], U[c], umax, inv, alpha);
}

hipError_t launch_erwa(int m, const int32_t *U, float *w, float alpha, const float *alpha_dev, int32_t *part,
                       hipStream_t s)
{
    if (m <= ERWA_ONE_BLOCK) {
        hipLaunchKernelGGL(k_erwa_one, dim3((m + 1023) / 1024), dim3(1024), 0, s, m, U, w, alpha, alpha_dev);
        return hipGetLastError();
    }
    const int nparts = std::min(1024, (m + 8191) / 8192);
    hipLaunchKernelGGL(k_umax_part, dim3(nparts), dim3(1024), 0, s, m, U, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_erwa_apply, dim3(nparts), dim3(1024), 0, s, m, nparts, part, U, w, alpha, alpha_dev);
    return hipGetLastError();
}

// ---------------------------------------------------------------- weight gradient

__global__ __launch_bounds__(256) void k_wgrad(int m, int B, const float *__restrict__ con_val,
                                               const float *__restrict__ gF, float *gw)
{
    const int lane = threadIdx.x & 63;
    const int c = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    if (c >= m) return;
    double acc = 0.0;
    for (int b = lane; b < B; b += 64) acc += (double)gF[b] * (double)con_val[(size_t)c * B + b];
#pragma unroll
    for (int d = 32; d > 0; d >>= 1) acc += __shfl_xor(acc, d, 64);
    if (lane == 0) gw[c] = (float)acc;
}

hipError_t launch_wgrad(int m, int B, const float *con_val, const float *gF, float *gw,
                        hipStream_t s)
{
    hipLaunchKernelGGL(k_wgrad, dim3((unsigned)((m + 3) / 4)), dim3(256), 0, s, m, B, con_val, gF,
                       gw);
    return hipGetLastError();
}

// ---------------------------------------------------------------- vector-Jacobian product

// gx[v][b] = gF[b] * grad[v][b]: the gradient of sum_b gF_b F_b with respect to x
__global__ void k_scale_restarts(int64_t total, int B, const float *__restrict__ grad, const float *__restrict__ gF,
                                 float *gx)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= total) return;
    gx[i] = gF[i % B] * grad[i];
}

hipError_t launch_scale_restarts(int64_t total, int B, const float *grad, const float *gF, float *gx, hipStream_t s)
{
    if (total <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_scale_restarts, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, total, B, grad, gF,
                       gx);
    return hipGetLastError();
}

// ---------------------------------------------------------------- restarts

// SplitMix64 (Steele, Lea, Flood, "Fast splittable pseudorandom number
// generators", OOPSLA 2014): the output function applied to seed + (i+1) *
// golden gamma; the top 24 bits give a uniform float in [-1, 1).
__device__ __forceinline__ uint64_t splitmix64(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

// Rephasing of selected restarts (App. Restart Heuristics): mode 0 keeps x
// (original phase), 1 flips it (x <- -x), 2 redraws it uniformly in [-1, 1].
// mask[b] != 0 selects restart b (mask may be null: all restarts).
__global__ void k_rephase(int64_t total, int B, float *x, int mode, uint64_t seed, const int32_t *__restrict__ mask)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= total) return;
    if (mask != nullptr && mask[i % B] == 0) return;
    if (mode == 1) {
        x[i] = -x[i];
    } else if (mode == 2) {
        const uint64_t r = splitmix64(seed + (uint64_t)(i + 1) * 0x9e3779b97f4a7c15ull);
        x[i] = (float)(r >> 40) * (2.0f / 16777216.0f) - 1.0f;
    }
}

hipError_t launch_rephase(int64_t total, int B, float *x, int mode, uint64_t seed, const int32_t *mask, hipStream_t s)
{
    if (total <= 0 || mode == 0) return hipSuccess;
    hipLaunchKernelGGL(k_rephase, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, total, B, x, mode, seed,
                       mask);
    return hipGetLastError();
}

// ---------------------------------------------------------------- utilities

template <typename IO>
__global__ void k_nonfinite(int64_t total, const IO *x, int32_t *flag)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= total) return;
    const IO v = x[i];
    if (!(v == v) || v - v != IO(0)) atomicOr(flag, 1);
}

hipError_t launch_nonfinite_f32(int64_t total, const float *x, int32_t *flag, hipStream_t s)
{
    hipLaunchKernelGGL((k_nonfinite<float>), dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s,
                       total, x, flag);
    return hipGetLastError();
}
hipError_t launch_nonfinite_f64(int64_t total, const double *x, int32_t *flag, hipStream_t s)
{
    hipLaunchKernelGGL((k_nonfinite<double>), dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s,
                       total, x, flag);
    return hipGetLastError();
}

// deterministic pseudo-random points in [-1, 1] for the autotuner
__global__ void k_scratch_points(float *x, int64_t total, uint32_t seed)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= total) return;
    uint32_t h = (uint32_t)i * 2654435761u ^ seed;
    h ^= h >> 16; h *= 0x7feb352du; h ^= h >> 15; h *= 0x846ca68bu; h ^= h >> 16;
    x[i] = (float)(h >> 8) * (2.0f / 16777216.0f) - 1.0f;
}

hipError_t launch_scratch_points(float *x, int64_t total, uint32_t seed, hipStream_t s)
{
    hipLaunchKernelGGL(k_scratch_points, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, x,
                       total, seed);
    return hipGetLastError();
}

}  // namespace ffsat

// ---------------------------------------------------------------- FISTA with backtracking
// Per restart b (columns of [n][B] arrays): see ffsat_fista in ffsat.h.

namespace ffsat {

constexpr float FISTA_ETA_MIN = 1e-12f;

__global__ void k_fista_begin(int B, const float *__restrict__ eta, int32_t *active, int32_t *searching,
                              int32_t *n_active)
{
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= B) return;
    const int32_t a = eta[b] >= FISTA_ETA_MIN ? 1 : 0;
    active[b] = a;
    searching[b] = a;
    if (a) atomicAdd(n_active, 1);
}

// z = clip(y - eta_b g) for the restarts still searching, and per (chunk of
// `rows` variables, restart) partial sums of g.(z - y) and |z - y|^2.
// skip: restarts still searching before this trial (0: nothing to do).
__global__ __launch_bounds__(256) void k_fista_trial(int n, int B, int rows, int chunks, const float *__restrict__ y,
                                                     const float *__restrict__ g, const float *__restrict__ eta,
                                                     const int32_t *__restrict__ searching, float *z, float *part,
                                                     const int32_t *__restrict__ skip)
{
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= B || *skip == 0 || !searching[b]) return;
    const float e = eta[b];
    const int v0 = blockIdx.y * rows, v1 = min(n, v0 + rows);
    float dot = 0.f, sq = 0.f;
    for (int v = v0; v < v1; ++v) {
        const size_t i = (size_t)v * B + b;
        const float yv = y[i], gv = g[i];
        const float zv = fminf(fmaxf(yv - e * gv, -1.f), 1.f);
        z[i] = zv;
        const float d = zv - yv;
        dot = fmaf(gv, d, dot);
        sq = fmaf(d, d, sq);
    }
    part[(size_t)blockIdx.y * B + b] = dot;
    part[((size_t)chunks + blockIdx.y) * B + b] = sq;
}

// sufficient-decrease test per searching restart; partial sums in a fixed
// order (FP64); on failure eta halves; after the last trial the point is
// taken anyway.  pending counts the restarts still searching after this trial.
__global__ void k_fista_accept(int B, int chunks, const float *__restrict__ part, const float *__restrict__ Fy,
                               const float *__restrict__ Fz, float *eta, int32_t *searching, float *Fout, int last,
                               int32_t *pending, const int32_t *__restrict__ skip)
{
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= B || *skip == 0 || !searching[b]) return;
    double dot = 0.0, sq = 0.0;
    for (int c = 0; c < chunks; ++c) {
        dot += (double)part[(size_t)c * B + b];
        sq += (double)part[((size_t)chunks + c) * B + b];
    }
    const float e = eta[b];
    const double bound = (double)Fy[b] + dot + sq / (2.0 * (double)e);
    const bool ok = (double)Fz[b] <= bound;
    if (!ok) eta[b] = 0.5f * e;
    if (ok || last) {
        searching[b] = 0;
        if (Fout) Fout[b] = Fz[b];
    } else {
        atomicAdd(pending, 1);
    }
}

__global__ void k_fista_coef(int B, const int32_t *__restrict__ active, float *t, float *coef)
{
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= B) return;
    if (!active[b]) {
        coef[b] = 0.f;
        return;
    }
    const float tk = t[b];
    const float tn = 0.5f * (1.f + sqrtf(1.f + 4.f * tk * tk));
    coef[b] = (tk - 1.f) / tn;
    t[b] = tn;
}

__global__ void k_fista_momentum(int64_t total, int B, const int32_t *__restrict__ active,
                                 const float *__restrict__ coef, const float *__restrict__ z, float *x, float *y)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= total) return;
    const int b = (int)(i % B);
    if (!active[b]) return;
    const float zv = z[i], xv = x[i];
    y[i] = fmaf(coef[b], zv - xv, zv);
    x[i] = zv;
}

int fista_rows(int n, int B)
{
    // enough (chunk, restart-tile) blocks to cover the chip, at least 8 variables per chunk
    const int tiles = (B + 255) / 256;
    int rows = (int)std::max<int64_t>(8, ((int64_t)n * tiles + 2047) / 2048);
    return std::min(rows, std::max(n, 1));
}

hipError_t launch_fista_begin(int B, const float *eta, int32_t *active, int32_t *searching, int32_t *n_active,
                              hipStream_t s)
{
    hipLaunchKernelGGL(k_fista_begin, dim3((B + 255) / 256), dim3(256), 0, s, B, eta, active, searching, n_active);
    return hipGetLastError();
}

hipError_t launch_fista_trial(int n, int B, const float *y, const float *g, const float *eta, const int32_t *searching,
                              float *z, float *part, const int32_t *skip, hipStream_t s)
{
    const int rows = fista_rows(n, B);
    const int chunks = (n + rows - 1) / rows;
    hipLaunchKernelGGL(k_fista_trial, dim3((B + 255) / 256, chunks), dim3(256), 0, s, n, B, rows, chunks, y, g, eta,
                       searching, z, part, skip);
    return hipGetLastError();
}

hipError_t launch_fista_accept(int n, int B, const float *part, const float *Fy, const float *Fz, float *eta,
                               int32_t *searching, float *Fout, int last, int32_t *pending, const int32_t *skip,
                               hipStream_t s)
{
    const int rows = fista_rows(n, B);
    const int chunks = (n + rows - 1) / rows;
    hipLaunchKernelGGL(k_fista_accept, dim3((B + 255) / 256), dim3(256), 0, s, B, chunks, part, Fy, Fz, eta, searching,
                       Fout, last, pending, skip);
    return hipGetLastError();
}

hipError_t launch_fista_finish(int n, int B, const int32_t *active, float *t, float *coef, const float *z, float *x,
                               float *y, hipStream_t s)
{
    hipLaunchKernelGGL(k_fista_coef, dim3((B + 255) / 256), dim3(256), 0, s, B, active, t, coef);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int64_t total = (int64_t)n * B;
    hipLaunchKernelGGL(k_fista_momentum, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, total, B, active, coef,
                       z, x, y);
    return hipGetLastError();
}

}  // namespace ffsat

// ---------------------------------------------------------------- satisfied weight

namespace ffsat {

// score[b] = sum_c w_c [constraint c holds at restart b's rounded point],
// from the unsat bits of ffsat_round_check ([B][ceil(m/32)]); w = NULL: all
// ones.  One wave per restart, FP64 accumulation in constraint order per
// lane, then a fixed-order wave reduction.
__global__ __launch_bounds__(256) void k_sat_weight(int m, int B, int wm, const uint32_t *__restrict__ bits,
                                                    const float *__restrict__ w, double *score)
{
    const int b = blockIdx.x * (blockDim.x >> 6) + (int)(threadIdx.x >> 6);
    if (b >= B) return;
    const int lane = threadIdx.x & 63;
    double acc = 0.0;
    for (int q = lane; q < wm; q += 64) {
        const uint32_t u = bits[(size_t)b * wm + q];
        const int c0 = q * 32, c1 = min(m, c0 + 32);
        for (int c = c0; c < c1; ++c)
            if (!((u >> (c - c0)) & 1u)) acc += w ? (double)w[c] : 1.0;
    }
#pragma unroll
    for (int d = 32; d > 0; d >>= 1) acc += __shfl_xor(acc, d, 64);
    if (lane == 0) score[b] = acc;
}

hipError_t launch_sat_weight(int m, int B, const uint32_t *bits, const float *w, double *score, hipStream_t s)
{
    const int wm = (m + 31) / 32;
    hipLaunchKernelGGL(k_sat_weight, dim3((B + 3) / 4), dim3(256), 0, s, m, B, wm, bits, w, score);
    return hipGetLastError();
}

}  // namespace ffsat
