// Reductions and the per-round kernels around the evaluation:
//  * segmented reduction of per-literal slots into the gradient over the
//    variable-major transpose (fixed order, deterministic), optionally
//    fused with the projected step (App. A.3, Alg. 5: clip to [-1,1]);
//  * two-level deterministic sum of objective partials (Def. 3);
//  * projected step; exact round-and-check (Alg. 1, Thm. 2); adaptive
//    weights (Prop. 3); weight gradient; small utilities.
#include "internal.h"

namespace ffsat {

static constexpr int RED_BLOCK = 256;
static constexpr int F_ROWS_PER_SPLIT = 32;

int f_splits(int rows) { return (rows + F_ROWS_PER_SPLIT - 1) / F_ROWS_PER_SPLIT; }

template <typename IO, bool STEP>
__global__ __launch_bounds__(RED_BLOCK) void k_reduce(int n, int B, const int32_t *__restrict__ vptr,
                                                      const int32_t *__restrict__ vslot,
                                                      const IO *__restrict__ slot, IO *grad, IO *x,
                                                      IO eta, int n_gblocks,
                                                      const IO *__restrict__ fpart, int rows,
                                                      IO *ftmp)
{
    const int bid = blockIdx.x;
    if (bid < n_gblocks) {
        const int64_t idx = (int64_t)bid * RED_BLOCK + threadIdx.x;
        if (idx >= (int64_t)n * B) return;
        const int v = (int)(idx / B);
        const int b = (int)(idx - (int64_t)v * B);
        double acc = 0.0;
        const int e1 = vptr[v + 1];
        for (int e = vptr[v]; e < e1; ++e) acc += (double)slot[(size_t)vslot[e] * B + b];
        if constexpr (STEP) {
            // same rounding as evaluating the gradient, then the step
            const float g = (float)acc;
            const float y = __builtin_fmaf(-(float)eta, g, (float)x[idx]);
            x[idx] = (IO)fminf(fmaxf(y, -1.0f), 1.0f);
        } else {
            grad[idx] = (IO)acc;
        }
    } else {
        // level 1 of the objective sum: one split of F_ROWS_PER_SPLIT rows
        const int fb = bid - n_gblocks;
        const int nbb = (B + RED_BLOCK - 1) / RED_BLOCK;
        const int split = fb / nbb;
        const int b = (fb - split * nbb) * RED_BLOCK + threadIdx.x;
        if (b >= B) return;
        const int r0 = split * F_ROWS_PER_SPLIT;
        const int r1 = min(rows, r0 + F_ROWS_PER_SPLIT);
        double acc = 0.0;
        for (int r = r0; r < r1; ++r) acc += (double)fpart[(size_t)r * B + b];
        ftmp[(size_t)split * B + b] = (IO)acc;
    }
}

template <typename IO>
__global__ __launch_bounds__(RED_BLOCK) void k_fsum2(int B, int splits, const IO *__restrict__ ftmp,
                                                     IO *F)
{
    const int b = blockIdx.x * RED_BLOCK + threadIdx.x;
    if (b >= B) return;
    double acc = 0.0;
    for (int s = 0; s < splits; ++s) acc += (double)ftmp[(size_t)s * B + b];
    F[b] = (IO)acc;
}

template <typename IO, bool STEP>
static hipError_t reduce_impl(int n, int B, const int32_t *vptr, const int32_t *vslot,
                              const IO *slot, IO *grad, IO *x, IO eta, const IO *fpart, int rows,
                              IO *ftmp, IO *F, hipStream_t s)
{
    const bool want_g = STEP ? (x != nullptr) : (grad != nullptr);
    const int64_t ng = want_g ? ((int64_t)n * B + RED_BLOCK - 1) / RED_BLOCK : 0;
    const int splits = F ? f_splits(rows) : 0;
    const int nbb = (B + RED_BLOCK - 1) / RED_BLOCK;
    const int64_t nf = (int64_t)splits * nbb;
    if (ng + nf > 0) {
        hipLaunchKernelGGL((k_reduce<IO, STEP>), dim3((unsigned)(ng + nf)), dim3(RED_BLOCK), 0, s, n,
                           B, vptr, vslot, slot, grad, x, eta, (int)ng, fpart, rows, ftmp);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    if (F) {
        hipLaunchKernelGGL((k_fsum2<IO>), dim3(nbb), dim3(RED_BLOCK), 0, s, B, splits, ftmp, F);
        return hipGetLastError();
    }
    return hipSuccess;
}

hipError_t launch_reduce_f32(int n, int B, const int32_t *vptr, const int32_t *vslot,
                             const float *slot, float *grad, float *x_step, float eta,
                             const float *fpart, int rows, float *ftmp, float *F, hipStream_t s)
{
    if (x_step)
        return reduce_impl<float, true>(n, B, vptr, vslot, slot, nullptr, x_step, eta, fpart, rows,
                                        ftmp, F, s);
    return reduce_impl<float, false>(n, B, vptr, vslot, slot, grad, nullptr, 0.f, fpart, rows, ftmp,
                                     F, s);
}

hipError_t launch_reduce_f64(int n, int B, const int32_t *vptr, const int32_t *vslot,
                             const double *slot, double *grad, const double *fpart, int rows,
                             double *ftmp, double *F, hipStream_t s)
{
    return reduce_impl<double, false>(n, B, vptr, vslot, slot, grad, nullptr, 0.0, fpart, rows,
                                      ftmp, F, s);
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

// ---------------------------------------------------------------- round and check

// One wave per (word of 32 consecutive original constraints, 64 restarts).
// Variable v is True iff x_v < 0; literal -v is True iff v is not.
template <typename IO>
__global__ __launch_bounds__(256) void k_check(int m, int B, const IO *__restrict__ x,
                                               const int32_t *__restrict__ pos,
                                               const ConDesc *__restrict__ con,
                                               const int32_t *__restrict__ lit,
                                               const int32_t *__restrict__ kind,
                                               const int32_t *__restrict__ param,
                                               int32_t *n_sat, uint32_t *unsat_bits, int32_t *U)
{
    const int lane = threadIdx.x & 63;
    const int unit = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    const int n_rb = (B + 63) / 64;
    const int wm = (m + 31) / 32;
    if (unit >= wm * n_rb) return;
    const int word = unit / n_rb;
    const int rb = unit - word * n_rb;
    const int b = rb * 64 + lane;
    const bool bok = b < B;
    const int bb = bok ? b : B - 1;
    uint32_t bits = 0;
    int nsat = 0;
    for (int q = 0; q < 32; ++q) {
        const int c = word * 32 + q;
        if (c >= m) break;
        const ConDesc d = con[pos[c]];
        int ntrue = 0;
        for (int i = 0; i < d.k; ++i) {
            const int l = lit[d.off + i];
            const int v = l & 0x7fffffff;
            const bool vt = x[(size_t)v * B + bb] < IO(0);
            ntrue += (l < 0) ? (vt ? 0 : 1) : (vt ? 1 : 0);
        }
        const int kd = kind[c], pr = param[c];
        bool sat;
        if (kd == FFSAT_KIND_OR) sat = ntrue >= 1;
        else if (kd == FFSAT_KIND_XOR) sat = (ntrue & 1) == (pr & 1);
        else sat = ntrue >= pr;
        if (!sat) bits |= 1u << q;
        nsat += sat ? 1 : 0;
        if (U != nullptr) {
            const unsigned long long bal = __ballot((!sat) && bok);
            if (lane == 0 && bal != 0ull) atomicAdd(&U[c], (int)__popcll(bal));
        }
    }
    if (bok) {
        if (unsat_bits != nullptr) unsat_bits[(size_t)b * wm + word] = bits;
        if (n_sat != nullptr) atomicAdd(&n_sat[b], nsat);
    }
}

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

hipError_t launch_fill_i32(int32_t *p, int64_t n, int32_t v, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_i32, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, n, v);
    return hipGetLastError();
}

template <typename IO>
static hipError_t check_impl(const ffsat_problem *p, int B, const IO *x, uint32_t *assign_bits,
                             int32_t *n_sat, uint32_t *unsat_bits, int32_t *U, hipStream_t s)
{
    const Layout &L = p->lay[IO_F32];
    hipError_t e;
    if (U) {
        if ((e = launch_fill_i32(U, p->m, 0, s)) != hipSuccess) return e;
    }
    if (n_sat) {
        if ((e = launch_fill_i32(n_sat, B, 0, s)) != hipSuccess) return e;
    }
    if (n_sat || unsat_bits || U) {
        const int64_t units = (int64_t)((p->m + 31) / 32) * ((B + 63) / 64);
        hipLaunchKernelGGL((k_check<IO>), dim3((unsigned)((units + 3) / 4)), dim3(256), 0, s, p->m, B,
                           x, L.d_pos, L.d_con, L.d_lit, p->d_kind, p->d_param, n_sat, unsat_bits,
                           U);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    if (assign_bits) {
        const int64_t tot = (int64_t)((p->n + 31) / 32) * B;
        hipLaunchKernelGGL((k_assign_bits<IO>), dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s,
                           p->n, B, x, assign_bits);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_check_f32(const ffsat_problem *p, int B, const float *x, uint32_t *assign_bits,
                            int32_t *n_sat, uint32_t *unsat_bits, int32_t *U, hipStream_t s)
{
    return check_impl<float>(p, B, x, assign_bits, n_sat, unsat_bits, U, s);
}
hipError_t launch_check_f64(const ffsat_problem *p, int B, const double *x,
                            uint32_t *assign_bits, int32_t *n_sat, uint32_t *unsat_bits,
                            int32_t *U, hipStream_t s)
{
    return check_impl<double>(p, B, x, assign_bits, n_sat, unsat_bits, U, s);
}

// ---------------------------------------------------------------- adaptive weights

__global__ __launch_bounds__(1024) void k_erwa(int m, const int32_t *__restrict__ U, float *w,
                                               float alpha)
{
    __shared__ int32_t red[1024];
    int32_t mx = 0;
    for (int c = threadIdx.x; c < m; c += blockDim.x) mx = max(mx, U[c]);
    red[threadIdx.x] = mx;
    __syncthreads();
    for (int h = blockDim.x / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) red[threadIdx.x] = max(red[threadIdx.x], red[threadIdx.x + h]);
        __syncthreads();
    }
    const int32_t umax = red[0];
    const float inv = umax > 0 ? 1.0f / (float)umax : 0.0f;
    for (int c = threadIdx.x; c < m; c += blockDim.x) {
        const float r = umax > 0 ? (float)U[c] * inv : 0.0f;
        w[c] = (1.0f - alpha) * w[c] + alpha * r;
    }
}

hipError_t launch_erwa(int m, const int32_t *U, float *w, float alpha, hipStream_t s)
{
    hipLaunchKernelGGL(k_erwa, dim3(1), dim3(1024), 0, s, m, U, w, alpha);
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
