// Gradient of the short transform-free constraints by gathering instead of
// scattering, fused with the reduction of every other constraint's slots
// and the projected step.
//
// For a variable v that sits at position i of an OR / AND / XOR constraint
// c, the term of dF/dx_v is w_c s_i c1 prod_{j != i} (alpha + beta l_j)
// (the closed forms of App. B differentiated as in Eq. chain; s_i = -1 for
// a negated literal).  The slot path computes it constraint by constraint,
// writes it to a [nnz][B] slot buffer and reads it back per variable: two
// passes over 4 bytes per (literal, restart) through HBM.  Here a wave owns
// a chunk of variables and 64 restarts and, for each variable, walks a list
// of entries {constraint, meta, the other literals} in a fixed order,
// gathers the other literals' points and adds the term in FP64 after the
// variable's remaining slots (longer constraints).  The objective term
// w_c WE_c and the exact check of c (Alg. 1: x < 0 is True) are taken once,
// at the entry of its first literal.
//
// Meta word: bits 0-2 transform-free kind, 3-5 k - 1, 6-9 check threshold
// + 2 (>= 0: at least that many true literals; -1 / -2: even / odd
// count), bit 10 this literal negated, bit 11 first literal of c.
#include "internal.h"

namespace ffsat {

// Mapping: a wave owns a chunk of at most PULL_VC_MAX variables and RPL
// blocks of 64 restarts (a lane holds restarts b, b + 64, ..): the decoding
// of an entry (readlane of its fields, kind coefficients, weight) is paid
// once for 64 * RPL restarts.  The chunk's list bounds are read with one
// lane-parallel load; per variable, the other constraints' slots and then
// the pulled entries are read in batches (one lane-parallel load of slot
// indices or entry words, broadcast with readlane), all gathers of a batch
// are issued before any term is added, and the terms are added in list
// order.  Batches past a list's end read null entries (kind 7: every
// coefficient zero) so that no term needs a branch.  Gathers are buffer
// loads: the variable's row offset is scalar, the restart offset per lane.
constexpr int RK_NULL = 7;
constexpr int BUF_DW3 = 0x00020000;   // gfx9 buffer resource word 3 (raw 32-bit loads)

__device__ __forceinline__ int lane_bcast(int v, int l) { return __builtin_amdgcn_readlane(v, l); }
// one float of a buffer: lane offset (bytes) plus scalar offset (bytes)
__device__ __forceinline__ float ldf(__amdgpu_buffer_rsrc_t r, int voff, unsigned soff)
{
    return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, voff, (int)soff, 0));
}

// Read-only arrays are separate __restrict__ arguments, so that the
// compiler reads the uniform ones (kind table, weights) through the scalar
// cache.
template <int E, int RPL, bool STEP>
__global__ __launch_bounds__(256) void k_pull(PullArgs a, const float *__restrict__ rkt, const float *__restrict__ wts,
                                              const int32_t *__restrict__ pent, const int32_t *__restrict__ pptr,
                                              const int32_t *__restrict__ vslot, const int32_t *__restrict__ vptr)
{
    constexpr int NO = E - 2;                              // other literals per entry
    constexpr int NB = (64 / E) < (64 / (NO * RPL)) ? (64 / E) : (64 / (NO * RPL));   // entries per batch
    constexpr int NS = 16 / RPL;                           // slots per batch
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int chunk = (int)blockIdx.x * 4 + wave;
    const int n_chunks = (a.n + a.vc - 1) / a.vc;
    if (chunk >= n_chunks) return;                   // whole wave
    if (a.skip != nullptr && *a.skip == 0) return;   // uniform
    const unsigned bstride = (unsigned)a.B * 4u;     // bytes per variable row
    const __amdgpu_buffer_rsrc_t rx = __builtin_amdgcn_make_buffer_rsrc(const_cast<float *>(a.x), (short)0,
                                                                          (int)a.x_bytes, BUF_DW3);
    int bl[RPL], lo[RPL];   // restart of each 64-block, and its load offset (clamped into the row)
    bool bok[RPL];
#pragma unroll
    for (int r = 0; r < RPL; ++r) {
        bl[r] = ((int)blockIdx.y * RPL + r) * 64 + lane;
        bok[r] = bl[r] < a.B;
        lo[r] = (bok[r] ? bl[r] : a.B - 1) * 4;
    }
    const int v0 = chunk * a.vc;
    const int nv = min(a.vc, a.n - v0);
    const int pb = lane <= nv ? pptr[v0 + lane] : 0;
    const int sb = lane <= nv ? vptr[v0 + lane] : 0;
    float facc[RPL];
    int nuns[RPL];
#pragma unroll
    for (int r = 0; r < RPL; ++r) {
        facc[r] = 0.f;
        nuns[r] = 0;
    }
    const float eta = STEP ? (a.eta_dev != nullptr ? *a.eta_dev : a.eta) : 0.f;
#pragma unroll 1
    for (int j = 0; j < nv; ++j) {
        const unsigned row = (unsigned)(v0 + j) * bstride;
        float xv[RPL];
        double acc[RPL];
#pragma unroll
        for (int r = 0; r < RPL; ++r) {
            xv[r] = ldf(rx, lo[r], row);
            acc[r] = 0.0;
        }
        // the other constraints' slots, ascending slot order
        const int e0 = lane_bcast(sb, j), e1 = lane_bcast(sb, j + 1);
#pragma unroll 1
        for (int e = e0; e < e1; e += NS) {
            const int idx = lane < NS && e + lane < e1 ? vslot[e + lane] : 0;
            float sv[NS][RPL];
#pragma unroll
            for (int q = 0; q < NS; ++q) {
                // the slot buffer may pass 2^31 bytes: 64-bit addresses
                const float *srow = a.slot + (size_t)lane_bcast(idx, q) * (size_t)a.B;
#pragma unroll
                for (int r = 0; r < RPL; ++r) sv[q][r] = srow[lo[r] >> 2];
            }
#pragma unroll
            for (int q = 0; q < NS; ++q) {
                const bool in = e + q < e1;   // uniform
#pragma unroll
                for (int r = 0; r < RPL; ++r) acc[r] += in ? (double)sv[q][r] : 0.0;
            }
        }
        // pulled entries, list order
        const int p0 = lane_bcast(pb, j), p1 = lane_bcast(pb, j + 1);
#pragma unroll 1
        for (int p = p0; p < p1; p += NB) {
            const int w = p * E + lane;
            const int ev = lane < NB * E ? (w < p1 * E ? pent[w] : ((lane % E) == 1 ? RK_NULL : 0)) : 0;
            float xo[NB][NO][RPL];
#pragma unroll
            for (int q = 0; q < NB; ++q) {
#pragma unroll
                for (int t = 0; t < NO; ++t) {
                    const unsigned so = (unsigned)(lane_bcast(ev, q * E + 2 + t) & 0x7fffffff) * bstride;
#pragma unroll
                    for (int r = 0; r < RPL; ++r)
                        xo[q][t][r] = ldf(rx, lo[r], so);
                }
            }
#pragma unroll
            for (int q = 0; q < NB; ++q) {
                const int orig = lane_bcast(ev, q * E);
                const int meta = lane_bcast(ev, q * E + 1);
                const int rk = meta & 7;
                const int km1 = (meta >> 3) & 7;
                const bool own_neg = (meta >> 10) & 1;
                const float al = rkt[rk], be = rkt[8 + rk], c1 = rkt[24 + rk];
                const float wc = wts[orig];
                float prod[RPL];
#pragma unroll
                for (int r = 0; r < RPL; ++r) prod[r] = 1.f;
#pragma unroll
                for (int t = 0; t < NO; ++t) {
                    if (t < km1) {   // uniform
                        const bool neg = lane_bcast(ev, q * E + 2 + t) < 0;
#pragma unroll
                        for (int r = 0; r < RPL; ++r) {
                            const float xval = xo[q][t][r];
                            prod[r] *= __builtin_fmaf(be, neg ? -xval : xval, al);
                        }
                    }
                }
                const float wc1 = wc * c1;
#pragma unroll
                for (int r = 0; r < RPL; ++r) {
                    const float gterm = wc1 * prod[r];
                    acc[r] += (double)(own_neg ? -gterm : gterm);
                }
                if ((meta >> 11) & 1) {   // first literal of the constraint: value and check
                    const float c0 = rkt[16 + rk], cst = rkt[32 + rk];
                    int nbad = 0;
#pragma unroll
                    for (int r = 0; r < RPL; ++r) {
                        const float lown = own_neg ? -xv[r] : xv[r];
                        const float we = __builtin_fmaf(c0, prod[r] * __builtin_fmaf(be, lown, al), cst);
                        facc[r] = __builtin_fmaf(wc, we, facc[r]);
                        if (a.want_check) {
                            // true literals (x < 0 is True; a negated literal flips it)
                            int c = (own_neg != (xv[r] < 0.f)) ? 1 : 0;
#pragma unroll
                            for (int t = 0; t < NO; ++t)
                                if (t < km1) c += ((lane_bcast(ev, q * E + 2 + t) < 0) != (xo[q][t][r] < 0.f)) ? 1 : 0;
                            const int chk = ((meta >> 6) & 15) - 2;
                            const bool sat = chk >= 0 ? (c >= chk) : ((c & 1) == (chk == -2 ? 1 : 0));
                            const bool uns = !sat && bok[r];
                            nuns[r] += uns ? 1 : 0;
                            if (a.unsat_bits != nullptr && uns)
                                atomicOr(&a.unsat_bits[(size_t)bl[r] * a.wm + (orig >> 5)], 1u << (orig & 31));
                            nbad += (int)__popcll(__ballot(uns));
                        }
                    }
                    if (a.U != nullptr && a.want_check && lane == 0 && nbad > 0) atomicAdd(&a.U[orig], nbad);
                }
            }
        }
#pragma unroll
        for (int r = 0; r < RPL; ++r) {
            if (!bok[r]) continue;
            const size_t idx = (size_t)(v0 + j) * (size_t)a.B + (size_t)bl[r];
            const float g = (float)acc[r];
            if constexpr (STEP) {
                // same rounding as the gradient, then the projected step
                const float y = __builtin_fmaf(-eta, g, xv[r]);
                a.x_out[idx] = fminf(fmaxf(y, -1.0f), 1.0f);
            } else {
                a.grad[idx] = g;
            }
        }
    }
#pragma unroll
    for (int r = 0; r < RPL; ++r) {
        if (!bok[r]) continue;
        const size_t rowi = (size_t)(a.row0 + chunk) * (size_t)a.B + (size_t)bl[r];
        a.fpart[rowi] = facc[r];
        if (a.want_check) a.cpart[rowi] = nuns[r];
    }
}

template <int E, int RPL>
static void launch_pull_t(const PullArgs &a, hipStream_t s)
{
    const int chunks = (a.n + a.vc - 1) / a.vc;
    const dim3 grid((unsigned)((chunks + 3) / 4), (unsigned)((a.B + 64 * RPL - 1) / (64 * RPL)));
    if (a.x_out)
        hipLaunchKernelGGL((k_pull<E, RPL, true>), grid, dim3(256), 0, s, a, a.rk, a.w, a.pent, a.pptr, a.vslot, a.vptr);
    else
        hipLaunchKernelGGL((k_pull<E, RPL, false>), grid, dim3(256), 0, s, a, a.rk, a.w, a.pent, a.pptr, a.vslot, a.vptr);
}

hipError_t launch_pull(int E, const PullArgs &a, hipStream_t s)
{
    if (a.n <= 0 || a.B <= 0) return hipSuccess;
    if ((a.x_out == nullptr) == (a.grad == nullptr) || a.x_out == a.x) return hipErrorInvalidValue;
    if (a.vc < 1 || a.vc > PULL_VC_MAX || a.x_bytes > 0x7fffffffll) return hipErrorInvalidValue;
    // restarts per lane: as many 64-blocks as the batch fills, up to 4
    const int rpl = a.B > 192 ? 4 : (a.B > 64 ? 2 : 1);
    if (E == 4) {
        if (rpl == 4) launch_pull_t<4, 4>(a, s);
        else if (rpl == 2) launch_pull_t<4, 2>(a, s);
        else launch_pull_t<4, 1>(a, s);
    } else if (E == 8) {
        if (rpl == 4) launch_pull_t<8, 4>(a, s);
        else if (rpl == 2) launch_pull_t<8, 2>(a, s);
        else launch_pull_t<8, 1>(a, s);
    } else {
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// Persistent loop of T fused iterations (App. A.3, Alg. 5; with the exact
// check of Alg. 1 and the weight update of Prop. 3) of a small problem whose
// constraints are all pulled (short transform-free chains): one workgroup
// holds the points, the weights, the violation counts U and the entry lists
// in LDS and runs all T iterations in one launch.  Per iteration:
//  1. one thread per (entry, restart) pair forms the entry's gradient term
//     (the weighted leave-one-out product of its constraint) and, at the
//     entries of first literals, the constraint's value and the exact check
//     (U and the restart's violation count by LDS integer atomics, which
//     are order-free);
//  2. one thread per (variable, restart) pair adds its entries' terms in
//     list order in FP64, rounds to FP32 as the evaluation does, and takes
//     the projected step in place;
//  3. with erwa, the maximum of U and the weight update; U cleared.
// The last iteration's F is summed per variable over its first-literal
// entries in list order (FP32), then over the variables in order (FP64):
// every result equals that of a thread walking each pair's list alone.
template <int E>
__global__ __launch_bounds__(1024) void k_iters_small(PullArgs a, int m, int T, float *F, int32_t *n_sat,
                                                      int32_t *Uout, float *wg, int erwa,
                                                      const float *__restrict__ alpha_dev,
                                                      const float *__restrict__ rkt_g,
                                                      const int32_t *__restrict__ pent_g,
                                                      const int32_t *__restrict__ pptr_g)
{
    constexpr int NO = E - 2;
    extern __shared__ float sm[];
    __shared__ int32_t red[16];
    __shared__ float rkt[RK_TABLE];
    const int B = a.B;
    const int nB = a.n * B;
    const int n_ent = pptr_g[a.n];
    const int eB = n_ent * B;
    float *xs = sm;                                           // [n][B] points
    float *fv = xs + nB;                                      // [n][B] objective sums of owned constraints
    float *tg = fv + nB;                                      // [n_ent][B] gradient terms
    float *fe = tg + eB;                                      // [m][B] constraint values
    float *ws = fe + (size_t)m * B;                           // [m] weights
    int32_t *us = reinterpret_cast<int32_t *>(ws + m);        // [m] violations per constraint
    int32_t *nu = us + m;                                     // [B] violated constraints per restart
    int32_t *pptr = nu + B;                                   // [n + 1] entry bounds
    int32_t *own = pptr + a.n + 1;                            // [n_ent] owning variable
    int32_t *pent = own + n_ent;                              // [n_ent][E] entries
    float *xg = const_cast<float *>(a.x);
    const bool check = n_sat != nullptr || Uout != nullptr || erwa;
    for (int i = threadIdx.x; i < nB; i += blockDim.x) xs[i] = xg[i];
    for (int c = threadIdx.x; c < m; c += blockDim.x) {
        ws[c] = wg[c];
        us[c] = 0;
    }
    for (int b = threadIdx.x; b < B; b += blockDim.x) nu[b] = 0;
    for (int i = threadIdx.x; i <= a.n; i += blockDim.x) pptr[i] = pptr_g[i];
    for (int i = threadIdx.x; i < n_ent * E; i += blockDim.x) pent[i] = pent_g[i];
    for (int i = threadIdx.x; i < RK_TABLE; i += blockDim.x) rkt[i] = rkt_g[i];
    for (int v = threadIdx.x; v < a.n; v += blockDim.x)
        for (int p = pptr_g[v]; p < pptr_g[v + 1]; ++p) own[p] = v;
    __syncthreads();
    const float eta = a.eta_dev != nullptr ? *a.eta_dev : a.eta;
    const float alpha = alpha_dev != nullptr ? *alpha_dev : 0.f;
#pragma unroll 1
    for (int it = 0; it < T; ++it) {
        // 1. entry terms at x_t
        for (int i = threadIdx.x; i < eB; i += blockDim.x) {
            const int p = i / B, b = i - p * B;
            const int32_t *en = pent + (size_t)p * E;
            const int orig = en[0], meta = en[1];
            const int rk = meta & 7, km1 = (meta >> 3) & 7;
            const bool own_neg = (meta >> 10) & 1;
            const float al = rkt[rk], be = rkt[8 + rk];
            float prod = 1.f;
            int cnt = 0;
#pragma unroll
            for (int t = 0; t < NO; ++t) {
                if (t < km1) {
                    const int o = en[2 + t];
                    const float xo = xs[(o & 0x7fffffff) * B + b];
                    prod *= __builtin_fmaf(be, o < 0 ? -xo : xo, al);
                    cnt += ((o < 0) != (xo < 0.f)) ? 1 : 0;
                }
            }
            const float gterm = ws[orig] * (rkt[24 + rk] * prod);
            tg[i] = own_neg ? -gterm : gterm;
            if ((meta >> 11) & 1) {
                const float xv = xs[own[p] * B + b];
                const float lown = own_neg ? -xv : xv;
                fe[(size_t)orig * B + b] = __builtin_fmaf(rkt[16 + rk], prod * __builtin_fmaf(be, lown, al), rkt[32 + rk]);
                if (check) {
                    cnt += (own_neg != (xv < 0.f)) ? 1 : 0;
                    const int chk = ((meta >> 6) & 15) - 2;
                    const bool sat = chk >= 0 ? (cnt >= chk) : ((cnt & 1) == (chk == -2 ? 1 : 0));
                    if (!sat) {
                        atomicAdd(&us[orig], 1);
                        atomicAdd(&nu[b], 1);
                    }
                }
            }
        }
        __syncthreads();
        // 2. ordered sums and the step; the last iteration's objective sums
        const bool last = it == T - 1;
        for (int i = threadIdx.x; i < nB; i += blockDim.x) {
            const int v = i / B, b = i - v * B;
            const int p0 = pptr[v], p1 = pptr[v + 1];
            double acc = 0.0;
            int p = p0;
            for (; p + 4 <= p1; p += 4) {
                const float t0 = tg[(p + 0) * B + b], t1 = tg[(p + 1) * B + b];
                const float t2 = tg[(p + 2) * B + b], t3 = tg[(p + 3) * B + b];
                acc += (double)t0;
                acc += (double)t1;
                acc += (double)t2;
                acc += (double)t3;
            }
            for (; p < p1; ++p) acc += (double)tg[p * B + b];
            if (last) {
                float facc = 0.f;
                for (int q = p0; q < p1; ++q) {
                    const int32_t *en = pent + (size_t)q * E;
                    if ((en[1] >> 11) & 1) facc = __builtin_fmaf(ws[en[0]], fe[(size_t)en[0] * B + b], facc);
                }
                fv[i] = facc;
            }
            const float g = (float)acc;   // same rounding as the evaluation's gradient
            const float y = __builtin_fmaf(-eta, g, xs[i]);
            xs[i] = fminf(fmaxf(y, -1.0f), 1.0f);
        }
        if (last) {
            __syncthreads();
            for (int b = threadIdx.x; b < B; b += blockDim.x) {
                double f = 0.0;
                for (int v = 0; v < a.n; ++v) f += (double)fv[v * B + b];
                if (F != nullptr) F[b] = (float)f;
                if (n_sat != nullptr) n_sat[b] = m - nu[b];
            }
            if (Uout != nullptr)
                for (int c = threadIdx.x; c < m; c += blockDim.x) Uout[c] = us[c];
        }
        // 3. weights (the counts are complete since the barrier after 1.;
        // the weights were last read in 2.)
        if (erwa) {
            int32_t mx = 0;
            for (int c = threadIdx.x; c < m; c += blockDim.x) mx = max(mx, us[c]);
            const int32_t umax = block_max_1024(mx, red);
            const float inv = umax > 0 ? 1.0f / (float)umax : 0.0f;
            for (int c = threadIdx.x; c < m; c += blockDim.x) ws[c] = erwa_weight(ws[c], us[c], umax, inv, alpha);
        }
        __syncthreads();   // every count read before it is cleared; the step and weights before the next terms
        if (check) {
            for (int c = threadIdx.x; c < m; c += blockDim.x) us[c] = 0;
            for (int b = threadIdx.x; b < B; b += blockDim.x) nu[b] = 0;
        }
        __syncthreads();
    }
    for (int i = threadIdx.x; i < nB; i += blockDim.x) xg[i] = xs[i];
    if (erwa)
        for (int c = threadIdx.x; c < m; c += blockDim.x) wg[c] = ws[c];
}

size_t iters_small_lds(int E, int n, int B, int m, int64_t n_ent)
{
    return (size_t)8 * n * B + (size_t)4 * n_ent * B + (size_t)4 * m * B + (size_t)8 * m + (size_t)4 * B +
           (size_t)4 * (n + 1) + (size_t)4 * n_ent + (size_t)4 * E * n_ent;
}

hipError_t launch_iters_small(int E, const PullArgs &a, int m, int64_t n_ent, int T, float *F, int32_t *n_sat,
                              int32_t *U, float *w, bool erwa, const float *alpha_dev, hipStream_t s)
{
    if (T <= 0) return hipSuccess;
    const int64_t work = std::max<int64_t>(std::max<int64_t>(n_ent * a.B, (int64_t)a.n * a.B), m);
    const size_t lds = iters_small_lds(E, a.n, a.B, m, n_ent);
    if (lds > (size_t)ITERS_SMALL_LDS) return hipErrorInvalidValue;
    const int threads = work >= 1024 ? 1024 : (int)((work + 63) / 64) * 64;
    if (E == 4)
        hipLaunchKernelGGL((k_iters_small<4>), dim3(1), dim3(threads), lds, s, a, m, T, F, n_sat, U, w, erwa ? 1 : 0,
                           alpha_dev, a.rk, a.pent, a.pptr);
    else if (E == 8)
        hipLaunchKernelGGL((k_iters_small<8>), dim3(1), dim3(threads), lds, s, a, m, T, F, n_sat, U, w, erwa ? 1 : 0,
                           alpha_dev, a.rk, a.pent, a.pptr);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

__global__ void k_copy_f32(float *dst, const float *src, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = src[i];
}

hipError_t launch_copy_f32(float *dst, const float *src, int64_t n, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_copy_f32, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, dst, src, n);
    return hipGetLastError();
}

}  // namespace ffsat
