// Objective and per-literal gradient of every constraint, for a batch of
// restarts (paper: Alg. 2 steps i-iii for the value, Eq. chain / Thm. 4 for
// the reverse traversal; App. B for the transform-free OR/XOR products).
//
// Mapping on CDNA4 (wave64): a wave owns one restart block and walks a
// chunk of `cpw` constraints of one bin.  Lane = (restart r, segment j):
// L adjacent lanes split the literals of a constraint into L segments of
// s = ceil(k/L) <= SEG literals, so literal values, prefix products and
// gradient accumulators of a segment live in registers (fully unrolled
// over SEG).  The per-frequency leave-one-out product of literal i is
//     (prefix inside its segment) * (product of earlier segments)
//   * (product of later segments) * (suffix inside its segment),
// the segment products being exchanged by exclusive prefix/suffix scans
// over the L lanes.  Constraint descriptors and coefficient tables are
// wave-uniform (scalar loads); literal values are gathered from x[v][b]
// with restarts contiguous, so a wave reads 64/L consecutive restarts of a
// variable per load.
//
// Per-literal results go to a slot buffer [nnz][B] (value w_c * s_i *
// dWE_c/dl_i) that a segmented reduction over the variable-major transpose
// turns into the gradient, in a fixed order (deterministic).  Objective
// partials go to fpart[row][B], one row per (bin, chunk).
#include "internal.h"

namespace ffsat {

template <typename T>
__device__ __forceinline__ T fmaT(T a, T b, T c);
template <>
__device__ __forceinline__ float fmaT<float>(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
template <>
__device__ __forceinline__ double fmaT<double>(double a, double b, double c) { return __builtin_fma(a, b, c); }

// exclusive prefix and suffix products (complex) over the L lanes of a group
template <typename CT, int L>
__device__ __forceinline__ void group_scan_cplx(int j, CT tr, CT ti, CT &pr, CT &pi, CT &sr, CT &si)
{
    if constexpr (L == 1) {
        pr = 1; pi = 0; sr = 1; si = 0;
    } else {
        CT ar = tr, ai = ti;
#pragma unroll
        for (int d = 1; d < L; d <<= 1) {
            CT yr = __shfl_up(ar, d, L), yi = __shfl_up(ai, d, L);
            if (j >= d) {
                CT nr = fmaT(yr, ar, -yi * ai);
                CT ni = fmaT(yr, ai, yi * ar);
                ar = nr; ai = ni;
            }
        }
        CT er = __shfl_up(ar, 1, L), ei = __shfl_up(ai, 1, L);
        pr = j > 0 ? er : CT(1);
        pi = j > 0 ? ei : CT(0);
        CT br = tr, bi = ti;
#pragma unroll
        for (int d = 1; d < L; d <<= 1) {
            CT yr = __shfl_down(br, d, L), yi = __shfl_down(bi, d, L);
            if (j + d < L) {
                CT nr = fmaT(yr, br, -yi * bi);
                CT ni = fmaT(yr, bi, yi * br);
                br = nr; bi = ni;
            }
        }
        CT fr = __shfl_down(br, 1, L), fi = __shfl_down(bi, 1, L);
        sr = j < L - 1 ? fr : CT(1);
        si = j < L - 1 ? fi : CT(0);
    }
}

template <typename CT, int L>
__device__ __forceinline__ void group_scan_real(int j, CT t, CT &pre, CT &suf)
{
    if constexpr (L == 1) {
        pre = 1; suf = 1;
    } else {
        CT a = t;
#pragma unroll
        for (int d = 1; d < L; d <<= 1) {
            CT y = __shfl_up(a, d, L);
            if (j >= d) a = y * a;
        }
        CT e = __shfl_up(a, 1, L);
        pre = j > 0 ? e : CT(1);
        CT b = t;
#pragma unroll
        for (int d = 1; d < L; d <<= 1) {
            CT y = __shfl_down(b, d, L);
            if (j + d < L) b = y * b;
        }
        CT f = __shfl_down(b, 1, L);
        suf = j < L - 1 ? f : CT(1);
    }
}

template <typename IO, typename CT, int SEG, int L, bool CPLX>
__global__ __launch_bounds__(256) void k_eval(EvalArgs<IO> a)
{
    constexpr int RPW = 64 / L;
    const int lane = threadIdx.x & 63;
    const int unit = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    const int n_chunks = (a.count + a.cpw - 1) / a.cpw;
    if (unit >= n_chunks * a.n_rb) return;   // whole wave leaves together
    const int chunk = unit / a.n_rb;
    const int rb = unit - chunk * a.n_rb;
    const int j = lane & (L - 1);
    const int r = lane / L;
    const int b = rb * RPW + r;
    const bool bok = b < a.B;
    const int bb = bok ? b : a.B - 1;
    const TypeT<CT> *types = reinterpret_cast<const TypeT<CT> *>(a.types);
    const FreqT<CT> *freqs = reinterpret_cast<const FreqT<CT> *>(a.freqs);

    CT facc = 0;
    const int c_begin = chunk * a.cpw;
    const int c_end = min(c_begin + a.cpw, a.count);
    for (int ci = c_begin; ci < c_end; ++ci) {
        const ConDesc d = a.con[a.first + ci];
        const TypeT<CT> ty = types[d.type];
        const int k = d.k;
        const int s = (L == 1) ? k : (k + L - 1) / L;
        const int i0 = j * s;

        // step i input: gather literal values of this lane's segment
        CT lv[SEG], gr[SEG];
        uint32_t negm = 0;
#pragma unroll
        for (int t = 0; t < SEG; ++t) {
            gr[t] = 0;
            lv[t] = ty.pad;
            if (t < s) {
                const int i = i0 + t;
                if (i < k) {
                    const int lit = a.lit[d.off + i];
                    const int v = lit & 0x7fffffff;
                    const CT xv = (CT)a.x[(size_t)v * a.B + bb];
                    lv[t] = lit < 0 ? -xv : xv;
                    negm |= (lit < 0 ? 1u : 0u) << t;
                }
            }
        }

        CT we = 0;
        if constexpr (CPLX) {
            const int nf = ty.n1 + ty.n2;
            for (int f = 0; f < nf; ++f) {
                const FreqT<CT> fr = freqs[ty.tab + f];
                const bool form1 = f < ty.n1;
                const CT tk = fr.tk;
                CT pr[SEG], pi[SEG];
                CT Pr = fr.init, Pi = 0;
                // steps i-ii: affine factors and their running product
                if (form1) {
#pragma unroll
                    for (int t = 0; t < SEG; ++t) {
                        if (t < s) {
                            pr[t] = Pr; pi[t] = Pi;
                            const CT u = tk * lv[t];
                            const CT nr = fmaT(Pi, u, Pr);
                            const CT ni = fmaT(-Pr, u, Pi);
                            Pr = nr; Pi = ni;
                        }
                    }
                } else {
#pragma unroll
                    for (int t = 0; t < SEG; ++t) {
                        if (t < s) {
                            pr[t] = Pr; pi[t] = Pi;
                            const CT l = lv[t];
                            const CT nr = fmaT(Pi, l, tk * Pr);
                            const CT ni = fmaT(-Pr, l, tk * Pi);
                            Pr = nr; Pi = ni;
                        }
                    }
                }
                CT er, ei, sr, si;
                group_scan_cplx<CT, L>(j, Pr, Pi, er, ei, sr, si);
                // step iii (lane j == 0 holds the full product T0 * suffix)
                const CT Gr = fmaT(Pr, sr, -Pi * si);
                const CT Gi = fmaT(Pr, si, Pi * sr);
                we += fmaT(fr.c0re, Gr, -fr.c0im * Gi);
                // reverse traversal seeded with c1 * (other segments)
                const CT qr = fmaT(er, sr, -ei * si);
                const CT qi = fmaT(er, si, ei * sr);
                CT Sr = fmaT(fr.c1re, qr, -fr.c1im * qi);
                CT Si = fmaT(fr.c1re, qi, fr.c1im * qr);
                if (form1) {
#pragma unroll
                    for (int t = SEG - 1; t >= 0; --t) {
                        if (t < s) {
                            gr[t] = fmaT(pr[t], Sr, fmaT(-pi[t], Si, gr[t]));
                            const CT u = tk * lv[t];
                            const CT nr = fmaT(Si, u, Sr);
                            const CT ni = fmaT(-Sr, u, Si);
                            Sr = nr; Si = ni;
                        }
                    }
                } else {
#pragma unroll
                    for (int t = SEG - 1; t >= 0; --t) {
                        if (t < s) {
                            gr[t] = fmaT(pr[t], Sr, fmaT(-pi[t], Si, gr[t]));
                            const CT l = lv[t];
                            const CT nr = fmaT(Si, l, tk * Sr);
                            const CT ni = fmaT(-Sr, l, tk * Si);
                            Sr = nr; Si = ni;
                        }
                    }
                }
            }
        }
        if (ty.has_real) {
            // real chain: prod (alpha + beta l)
            CT q[SEG];
            CT P = 1;
#pragma unroll
            for (int t = 0; t < SEG; ++t) {
                if (t < s) {
                    q[t] = P;
                    P = P * fmaT(ty.beta, lv[t], ty.alpha);
                }
            }
            CT pre, suf;
            group_scan_real<CT, L>(j, P, pre, suf);
            we += ty.c0r * (P * suf);
            CT S = ty.c1r * (pre * suf);
#pragma unroll
            for (int t = SEG - 1; t >= 0; --t) {
                if (t < s) {
                    gr[t] = fmaT(q[t], S, gr[t]);
                    S = S * fmaT(ty.beta, lv[t], ty.alpha);
                }
            }
        }
        we += ty.cst;
        const CT wc = (CT)a.w[d.orig];
        if (j == 0) facc = fmaT(wc, we, facc);
        if (a.con_val != nullptr && j == 0 && bok) a.con_val[(size_t)d.orig * a.B + b] = (IO)we;
        if (a.want_grad && bok) {
#pragma unroll
            for (int t = 0; t < SEG; ++t) {
                if (t < s) {
                    const int i = i0 + t;
                    if (i < k) {
                        const CT gv = ((negm >> t) & 1u) ? -gr[t] : gr[t];
                        a.slot[(size_t)(d.off + i) * a.B + b] = (IO)(wc * gv);
                    }
                }
            }
        }
    }
    if (j == 0 && bok) a.fpart[(size_t)(a.fpart_row0 + chunk) * a.B + b] = (IO)facc;
}

template <typename IO>
using EvalFn = void (*)(EvalArgs<IO>);

template <typename IO, typename CT, bool CPLX>
static EvalFn<IO> pick_seg(int seg, int L)
{
    if (seg == 8 && L == 1) return &k_eval<IO, CT, 8, 1, CPLX>;
    if (seg == 16) {
        switch (L) {
        case 1: return &k_eval<IO, CT, 16, 1, CPLX>;
        default: break;
        }
        if constexpr (sizeof(CT) == 8) {
            switch (L) {
            case 2: return &k_eval<IO, CT, 16, 2, CPLX>;
            case 4: return &k_eval<IO, CT, 16, 4, CPLX>;
            case 8: return &k_eval<IO, CT, 16, 8, CPLX>;
            case 16: return &k_eval<IO, CT, 16, 16, CPLX>;
            case 32: return &k_eval<IO, CT, 16, 32, CPLX>;
            default: break;
            }
        }
    }
    if constexpr (sizeof(CT) == 4) {
        if (seg == 32) {
            switch (L) {
            case 1: return &k_eval<IO, CT, 32, 1, CPLX>;
            case 2: return &k_eval<IO, CT, 32, 2, CPLX>;
            case 4: return &k_eval<IO, CT, 32, 4, CPLX>;
            case 8: return &k_eval<IO, CT, 32, 8, CPLX>;
            case 16: return &k_eval<IO, CT, 32, 16, CPLX>;
            default: break;
            }
        }
    }
    return nullptr;
}

template <typename IO>
static EvalFn<IO> pick(int ct, int cls, int seg, int L)
{
    if constexpr (sizeof(IO) == 4) {
        if (ct == CT_F32) return cls == CLASS_DFT ? pick_seg<IO, float, true>(seg, L)
                                                  : pick_seg<IO, float, false>(seg, L);
        if (ct == CT_F64 && cls == CLASS_DFT) return pick_seg<IO, double, true>(seg, L);
        return nullptr;
    } else {
        if (ct != CT_F64) return nullptr;
        return cls == CLASS_DFT ? pick_seg<IO, double, true>(seg, L)
                                : pick_seg<IO, double, false>(seg, L);
    }
}

bool eval_variant_exists(int io, int ct, int cls, int seg, int L)
{
    if (io == IO_F32) return pick<float>(ct, cls, seg, L) != nullptr;
    return pick<double>(ct, cls, seg, L) != nullptr;
}

template <typename IO>
static hipError_t launch_bin(const Bin &bin, const EvalArgs<IO> &a, hipStream_t s)
{
    EvalFn<IO> fn = pick<IO>(bin.ct, bin.cls, bin.seg, bin.L);
    if (!fn) return hipErrorInvalidValue;
    const int n_chunks = (a.count + a.cpw - 1) / a.cpw;
    const int64_t units = (int64_t)n_chunks * a.n_rb;
    if (units <= 0) return hipSuccess;
    const int wpb = bin.wpb;
    const int64_t blocks = (units + wpb - 1) / wpb;
    hipLaunchKernelGGL(fn, dim3((unsigned)blocks), dim3(64 * wpb), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_eval_bin_f32(const Bin &bin, const EvalArgs<float> &a, hipStream_t s)
{
    return launch_bin<float>(bin, a, s);
}
hipError_t launch_eval_bin_f64(const Bin &bin, const EvalArgs<double> &a, hipStream_t s)
{
    return launch_bin<double>(bin, a, s);
}

}  // namespace ffsat
