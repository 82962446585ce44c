// The root-of-unity evaluation in the paper's own form, kept as an ablation
// of the bounded basis: factors w^a + l on the unit circle (Eq. forward),
// their product per frequency (Eq. reduction) and the conjugated Walsh
// coefficients f~ = f^ W^-1 (Eq. inverse), with no rescaling of the running
// products.  Lane layout, scans, gradient traversal and check are those of
// the main kernels; only the factor form differs.  Segment shapes: L = 1
// with SEG in {4, 8, 16}, SEG = 16 at L = 2..32.
#include "eval_kernel.h"

namespace ffsat {

template <typename IO, typename CT, int SEG, int L>
__global__ __launch_bounds__(256) void k_eval_uc(EvalArgs<IO> a, const IO *__restrict__ xin,
                                                 const ConDesc *__restrict__ con,
                                                 const int32_t *__restrict__ lits,
                                                 const float *__restrict__ wts,
                                                 const TypeT<CT> *__restrict__ types,
                                                 const FreqT<CT> *__restrict__ freqs)
{
    extern __shared__ __align__(16) char uc_lds[];
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const bool split = a.fg > 1;
    const int unit = split ? (int)blockIdx.x : (int)blockIdx.x * (int)(blockDim.x >> 6) + wave;
    const Span sp{a.first, a.count, a.cpw, a.n_rb, a.fpart_row0};
    eval_unit<IO, CT, SEG, L, true, true>(a, sp, unit, xin, con, lits, wts, types, freqs, split ? a.fg : 1,
                                          split ? wave : 0, uc_lds);
}

template <typename IO, typename CT, int SEG, int L>
static EvalFn<IO> uc_handle()
{
    EvalFn<IO> h;
    h.fn = reinterpret_cast<const void *>(&k_eval_uc<IO, CT, SEG, L>);
    h.ct = sizeof(CT) == 4 ? CT_F32 : CT_F64;
    return h;
}

template <typename IO, typename CT>
static EvalFn<IO> uc_pick(int seg, int L)
{
    if (L == 1) {
        if (seg == 4) return uc_handle<IO, CT, 4, 1>();
        if (seg == 8) return uc_handle<IO, CT, 8, 1>();
        if (seg == 16) return uc_handle<IO, CT, 16, 1>();
        return EvalFn<IO>{};
    }
    if (seg != 16) return EvalFn<IO>{};
    switch (L) {
    case 2: return uc_handle<IO, CT, 16, 2>();
    case 4: return uc_handle<IO, CT, 16, 4>();
    case 8: return uc_handle<IO, CT, 16, 8>();
    case 16: return uc_handle<IO, CT, 16, 16>();
    case 32: return uc_handle<IO, CT, 16, 32>();
    default: return EvalFn<IO>{};
    }
}

EvalFn<float> pick_uc_f32(int ct, int seg, int L)
{
    return ct == CT_F32 ? uc_pick<float, float>(seg, L) : uc_pick<float, double>(seg, L);
}

EvalFn<double> pick_uc_f64(int seg, int L) { return uc_pick<double, double>(seg, L); }

}  // namespace ffsat
