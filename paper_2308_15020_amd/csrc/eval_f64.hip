// Evaluation kernels with FP64 inputs and arithmetic (the FP64 evaluation),
// and the launch entry points of all evaluation kernels.
#include "eval_kernel.h"

namespace ffsat {

EvalFn<float> pick_f32_f32(int cls, int seg, int L);
EvalFn<float> pick_f32_f64(int cls, int seg, int L);
EvalFn<float> pick_uc_f32(int ct, int seg, int L);
EvalFn<double> pick_uc_f64(int seg, int L);

static EvalFn<double> pick_f64(int cls, int seg, int L)
{
    return cls == CLASS_DFT ? pick_seg<double, double, true>(seg, L) : pick_seg<double, double, false>(seg, L);
}

static EvalFn<float> pick_f32(int ct, int cls, int seg, int L)
{
    if (ct == CT_F32) return pick_f32_f32(cls, seg, L);
    return pick_f32_f64(cls, seg, L);
}

bool eval_variant_exists(int io, int ct, int cls, int seg, int L, bool uc)
{
    if (uc && cls == CLASS_DFT) return io == IO_F32 ? (bool)pick_uc_f32(ct, seg, L) : (ct == CT_F64 && (bool)pick_uc_f64(seg, L));
    if (io == IO_F32) return (bool)pick_f32(ct, cls, seg, L);
    return ct == CT_F64 && (bool)pick_f64(cls, seg, L);
}

hipError_t launch_eval_bin_f32(const Bin &bin, const EvalArgs<float> &a, hipStream_t s)
{
    if (bin.uc) return launch_fn<float>(pick_uc_f32(bin.ct, bin.seg, bin.L), bin, a, s);
    return launch_fn<float>(pick_f32(bin.ct, bin.cls, bin.seg, bin.L), bin, a, s);
}

hipError_t launch_eval_bin_f64(const Bin &bin, const EvalArgs<double> &a, hipStream_t s)
{
    if (bin.ct != CT_F64) return hipErrorInvalidValue;
    if (bin.uc) return launch_fn<double>(pick_uc_f64(bin.seg, bin.L), bin, a, s);
    return launch_fn<double>(pick_f64(bin.cls, bin.seg, bin.L), bin, a, s);
}

}  // namespace ffsat
