// Evaluation kernels with FP32 inputs and FP64 arithmetic: root-of-unity
// products of long constraints in the FP32 evaluation.
#include "eval_kernel.h"

namespace ffsat {

EvalFn<float> pick_f32_f64(int cls, int seg, int L)
{
    return cls == CLASS_DFT ? pick_seg<float, double, true>(seg, L) : EvalFn<float>{};
}

}  // namespace ffsat
