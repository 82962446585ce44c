// Evaluation kernels with FP32 inputs and FP32 arithmetic (all bins of the
// FP32 evaluation except long root-of-unity products).
#include "eval_kernel.h"

namespace ffsat {

EvalFn<float> pick_f32_f32(int cls, int seg, int L)
{
    return cls == CLASS_DFT ? pick_seg<float, float, true>(seg, L) : pick_seg<float, float, false>(seg, L);
}

}  // namespace ffsat
