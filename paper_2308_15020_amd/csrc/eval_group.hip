// Grouped evaluation launches: every FP32-arithmetic bin of the FP32
// evaluation in one grid, and the long FP64-arithmetic root-of-unity bins in
// another.  A host-built block table gives each 4-wave block
// its bin (entry) and first unit; the host orders the blocks longest-first
// with the memory-bound real-chain blocks spread among them.  One launch
// keeps all CUs busy across bins of very different cost, with no
// cross-stream synchronisation.
#include "eval_kernel.h"

namespace ffsat {

// Kernel variants of a grouped launch (FP32 arithmetic, the shapes of the
// FP32 shape rule): (SEG, L) for L = 1 with SEG in {4, 8, ..., 24}, and for
// L in {2, 4, 8, 16} with SEG in {16, 20, 24}; real chains first, then
// root-of-unity products.
#define FFSAT_GROUP_SHAPES(X, CPLX, BASE)                                                              \
    X(BASE + 0, 4, 1, CPLX) X(BASE + 1, 8, 1, CPLX) X(BASE + 2, 12, 1, CPLX) X(BASE + 3, 16, 1, CPLX)  \
    X(BASE + 4, 20, 1, CPLX) X(BASE + 5, 24, 1, CPLX) X(BASE + 6, 16, 2, CPLX) X(BASE + 7, 20, 2, CPLX) \
    X(BASE + 8, 24, 2, CPLX) X(BASE + 9, 16, 4, CPLX) X(BASE + 10, 20, 4, CPLX)                        \
    X(BASE + 11, 24, 4, CPLX) X(BASE + 12, 16, 8, CPLX) X(BASE + 13, 20, 8, CPLX)                      \
    X(BASE + 14, 24, 8, CPLX) X(BASE + 15, 16, 16, CPLX) X(BASE + 16, 20, 16, CPLX)                    \
    X(BASE + 17, 24, 16, CPLX)
constexpr int GROUP_SHAPES = 18;

int group_variant(int ct, int cls, int seg, int L)
{
    if (ct != CT_F32) return -1;
    const int base = cls == CLASS_DFT ? GROUP_SHAPES : 0;
#define X(ID, S, LL, C) \
    if (seg == S && L == LL) return ID + base;
    FFSAT_GROUP_SHAPES(X, false, 0)
#undef X
    return -1;
}

// Each 256-thread block: entry blk.x; fg == 1: units blk.y .. blk.y + 3,
// one per wave; fg == 4: unit blk.y, its frequencies over the 4 waves.
// Register budget of 4 waves per SIMD (128 VGPRs; the longest variants spill
// a few values outside their inner loops): measured faster than 3 waves
// without spills.
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4, 8))) void k_eval_group(EvalArgs<float> a, const float *__restrict__ xin,
                                                    const ConDesc *__restrict__ con,
                                                    const int32_t *__restrict__ lits,
                                                    const float *__restrict__ wts,
                                                    const TypeT<float> *__restrict__ types,
                                                    const FreqT<float> *__restrict__ freqs,
                                                    const GroupEntry *__restrict__ ent,
                                                    const int2 *__restrict__ blk)
{
    extern __shared__ __align__(16) char group_lds[];
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int2 bw = blk[blockIdx.x];
    const GroupEntry e = ent[__builtin_amdgcn_readfirstlane(bw.x)];
    const Span sp{e.first, e.count, e.cpw, e.n_rb, e.fpart_row0};
    const int fg = e.fg;
    const int unit = fg > 1 ? bw.y : bw.y + wave;
    const int wg = fg > 1 ? wave : 0;
    switch (e.variant) {
#define X(ID, S, LL, C)                                                                                    \
    case ID:                                                                                               \
        eval_unit<float, float, S, LL, C>(a, sp, unit, xin, con, lits, wts, types, freqs, fg, wg, group_lds); \
        break;
        FFSAT_GROUP_SHAPES(X, false, 0)
        FFSAT_GROUP_SHAPES(X, true, GROUP_SHAPES)
#undef X
    default: break;
    }
}

// The root-of-unity bins with FP64 arithmetic (k >= 128 by default) in one
// grid as well: the ramp and tail of a launch are paid once instead of once
// per bin.  (SEG, L): 14..32 at L = 16, 16, 20, 24 and 25..32 at L = 8.  Compiled for
// 3 waves per SIMD (168 VGPRs): the variants of more than 28 positions spill
// a few per-constraint values, none in their frequency loops, and the grid
// runs 20% faster than at the 2 waves their full register count would give.
#define FFSAT_GROUP64_SHAPES(X)                                                                           \
    X(0, 17, 16) X(1, 18, 16) X(2, 19, 16) X(3, 20, 16) X(4, 21, 16) X(5, 22, 16) X(6, 23, 16)           \
    X(7, 24, 16) X(8, 25, 16) X(9, 26, 16) X(10, 27, 16) X(11, 28, 16) X(12, 29, 16) X(13, 30, 16)       \
    X(14, 31, 16) X(15, 32, 16) X(16, 14, 16) X(17, 15, 16) X(18, 16, 16) X(19, 16, 8) X(20, 20, 8)      \
    X(21, 24, 8) X(22, 25, 8) X(23, 26, 8) X(24, 27, 8) X(25, 28, 8) X(26, 29, 8) X(27, 30, 8)          \
    X(28, 31, 8) X(29, 32, 8)

int group_variant64(int seg, int L)
{
#define X(ID, S, LL) \
    if (seg == S && L == LL) return ID;
    FFSAT_GROUP64_SHAPES(X)
#undef X
    return -1;
}

__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3))) void k_eval_group64(EvalArgs<float> a, const float *__restrict__ xin,
                                                      const ConDesc *__restrict__ con,
                                                      const int32_t *__restrict__ lits,
                                                      const float *__restrict__ wts,
                                                      const TypeT<double> *__restrict__ types,
                                                      const FreqT<double> *__restrict__ freqs,
                                                      const GroupEntry *__restrict__ ent,
                                                      const int2 *__restrict__ blk)
{
    extern __shared__ __align__(16) char group_lds[];
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int2 bw = blk[blockIdx.x];
    const GroupEntry e = ent[__builtin_amdgcn_readfirstlane(bw.x)];
    const Span sp{e.first, e.count, e.cpw, e.n_rb, e.fpart_row0};
    const int fg = e.fg;
    const int unit = fg > 1 ? bw.y : bw.y + wave;
    const int wg = fg > 1 ? wave : 0;
    switch (e.variant) {
#define X(ID, S, LL)                                                                                          \
    case ID:                                                                                                  \
        eval_unit<float, double, S, LL, true>(a, sp, unit, xin, con, lits, wts, types, freqs, fg, wg, group_lds); \
        break;
        FFSAT_GROUP64_SHAPES(X)
#undef X
    default: break;
    }
}

hipError_t launch_eval_group64_f32(const EvalArgs<float> &a, const GroupEntry *ent, const int2 *blk, int nblk,
                                   size_t lds, hipStream_t s)
{
    if (nblk <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_eval_group64, dim3((unsigned)nblk), dim3(256), lds, s, a, a.x, a.con, a.lit, a.w,
                       reinterpret_cast<const TypeT<double> *>(a.types),
                       reinterpret_cast<const FreqT<double> *>(a.freqs), ent, blk);
    return hipGetLastError();
}

hipError_t launch_eval_group_f32(const EvalArgs<float> &a, const GroupEntry *ent, const int2 *blk, int nblk,
                                 size_t lds, hipStream_t s)
{
    if (nblk <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_eval_group, dim3((unsigned)nblk), dim3(256), lds, s, a, a.x, a.con, a.lit, a.w,
                       reinterpret_cast<const TypeT<float> *>(a.types),
                       reinterpret_cast<const FreqT<float> *>(a.freqs), ent, blk);
    return hipGetLastError();
}

}  // namespace ffsat
