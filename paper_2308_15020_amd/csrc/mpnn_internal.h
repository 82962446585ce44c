// Internal declarations of the message-passing initialiser.
#pragma once

#include <algorithm>

#include "internal.h"

namespace ffsat {

hipError_t gemm(bool ta, bool tb, int epi, int M, int N, int K, const float *A, int lda, const float *B, int ldb,
                float *C, int ldc, const float *bias, int splits, size_t slice_stride, hipStream_t s);
// number of reduction slices gemm() writes for `splits` requested over K terms
int gemm_slices(int K, int splits);
hipError_t sum_slices(int64_t len, int S, const float *part, size_t stride, float *out, bool add, hipStream_t s);
hipError_t gather(int rows, int H, const int32_t *row_ptr, const int32_t *edges, const int32_t *src_of,
                  const int32_t *lit, const float *w, const float *src, int sstride, int spos, int sneg, float *dst,
                  int dstride, int dpos, int dneg, int mode, hipStream_t s, const float *hcopy = nullptr);
hipError_t relu_back(int rows, int H, float *dH, const float *Y, const float *dx, int dxstride, hipStream_t s);
hipError_t colsum(int rows, int H, const float *X, float *part, int max_slices, float *out, hipStream_t s);
hipError_t head(int n, int H, const float *hv, const float *wo, const float *bo, float *mu, hipStream_t s);
hipError_t head_back(int n, int H, const float *mu, const float *t, const float *wo, float *dz, float *lterm,
                     float *dH, hipStream_t s);
hipError_t dwo(int n, int H, const float *dz, const float *hv, float *part, int max_slices, float *out,
               hipStream_t s);
hipError_t adam(int64_t P, float *w, const float *g, float *m1, float *m2, float lr, float b1, float b2, float eps,
                int step, hipStream_t s);
hipError_t propose(int64_t total, int B, int nl, const float *mu, float sigma, uint64_t seed, float *x,
                   hipStream_t s);

// Incidence graph of a problem in original constraint order, on the device.
struct MpnnGraph {
    int n = 0, m = 0, nnz = 0;
    void *buf = nullptr;          // one device allocation holding every array below
    int32_t *con_ptr = nullptr;   // [m+1]
    int32_t *lit = nullptr;       // [nnz] var | negated << 31
    int32_t *var_of = nullptr;    // [nnz] variable of each slot
    int32_t *con_of = nullptr;    // [nnz] constraint of each slot
    int32_t *vptr = nullptr;      // [n+1] variable -> slots
    int32_t *vslots = nullptr;    // [nnz]
    float *wk = nullptr;          // [nnz] 1 / k of the slot's constraint
    float *wd = nullptr;          // [nnz] 1 / max(d, 1) of the slot's variable
    float *fv = nullptr;          // [n][8] variable features
    float *fc = nullptr;          // [m][8] constraint features
};

}  // namespace ffsat

namespace ffsat {
hipError_t fill_f32(int64_t n, float *p, float v, hipStream_t s);
hipError_t take_cols(int rows, int H, const float *X, int xstride, float *dst, hipStream_t s);
}  // namespace ffsat
