// Kernel template: objective and per-literal gradient of every constraint, for a batch of
// restarts (paper: Alg. 2 steps i-iii for the value, Eq. chain / Thm. 4 for
// the reverse traversal; App. B for the transform-free OR/XOR products),
// fused with the exact round-and-check of the same point (Alg. 1).
//
// Mapping on CDNA4 (wave64): a wave owns one restart block and walks a
// chunk of `cpw` constraints of one bin.  Lane = (restart r, segment j):
// L adjacent lanes split the literals of a constraint into L segments of
// s = ceil(k/L) <= SEG literals, so literal values, prefix products and
// gradient accumulators of a segment live in registers (fully unrolled
// over SEG; every lane processes exactly SEG positions, padded past the
// constraint's end, so the arithmetic is straight-line code).  The
// per-frequency leave-one-out product of literal i is
//     (prefix inside its segment) * (product of earlier segments)
//   * (product of later segments) * (suffix inside its segment),
// the segment products being exchanged by exclusive prefix/suffix scans
// over the L lanes (DPP row shifts for L <= 16).  FP64 root-of-unity bins
// evaluate each segment's product as a polynomial in the frequency's factor
// coefficient and accumulate per-degree moments for the gradient (the
// polynomial form, below).  Constraint descriptors and
// coefficient tables are wave-uniform (scalar loads, the next frequency's
// entry prefetched); literal values are gathered from x[v][b] with restarts
// contiguous, so a wave reads 64/L consecutive restarts of a variable per
// load.
//
// Per-literal results go to a slot buffer [nnz][B] (value w_c * s_i *
// dWE_c/dl_i) that a segmented reduction over the variable-major transpose
// turns into the gradient, in a fixed order (deterministic).  Objective
// partials and violated-constraint counts go to per-(bin, chunk) rows.
#pragma once
#include "internal.h"

namespace ffsat {

template <typename T>
__device__ __forceinline__ T fmaT(T a, T b, T c);
template <>
__device__ __forceinline__ float fmaT<float>(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
template <>
__device__ __forceinline__ double fmaT<double>(double a, double b, double c) { return __builtin_fma(a, b, c); }

// lane (j - D) / (j + D) inside a group of L lanes; only read where valid.
// Groups of L <= 16 lanes never straddle a DPP row, so row shifts suffice.
// bound_ctrl: lanes whose source is outside the row read 0 (never used by
// the scans, which select on j >= D), so no "old" operand has to be set up
template <int CTRL>
__device__ __forceinline__ float dpp_f32(float v)
{
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), CTRL, 0xF, 0xF, true));
}
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v)
{
    const long long u = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_mov_dpp((int)(u & 0xffffffffll), CTRL, 0xF, 0xF, true);
    const int hi = __builtin_amdgcn_mov_dpp((int)(u >> 32), CTRL, 0xF, 0xF, true);
    return __longlong_as_double((long long)(unsigned)lo | ((long long)hi << 32));
}
template <int D, int L, typename CT>
__device__ __forceinline__ CT from_lower(CT v)
{
    if constexpr (L <= 16) {
        if constexpr (sizeof(CT) == 4) return dpp_f32<0x110 + D>(v);
        else return dpp_f64<0x110 + D>(v);
    } else {
        return __shfl_up(v, D, L);
    }
}
template <int D, int L, typename CT>
__device__ __forceinline__ CT from_upper(CT v)
{
    if constexpr (L <= 16) {
        if constexpr (sizeof(CT) == 4) return dpp_f32<0x100 + D>(v);
        else return dpp_f64<0x100 + D>(v);
    } else {
        return __shfl_down(v, D, L);
    }
}

template <typename CT, int L, int D>
__device__ __forceinline__ void scan_up_cplx(int j, CT &ar, CT &ai)
{
    if constexpr (D < L) {
        const CT yr = from_lower<D, L>(ar), yi = from_lower<D, L>(ai);
        if (j >= D) {
            const CT nr = fmaT(yr, ar, -yi * ai);
            const CT ni = fmaT(yr, ai, yi * ar);
            ar = nr; ai = ni;
        }
        scan_up_cplx<CT, L, 2 * D>(j, ar, ai);
    }
}
template <typename CT, int L, int D>
__device__ __forceinline__ void scan_down_cplx(int j, CT &br, CT &bi)
{
    if constexpr (D < L) {
        const CT yr = from_upper<D, L>(br), yi = from_upper<D, L>(bi);
        if (j + D < L) {
            const CT nr = fmaT(yr, br, -yi * bi);
            const CT ni = fmaT(yr, bi, yi * br);
            br = nr; bi = ni;
        }
        scan_down_cplx<CT, L, 2 * D>(j, br, bi);
    }
}

// Lane 15 of each even row broadcast to the following (odd) row; the even
// rows receive 1.  For 32-lane groups: the lower row's value to the upper.
__device__ __forceinline__ float bcast15_f32(float v)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(1.0f), __float_as_int(v), 0x142, 0xA, 0xF, false));
}
__device__ __forceinline__ double bcast15_f64(double v)
{
    const long long u = __double_as_longlong(v);
    const long long one = __double_as_longlong(1.0);
    const int lo = __builtin_amdgcn_update_dpp((int)(one & 0xffffffffll), (int)(u & 0xffffffffll), 0x142, 0xA, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp((int)(one >> 32), (int)(u >> 32), 0x142, 0xA, 0xF, false);
    return __longlong_as_double((long long)(unsigned)lo | ((long long)hi << 32));
}
template <typename CT>
__device__ __forceinline__ CT bcast15(CT v)
{
    if constexpr (sizeof(CT) == 4) return bcast15_f32(v);
    else return bcast15_f64(v);
}

// 32-lane groups: scans inside each 16-lane row with DPP; the lower row's
// total joins the upper row's prefixes through a row broadcast, and the
// upper row's total (one lane read) joins the lower row's suffixes.
template <typename CT>
__device__ __forceinline__ void group_scan_cplx32(int j, CT tr, CT ti, CT &er, CT &ei, CT &sr, CT &si)
{
    const int jr = j & 15;
    const bool upper = j >= 16;
    CT ar = tr, ai = ti, br = tr, bi = ti;
    scan_up_cplx<CT, 16, 1>(jr, ar, ai);      // inclusive prefix inside the row
    scan_down_cplx<CT, 16, 1>(jr, br, bi);    // inclusive suffix inside the row
    const CT t0r = bcast15(ar), t0i = bcast15(ai);           // lower row's total (upper rows)
    const int src = (int)(threadIdx.x & 63 & ~31) | 31;
    const CT t1r = __shfl(ar, src, 64), t1i = __shfl(ai, src, 64);   // upper row's total
    // inclusive prefix / suffix over the whole group
    CT pr = ar, pi = ai, qr = br, qi = bi;
    if (upper) {
        pr = fmaT(t0r, ar, -t0i * ai);
        pi = fmaT(t0r, ai, t0i * ar);
    } else {
        qr = fmaT(br, t1r, -bi * t1i);
        qi = fmaT(br, t1i, bi * t1r);
    }
    // exclusive: the neighbour's inclusive value inside the row, the row
    // totals across the boundary, 1 at the ends
    const CT xr = from_lower<1, 16>(pr), xi = from_lower<1, 16>(pi);
    const CT yr = from_upper<1, 16>(qr), yi = from_upper<1, 16>(qi);
    er = jr > 0 ? xr : (upper ? t0r : CT(1));
    ei = jr > 0 ? xi : (upper ? t0i : CT(0));
    sr = jr < 15 ? yr : (upper ? CT(1) : t1r);
    si = jr < 15 ? yi : (upper ? CT(0) : t1i);
}

// exclusive prefix (e) and suffix (s) products of the segment totals t
template <typename CT, int L>
__device__ __forceinline__ void group_scan_cplx(int j, CT tr, CT ti, CT &er, CT &ei, CT &sr, CT &si)
{
    if constexpr (L == 32) {
        group_scan_cplx32<CT>(j, tr, ti, er, ei, sr, si);
    } else if constexpr (L == 1) {
        er = 1; ei = 0; sr = 1; si = 0;
    } else {
        CT ar = tr, ai = ti, br = tr, bi = ti;
        scan_up_cplx<CT, L, 1>(j, ar, ai);
        scan_down_cplx<CT, L, 1>(j, br, bi);
        const CT pr = from_lower<1, L>(ar), pi = from_lower<1, L>(ai);
        const CT qr = from_upper<1, L>(br), qi = from_upper<1, L>(bi);
        er = j > 0 ? pr : CT(1);
        ei = j > 0 ? pi : CT(0);
        sr = j < L - 1 ? qr : CT(1);
        si = j < L - 1 ? qi : CT(0);
    }
}

template <typename CT, int L, int D>
__device__ __forceinline__ void scan_up_real(int j, CT &a)
{
    if constexpr (D < L) {
        const CT y = from_lower<D, L>(a);
        if (j >= D) a = y * a;
        scan_up_real<CT, L, 2 * D>(j, a);
    }
}
template <typename CT, int L, int D>
__device__ __forceinline__ void scan_down_real(int j, CT &b)
{
    if constexpr (D < L) {
        const CT y = from_upper<D, L>(b);
        if (j + D < L) b = y * b;
        scan_down_real<CT, L, 2 * D>(j, b);
    }
}

template <typename CT>
__device__ __forceinline__ void group_scan_real32(int j, CT t, CT &pre, CT &suf)
{
    const int jr = j & 15;
    const bool upper = j >= 16;
    CT a = t, b = t;
    scan_up_real<CT, 16, 1>(jr, a);
    scan_down_real<CT, 16, 1>(jr, b);
    const CT t0 = bcast15(a);
    const int src = (int)(threadIdx.x & 63 & ~31) | 31;
    const CT t1 = __shfl(a, src, 64);
    const CT p = upper ? t0 * a : a;
    const CT q = upper ? b : b * t1;
    const CT x = from_lower<1, 16>(p), y = from_upper<1, 16>(q);
    pre = jr > 0 ? x : (upper ? t0 : CT(1));
    suf = jr < 15 ? y : (upper ? CT(1) : t1);
}

template <typename CT, int L>
__device__ __forceinline__ void group_scan_real(int j, CT t, CT &pre, CT &suf)
{
    if constexpr (L == 32) {
        group_scan_real32<CT>(j, t, pre, suf);
    } else if constexpr (L == 1) {
        pre = 1; suf = 1;
    } else {
        CT a = t, b = t;
        scan_up_real<CT, L, 1>(j, a);
        scan_down_real<CT, L, 1>(j, b);
        const CT p = from_lower<1, L>(a), q = from_upper<1, L>(b);
        pre = j > 0 ? p : CT(1);
        suf = j < L - 1 ? q : CT(1);
    }
}

template <int L>
__device__ __forceinline__ int group_sum_int(int v)
{
#pragma unroll
    for (int d = 1; d < L; d <<= 1) v += __shfl_xor(v, d, L);
    return v;
}

// Butterfly product over groups of L lanes (FP64 complex): quad
// permutations for partners 1 and 2, half-row and row mirrors for 4 and 8
// (after the earlier stages every lane of a quad / half-row holds the same
// product, so a mirror reaches the other half), and the gfx950 row swap for
// 16.  Every lane ends with the product of its group (rounded in its own
// order).
template <int CTRL>
__device__ __forceinline__ void cmul_by_dpp(double &ar, double &ai)
{
    const double yr = dpp_f64<CTRL>(ar), yi = dpp_f64<CTRL>(ai);
    const double nr = fmaT(yr, ar, -yi * ai);
    const double ni = fmaT(yr, ai, yi * ar);
    ar = nr;
    ai = ni;
}
// this lane's value and the one of the same lane in the paired row (rows 0-1, 2-3)
__device__ __forceinline__ void swap_rows16(double v, double &a, double &b)
{
    const long long u = __double_as_longlong(v);
    const auto lo = __builtin_amdgcn_permlane16_swap((unsigned)(u & 0xffffffffll), (unsigned)(u & 0xffffffffll),
                                                     false, false);
    const auto hi = __builtin_amdgcn_permlane16_swap((unsigned)(u >> 32), (unsigned)(u >> 32), false, false);
    a = __longlong_as_double((long long)lo[0] | ((long long)hi[0] << 32));
    b = __longlong_as_double((long long)lo[1] | ((long long)hi[1] << 32));
}
template <int L>
__device__ __forceinline__ void allreduce_prod_f64(double &ar, double &ai)
{
    if constexpr (L >= 2) cmul_by_dpp<0xB1>(ar, ai);    // quad_perm [1,0,3,2]
    if constexpr (L >= 4) cmul_by_dpp<0x4E>(ar, ai);    // quad_perm [2,3,0,1]
    if constexpr (L >= 8) cmul_by_dpp<0x141>(ar, ai);   // row_half_mirror
    if constexpr (L >= 16) cmul_by_dpp<0x140>(ar, ai);  // row_mirror
    if constexpr (L >= 32) {
        double pr, pi, qr, qi;
        swap_rows16(ar, pr, qr);
        swap_rows16(ai, pi, qi);
        // {p, q} = {own, paired row's}: the same product on both rows
        ar = fmaT(pr, qr, -pi * qi);
        ai = fmaT(pr, qi, pi * qr);
    }
    static_assert(L <= 32, "groups of at most 32 lanes");
}
// 1 / v for v in the normal range: hardware estimate and one Newton step
// (the step squares the estimate's relative error; from at most 2^-22 that
// leaves below 2^-44, far inside what the leave-one-out products need)
__device__ __forceinline__ double recip_f64(double v)
{
    const double r = __builtin_amdgcn_rcp(v);
    const double e = fmaT(-v, r, 1.0);
    return fmaT(r, e, r);
}

// One complex frequency of a constraint: steps i-ii (affine factors psi and
// their running product), step iii (value term Re(c0 * prod psi)) and the
// reverse traversal that adds Re(c1 * leave-one-out product) to every
// position's gradient.  FORM 1: psi = 1 - i tk l; FORM 2: psi = tk - i l;
// FORM 3 (the unit-circle form of Eq. forward): psi = (tk + l) + i p0 with
// (tk, p0) = (cos, sin) of the frequency's root, so that c1 = c0.  FP32
// bins and the unit-circle form; FP64 bounded-basis bins take the polynomial
// form below.  The other lanes' products come from exclusive scans.
template <typename CT, int SEG, int L, int FORM>
__device__ __forceinline__ void freq_pass(const int j, const CT (&lv)[SEG], CT (&gr)[SEG], const FreqT<CT> &fr,
                                          CT &we)
{
    static_assert(sizeof(CT) == 4 || FORM == 3, "FP64 bounded-basis bins use freq_pass_poly");
    // form-1 segments of at most 16: the reverse pass reuses the forward
    // pass's tau * l (SEG more VGPRs, one multiply less per position)
    constexpr bool KEEP_U = FORM == 1 && SEG <= 16;
    const CT tk = fr.tk;
    CT pr[SEG], pi[SEG];
    CT uk[KEEP_U ? SEG : 1];
    CT Pr = fr.init, Pi = 0;
#pragma unroll
    for (int t = 0; t < SEG; ++t) {
        pr[t] = Pr; pi[t] = Pi;
        if constexpr (FORM == 1) {
            const CT u = tk * lv[t];
            if constexpr (KEEP_U) uk[t] = u;
            const CT nr = fmaT(Pi, u, Pr);
            const CT ni = fmaT(-Pr, u, Pi);
            Pr = nr; Pi = ni;
        } else if constexpr (FORM == 2) {
            const CT l = lv[t];
            const CT nr = fmaT(Pi, l, tk * Pr);
            const CT ni = fmaT(-Pr, l, tk * Pi);
            Pr = nr; Pi = ni;
        } else {
            const CT u = tk + lv[t];
            const CT nr = fmaT(Pr, u, -Pi * fr.p0);
            const CT ni = fmaT(Pi, u, Pr * fr.p0);
            Pr = nr; Pi = ni;
        }
    }
    // product of the other lanes' segments (exclusive prefix times exclusive suffix)
    CT er, ei, sr, si;
    group_scan_cplx<CT, L>(j, Pr, Pi, er, ei, sr, si);
    const CT Gr = fmaT(Pr, sr, -Pi * si);
    const CT Gi = fmaT(Pr, si, Pi * sr);
    we += fmaT(fr.c0re, Gr, -fr.c0im * Gi);
    const CT qr = fmaT(er, sr, -ei * si);
    const CT qi = fmaT(er, si, ei * sr);
    // the factors are recomputed from an opaque copy of tk so that the
    // forward products are not kept alive across both passes
    CT tkb = tk;
    asm volatile("" : "+v"(tkb));
    CT Sr = fmaT(fr.c1re, qr, -fr.c1im * qi);
    CT Si = fmaT(fr.c1re, qi, fr.c1im * qr);
#pragma unroll
    for (int t = SEG - 1; t >= 0; --t) {
        gr[t] = fmaT(pr[t], Sr, fmaT(-pi[t], Si, gr[t]));
        if (t > 0) {
            if constexpr (FORM == 1) {
                const CT u = KEEP_U ? uk[t] : tkb * lv[t];
                const CT nr = fmaT(Si, u, Sr);
                const CT ni = fmaT(-Sr, u, Si);
                Sr = nr; Si = ni;
            } else if constexpr (FORM == 2) {
                const CT l = lv[t];
                const CT nr = fmaT(Si, l, tkb * Sr);
                const CT ni = fmaT(-Sr, l, tkb * Si);
                Sr = nr; Si = ni;
            } else {
                const CT u = tkb + lv[t];
                const CT nr = fmaT(Sr, u, -Si * fr.p0);
                const CT ni = fmaT(Si, u, Sr * fr.p0);
                Sr = nr; Si = ni;
            }
        }
    }
}

// ---- FP64 root-of-unity products in the polynomial form
//
// A lane's segment product of form-1 factors, init * prod_t (1 - i tau l_t),
// is init * sum_m e_m z^m at z = -i tau, e_m the elementary symmetric
// polynomials of the segment's literals: they do not depend on the
// frequency, so the lane forms them once per constraint and each frequency
// evaluates two real polynomials in sg = z^2 = -tau^2 (Horner), about SEG
// FP64 operations instead of 3 SEG for the running product.  The leave-one-out
// product of position t is init * sum_m e^(-t)_m z^m (e^(-t): the elementary
// symmetric polynomials of the other positions), so each position's gradient,
// sum over frequencies of Re(C z^m) e^(-t)_m with C = c1 * (product of the
// other lanes) * init, only needs the moments H_m = sum_f Re(C_f z_f^m): 1.5
// operations per position and frequency; the positions' gradients follow
// from H once per constraint (seg_grad_from_moments).  Rounding: every
// quantity is a sum of products of nonnegative weights (the polynomials of
// |l|) with the exact terms, so the error of a frequency's contribution is
// within about SEG eps prod_t (1 + |tau l_t|) <= SEG eps 2^(SEG/2) |prod_t
// (1 - i tau l_t)|: below 1e-9 relative for SEG <= 32 in FP64 (not in FP32,
// which keeps the running products).

// e[0..SEG]: elementary symmetric polynomials of v[0..SEG-1]
template <int SEG>
__device__ __forceinline__ void seg_esp(const double (&v)[SEG], double (&e)[SEG + 1])
{
    e[0] = 1.0;
#pragma unroll
    for (int m = 1; m <= SEG; ++m) e[m] = 0.0;
#pragma unroll
    for (int t = 0; t < SEG; ++t) {
#pragma unroll
        for (int m = SEG; m >= 1; --m)
            if (m <= t + 1) e[m] = fmaT(v[t], e[m - 1], e[m]);
    }
}

// One frequency: value term Re(c0 T) into we (T: the product over the
// group's L lanes) and the moments H_m += Re(c1 (T / P) init z^m), P this
// lane's segment product.  With W = c1 init T / P and c0 = i c1 / tau,
// Re(c0 T) = Re(W (A - i tau B) i / tau) = B Re(W) + A tau Im(W) / sg.
template <int SEG, int L>
__device__ __forceinline__ void freq_pass_poly(const double (&e)[SEG + 1], double (&H)[SEG], const FreqPoly &fr,
                                               double &we)
{
    const double sg = fr.sg;
    constexpr int NE = SEG / 2;         // highest even degree 2 NE <= SEG
    constexpr int NO = (SEG - 1) / 2;   // highest odd degree 2 NO + 1 <= SEG
    double A = e[2 * NE];
#pragma unroll
    for (int n = NE - 1; n >= 0; --n) A = fmaT(A, sg, e[2 * n]);
    double Bo = e[2 * NO + 1];
#pragma unroll
    for (int n = NO - 1; n >= 0; --n) Bo = fmaT(Bo, sg, e[2 * n + 1]);
    const double Pr = fr.init * A;   // P = init (A - i tau B)
    const double Pi = -fr.itau * Bo;
    double qr = 1.0, qi = 0.0;       // T / P: the other lanes' product
    if constexpr (L >= 2) {
        double Tr = Pr, Ti = Pi;
        allreduce_prod_f64<L>(Tr, Ti);
        const double nrm = fmaT(Pr, Pr, Pi * Pi);
        const double rinv = recip_f64(nrm);
        const double ir = Pr * rinv, ii = -Pi * rinv;
        qr = fmaT(Tr, ir, -Ti * ii);
        qi = fmaT(Tr, ii, Ti * ir);
    }
    // Re(W) and tau Im(W); Re(W z^(2n)) = sg^n Re(W), Re(W z^(2n+1)) = sg^n tau Im(W)
    const double Cr = fmaT(fr.c1ire, qr, -fr.c1iim * qi);
    const double Ci = fmaT(fr.c1tre, qi, fr.c1tim * qr);
    we = fmaT(Cr, Bo, we);
    we = fmaT(Ci * fr.isg, A, we);
    double pw = 1.0;
#pragma unroll
    for (int n = 0; 2 * n < SEG; ++n) {
        H[2 * n] = fmaT(pw, Cr, H[2 * n]);
        if (2 * n + 1 < SEG) H[2 * n + 1] = fmaT(pw, Ci, H[2 * n + 1]);
        if (2 * n + 2 < SEG) pw *= sg;
    }
}

// out(t, sum_m e^(-t)_m H_m) for every position t of the segment, with no
// division (no cancellation beyond the bound above).  Blocks of GB positions,
// last block first.  R = the moments taken through the positions after the
// block (R_q = sum_j S_j H_(q+j), S the polynomials of those positions; one
// in-place step R_q += v_u R_(q+1) per position, so R starts as H); K_a =
// sum_i P_i R_(a+i) with P the polynomials of the positions before the block;
// inside the block the same once more: G = K taken through the block's
// positions after t, and out(t, sum_i Q_i G_i), Q the polynomials of the
// block's positions before t.  About 2 SEG^2 FMAs per lane (SEG = 32), once
// per constraint.  H is overwritten.
template <int SEG, typename V, typename Out>
__device__ __forceinline__ void seg_grad_from_moments(V (&v)[SEG], double (&H)[SEG], Out &&out)
{
    // every loop has a constant trip count with the bounds as conditions in
    // the body, so that full unrolling never leaves an indexed array behind
    constexpr int GB = 8;
    constexpr int NBLK = (SEG + GB - 1) / GB;
#pragma unroll
    for (int bi = NBLK - 1; bi >= 0; --bi) {
        const int lo = bi * GB;
        const int nb = lo + GB <= SEG ? GB : SEG - lo;
        const int hi = lo + nb;
        // one block at a time: opaque inputs keep the scheduler from
        // interleaving the blocks (each holds its own P, K and G)
#pragma unroll
        for (int u = 0; u < SEG; ++u) asm volatile("" : "+v"(v[u]), "+v"(H[u]));
        double P[SEG + 1];
        P[0] = 1.0;
#pragma unroll
        for (int m = 1; m <= SEG; ++m) P[m] = 0.0;
#pragma unroll
        for (int u = 0; u < SEG; ++u) {
            if (u < lo) {
                const double vu = (double)v[u];
#pragma unroll
                for (int m = SEG; m >= 1; --m)
                    if (m <= u + 1) P[m] = fmaT(vu, P[m - 1], P[m]);
            }
        }
        double G[GB];
#pragma unroll
        for (int a2 = 0; a2 < GB; ++a2) {
            double acc = 0.0;
#pragma unroll
            for (int i = 0; i <= SEG; ++i)
                if (a2 < nb && i <= lo) acc = fmaT(P[i], H[a2 + i < SEG ? a2 + i : 0], acc);
            G[a2] = acc;
        }
#pragma unroll
        for (int tl = GB - 1; tl >= 0; --tl) {
            if (tl < nb) {
                double Q[GB];
                Q[0] = 1.0;
#pragma unroll
                for (int m = 1; m < GB; ++m) Q[m] = 0.0;
#pragma unroll
                for (int u = 0; u < GB; ++u) {
                    if (u < tl) {
                        const double vu = (double)v[lo + u < SEG ? lo + u : 0];
#pragma unroll
                        for (int m = GB - 1; m >= 1; --m)
                            if (m <= u + 1) Q[m] = fmaT(vu, Q[m - 1], Q[m]);
                    }
                }
                double g = 0.0;
#pragma unroll
                for (int i = 0; i < GB; ++i)
                    if (i <= tl) g = fmaT(Q[i], G[i], g);
                out(lo + tl, g);
                const double vt = (double)v[lo + tl < SEG ? lo + tl : 0];
#pragma unroll
                for (int i = 0; i < GB - 1; ++i)
                    if (i < tl) G[i] = fmaT(vt, G[i + 1], G[i]);
            }
        }
        // R for the previous block: the moments taken through this block too
#pragma unroll
        for (int u = 0; u < GB; ++u) {
            if (bi > 0 && u < nb) {
                const double vu = (double)v[lo + u < SEG ? lo + u : 0];
                const int len = hi - u;
#pragma unroll
                for (int q = 0; q < SEG - 1; ++q)
                    if (q < len - 1) H[q] = fmaT(vu, H[q + 1], H[q]);
            }
        }
    }
}

// First frequency of wave w of fg that split a constraint's n1 form-1 and
// nf - n1 form-2 frequencies (and the real chain, on the last wave) into
// shares of about equal estimated VALU work.  Wave-uniform integer arithmetic.
__device__ __forceinline__ int freq_bound(int w, int fg, int n1, int nf, int has_real)
{
    if (w <= 0) return 0;
    if (w >= fg) return nf;
    const int total = 4 * n1 + 5 * (nf - n1) + (has_real ? 4 : 0);
    const int tgt = (total * w + fg / 2) / fg;
    const int f = tgt <= 4 * n1 ? (tgt + 3) / 4 : n1 + (tgt - 4 * n1 + 4) / 5;
    return min(f, nf);
}

// Partial sums of the fg waves of a workgroup that split a constraint's
// frequencies (v[] and we), added in wave order by wave 0.  One base index
// per wave, positions at constant offsets; the index (not the pointer, which
// must stay an LDS pointer) is opaque so that the compiler does not hoist SEG
// addresses.
template <typename CT, int SEG>
__device__ __forceinline__ void waves_reduce(void *lds, int wg, int fg, int lane, CT (&v)[SEG], CT &we)
{
    CT *red = reinterpret_cast<CT *>(lds);
    if (wg > 0) {
        int base = (wg - 1) * (SEG + 1) * 64 + lane;
        asm volatile("" : "+v"(base));
#pragma unroll
        for (int t = 0; t < SEG; ++t) red[base + t * 64] = v[t];
        red[base + SEG * 64] = we;
    }
    __syncthreads();
    if (wg == 0) {
#pragma unroll
        for (int q = 1; q < 4; ++q) {
            if (q < fg) {
                int base = (q - 1) * (SEG + 1) * 64 + lane;
                asm volatile("" : "+v"(base));
#pragma unroll
                for (int t = 0; t < SEG; ++t) v[t] += red[base + t * 64];
                we += red[base + SEG * 64];
            }
        }
    }
    __syncthreads();   // the next constraint reuses the buffer
}

// The work of one wave: unit = (chunk of sp.cpw constraints of the range
// sp.first .. sp.first + sp.count, restart block rb).  `unit` must be
// wave-uniform.  Root-of-unity kernels may split a unit's frequencies over
// fg <= 4 waves of one workgroup (wave wg takes a contiguous share, the
// last one also the real chain); waves 1.. pass their partial gradients and
// values through LDS (`lds`: (fg - 1) * (SEG + 1) * 64 values) and wave 0
// adds them in wave order and writes the results.  Read-only inputs are
// separate __restrict__ arguments: the compiler may then read uniform
// descriptors and coefficients through the scalar cache.  UC: the
// root-of-unity bins take the unit-circle form (every frequency FORM 3).
template <typename IO, typename CT, int SEG, int L, bool CPLX, bool UC = false>
__device__ __forceinline__ void eval_unit(const EvalArgs<IO> &a, const Span sp, const int unit,
                                          const IO *__restrict__ xin, const ConDesc *__restrict__ con,
                                          const int32_t *__restrict__ lits, const float *__restrict__ wts,
                                          const TypeT<CT> *__restrict__ types,
                                          const FreqT<CT> *__restrict__ freqs, const int fg_in, const int wg_in,
                                          void *lds)
{
    const int fg = CPLX ? fg_in : 1;
    const int wg = CPLX ? wg_in : 0;
    // FP64 root-of-unity bins take the polynomial form (seg_esp / freq_pass_poly)
    constexpr bool POLY = CPLX && !UC && sizeof(CT) == 8 && SEG <= 32;
    constexpr int RPW = 64 / L;
    const int lane = threadIdx.x & 63;
    const int n_chunks = (sp.count + sp.cpw - 1) / sp.cpw;
    if (unit >= n_chunks * sp.n_rb) return;   // whole wave leaves together
    if (a.skip != nullptr && *a.skip == 0) return;   // uniform: every wave of the launch leaves
    const int chunk = unit / sp.n_rb;
    const int rb = unit - chunk * sp.n_rb;
    const int j = lane & (L - 1);
    const int r = lane / L;
    const int b = rb * RPW + r;
    const bool bok = b < a.B;
    const int bb = bok ? b : a.B - 1;
    const int i0 = j * SEG;
    CT facc = 0;
    int nunsat = 0;
    const int c_begin = chunk * sp.cpw;
    const int c_end = min(c_begin + sp.cpw, sp.count);
#pragma unroll 1
    for (int ci = c_begin; ci < c_end; ++ci) {
        const ConDesc d = con[sp.first + ci];
        const TypeT<CT> ty = types[d.type];
        const int k = d.k;

        // step i input: this lane's SEG positions j*SEG .. j*SEG+SEG-1; the
        // positions past the constraint's end hold the padding value (count
        // neutral; its factor is divided out of the coefficients on the
        // host).  Also the rounded truth of each literal (x_v < 0: True).
        // Branch-free: all literal loads (indices clamped into the
        // constraint), then all point loads, so that a lane waits for two
        // memory round trips per constraint rather than two per position.
        // kernels with long constraints: per-constraint copies the compiler cannot
        // hoist; otherwise it keeps i0 + t and the bit constants 1 << t in
        // SEG registers each across the whole kernel (real-chain kernels run
        // many constraints per wave and profit from the hoisting)
        int i0c = i0;
        uint32_t one = 1u;
        if constexpr (CPLX || L > 1) asm volatile("" : "+v"(i0c), "+v"(one));
        int nv = min(max(k - i0c, 0), SEG);   // positions of this lane inside the constraint
        int lt[SEG];
#pragma unroll
        for (int t = 0; t < SEG; ++t) lt[t] = lits[d.off + min(i0c + t, k - 1)];
        IO xr[SEG];
#pragma unroll
        for (int t = 0; t < SEG; ++t) xr[t] = xin[(size_t)(lt[t] & 0x7fffffff) * a.B + bb];
        CT lv[SEG];
        uint32_t negm = 0, tmask = 0;
#pragma unroll
        for (int t = 0; t < SEG; ++t) {
            const bool in = t < nv;
            const bool neg = lt[t] < 0;
            const CT xv = (CT)xr[t];
            lv[t] = in ? (neg ? -xv : xv) : ty.pad;
            const bool vt = xr[t] < IO(0);
            negm |= ((in && neg) ? one : 0u) << t;
            tmask |= ((in && (neg != vt)) ? one : 0u) << t;
        }
        // opaque: otherwise the stores re-derive the sign bits from the
        // loaded literals, which then stay live across the frequency loop
        asm volatile("" : "+v"(negm));
        if (a.want_check && wg == 0) {
            const int cnt = group_sum_int<L>(__popc(tmask));
            const bool sat = d.chk >= 0 ? (cnt >= d.chk) : ((cnt & 1) == (d.chk == -2 ? 1 : 0));
            const bool uns = !sat && bok && j == 0;
            nunsat += uns ? 1 : 0;
            if (a.unsat_bits != nullptr && uns)
                atomicOr(&a.unsat_bits[(size_t)b * a.wm + (d.orig >> 5)], 1u << (d.orig & 31));
            if (a.U != nullptr) {
                const unsigned long long bal = __ballot(uns);
                if (lane == 0 && bal != 0ull) atomicAdd(&a.U[d.orig], (int)__popcll(bal));
            }
        }
        if (!a.do_value) continue;

        CT gr[SEG];
        CT we = 0;
        if constexpr (POLY) {
            // FP64 root-of-unity products in the polynomial form: moments of
            // every frequency, then the positions' gradients from them
            double e[SEG + 1];
            seg_esp<SEG>(lv, e);
            double H[SEG];
#pragma unroll
            for (int t = 0; t < SEG; ++t) {
                H[t] = 0;
                asm volatile("" : "+v"(H[t]));
            }
            const int n1 = ty.n1, nf = ty.n1 + ty.n2;
            const int f0 = freq_bound(wg, fg, n1, nf, ty.has_real);
            const int f1 = freq_bound(wg + 1, fg, n1, nf, ty.has_real);
            // two frequencies per iteration: their Horner chains, butterflies
            // and divisions interleave (a loop with cross-lane moves is not
            // unrolled by the compiler), one wait for both coefficient loads
            const FreqPoly *fp = reinterpret_cast<const FreqPoly *>(freqs) + ty.tab;
            int f = f0;
#pragma unroll 1
            for (; f + 1 < f1; f += 2) {
                const FreqPoly fa = fp[f], fb = fp[f + 1];
                freq_pass_poly<SEG, L>(e, H, fa, we);
                freq_pass_poly<SEG, L>(e, H, fb, we);
            }
            if (f < f1) freq_pass_poly<SEG, L>(e, H, fp[f], we);
            if (ty.has_real && wg == fg - 1) {
                // the chain prod l of the root z = -1 (alpha = 0, beta = 1;
                // padding factors 1): its segment product is e_SEG and the
                // leave-one-out products inside the segment are e^(-t)_(SEG-1)
                CT pre, suf;
                group_scan_real<CT, L>(j, e[SEG], pre, suf);
                we += ty.c0r * (e[SEG] * suf);
                H[SEG - 1] = fmaT(ty.c1r, pre * suf, H[SEG - 1]);
            }
            if (fg > 1) {
                waves_reduce<CT, SEG>(lds, wg, fg, lane, H, we);
                if (wg > 0) continue;
            }
            we += ty.cst;
            const CT wc = (CT)wts[d.orig];
            if (j == 0) facc = fmaT(wc, we, facc);
            if (a.con_val != nullptr && j == 0 && bok) a.con_val[(size_t)d.orig * a.B + b] = (IO)we;
            if (a.want_grad && bok) {
                asm volatile("" : "+v"(nv));
                // the literals again, from memory (L2): keeping them across
                // the frequency loop would cost SEG registers there.  The
                // opaque index keeps the compiler from reusing the first loads.
                int ib = i0;
                asm volatile("" : "+v"(ib));
                int lr[SEG];
#pragma unroll
                for (int t = 0; t < SEG; ++t) lr[t] = lits[d.off + min(ib + t, k - 1)];
                IO lio[SEG];
#pragma unroll
                for (int t = 0; t < SEG; ++t) {
                    const IO xv = xin[(size_t)(lr[t] & 0x7fffffff) * a.B + bb];
                    lio[t] = t < nv ? (lr[t] < 0 ? -xv : xv) : (IO)ty.pad;
                }
                seg_grad_from_moments<SEG>(lio, H, [&](int t, double g) {
                    if (t < nv) {
                        const CT gv = ((negm >> t) & 1u) ? -g : g;
                        a.slot[(size_t)(d.off + i0 + t) * a.B + b] = (IO)(wc * gv);
                    }
                });
            }
            continue;
        } else {
#pragma unroll
            for (int t = 0; t < SEG; ++t) {
                gr[t] = 0;
                // materialised here, once: keeps one register set for the
                // accumulators across both frequency loops (no bypass copies)
                if constexpr (CPLX) asm volatile("" : "+v"(gr[t]));
            }
            if constexpr (CPLX && UC) {
                const int nf = ty.n1;
                const int f0 = (nf * wg) / fg, f1 = (nf * (wg + 1)) / fg;
                FreqT<CT> fr = freqs[ty.tab + f0];
#pragma unroll 1
                for (int f = f0; f < f1; ++f) {
                    const FreqT<CT> nxt = freqs[ty.tab + f + 1];
                    freq_pass<CT, SEG, L, 3>(j, lv, gr, fr, we);
                    fr = nxt;
                }
            } else if constexpr (CPLX) {
                const int n1 = ty.n1, nf = ty.n1 + ty.n2;
                // this wave's frequencies: equal shares of the estimated work
                // (4 units per form-1 frequency, 5 per form-2 one, 4 for the real
                // chain, which the last wave takes)
                const int f0 = freq_bound(wg, fg, n1, nf, ty.has_real);
                const int f1 = freq_bound(wg + 1, fg, n1, nf, ty.has_real);
                FreqT<CT> fr = freqs[ty.tab + f0];
#pragma unroll 1
                for (int f = f0; f < min(f1, n1); ++f) {
                    const FreqT<CT> nxt = freqs[ty.tab + f + 1];   // table has one entry of padding
                    freq_pass<CT, SEG, L, 1>(j, lv, gr, fr, we);
                    fr = nxt;
                }
#pragma unroll 1
                for (int f = max(f0, n1); f < f1; ++f) {
                    const FreqT<CT> nxt = freqs[ty.tab + f + 1];
                    freq_pass<CT, SEG, L, 2>(j, lv, gr, fr, we);
                    fr = nxt;
                }
            }
            if (ty.has_real && wg == fg - 1) {
                // real chain: prod (alpha + beta l); padding factors are exactly 1
                CT q[SEG];
                CT P = 1;
#pragma unroll
                for (int t = 0; t < SEG; ++t) {
                    q[t] = P;
                    P = P * fmaT(ty.beta, lv[t], ty.alpha);
                }
                CT pre, suf;
                group_scan_real<CT, L>(j, P, pre, suf);
                we += ty.c0r * (P * suf);
                CT S = ty.c1r * (pre * suf);
#pragma unroll
                for (int t = SEG - 1; t >= 0; --t) {
                    gr[t] = fmaT(q[t], S, gr[t]);
                    if (t > 0) S = S * fmaT(ty.beta, lv[t], ty.alpha);
                }
            }
            if constexpr (CPLX) {
                if (fg > 1) {
                    waves_reduce<CT, SEG>(lds, wg, fg, lane, gr, we);
                    if (wg > 0) continue;
                }
            }
        }
        we += ty.cst;
        const CT wc = (CT)wts[d.orig];
        if (j == 0) facc = fmaT(wc, we, facc);
        if (a.con_val != nullptr && j == 0 && bok) a.con_val[(size_t)d.orig * a.B + b] = (IO)we;
        if (a.want_grad && bok) {
            // fresh predicates: keep the load phase's lane masks from living
            // across the frequency loop
            asm volatile("" : "+v"(nv));
#pragma unroll
            for (int t = 0; t < SEG; ++t) {
                const int i = i0 + t;
                if (t < nv) {
                    const CT gv = ((negm >> t) & 1u) ? -gr[t] : gr[t];
                    a.slot[(size_t)(d.off + i) * a.B + b] = (IO)(wc * gv);
                }
            }
        }
    }
    if (j == 0 && bok && wg == 0) {
        const size_t row = (size_t)(sp.fpart_row0 + chunk) * a.B + b;
        if (a.do_value) a.fpart[row] = (IO)facc;
        if (a.want_check) a.cpart[row] = nunsat;
    }
}

// One bin per launch.
template <typename IO, typename CT, int SEG, int L, bool CPLX>
__global__ __launch_bounds__(256) void k_eval(EvalArgs<IO> a, const IO *__restrict__ xin,
                                              const ConDesc *__restrict__ con,
                                              const int32_t *__restrict__ lits,
                                              const float *__restrict__ wts,
                                              const TypeT<CT> *__restrict__ types,
                                              const FreqT<CT> *__restrict__ freqs)
{
    extern __shared__ __align__(16) char eval_lds[];
    // the wave index is uniform: say so, so that everything derived from it
    // (constraint descriptors, coefficient tables, loop bounds) stays scalar
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const bool split = CPLX && a.fg > 1;   // one unit per block, its frequencies over the waves
    const int unit = split ? (int)blockIdx.x : (int)blockIdx.x * (int)(blockDim.x >> 6) + wave;
    const Span sp{a.first, a.count, a.cpw, a.n_rb, a.fpart_row0};
    eval_unit<IO, CT, SEG, L, CPLX>(a, sp, unit, xin, con, lits, wts, types, freqs, split ? a.fg : 1,
                                    split ? wave : 0, eval_lds);
}

template <typename IO>
struct EvalFnT {
    template <typename CT>
    using type = void (*)(EvalArgs<IO>, const IO *, const ConDesc *, const int32_t *, const float *,
                          const TypeT<CT> *, const FreqT<CT> *);
};
// type-erased kernel handle: the kernel and the arithmetic type it expects
template <typename IO>
struct EvalFn {
    const void *fn = nullptr;
    int ct = 0;
    explicit operator bool() const { return fn != nullptr; }
};

// Segment shapes.  FP32 arithmetic: L = 1 with SEG in {4, 8, ..., 32}, L >= 2
// with SEG in {16, 20, 24, 28, 32}.  FP64 arithmetic: L = 1 with SEG in
// {4, 8, ..., 24}; L = 2..8 with SEG in {16, 20, 24}, L = 8 also with every
// SEG from 25 to 32; L = 16 with every SEG from 14 to 32 (the long root-of-unity bins: a padding position costs as
// much as a literal in every frequency, and in the polynomial form the
// per-frequency cost of a lane, about 2.5 SEG operations plus a butterfly
// stage per doubling of L, favours long segments; 32 positions still fit 2
// waves per SIMD).
template <typename IO, typename CT, int SEG, int L, bool CPLX>
static EvalFn<IO> handle()
{
    EvalFn<IO> h;
    h.fn = reinterpret_cast<const void *>(&k_eval<IO, CT, SEG, L, CPLX>);
    h.ct = sizeof(CT) == 4 ? CT_F32 : CT_F64;
    return h;
}

template <typename IO, typename CT, bool CPLX, int L>
static EvalFn<IO> pick_L(int seg)
{
    constexpr bool F64 = sizeof(CT) == 8;
    switch (seg) {
    case 4: if constexpr (L == 1) return handle<IO, CT, 4, L, CPLX>(); break;
    case 8: if constexpr (L == 1) return handle<IO, CT, 8, L, CPLX>(); break;
    case 12: if constexpr (L == 1) return handle<IO, CT, 12, L, CPLX>(); break;
    case 14: if constexpr (F64 && L == 16) return handle<IO, CT, 14, L, CPLX>(); break;
    case 15: if constexpr (F64 && L == 16) return handle<IO, CT, 15, L, CPLX>(); break;
    case 16: if constexpr (!F64 || L <= 16) return handle<IO, CT, 16, L, CPLX>(); break;
    case 17: if constexpr (F64 && L == 16) return handle<IO, CT, 17, L, CPLX>(); break;
    case 18: if constexpr (F64 && L == 16) return handle<IO, CT, 18, L, CPLX>(); break;
    case 19: if constexpr (F64 && L == 16) return handle<IO, CT, 19, L, CPLX>(); break;
    case 20: if constexpr (!F64 || L <= 16) return handle<IO, CT, 20, L, CPLX>(); break;
    case 21: if constexpr (F64 && L == 16) return handle<IO, CT, 21, L, CPLX>(); break;
    case 22: if constexpr (F64 && L == 16) return handle<IO, CT, 22, L, CPLX>(); break;
    case 23: if constexpr (F64 && L == 16) return handle<IO, CT, 23, L, CPLX>(); break;
    case 24: if constexpr (!F64 || L <= 16) return handle<IO, CT, 24, L, CPLX>(); break;
    case 25: if constexpr (F64 && (L == 8 || L == 16)) return handle<IO, CT, 25, L, CPLX>(); break;
    case 26: if constexpr (F64 && (L == 8 || L == 16)) return handle<IO, CT, 26, L, CPLX>(); break;
    case 27: if constexpr (F64 && (L == 8 || L == 16)) return handle<IO, CT, 27, L, CPLX>(); break;
    case 28: if constexpr (!F64 || L == 8 || L == 16) return handle<IO, CT, 28, L, CPLX>(); break;
    case 29: if constexpr (F64 && (L == 8 || L == 16)) return handle<IO, CT, 29, L, CPLX>(); break;
    case 30: if constexpr (F64 && (L == 8 || L == 16)) return handle<IO, CT, 30, L, CPLX>(); break;
    case 31: if constexpr (F64 && (L == 8 || L == 16)) return handle<IO, CT, 31, L, CPLX>(); break;
    case 32: if constexpr (!F64 || L == 8 || L == 16) return handle<IO, CT, 32, L, CPLX>(); break;
    default: break;
    }
    return EvalFn<IO>{};
}

template <typename IO, typename CT, bool CPLX>
static EvalFn<IO> pick_seg(int seg, int L)
{
    switch (L) {
    case 1: return pick_L<IO, CT, CPLX, 1>(seg);
    case 2: return pick_L<IO, CT, CPLX, 2>(seg);
    case 4: return pick_L<IO, CT, CPLX, 4>(seg);
    case 8: return pick_L<IO, CT, CPLX, 8>(seg);
    case 16: return pick_L<IO, CT, CPLX, 16>(seg);
    case 32: if constexpr (sizeof(CT) == 8) return pick_L<IO, CT, CPLX, 32>(seg); break;
    default: break;
    }
    return EvalFn<IO>{};
}

template <typename IO>
static hipError_t launch_fn(EvalFn<IO> fn, const Bin &bin, const EvalArgs<IO> &a, hipStream_t s)
{
    if (!fn) return hipErrorInvalidValue;
    const int n_chunks = (a.count + a.cpw - 1) / a.cpw;
    const int64_t units = (int64_t)n_chunks * a.n_rb;
    if (units <= 0) return hipSuccess;
    const bool split = bin.cls == CLASS_DFT && a.fg > 1;
    const int wpb = split ? a.fg : bin.wpb;
    const int64_t blocks = split ? units : (units + wpb - 1) / wpb;
    const size_t lds = split ? (size_t)(a.fg - 1) * (bin.seg + 1) * 64 * (fn.ct == CT_F32 ? 4 : 8) : 0;
    if (fn.ct == CT_F32) {
        auto k = reinterpret_cast<typename EvalFnT<IO>::template type<float>>(const_cast<void *>(fn.fn));
        hipLaunchKernelGGL(k, dim3((unsigned)blocks), dim3(64 * wpb), lds, s, a, a.x, a.con, a.lit, a.w,
                           reinterpret_cast<const TypeT<float> *>(a.types),
                           reinterpret_cast<const FreqT<float> *>(a.freqs));
    } else {
        auto k = reinterpret_cast<typename EvalFnT<IO>::template type<double>>(const_cast<void *>(fn.fn));
        hipLaunchKernelGGL(k, dim3((unsigned)blocks), dim3(64 * wpb), lds, s, a, a.x, a.con, a.lit, a.w,
                           reinterpret_cast<const TypeT<double> *>(a.types),
                           reinterpret_cast<const FreqT<double> *>(a.freqs));
    }
    return hipGetLastError();
}

}  // namespace ffsat
