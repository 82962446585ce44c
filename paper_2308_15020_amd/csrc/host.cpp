// Host runtime of the ffsat library: validation, CSR / transpose / bins,
// conjugated coefficient tables in FP64, plans and their workspace,
// graph capture of the step loop, the tile-shape autotuner, and every
// C-ABI entry point declared in include/ffsat.h.
#include <algorithm>
#include <cmath>
#include <complex>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <sstream>
#include <tuple>
#include <string>
#include <vector>

#include "internal.h"

using namespace ffsat;

// ------------------------------------------------------------------ errors

static thread_local std::string g_last_error;

static ffsat_status fail(ffsat_status st, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return st;
}

ffsat_status ffsat_fail_external(ffsat_status st, const char *msg) { return fail(st, "%s", msg); }

#define HIPCHK(call)                                                                      \
    do {                                                                                  \
        hipError_t e_ = (call);                                                           \
        if (e_ != hipSuccess)                                                             \
            return fail(e_ == hipErrorOutOfMemory ? FFSAT_E_NOMEM : FFSAT_E_HIP,          \
                        "%s failed: %s", #call, hipGetErrorString(e_));                   \
    } while (0)

extern "C" const char *ffsat_status_string(ffsat_status s)
{
    switch (s) {
    case FFSAT_OK: return "ok";
    case FFSAT_E_INVALID_ARG: return "invalid argument";
    case FFSAT_E_VAR_RANGE: return "literal out of variable range";
    case FFSAT_E_DUP_VAR: return "variable repeated in a constraint";
    case FFSAT_E_EMPTY_CONSTRAINT: return "empty constraint";
    case FFSAT_E_BAD_KIND: return "unknown constraint kind";
    case FFSAT_E_DEVICE_MISMATCH: return "device mismatch";
    case FFSAT_E_NOMEM: return "out of memory";
    case FFSAT_E_HIP: return "HIP runtime error";
    case FFSAT_E_NONFINITE: return "non-finite input";
    case FFSAT_E_UNSUPPORTED: return "unsupported";
    default: return "unknown status";
    }
}

extern "C" const char *ffsat_last_error(void) { return g_last_error.c_str(); }
extern "C" const char *ffsat_version(void) { return "ffsat 0.1.0 (gfx950)"; }

// ------------------------------------------------------------------ coefficients

namespace {

constexpr long double PI_L = 3.141592653589793238462643383279502884L;

double truth(int kind, int param, int c)
{
    switch (kind) {
    case FFSAT_KIND_OR: return c >= 1 ? -1.0 : 1.0;
    case FFSAT_KIND_XOR: return (c % 2) == (param & 1) ? -1.0 : 1.0;
    default: return c >= param ? -1.0 : 1.0;
    }
}

using cld = std::complex<long double>;

// All conjugated coefficients h_a = (1/N) sum_c f(c) exp(-2 pi i a c / N),
// a = 0..floor(N/2), N = k + 1.  f is a step function of the count c, so
// with its jumps d_j = f(j) - f(j-1) (j = 1..k) and z = exp(-2 pi i a / N),
// z != 1, the sum over all N roots vanishes and
//     h_a = (1/N) sum_j d_j (z^j - 1) / (1 - z),
// one term per jump (OR and at-least-t have a single jump).  Angles are
// reduced exactly in integers; arithmetic in long double.
std::vector<cld> conj_coeffs(int kind, int param, int k)
{
    const long long N = k + 1;
    std::vector<double> fv((size_t)k + 1);
    for (int c = 0; c <= k; ++c) fv[(size_t)c] = truth(kind, param, c);
    std::vector<std::pair<int, double>> jumps;
    for (int j = 1; j <= k; ++j)
        if (fv[(size_t)j] != fv[(size_t)j - 1]) jumps.emplace_back(j, fv[(size_t)j] - fv[(size_t)j - 1]);
    auto root = [&](long long e) {   // exp(-2 pi i e / N)
        const long long r = ((e % N) + N) % N;
        const long double ang = -2.0L * PI_L * (long double)r / (long double)N;
        return cld(cosl(ang), sinl(ang));
    };
    std::vector<cld> h((size_t)(N / 2) + 1);
    long double s0 = 0;
    for (int c = 0; c <= k; ++c) s0 += fv[(size_t)c];
    h[0] = cld(s0 / N, 0.0L);
    for (long long a = 1; a <= N / 2; ++a) {
        const cld z = root(a);
        const cld den = 1.0L - z;
        cld acc = 0.0L;
        for (const auto &jd : jumps) acc += (long double)jd.second * (root(a * jd.first) - 1.0L);
        h[(size_t)a] = acc / den / (long double)N;
    }
    return h;
}

struct FreqD {
    double tk, init, c0re, c0im, c1re, c1im;
    double p0 = 0.0;   // form 3: imaginary part of the root
};

struct TypeD {
    int cls = CLASS_REAL;
    double cst = 0, alpha = 0, beta = 0, c0r = 0, c1r = 0, pad = 1;
    int has_real = 0;
    int n1 = 0, n2 = 0;
    bool poly = false;   // FP64 root-of-unity type: its FP64 table takes the FreqPoly layout
    std::vector<FreqD> fr;
};

// Transform-free product chains (App. B and its footnote for OR).
TypeD real_or() { TypeD t; t.has_real = 1; t.alpha = 0.5; t.beta = 0.5; t.c0r = 2; t.c1r = 1; t.cst = -1; t.pad = 1; return t; }
TypeD real_and() { TypeD t; t.has_real = 1; t.alpha = 0.5; t.beta = -0.5; t.c0r = -2; t.c1r = 1; t.cst = 1; t.pad = -1; return t; }
TypeD real_xor(int p) { TypeD t; t.has_real = 1; t.alpha = 0; t.beta = 1; t.c0r = t.c1r = (p & 1) ? 1.0 : -1.0; t.cst = 0; t.pad = 1; return t; }
TypeD real_const(double v) { TypeD t; t.cst = v; t.pad = 1; return t; }

// Factor, value and gradient coefficients of every transform-free kind (the
// same constants as the slot path's type tables), laid out for k_pull.
static std::vector<float> rkind_table()
{
    const TypeD t[RKIND_N] = {real_or(), real_and(), real_xor(1), real_xor(0), real_const(-1.0), real_const(1.0)};
    std::vector<float> r(RK_TABLE, 0.f);
    for (int i = 0; i < RKIND_N; ++i) {
        r[(size_t)i] = (float)t[i].alpha;
        r[(size_t)8 + i] = (float)t[i].beta;
        r[(size_t)16 + i] = t[i].has_real ? (float)t[i].c0r : 0.f;
        r[(size_t)24 + i] = t[i].has_real ? (float)t[i].c1r : 0.f;
        r[(size_t)32 + i] = (float)t[i].cst;
    }
    return r;
}

// Root-of-unity evaluation of a symmetric constraint (Alg. 2), with the
// factor of literal i at frequency a taken in the bounded basis
//   q_i + p_i z = (1+z)/2 + l_i (1-z)/2,  z = exp(2 pi i a / N)
//              = e^{i th/2} (C - i S l_i),  th = 2 pi a / N,
// rescaled to psi = 1 - i (S/C) l (form 1, C >= S) or (C/S) - i l (form 2);
// the removed factor e^{i k th/2} C^k (or S^k), the padding literals of the
// segment layout (value +1, count-neutral) and the power-of-two start value
// of every segment are folded into c0 / c1 here, in long double.
//
// FP64 tables (f64 = true) run every frequency with form 1's factor (the
// polynomial form evaluates at z = -i tau), FP32 tables of segments of at
// most 16 too where the start value stays above 1e-30: a form-2 factor is
// kappa (1 - i l / kappa), kappa = C/S, so its lane takes tau = S/C and
// starts from kappa^s times the usual start value; each segment product is
// then exactly the form-2 one (FP64 holds kappa^s, >= 1e-81 for k <= 512 and
// s <= 32), and the leave-one-out products carry one extra factor kappa,
// divided out of c1.
TypeD dft_type(const std::vector<cld> &hv, int k, int L, int s, bool f64)
{
    TypeD t;
    t.cls = CLASS_DFT;
    t.poly = f64;
    const int N = k + 1;
    const int npad = L * s - k;
    t.cst = (double)hv[0].real();
    t.pad = 1.0;
    std::vector<FreqD> f1, f2;
    for (int a = 1; a <= k / 2; ++a) {
        const cld h = hv[(size_t)a];
        if (std::abs(h) < 1e-15L) continue;
        const long double half = PI_L * a / N;
        const long double C = cosl(half), S = sinl(half);
        const bool form1 = C >= S;
        const long double tk = form1 ? S / C : C / S;
        const long double base = form1 ? C : S;
        const long double mag2 = 1.0L + tk * tk;
        const int e = (int)floorl((long double)s * log2l(mag2) / 4.0L);
        const long long r2 = ((long long)a * k) % (2LL * N);   // phase k*th/2 = pi a k / N
        const long double ph = PI_L * (long double)r2 / (long double)N;
        const cld sigma = cld(cosl(ph), sinl(ph)) * powl(base, (long double)k);
        const cld psipad = form1 ? cld(1.0L, -tk) : cld(tk, -1.0L);
        cld corr = 1.0L;
        for (int q = 0; q < npad; ++q) corr /= psipad;
        const cld c0 = 2.0L * h * sigma * corr * ldexpl(1.0L, L * e);
        const cld c1 = c0 * (form1 ? cld(0.0L, -tk) : cld(0.0L, -1.0L));
        // FP32 takes the same route where its range allows: segments of at
        // most 16 (the kernels keep tau * l for the reverse pass there, so a
        // factor costs 3 + 4 operations instead of 4 + 6) and a start value
        // far inside the normal range
        const bool via1 = f64 || (s <= 16 && ldexpl(1.0L, -e) * powl(tk, (long double)s) >= 1e-30L);
        if (via1 && !form1) {
            // form 2 through form 1's code (see above)
            const cld c1r = c1 / tk;
            FreqD fd{(double)(1.0L / tk), (double)(ldexpl(1.0L, -e) * powl(tk, (long double)s)), (double)c0.real(),
                     (double)c0.imag(), (double)c1r.real(), (double)c1r.imag()};
            f1.push_back(fd);
            continue;
        }
        FreqD fd{(double)tk, (double)ldexpl(1.0L, -e), (double)c0.real(), (double)c0.imag(),
                 (double)c1.real(), (double)c1.imag()};
        (form1 ? f1 : f2).push_back(fd);
    }
    t.n1 = (int)f1.size();
    t.n2 = (int)f2.size();
    t.fr = f1;
    t.fr.insert(t.fr.end(), f2.begin(), f2.end());
    if (k % 2 == 1) {
        // z = -1 (N even): the factor is l_i itself, a real product chain
        const long double hn = hv[(size_t)N / 2].real();
        if (fabsl(hn) >= 1e-15L) {
            t.has_real = 1;
            t.alpha = 0;
            t.beta = 1;
            t.c0r = t.c1r = (double)hn;
        }
    }
    return t;
}

// ---- the unit-circle form (ablation of the basis above)

// Signed integers of any size, with just the operations the Krawtchouk
// recurrences below need: multiply by a small integer, add, exact division
// by a small integer, conversion to long double.
struct BigInt {
    int sign = 0;                  // -1, 0, +1
    std::vector<uint32_t> mag;     // little-endian base 2^32, no leading zero limb

    static BigInt of(long long v)
    {
        BigInt r;
        if (v == 0) return r;
        r.sign = v < 0 ? -1 : 1;
        unsigned long long u = v < 0 ? 0ULL - (unsigned long long)v : (unsigned long long)v;
        while (u) { r.mag.push_back((uint32_t)u); u >>= 32; }
        return r;
    }
    void trim()
    {
        while (!mag.empty() && mag.back() == 0) mag.pop_back();
        if (mag.empty()) sign = 0;
    }
    BigInt mul(long long m) const
    {
        BigInt r;
        if (sign == 0 || m == 0) return r;
        const unsigned long long um = m < 0 ? 0ULL - (unsigned long long)m : (unsigned long long)m;
        r.sign = (m < 0) ? -sign : sign;
        r.mag.assign(mag.size() + 2, 0u);
        for (int part = 0; part < 2; ++part) {   // um < 2^64: two 32-bit halves
            const uint64_t mm = (uint32_t)(um >> (32 * part));
            uint64_t carry = 0;
            for (size_t i = 0; i < mag.size(); ++i) {
                const uint64_t t = (uint64_t)mag[i] * mm + r.mag[i + part] + carry;
                r.mag[i + part] = (uint32_t)t;
                carry = t >> 32;
            }
            for (size_t i = mag.size() + part; carry; ++i) {
                const uint64_t t = (uint64_t)r.mag[i] + carry;
                r.mag[i] = (uint32_t)t;
                carry = t >> 32;
            }
        }
        r.trim();
        return r;
    }
    static int cmp_mag(const BigInt &a, const BigInt &b)
    {
        if (a.mag.size() != b.mag.size()) return a.mag.size() < b.mag.size() ? -1 : 1;
        for (size_t i = a.mag.size(); i-- > 0;)
            if (a.mag[i] != b.mag[i]) return a.mag[i] < b.mag[i] ? -1 : 1;
        return 0;
    }
    BigInt add(const BigInt &b) const
    {
        if (b.sign == 0) return *this;
        if (sign == 0) return b;
        BigInt r;
        if (sign == b.sign) {
            r.sign = sign;
            r.mag.assign(std::max(mag.size(), b.mag.size()) + 1, 0u);
            uint64_t carry = 0;
            for (size_t i = 0; i < r.mag.size(); ++i) {
                const uint64_t t = (uint64_t)(i < mag.size() ? mag[i] : 0u) + (i < b.mag.size() ? b.mag[i] : 0u) + carry;
                r.mag[i] = (uint32_t)t;
                carry = t >> 32;
            }
        } else {
            const int c = cmp_mag(*this, b);
            if (c == 0) return r;
            const BigInt &hi = c > 0 ? *this : b, &lo = c > 0 ? b : *this;
            r.sign = hi.sign;
            r.mag.assign(hi.mag.size(), 0u);
            int64_t borrow = 0;
            for (size_t i = 0; i < hi.mag.size(); ++i) {
                int64_t t = (int64_t)hi.mag[i] - (i < lo.mag.size() ? lo.mag[i] : 0u) - borrow;
                borrow = t < 0 ? 1 : 0;
                r.mag[i] = (uint32_t)(t + (borrow << 32));
            }
        }
        r.trim();
        return r;
    }
    BigInt neg() const { BigInt r = *this; r.sign = -r.sign; return r; }
    // exact division by d > 0 (the caller guarantees divisibility)
    BigInt div_exact(uint32_t d) const
    {
        BigInt r = *this;
        uint64_t rem = 0;
        for (size_t i = r.mag.size(); i-- > 0;) {
            const uint64_t cur = (rem << 32) | r.mag[i];
            r.mag[i] = (uint32_t)(cur / d);
            rem = cur % d;
        }
        r.trim();
        return r;
    }
    long double to_ld() const
    {
        long double v = 0.0L;
        for (size_t i = mag.size(); i-- > 0;) v = v * 4294967296.0L + (long double)mag[i];
        return sign < 0 ? -v : v;
    }
};

// Walsh coefficients fhat[j] of a symmetric constraint: the coefficient of
// the elementary symmetric polynomial e_j in its Walsh expansion (Def. 2 and
// Eq. effi_eval), j = 0..k, f = -1 on satisfying count vectors.  Exact up to
// the final rounding:
//   XOR with parity p: only e_k, with coefficient 2p - 1;
//   at least t (OR: t = 1), 1 <= t <= k: fhat_0 = 1 - 2^(1-k) sum_{c>=t} C(k,c)
//     and, for j >= 1, fhat_j = 2^(1-k) K_{t-1}(j-1; k-1), a binary Krawtchouk
//     value (the derivative of the tail sum of the Krawtchouk generating
//     function (1-z)^c (1+z)^(k-c) over c >= t telescopes to one term).
//     With K = k-1, n = t-1: D_x = C(K,x) K_n(x) = C(K,n) K_x(n) satisfies
//     (x+1) D_{x+1} = (K-2n) D_x - (K-x+1) D_{x-1}, D_0 = C(K,n),
//     D_1 = (K-2n) C(K,n), all integers; fhat_j = 2^(1-k) D_{j-1} / C(K,j-1).
//   t <= 0 or t > k: constant -1 or +1.
std::vector<long double> walsh_exact(int kind, int param, int k)
{
    std::vector<long double> fh((size_t)k + 1, 0.0L);
    if (kind == FFSAT_KIND_XOR) {
        fh[(size_t)k] = (param & 1) ? 1.0L : -1.0L;
        return fh;
    }
    const int t = kind == FFSAT_KIND_OR ? 1 : param;
    if (t <= 0) { fh[0] = -1.0L; return fh; }
    if (t > k) { fh[0] = 1.0L; return fh; }
    // binomials C(k, c) and the tail sum
    BigInt C = BigInt::of(1), tail;
    for (int c = 0; c <= k; ++c) {
        if (c >= t) tail = tail.add(C);
        if (c < k) C = C.mul(k - c).div_exact((uint32_t)(c + 1));
    }
    // fhat_0 = (2^k - 2 tail) / 2^k
    BigInt two_k = BigInt::of(1);
    for (int i = 0; i < k; ++i) two_k = two_k.mul(2);
    fh[0] = ldexpl(two_k.add(tail.mul(-2)).to_ld(), -k);
    const int K = k - 1, n = t - 1;
    BigInt CKn = BigInt::of(1);
    for (int i = 0; i < n; ++i) CKn = CKn.mul(K - i).div_exact((uint32_t)(i + 1));
    BigInt Dm1, D = CKn, CKx = BigInt::of(1);   // D_{x-1}, D_x, C(K, x)
    for (int x = 0; x <= K; ++x) {
        fh[(size_t)x + 1] = ldexpl(D.to_ld() / CKx.to_ld(), 1 - k);
        if (x == K) break;
        BigInt Dn = (x == 0) ? CKn.mul(K - 2 * n)
                             : D.mul(K - 2 * n).add(Dm1.mul(-(long long)(K - x + 1))).div_exact((uint32_t)(x + 1));
        Dm1 = D;
        D = Dn;
        CKx = CKx.mul(K - x).div_exact((uint32_t)(x + 1));
    }
    return fh;
}

// Conjugated Walsh coefficients of the unit-circle form, f~ = f^ W^-1
// (Eq. inverse): with the ESP sequence ordered e_k .. e_0 (the order the
// convolution of [l_i, 1] produces), omega = exp(-2 pi i / N), N = k + 1,
//   f~[a] = (1/N) sum_j fhat_{k-j} omega^(-j a),  a = 0..k,
// so that WE = sum_a f~[a] prod_i (omega^a + l_i).  Angles are reduced
// exactly in integers; arithmetic in long double.
std::vector<cld> uc_coeffs(int kind, int param, int k)
{
    const std::vector<long double> fh = walsh_exact(kind, param, k);
    const long long N = k + 1;
    std::vector<cld> roots((size_t)N);
    for (long long r = 0; r < N; ++r) {
        const long double ang = 2.0L * PI_L * (long double)r / (long double)N;   // omega^(-r)
        roots[(size_t)r] = cld(cosl(ang), sinl(ang));
    }
    std::vector<cld> ft((size_t)N);
    for (long long a = 0; a < N; ++a) {
        cld acc = 0.0L;
        for (long long j = 0; j <= k; ++j) {
            const long double f = fh[(size_t)(k - j)];
            if (f != 0.0L) acc += f * roots[(size_t)((j * a) % N)];
        }
        ft[(size_t)a] = acc / (long double)N;
    }
    return ft;
}

// Kernel tables of the unit-circle form.  Frequency a = 0 (omega^0 = 1) is
// the real chain prod (1 + l); a = 1..ceil(k/2)-1 are complex (weight 2 by
// conjugate symmetry, f~[N-a] = conj f~[a]); for odd k, a = N/2 is the factor
// l - 1, taken as a complex entry with zero imaginary part.  Padding literals
// hold 0: factor 1 in the real chain and omega^a elsewhere, divided out of
// the coefficients.  Running products start at 1 (no rescaling, as printed).
TypeD uc_type(const std::vector<cld> &ft, int k, int L, int s)
{
    TypeD t;
    t.cls = CLASS_DFT;
    const long long N = k + 1;
    const long long npad = (long long)L * s - k;
    t.cst = 0.0;
    t.pad = 0.0;
    t.has_real = 1;
    t.alpha = 1.0;
    t.beta = 1.0;
    t.c0r = t.c1r = (double)ft[0].real();
    for (long long a = 1; 2 * a <= N; ++a) {
        const bool mid = 2 * a == N;
        const long double th = 2.0L * PI_L * (long double)a / (long double)N;
        const long double cr = mid ? -1.0L : cosl(th), si = mid ? 0.0L : -sinl(th);   // omega^a
        const long long r = (a * npad) % N;   // divide by omega^(a npad)
        const long double ph = 2.0L * PI_L * (long double)r / (long double)N;
        const cld corr = mid ? cld((npad & 1) ? -1.0L : 1.0L, 0.0L) : cld(cosl(ph), sinl(ph));
        const cld c0 = (mid ? 1.0L : 2.0L) * ft[(size_t)a] * corr;
        FreqD fd{(double)cr, 1.0, (double)c0.real(), (double)c0.imag(), (double)c0.real(), (double)c0.imag()};
        fd.p0 = (double)si;
        t.fr.push_back(fd);
    }
    t.n1 = (int)t.fr.size();
    t.n2 = 0;
    return t;
}

// FLOPs (an FMA counts 2) of one restart of a root-of-unity constraint in
// the FP64 polynomial form, as the kernel runs it on L lanes of s positions
// with nf complex frequencies: per lane the segment's elementary symmetric
// polynomials (s(s+1)/2 FMAs); per lane and frequency two Horner
// evaluations (s FMAs), the segment product (2) and the butterfly over L
// lanes (6 log2 L), the quotient by the segment product (16, none on one
// lane), the moments' coefficients (6) and the value term (5), and the
// moments (s FMAs and (s+1)/2 - 1 powers of -tau^2); per lane once, the
// gradients from the moments (about 2 s^2 FMAs, seg_grad_from_moments).
double poly_flops(int s, int L, int nf)
{
    int lg = 0;
    while ((1 << lg) < L) ++lg;
    double tail = 0.0;   // FMAs of the gradient pass (seg_grad_from_moments)
    for (int lo = 0; lo < s; lo += 8) {
        const int nb = std::min(8, s - lo), hi = lo + nb;
        tail += 0.5 * lo * (lo + 1) + (double)nb * (lo + 1);
        for (int t = 0; t < nb; ++t) tail += 0.5 * t * (t + 1) + (t + 1) + t;
        if (lo > 0)
            for (int u = 0; u < nb; ++u) tail += hi - u - 1;
    }
    const double per_freq = 4.0 * s + (s + 1) / 2 - 1 + 13.0 + (L > 1 ? 16.0 : 0.0) + 6.0 * lg;
    return (double)L * ((double)s * (s + 1) + (double)nf * per_freq + 2.0 * tail);
}

// Segment shape of a unit-circle bin: L = 1 with SEG in {4, 8, 16}, else
// SEG = 16 and the smallest L in 2..32 with 16 L >= k.
void shape_for_uc(int k, int &seg, int &L)
{
    L = 1;
    while (16 * L < k) L <<= 1;
    seg = L > 1 ? 16 : (k <= 4 ? 4 : (k <= 8 ? 8 : 16));
}

// Segment shape of a constraint of length k: L lanes (a power of two) of SEG
// positions each, L * SEG >= k, the smallest such L and then the smallest
// SEG.  FP32 arithmetic: SEG in {4, 8, 16, 24} (32 past k = 384); products
// at roots of unity (dft) also take 12 on one lane and 20 on several.  FP64
// arithmetic: SEG up to 24 (multiples of 4 below 8 lanes and up to 24 at 8),
// 8-lane groups take every SEG from 25 to 32 (k <= 256) and 16-lane groups
// every SEG from 14 to 32 (k <= 512): in root-of-unity bins a padding
// position costs as much as a literal in every frequency, and each doubling
// of L adds a butterfly stage per frequency.  Real chains pay for padding once, so they keep the coarser
// steps: fewer distinct shapes mean fewer, larger kernel launches.
void shape_for(int ct, int k, int &seg, int &L, bool dft)
{
    if (ct == CT_F64) {
        L = 1;
        while ((k + L - 1) / L > 24 && L < 8) L <<= 1;
        // 8 lanes of up to 32 positions (k <= 256), then 16 lanes of up to 32
        // (k <= 512); longer constraints have no FP64 variant (32 lanes)
        if (L == 8 && (k + 7) / 8 > 32) L = 16;
        if (L == 16 && (k + 15) / 16 > 32) L = 32;
        const int s = (k + L - 1) / L;
        if (L >= 16) seg = std::max(14, s);   // every count: padding costs as much as a literal
        else if (L == 8 && s > 24) seg = s;
        else if (L > 1) seg = std::max(16, ((s + 3) / 4) * 4);
        else seg = s <= 4 ? 4 : ((s + 3) / 4) * 4;
        return;
    }
    // FP32: segments of at most 24 literals (the register budget of 3+ waves
    // per SIMD), 32 only where 16 lanes of 24 do not reach (k > 384); counts
    // in steps of 4 on one lane, 16, 20 or 24 on several for root-of-unity
    // products
    int smax = 24;
    L = 1;
    while ((k + L - 1) / L > smax) {
        if (L == 16) {
            smax = 32;
            break;
        }
        L <<= 1;
    }
    const int s = (k + L - 1) / L;
    if (s <= 4) seg = 4;
    else if (!dft) seg = s <= 8 ? 8 : ((s + 7) / 8) * 8;   // 8, 16, 24 (32)
    else if (L == 1) seg = ((s + 3) / 4) * 4;   // 8, 12, ..., 24
    else if (s <= 16) seg = 16;
    else if (s <= 20) seg = 20;
    else seg = ((s + 7) / 8) * 8;   // 24 (32 only past k = 384)
}

struct TypeKey {
    int cls, ct, kind, param, k, L, seg;
    bool operator<(const TypeKey &o) const
    {
        return std::tie(cls, ct, kind, param, k, L, seg) < std::tie(o.cls, o.ct, o.kind, o.param, o.k, o.L, o.seg);
    }
};

enum { RK_OR = 100, RK_XOR = 101, RK_AND = 102, RK_CONST = 103 };

template <typename T>
ffsat_status upload(T **dst, const std::vector<T> &src, int64_t &bytes)
{
    *dst = nullptr;
    if (src.empty()) return FFSAT_OK;
    HIPCHK(hipMalloc((void **)dst, src.size() * sizeof(T)));
    HIPCHK(hipMemcpy(*dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice));
    bytes += (int64_t)(src.size() * sizeof(T));
    return FFSAT_OK;
}

}  // namespace

extern "C" ffsat_status ffsat_coefficients(int32_t kind, int32_t k, int32_t param, double *h_out)
{
    if (!h_out || k < 1 || k > FFSAT_MAX_CONSTRAINT_LEN)
        return fail(FFSAT_E_INVALID_ARG, "ffsat_coefficients: bad argument");
    if (kind < 0 || kind > 2) return fail(FFSAT_E_BAD_KIND, "ffsat_coefficients: bad kind %d", kind);
    const std::vector<cld> h = conj_coeffs(kind, param, k);
    for (int a = 0; a <= (k + 1) / 2; ++a) {
        h_out[2 * a] = (double)h[(size_t)a].real();
        h_out[2 * a + 1] = (double)h[(size_t)a].imag();
    }
    return FFSAT_OK;
}

extern "C" ffsat_status ffsat_walsh_coefficients(int32_t kind, int32_t k, int32_t param, double *f_out)
{
    if (!f_out || k < 1 || k > FFSAT_MAX_CONSTRAINT_LEN)
        return fail(FFSAT_E_INVALID_ARG, "ffsat_walsh_coefficients: bad argument");
    if (kind < 0 || kind > 2) return fail(FFSAT_E_BAD_KIND, "ffsat_walsh_coefficients: bad kind %d", kind);
    const std::vector<long double> f = walsh_exact(kind, param, k);
    for (int j = 0; j <= k; ++j) f_out[j] = (double)f[(size_t)j];
    return FFSAT_OK;
}

extern "C" ffsat_status ffsat_unit_circle_coefficients(int32_t kind, int32_t k, int32_t param, double *ft_out)
{
    if (!ft_out || k < 1 || k > FFSAT_MAX_CONSTRAINT_LEN)
        return fail(FFSAT_E_INVALID_ARG, "ffsat_unit_circle_coefficients: bad argument");
    if (kind < 0 || kind > 2) return fail(FFSAT_E_BAD_KIND, "ffsat_unit_circle_coefficients: bad kind %d", kind);
    const std::vector<cld> ft = uc_coeffs(kind, param, k);
    for (int a = 0; a <= k; ++a) {
        ft_out[2 * a] = (double)ft[(size_t)a].real();
        ft_out[2 * a + 1] = (double)ft[(size_t)a].imag();
    }
    return FFSAT_OK;
}

// ------------------------------------------------------------------ problem

static ffsat_status validate(const ffsat_problem_desc *d)
{
    if (!d) return fail(FFSAT_E_INVALID_ARG, "problem description is NULL");
    if (d->n_vars < 1) return fail(FFSAT_E_INVALID_ARG, "n_vars must be >= 1 (got %d)", d->n_vars);
    if (d->n_cons < 1) return fail(FFSAT_E_INVALID_ARG, "n_cons must be >= 1 (got %d)", d->n_cons);
    if (!d->con_ptr || !d->lits || !d->kinds || !d->params)
        return fail(FFSAT_E_INVALID_ARG, "con_ptr, lits, kinds and params are required");
    if (d->con_ptr[0] != 0) return fail(FFSAT_E_INVALID_ARG, "con_ptr[0] must be 0");
    const int m = d->n_cons, n = d->n_vars;
    for (int c = 0; c < m; ++c) {
        const int64_t a = d->con_ptr[c], b = d->con_ptr[c + 1];
        if (b < a) return fail(FFSAT_E_INVALID_ARG, "con_ptr decreases at constraint %d", c);
        if (b == a) return fail(FFSAT_E_EMPTY_CONSTRAINT, "constraint %d has no literal", c);
        if (b - a > FFSAT_MAX_CONSTRAINT_LEN)
            return fail(FFSAT_E_UNSUPPORTED, "constraint %d has %lld literals (max %d)", c,
                        (long long)(b - a), FFSAT_MAX_CONSTRAINT_LEN);
        const int kd = d->kinds[c];
        if (kd != FFSAT_KIND_OR && kd != FFSAT_KIND_XOR && kd != FFSAT_KIND_CARD_GE)
            return fail(FFSAT_E_BAD_KIND, "constraint %d has kind %d", c, kd);
    }
    if (d->con_ptr[m] > (int64_t)INT32_MAX - 1)
        return fail(FFSAT_E_UNSUPPORTED, "more than 2^31-1 literals");
    std::vector<int32_t> stamp((size_t)n, -1);
    for (int c = 0; c < m; ++c) {
        for (int64_t i = d->con_ptr[c]; i < d->con_ptr[c + 1]; ++i) {
            const int32_t l = d->lits[i];
            if (l == 0 || l > n || l < -n)
                return fail(FFSAT_E_VAR_RANGE, "literal %d of constraint %d is out of range", l, c);
            const int v = (l > 0 ? l : -l) - 1;
            if (stamp[v] == c)
                return fail(FFSAT_E_DUP_VAR, "variable %d appears twice in constraint %d", v + 1, c);
            stamp[v] = c;
        }
    }
    if (d->weights) {
        for (int c = 0; c < m; ++c)
            if (!std::isfinite(d->weights[c]))
                return fail(FFSAT_E_INVALID_ARG, "weight %d is not finite", c);
    }
    if (d->fp64_min_len < 0) return fail(FFSAT_E_INVALID_ARG, "fp64_min_len must be >= 0");
    return FFSAT_OK;
}

static void free_layout(Layout &L)
{
    (void)hipFree(L.d_con);
    (void)hipFree(L.d_lit);
    (void)hipFree(L.d_vptr);
    (void)hipFree(L.d_vslot);
    (void)hipFree(L.d_pos);
    (void)hipFree(L.d_t32);
    (void)hipFree(L.d_t64);
    (void)hipFree(L.d_f32);
    (void)hipFree(L.d_f64);
    for (PullLayout &P : L.pull) {
        (void)hipFree(P.d_pptr);
        (void)hipFree(P.d_pent);
        (void)hipFree(P.d_vptr);
        (void)hipFree(P.d_vslot);
        (void)hipFree(P.d_rk);
    }
    L = Layout();
}

// The pulled-occurrence lists of pull class c (constraints of the FP32
// layout's bins with pk >= c): per variable, ascending (binned constraint,
// position), one entry {original constraint, meta, the other literals in
// constraint order, padded with the variable itself}; and the
// variable-major transpose of every other slot.  Built once per class.
static ffsat_status build_pull(ffsat_problem *p, int c)
{
    Layout &Ly = p->lay[IO_F32];
    PullLayout &P = Ly.pull[c];
    if (P.built) return FFSAT_OK;
    const int E = PULL_E[c];
    const int n = p->n, m = p->m;
    std::vector<char> pulled((size_t)m, 0);
    for (const Bin &b : Ly.bins)
        if (b.pk >= c)
            for (int q = b.first; q < b.first + b.count; ++q) pulled[(size_t)q] = 1;
    std::vector<int32_t> pptr((size_t)n + 1, 0), vptr((size_t)n + 1, 0);
    for (int q = 0; q < m; ++q) {
        const ConDesc &d = Ly.h_con[(size_t)q];
        for (int i = 0; i < d.k; ++i) {
            const int v = Ly.h_lit[(size_t)d.off + i] & 0x7fffffff;
            (pulled[(size_t)q] ? pptr : vptr)[(size_t)v + 1]++;
        }
    }
    for (int v = 0; v < n; ++v) {
        pptr[(size_t)v + 1] += pptr[(size_t)v];
        vptr[(size_t)v + 1] += vptr[(size_t)v];
    }
    std::vector<int32_t> pent((size_t)pptr[(size_t)n] * E), vslot((size_t)vptr[(size_t)n]);
    std::vector<int32_t> pfill(pptr.begin(), pptr.end() - 1), vfill(vptr.begin(), vptr.end() - 1);
    for (int q = 0; q < m; ++q) {
        const ConDesc &d = Ly.h_con[(size_t)q];
        const int32_t *cl = &Ly.h_lit[(size_t)d.off];
        if (!pulled[(size_t)q]) {
            for (int i = 0; i < d.k; ++i) vslot[(size_t)vfill[(size_t)(cl[i] & 0x7fffffff)]++] = d.off + i;
            continue;
        }
        const int rk = Ly.h_rk[(size_t)q];
        if (rk < 0 || d.k > PULL_K[c]) return fail(FFSAT_E_HIP, "pull layout: constraint %d is not pullable", d.orig);
        const int chk = std::min(std::max(d.chk, -2), d.k + 1);   // counts never exceed k
        for (int i = 0; i < d.k; ++i) {
            const int v = cl[i] & 0x7fffffff;
            int32_t *ent = &pent[(size_t)pfill[(size_t)v]++ * E];
            ent[0] = d.orig;
            ent[1] = rk | ((d.k - 1) << 3) | ((chk + 2) << 6) | ((cl[i] < 0 ? 1 : 0) << 10) | ((i == 0 ? 1 : 0) << 11);
            int t = 2;
            for (int j = 0; j < d.k; ++j)
                if (j != i) ent[t++] = cl[j];
            while (t < E) ent[t++] = v;
        }
    }
    ffsat_status st;
    if ((st = upload(&P.d_pptr, pptr, p->device_bytes)) != FFSAT_OK) return st;
    if (!pent.empty() && (st = upload(&P.d_pent, pent, p->device_bytes)) != FFSAT_OK) return st;
    if ((st = upload(&P.d_vptr, vptr, p->device_bytes)) != FFSAT_OK) return st;
    if (!vslot.empty() && (st = upload(&P.d_vslot, vslot, p->device_bytes)) != FFSAT_OK) return st;
    if ((st = upload(&P.d_rk, rkind_table(), p->device_bytes)) != FFSAT_OK) return st;
    P.n_ent = pptr[(size_t)n];
    P.n_rest = vptr[(size_t)n];
    for (int64_t e = 0; e < P.n_ent; ++e) P.n_gather += ((pent[(size_t)e * E + 1] >> 3) & 7);
    P.built = true;
    return FFSAT_OK;
}

using CoeffMemo = std::map<std::tuple<int, int, int>, std::vector<cld>>;

static ffsat_status build_layout(ffsat_problem *p, const ffsat_problem_desc *d, int io, CoeffMemo &memo)
{
    Layout &Ly = p->lay[io];
    Ly.io = io;
    const int m = p->m, n = p->n;
    const bool force_dft = (p->flags & FFSAT_FLAG_FORCE_DFT) != 0;
    const bool uc = (p->flags & FFSAT_FLAG_UNIT_CIRCLE) != 0;

    // 1. classify every constraint into a (type, bin)
    std::map<TypeKey, int> type_index;
    std::vector<TypeD> types;
    struct Item { int c, k, type, bin; double cost, alg; };
    std::vector<Item> items((size_t)m);
    struct BinKey {
        int cls, ct, seg, L, pk;
        bool operator<(const BinKey &o) const {
            return std::tie(cls, ct, seg, L, pk) < std::tie(o.cls, o.ct, o.seg, o.L, o.pk);
        }
    };
    std::vector<int8_t> rkind((size_t)m, -1);   // original order
    std::map<BinKey, int> bin_index;
    std::vector<Bin> bins;
    for (int c = 0; c < m; ++c) {
        const int k = (int)(d->con_ptr[c + 1] - d->con_ptr[c]);
        const int kind = d->kinds[c];
        const int prm = d->params[c];
        int cls, rk = -1, rparam = 0;
        if (kind == FFSAT_KIND_CARD_GE && prm <= 0) { cls = CLASS_REAL; rk = RK_CONST; rparam = -1; }
        else if (kind == FFSAT_KIND_CARD_GE && prm > k) { cls = CLASS_REAL; rk = RK_CONST; rparam = 1; }
        else if (!force_dft && (kind == FFSAT_KIND_OR || (kind == FFSAT_KIND_CARD_GE && prm == 1))) { cls = CLASS_REAL; rk = RK_OR; }
        else if (!force_dft && kind == FFSAT_KIND_XOR) { cls = CLASS_REAL; rk = RK_XOR; rparam = prm & 1; }
        else if (!force_dft && kind == FFSAT_KIND_CARD_GE && prm == k) { cls = CLASS_REAL; rk = RK_AND; }
        else cls = CLASS_DFT;
        int ct;
        if (io == IO_F64) ct = CT_F64;
        else ct = (cls == CLASS_DFT && k >= p->fp64_min_len) ? CT_F64 : CT_F32;
        int seg, L;
        if (uc && cls == CLASS_DFT) shape_for_uc(k, seg, L);
        else shape_for(ct, k, seg, L, cls == CLASS_DFT);
        if (!eval_variant_exists(io, ct, cls, seg, L, uc))
            return fail(FFSAT_E_UNSUPPORTED, "no kernel variant for constraint %d (k=%d)", c, k);
        TypeKey tk;
        if (cls == CLASS_REAL) tk = TypeKey{cls, ct, rk, rparam, 0, 0, 0};
        else {
            int nprm = kind == FFSAT_KIND_XOR ? (prm & 1) : (kind == FFSAT_KIND_OR ? 0 : prm);
            tk = TypeKey{cls, ct, kind, nprm, k, L, seg};
        }
        auto it = type_index.find(tk);
        int ti;
        if (it == type_index.end()) {
            TypeD td;
            if (cls == CLASS_DFT) {
                auto key = std::make_tuple(tk.kind, tk.param, k);
                auto mh = memo.find(key);
                if (mh == memo.end())
                    mh = memo.emplace(key, uc ? uc_coeffs(tk.kind, tk.param, k) : conj_coeffs(tk.kind, tk.param, k)).first;
                td = uc ? uc_type(mh->second, k, L, seg) : dft_type(mh->second, k, L, seg, ct == CT_F64);
            }
            else if (rk == RK_OR) td = real_or();
            else if (rk == RK_XOR) td = real_xor(rparam);
            else if (rk == RK_AND) td = real_and();
            else td = real_const((double)rparam);
            ti = (int)types.size();
            types.push_back(td);
            type_index[tk] = ti;
        } else {
            ti = it->second;
        }
        // pull class (FP32 layout): transform-free chains of length <= 3, 4..7
        const int pk = (io == IO_F32 && cls == CLASS_REAL && L == 1 && k <= PULL_K[PULL_LE7])
                           ? (k <= PULL_K[PULL_LE3] ? PULL_LE3 : PULL_LE7) : 0;
        if (cls == CLASS_REAL) {
            rkind[(size_t)c] = (int8_t)(rk == RK_OR ? RKIND_OR : rk == RK_AND ? RKIND_AND
                                        : rk == RK_XOR ? (rparam ? RKIND_XOR_ODD : RKIND_XOR_EVEN)
                                        : (rparam < 0 ? RKIND_TRUE : RKIND_FALSE));
        }
        BinKey bk{cls, ct, seg, L, pk};
        auto bi = bin_index.find(bk);
        int bidx;
        if (bi == bin_index.end()) {
            Bin b;
            b.cls = cls; b.ct = ct; b.seg = seg; b.L = L; b.pk = pk;
            b.uc = uc && cls == CLASS_DFT;
            bidx = (int)bins.size();
            bins.push_back(b);
            bin_index[bk] = bidx;
        } else {
            bidx = bi->second;
        }
        const double cost = cls == CLASS_DFT ? (double)k * (double)(types[ti].n1 + types[ti].n2 + 1) * 9.0
                                             : (double)k * 4.0;
        Bin &b = bins[(size_t)bidx];
        // Algorithmic work per restart.  Running products (FP32, and the
        // unit-circle form): per (literal, complex frequency) factor and
        // running product 5 FLOPs, reverse product 5, leave-one-out dot 4;
        // per frequency the step-iii dot 4; real chains 8 FLOPs per literal;
        // priced at 10 k^2 per root-of-unity constraint.  FP64 polynomial form
        // (eval_kernel.h): its own count, poly_flops.  Bytes: one gathered
        // value and one slot per literal.
        double alg = 0.0;
        {
            const TypeD &td = types[(size_t)ti];
            const double nfc = (double)(td.n1 + td.n2);
            if (cls == CLASS_DFT && ct == CT_F64 && !uc) {
                alg = poly_flops(seg, L, td.n1 + td.n2);
                b.flops += alg;
            } else {
                b.flops += 14.0 * k * nfc + 4.0 * nfc + (td.has_real ? 8.0 * k : 0.0);
                if (cls == CLASS_DFT) alg = 10.0 * (double)k * (double)k;
            }
            b.exec_pos += (double)L * seg;
            b.bytes += (io == IO_F32 ? 8.0 : 16.0) * k;
        }
        items[(size_t)c] = Item{c, k, ti, bidx, cost, alg};
        b.count += 1;
        b.maxk = std::max(b.maxk, k);
        b.cost += cost;
        b.lits += k;
        if (cls == CLASS_DFT) b.k2 += (double)k * (double)k;
        b.alg += alg;
    }

    // 2. order bins by pull class (pullable bins last, so that their objective
    // rows are the last rows), then by total cost (heaviest first);
    // constraints by cost inside a bin (transform-free: longest first)
    std::vector<int> border(bins.size());
    for (size_t i = 0; i < bins.size(); ++i) border[i] = (int)i;
    std::stable_sort(border.begin(), border.end(), [&](int a, int b) {
        if (bins[a].pk != bins[b].pk) return bins[a].pk < bins[b].pk;
        return bins[a].cost > bins[b].cost;
    });
    std::vector<int> rank(bins.size());
    for (size_t r = 0; r < border.size(); ++r) rank[(size_t)border[r]] = (int)r;
    std::stable_sort(items.begin(), items.end(), [&](const Item &a, const Item &b) {
        if (rank[a.bin] != rank[b.bin]) return rank[a.bin] < rank[b.bin];
        return a.cost > b.cost;
    });
    std::vector<Bin> sorted;
    int first = 0;
    for (int r : border) {
        Bin b = bins[(size_t)r];
        b.first = first;
        first += b.count;
        if (b.cls == CLASS_REAL) b.cpw = b.maxk <= 8 ? 16 : (b.maxk <= 32 ? 8 : 2);
        else b.cpw = 1;
        b.wpb = 4;
        sorted.push_back(b);
    }
    Ly.bins = sorted;

    Ly.cost_prefix.assign((size_t)m + 1, 0.0);
    for (int q = 0; q < m; ++q) Ly.cost_prefix[(size_t)q + 1] = Ly.cost_prefix[(size_t)q] + items[(size_t)q].cost;
    Ly.k2_prefix.assign((size_t)m + 1, 0.0);
    Ly.alg_prefix.assign((size_t)m + 1, 0.0);
    for (int q = 0; q < m; ++q) {
        const Item &it = items[(size_t)q];
        const double k2 = bins[(size_t)it.bin].cls == CLASS_DFT ? (double)it.k * (double)it.k : 0.0;
        Ly.k2_prefix[(size_t)q + 1] = Ly.k2_prefix[(size_t)q] + k2;
        Ly.alg_prefix[(size_t)q + 1] = Ly.alg_prefix[(size_t)q] + it.alg;
    }

    // 3. binned descriptors and literals, original -> binned positions
    std::vector<ConDesc> con((size_t)m);
    std::vector<int32_t> lit((size_t)p->nnz);
    std::vector<int32_t> pos((size_t)m);
    Ly.h_rk.assign((size_t)m, -1);
    int64_t off = 0;
    for (int q = 0; q < m; ++q) {
        const Item &it = items[(size_t)q];
        Ly.h_rk[(size_t)q] = rkind[(size_t)it.c];
        const int kd = d->kinds[it.c], pm = d->params[it.c];
        const int chk = kd == FFSAT_KIND_OR ? 1 : (kd == FFSAT_KIND_XOR ? ((pm & 1) ? -2 : -1) : std::max(pm, 0));
        con[(size_t)q] = ConDesc{(int32_t)off, it.k, it.type, it.c, chk, 0, 0, 0};
        pos[(size_t)it.c] = q;
        for (int i = 0; i < it.k; ++i) {
            const int32_t l = d->lits[d->con_ptr[it.c] + i];
            const int32_t v = (l > 0 ? l : -l) - 1;
            lit[(size_t)(off + i)] = v | (l < 0 ? (int32_t)0x80000000u : 0);
        }
        off += it.k;
    }
    // 4. variable-major transpose over binned slots (ascending slot per variable)
    std::vector<int32_t> vptr((size_t)n + 1, 0), vslot((size_t)p->nnz);
    for (int64_t s = 0; s < p->nnz; ++s) vptr[(size_t)(lit[(size_t)s] & 0x7fffffff) + 1]++;
    for (int v = 0; v < n; ++v) vptr[(size_t)v + 1] += vptr[(size_t)v];
    {
        std::vector<int32_t> fill(vptr.begin(), vptr.end() - 1);
        for (int64_t s = 0; s < p->nnz; ++s) vslot[(size_t)fill[(size_t)(lit[(size_t)s] & 0x7fffffff)]++] = (int32_t)s;
    }
    // 5. type and frequency tables in both precisions
    std::vector<TypeF32> t32;
    std::vector<TypeF64> t64;
    std::vector<FreqF32> f32;
    std::vector<FreqF64> f64;
    for (const TypeD &td : types) {
        const int tab = (int)f64.size();
        TypeF32 a{(float)td.cst, (float)td.alpha, (float)td.beta, (float)td.c0r, (float)td.c1r,
                  (float)td.pad, td.n1, td.n2, td.has_real, tab};
        TypeF64 b{td.cst, td.alpha, td.beta, td.c0r, td.c1r, td.pad, td.n1, td.n2, td.has_real, tab};
        t32.push_back(a);
        t64.push_back(b);
        for (const FreqD &f : td.fr) {
            f32.push_back(FreqF32{(float)f.tk, (float)f.init, (float)f.c0re, (float)f.c0im,
                                  (float)f.c1re, (float)f.c1im, (float)f.p0, 0.f});
            if (td.poly) {
                // FreqPoly layout (the kernel reads the entry through that type)
                const double sg = -(f.tk * f.tk), itau = f.init * f.tk;
                f64.push_back(FreqF64{sg, 1.0 / sg, f.init, itau, f.c1re * f.init, f.c1im * f.init,
                                      f.c1re * itau, f.c1im * itau});
            } else {
                f64.push_back(FreqF64{f.tk, f.init, f.c0re, f.c0im, f.c1re, f.c1im, f.p0, 0.0});
            }
        }
    }
    // one entry of padding: the kernels prefetch the entry after a type's last
    f32.push_back(FreqF32{});
    f64.push_back(FreqF64{});
    Ly.n_types = (int)types.size();
    Ly.n_freqs = (int64_t)f64.size();
    ffsat_status st;
    if ((st = upload(&Ly.d_con, con, p->device_bytes)) != FFSAT_OK) return st;
    if ((st = upload(&Ly.d_lit, lit, p->device_bytes)) != FFSAT_OK) return st;
    if (io == IO_F32) {
        Ly.h_con = con;
        Ly.h_lit = lit;
    }
    if ((st = upload(&Ly.d_vptr, vptr, p->device_bytes)) != FFSAT_OK) return st;
    if ((st = upload(&Ly.d_vslot, vslot, p->device_bytes)) != FFSAT_OK) return st;
    if ((st = upload(&Ly.d_pos, pos, p->device_bytes)) != FFSAT_OK) return st;
    if ((st = upload(&Ly.d_t32, t32, p->device_bytes)) != FFSAT_OK) return st;
    if ((st = upload(&Ly.d_t64, t64, p->device_bytes)) != FFSAT_OK) return st;
    if ((st = upload(&Ly.d_f32, f32, p->device_bytes)) != FFSAT_OK) return st;
    if ((st = upload(&Ly.d_f64, f64, p->device_bytes)) != FFSAT_OK) return st;
    return FFSAT_OK;
}


static void free_problem(ffsat_problem *p)
{
    if (!p) return;
    ffsat_free_mpnn_graph(p->mpnn_graph);
    free_layout(p->lay[0]);
    free_layout(p->lay[1]);
    (void)hipFree(p->d_w);
    (void)hipFree(p->d_kind);
    (void)hipFree(p->d_param);
    delete p;
}

extern "C" ffsat_status ffsat_problem_create(const ffsat_problem_desc *d, ffsat_problem **out)
{
    if (!out) return fail(FFSAT_E_INVALID_ARG, "out is NULL");
    ffsat_status st = validate(d);
    if (st != FFSAT_OK) return st;
    int ndev = 0, cur = -1;
    HIPCHK(hipGetDeviceCount(&ndev));
    if (d->device < 0 || d->device >= ndev)
        return fail(FFSAT_E_DEVICE_MISMATCH, "device %d not present (%d devices)", d->device, ndev);
    HIPCHK(hipGetDevice(&cur));
    if (cur != d->device)
        return fail(FFSAT_E_DEVICE_MISMATCH, "device %d is not the current device (%d)", d->device, cur);
    ffsat_problem *p = new ffsat_problem();
    p->n = d->n_vars;
    p->m = d->n_cons;
    p->nnz = d->con_ptr[d->n_cons];
    p->device = d->device;
    p->fp64_min_len = d->fp64_min_len > 0 ? d->fp64_min_len : 128;
    p->flags = d->flags;
    for (int c = 0; c < p->m; ++c)
        p->maxk = std::max(p->maxk, (int32_t)(d->con_ptr[c + 1] - d->con_ptr[c]));
    std::vector<float> w((size_t)p->m, 1.0f);
    if (d->weights) std::copy(d->weights, d->weights + p->m, w.begin());
    std::vector<int32_t> kinds(d->kinds, d->kinds + p->m), params(d->params, d->params + p->m);
    p->h_con_ptr.assign(d->con_ptr, d->con_ptr + p->m + 1);
    p->h_lits.assign(d->lits, d->lits + p->nnz);
    p->h_kinds = kinds;
    p->h_params = params;
    CoeffMemo memo;
    if ((st = upload(&p->d_w, w, p->device_bytes)) != FFSAT_OK ||
        (st = upload(&p->d_kind, kinds, p->device_bytes)) != FFSAT_OK ||
        (st = upload(&p->d_param, params, p->device_bytes)) != FFSAT_OK ||
        (st = build_layout(p, d, IO_F32, memo)) != FFSAT_OK ||
        (st = build_layout(p, d, IO_F64, memo)) != FFSAT_OK) {
        free_problem(p);
        return st;
    }
    *out = p;
    return FFSAT_OK;
}

extern "C" ffsat_status ffsat_problem_destroy(ffsat_problem *p)
{
    free_problem(p);
    return FFSAT_OK;
}

extern "C" ffsat_status ffsat_problem_info_get(const ffsat_problem *p, ffsat_problem_info *info)
{
    if (!p || !info) return fail(FFSAT_E_INVALID_ARG, "NULL argument");
    info->n_vars = p->n;
    info->n_cons = p->m;
    info->nnz = p->nnz;
    info->max_len = p->maxk;
    info->n_bins_f32 = (int32_t)p->lay[0].bins.size();
    info->n_bins_f64 = (int32_t)p->lay[1].bins.size();
    info->device = p->device;
    info->device_bytes = p->device_bytes;
    return FFSAT_OK;
}

extern "C" ffsat_status ffsat_set_weights(ffsat_problem *p, const float *w, int32_t on_device, void *stream)
{
    if (!p || !w) return fail(FFSAT_E_INVALID_ARG, "NULL argument");
    HIPCHK(hipMemcpyAsync(p->d_w, w, sizeof(float) * (size_t)p->m,
                          on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, (hipStream_t)stream));
    if (!on_device) HIPCHK(hipStreamSynchronize((hipStream_t)stream));
    return FFSAT_OK;
}

extern "C" ffsat_status ffsat_get_weights(const ffsat_problem *p, float *w, int32_t on_device, void *stream)
{
    if (!p || !w) return fail(FFSAT_E_INVALID_ARG, "NULL argument");
    HIPCHK(hipMemcpyAsync(w, p->d_w, sizeof(float) * (size_t)p->m,
                          on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, (hipStream_t)stream));
    if (!on_device) HIPCHK(hipStreamSynchronize((hipStream_t)stream));
    return FFSAT_OK;
}

// ------------------------------------------------------------------ plan

namespace ffsat {
int fpart_rows_of(const std::vector<Bin> &bins)
{
    int rows = 0;
    for (const Bin &b : bins) rows += (b.count + b.cpw - 1) / b.cpw;
    return rows;
}
}  // namespace ffsat

static ffsat_status ensure_workspace(ffsat_plan *pl, int io)
{
    if (pl->d_slot[io]) return FFSAT_OK;
    const size_t es = io == IO_F32 ? sizeof(float) : sizeof(double);
    const size_t B = (size_t)pl->B;
    // objective / count rows: at most one per constraint, plus one per
    // variable chunk of the pulled gradient
    const int max_rows = pl->p->m + pl->p->n;
    const size_t slot = (size_t)pl->p->nnz * B * es;
    const size_t fpart = (size_t)max_rows * B * es;
    const size_t ftmp = (size_t)f_splits(max_rows) * B * es;
    HIPCHK(hipMalloc(&pl->d_slot[io], slot));
    HIPCHK(hipMalloc(&pl->d_fpart[io], fpart));
    HIPCHK(hipMalloc(&pl->d_ftmp[io], ftmp));
    pl->device_bytes += (int64_t)(slot + fpart + ftmp);
    if (!pl->d_cpart) {
        const size_t cp = (size_t)max_rows * B * sizeof(int32_t);
        const size_t ct = (size_t)f_splits(max_rows) * B * sizeof(int32_t);
        HIPCHK(hipMalloc(&pl->d_cpart, cp));
        HIPCHK(hipMalloc(&pl->d_ctmp, ct));
        pl->device_bytes += (int64_t)(cp + ct);
    }
    return FFSAT_OK;
}

static std::string bin_key(const ffsat_plan *pl, const Bin &b, int io)
{
    char buf[256];
    snprintf(buf, sizeof buf, "gfx950|io%d|B%d|c%d%s|t%d|s%d|L%d|n%d|l%lld|k%d", io, pl->B, b.cls, b.uc ? "uc" : "",
             b.ct, b.seg, b.L, b.count, (long long)b.lits, b.maxk);
    return buf;
}

struct Shape {
    int cpw, wpb, fg;
};

static std::map<std::string, Shape> read_cache(const std::string &path)
{
    std::map<std::string, Shape> out;
    std::ifstream f(path);
    if (!f) return out;
    std::stringstream ss;
    ss << f.rdbuf();
    const std::string s = ss.str();
    // entries: "key": [cpw, wpb, fg] (fg optional, default 1); the launch
    // structure entries ("|mode|" keys) hold [structure, pull class,
    // grouped shapes coded as 8 * chain cpw + frequency split] instead
    size_t i = 0;
    while ((i = s.find('"', i)) != std::string::npos) {
        const size_t j = s.find('"', i + 1);
        if (j == std::string::npos) break;
        const std::string key = s.substr(i + 1, j - i - 1);
        const size_t lb = s.find('[', j), rb = s.find(']', j);
        if (lb == std::string::npos || rb == std::string::npos) break;
        int cpw = 0, wpb = 0, fg = 1;
        const int got = sscanf(s.c_str() + lb + 1, "%d , %d , %d", &cpw, &wpb, &fg);
        if (key.find("|mode|") != std::string::npos) {
            if (got == 3 && cpw >= MODE_PER_BIN && cpw <= MODE_GROUP_DFT && wpb >= PULL_OFF && wpb <= PULL_LE3 &&
                fg >= 0 && fg <= 8 * 64 + 7)
                out[key] = {cpw, wpb, fg};
        } else if (got >= 2 && cpw > 0 && wpb > 0 && (got == 2 || (fg == 1 || fg == 2 || fg == 4))) {
            out[key] = {cpw, wpb, got == 3 ? fg : 1};
        }
        i = rb + 1;
    }
    return out;
}

static void write_cache(const std::string &path, const std::map<std::string, Shape> &m)
{
    std::ofstream f(path);
    if (!f) return;
    f << "{\n";
    size_t q = 0;
    for (const auto &kv : m) {
        f << "  \"" << kv.first << "\": [" << kv.second.cpw << ", " << kv.second.wpb << ", " << kv.second.fg << "]"
          << (++q < m.size() ? ",\n" : "\n");
    }
    f << "}\n";
}

template <typename IO>
static EvalArgs<IO> base_args(ffsat_plan *pl, int io, const IO *x, IO *con_val, bool want_grad)
{
    const ffsat_problem *p = pl->p;
    const Layout &Ly = p->lay[io];
    EvalArgs<IO> a{};
    a.x = x;
    a.slot = (IO *)pl->d_slot[io];
    a.fpart = (IO *)pl->d_fpart[io];
    a.con_val = con_val;
    a.con = Ly.d_con;
    a.lit = Ly.d_lit;
    a.w = p->d_w;
    a.cpart = pl->d_cpart;
    a.B = pl->B;
    a.wm = (p->m + 31) / 32;
    a.want_grad = want_grad ? 1 : 0;
    a.do_value = 1;
    a.want_check = 0;
    a.fg = 1;
    return a;
}

static hipEvent_t prof_event(ffsat_plan *pl)
{
    if (!pl->prof_pool.empty()) {
        hipEvent_t e = pl->prof_pool.back();
        pl->prof_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

static bool prof_active(ffsat_plan *pl, hipStream_t s)
{
    if (!pl->profiling) return false;
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(s, &cs) != hipSuccess) return false;
    return cs == hipStreamCaptureStatusNone;
}

static void prof_begin(ffsat_plan *pl, hipStream_t s, bool on, ProfRec &r, int io, int bin)
{
    r = ProfRec{io, bin, nullptr, nullptr};
    if (!on) return;
    r.e0 = prof_event(pl);
    r.e1 = prof_event(pl);
    if (r.e0) (void)hipEventRecord(r.e0, s);
}

static void prof_end(ffsat_plan *pl, hipStream_t s, ProfRec &r)
{
    if (!r.e0 || !r.e1) return;
    (void)hipEventRecord(r.e1, s);
    pl->prof_pending.push_back(r);
}

// Root-of-unity bins with FP64 arithmetic that the FP64 grouped launch can hold.
static bool in_group64(const Bin &b)
{
    return !b.uc && b.ct == CT_F64 && b.cls == CLASS_DFT && group_variant64(b.seg, b.L) >= 0;
}

// Block table of the grouped FP32 evaluation (MODE_GROUP_ALL: every bin with
// a grouped variant; MODE_GROUP_DFT: the root-of-unity bins, the others run
// on a side stream beside it).  Units of a bin are (chunk,
// restart block); a block runs 4 units (fg = 1) or one unit with its
// frequencies over 4 waves (fg = 4).  Blocks are ordered longest first
// (estimated VALU work), with the real-chain blocks spread evenly among the
// root-of-unity ones so that every CU mixes memory- and ALU-bound waves.
// The FP64-arithmetic root-of-unity bins with a variant of the FP64 group
// get a block table of their own, longest first.
static ffsat_status build_groups(ffsat_plan *pl)
{
    (void)hipFree(pl->d_gent);
    (void)hipFree(pl->d_gblk);
    (void)hipFree(pl->d_gent64);
    (void)hipFree(pl->d_gblk64);
    pl->d_gent = nullptr;
    pl->d_gblk = nullptr;
    pl->d_gent64 = nullptr;
    pl->d_gblk64 = nullptr;
    pl->gblocks = 0;
    pl->glds = 0;
    pl->gblocks64 = 0;
    pl->glds64 = 0;
    pl->gsolo.clear();
    if (!pl->grouped) return FFSAT_OK;
    const std::vector<Bin> &bins = pl->bins[IO_F32];
    std::vector<GroupEntry> ent, ent64;
    struct Blk {
        int2 b;
        double cost;
    };
    std::vector<Blk> dft, real, f64;
    int row0 = 0;
    for (int i = 0; i < (int)bins.size(); ++i) {
        const Bin &b = bins[i];
        const int rows = (b.count + b.cpw - 1) / b.cpw;
        if (in_group64(b) && (b.fg == 1 || b.fg == 4)) {
            // the FP64 group: blocks of 4 units (fg 1) or one unit over 4
            // waves (fg 4), longest first
            const int rpw = 64 / b.L;
            const int n_rb = (pl->B + rpw - 1) / rpw;
            const int ei = (int)ent64.size();
            ent64.push_back(GroupEntry{group_variant64(b.seg, b.L), b.first, b.count, b.cpw, n_rb, row0, b.fg, 0});
            const int64_t units = (int64_t)rows * n_rb;
            const double unit_cost = b.cost / std::max(1, b.count) * b.cpw * rpw;
            for (int64_t u = 0; u < units; u += (b.fg == 4 ? 1 : 4))
                f64.push_back({make_int2(ei, (int)u), b.fg == 4 ? unit_cost : 4 * unit_cost});
            if (b.fg == 4) pl->glds64 = std::max(pl->glds64, (size_t)3 * (b.seg + 1) * 64 * sizeof(double));
            row0 += rows;
            continue;
        }
        const int v = b.uc ? -1 : group_variant(b.ct, b.cls, b.seg, b.L);
        const int fg = b.cls == CLASS_DFT ? b.fg : 1;
        if (v < 0 || (fg != 1 && fg != 4) || (pl->mode == MODE_GROUP_DFT && b.cls != CLASS_DFT)) {
            pl->gsolo.push_back(i);
            row0 += rows;
            continue;
        }
        const int rpw = 64 / b.L;
        const int n_rb = (pl->B + rpw - 1) / rpw;
        GroupEntry e{v, b.first, b.count, b.cpw, n_rb, row0, fg, 0};
        const int ei = (int)ent.size();
        ent.push_back(e);
        const int64_t units = (int64_t)rows * n_rb;
        const double unit_cost = b.cost / std::max(1, b.count) * b.cpw * rpw;
        if (fg == 4) {
            for (int64_t u = 0; u < units; ++u) dft.push_back({make_int2(ei, (int)u), unit_cost});
            pl->glds = std::max(pl->glds, (size_t)3 * (b.seg + 1) * 64 * sizeof(float));
        } else {
            for (int64_t u = 0; u < units; u += 4)
                (b.cls == CLASS_DFT ? dft : real).push_back({make_int2(ei, (int)u), 4 * unit_cost});
        }
        row0 += rows;
    }
    if (!ent64.empty()) {
        std::stable_sort(f64.begin(), f64.end(), [](const Blk &x, const Blk &y) { return x.cost > y.cost; });
        std::vector<int2> order64;
        order64.reserve(f64.size());
        for (const Blk &q : f64) order64.push_back(q.b);
        HIPCHK(hipMalloc(&pl->d_gent64, ent64.size() * sizeof(GroupEntry)));
        HIPCHK(hipMemcpy(pl->d_gent64, ent64.data(), ent64.size() * sizeof(GroupEntry), hipMemcpyHostToDevice));
        HIPCHK(hipMalloc(&pl->d_gblk64, order64.size() * sizeof(int2)));
        HIPCHK(hipMemcpy(pl->d_gblk64, order64.data(), order64.size() * sizeof(int2), hipMemcpyHostToDevice));
        pl->gblocks64 = (int)order64.size();
    }
    if (ent.empty()) return FFSAT_OK;
    std::stable_sort(dft.begin(), dft.end(), [](const Blk &x, const Blk &y) { return x.cost > y.cost; });
    std::vector<int2> order;
    order.reserve(dft.size() + real.size());
    size_t di = 0, ri = 0;
    const double nd = (double)dft.size(), nr = (double)real.size();
    while (di < dft.size() || ri < real.size()) {
        // keep the fraction of real blocks emitted equal to that of root-of-unity ones
        const bool take_real = ri < real.size() && (di >= dft.size() || (ri + 0.5) / nr <= (di + 0.5) / nd);
        order.push_back(take_real ? real[ri++].b : dft[di++].b);
    }
    HIPCHK(hipMalloc(&pl->d_gent, ent.size() * sizeof(GroupEntry)));
    HIPCHK(hipMemcpy(pl->d_gent, ent.data(), ent.size() * sizeof(GroupEntry), hipMemcpyHostToDevice));
    HIPCHK(hipMalloc(&pl->d_gblk, order.size() * sizeof(int2)));
    HIPCHK(hipMemcpy(pl->d_gblk, order.data(), order.size() * sizeof(int2), hipMemcpyHostToDevice));
    pl->gblocks = (int)order.size();
    return FFSAT_OK;
}

// Launches every bin of the evaluation.  With side streams, the bins are
// spread over them (heaviest first, each to the least loaded stream) after a
// fork event on s, and s waits for all of them: independent bins overlap,
// and under graph capture they become parallel branches.
// Bins of pull class >= pk_limit are skipped (their gradient, objective and
// check come from k_pull); they are the last bins, so the launched bins'
// objective rows are the first rows either way.
template <typename IO>
static hipError_t enqueue_bins(ffsat_plan *pl, int io, EvalArgs<IO> a, hipStream_t s, int pk_limit = 3)
{
    const Layout &Ly = pl->p->lay[io];
    const std::vector<Bin> &bins = pl->bins[io];
    if constexpr (sizeof(IO) == 4) {
        if (pl->grouped && (pl->gblocks > 0 || pl->gblocks64 > 0)) {
            // bins without a grouped variant: on a side stream beside the
            // grouped launch when there is one, else before it
            hipError_t e;
            hipStream_t ss = s;
            // while profiling, everything runs on s: each launch's time is its own
            const bool fork = pl->side[0] != nullptr && !pl->gsolo.empty() && !pl->profiling;
            if (fork) {
                if ((e = hipEventRecord(pl->ev_fork, s)) != hipSuccess) return e;
                if ((e = hipStreamWaitEvent(pl->side[0], pl->ev_fork, 0)) != hipSuccess) return e;
                ss = pl->side[0];
            }
            if (pl->gblocks64 > 0) {
                // the long FP64 root-of-unity bins first: the heaviest work
                a.types = (const void *)Ly.d_t64;
                a.freqs = (const void *)Ly.d_f64;
                ProfRec rec;
                prof_begin(pl, ss, prof_active(pl, s), rec, io, -4);
                e = launch_eval_group64_f32(a, pl->d_gent64, pl->d_gblk64, pl->gblocks64, pl->glds64, ss);
                prof_end(pl, ss, rec);
                if (e != hipSuccess) return e;
            }
            for (int bi : pl->gsolo) {
                const Bin &b = bins[bi];
                if (b.pk >= pk_limit) continue;
                int row0 = 0;
                for (int q = 0; q < bi; ++q) row0 += (bins[q].count + bins[q].cpw - 1) / bins[q].cpw;
                a.first = b.first;
                a.count = b.count;
                a.cpw = b.cpw;
                a.fg = b.fg;
                a.n_rb = (pl->B + (64 / b.L) - 1) / (64 / b.L);
                a.fpart_row0 = row0;
                a.types = b.ct == CT_F32 ? (const void *)Ly.d_t32 : (const void *)Ly.d_t64;
                a.freqs = b.ct == CT_F32 ? (const void *)Ly.d_f32 : (const void *)Ly.d_f64;
                ProfRec rec;
                prof_begin(pl, ss, prof_active(pl, s), rec, io, bi);
                e = launch_eval_bin_f32(b, a, ss);
                prof_end(pl, ss, rec);
                if (e != hipSuccess) return e;
            }
            if (pl->gblocks > 0) {
                a.types = (const void *)Ly.d_t32;
                a.freqs = (const void *)Ly.d_f32;
                ProfRec rec;
                prof_begin(pl, s, prof_active(pl, s), rec, io, -2);
                e = launch_eval_group_f32(a, pl->d_gent, pl->d_gblk, pl->gblocks, pl->glds, s);
                prof_end(pl, s, rec);
                if (e != hipSuccess) return e;
            }
            if (fork) {
                if ((e = hipEventRecord(pl->ev_join[0], pl->side[0])) != hipSuccess) return e;
                if ((e = hipStreamWaitEvent(s, pl->ev_join[0], 0)) != hipSuccess) return e;
            }
            return hipSuccess;
        }
    }
    const bool fork = pl->side[0] != nullptr && bins.size() > 1 && !pl->profiling;
    hipError_t e;
    constexpr int NS = ffsat_plan::N_SIDE + 1;   // slot 0 is the caller's stream
    double load[NS] = {};
    bool used[NS] = {};
    if (fork) {
        if ((e = hipEventRecord(pl->ev_fork, s)) != hipSuccess) return e;
    }
    int row0 = 0;
    int bi = 0;
    for (const Bin &b : bins) {
        if (b.pk >= pk_limit) break;   // pulled bins are last
        a.first = b.first;
        a.count = b.count;
        a.cpw = b.cpw;
        a.fg = b.fg;
        a.n_rb = (pl->B + (64 / b.L) - 1) / (64 / b.L);
        a.fpart_row0 = row0;
        a.types = b.ct == CT_F32 ? (const void *)Ly.d_t32 : (const void *)Ly.d_t64;
        a.freqs = b.ct == CT_F32 ? (const void *)Ly.d_f32 : (const void *)Ly.d_f64;
        hipStream_t bs = s;
        if (fork) {
            int q = 0;
            for (int i = 1; i < NS; ++i)
                if (load[i] < load[q]) q = i;
            if (q > 0 && !used[q]) {
                if ((e = hipStreamWaitEvent(pl->side[q - 1], pl->ev_fork, 0)) != hipSuccess) return e;
            }
            used[q] = true;
            load[q] += b.cost * (double)pl->B + 5.0e6;   // work plus a per-launch latency term
            bs = q == 0 ? s : pl->side[q - 1];
        }
        ProfRec rec;
        prof_begin(pl, bs, prof_active(pl, s), rec, io, bi);
        if constexpr (sizeof(IO) == 4) e = launch_eval_bin_f32(b, a, bs);
        else e = launch_eval_bin_f64(b, a, bs);
        prof_end(pl, bs, rec);
        if (e != hipSuccess) return e;
        row0 += (b.count + b.cpw - 1) / b.cpw;
        ++bi;
    }
    if (fork) {
        for (int q = 1; q < NS; ++q) {
            if (!used[q]) continue;
            if ((e = hipEventRecord(pl->ev_join[q - 1], pl->side[q - 1])) != hipSuccess) return e;
            if ((e = hipStreamWaitEvent(s, pl->ev_join[q - 1], 0)) != hipSuccess) return e;
        }
    }
    return hipSuccess;
}

// Splits every bin heavier than an eighth of the total work into
// cost-balanced contiguous constraint ranges, so that the streams can share
// the work of one heavy bin.
static std::vector<Bin> split_bins(const std::vector<Bin> &in, const std::vector<double> &pre,
                                   const std::vector<double> &k2pre, const std::vector<double> &algpre)
{
    double total = 0;
    for (const Bin &b : in) total += b.cost;
    const double target = total / 8.0;
    std::vector<Bin> out;
    for (const Bin &b : in) {
        const int parts = (int)std::min<double>(b.count, std::ceil(b.cost / std::max(target, 1e-30)));
        if (parts <= 1) {
            out.push_back(b);
            continue;
        }
        const double c0 = pre[(size_t)b.first], c1 = pre[(size_t)b.first + b.count];
        int start = b.first;
        for (int q = 1; q <= parts; ++q) {
            int end = b.first + b.count;
            if (q < parts) {
                const double goal = c0 + (c1 - c0) * q / parts;
                end = (int)(std::lower_bound(pre.begin() + start + 1, pre.begin() + b.first + b.count, goal) - pre.begin());
                end = std::max(end, start + 1);
            }
            if (end <= start) continue;
            Bin part = b;
            part.first = start;
            part.count = end - start;
            const double frac = (pre[(size_t)end] - pre[(size_t)start]) / std::max(c1 - c0, 1e-30);
            part.cost = b.cost * frac;
            part.flops = b.flops * frac;
            part.bytes = b.bytes * frac;
            part.exec_pos = b.exec_pos * frac;
            part.k2 = k2pre[(size_t)end] - k2pre[(size_t)start];
            part.alg = algpre[(size_t)end] - algpre[(size_t)start];
            part.lits = (int64_t)((double)b.lits * frac);
            out.push_back(part);
            start = end;
            if (start >= b.first + b.count) break;
        }
    }
    std::stable_sort(out.begin(), out.end(), [](const Bin &a, const Bin &b) {
        if (a.pk != b.pk) return a.pk < b.pk;   // pullable bins stay last
        return a.cost > b.cost;
    });
    return out;
}

// Longest run of constraints one wave takes in a transform-free bin.
static int real_cpw_cap(const Bin &b) { return b.maxk <= 8 ? 16 : (b.maxk <= 32 ? 8 : 2); }

// Shapes of the bins inside a grouped launch.  There they share the chip
// with each other, and short waves cost more than in a launch of their own,
// so the per-bin shapes (timed bin by bin, they favour 1-2 transform-free
// constraints per wave and split long root-of-unity constraints' frequencies
// over 4 waves) do not carry over.  Timed in the grouped launch on the mixed
// instances at B = 256 and 1024: 8 constraints per wave beat 1-2, 4 and 16,
// and one wave per root-of-unity unit beat 4.
constexpr int GROUP_REAL_CPW = 8;
constexpr int GROUP_DFT_FG = 1;
constexpr int GROUP_CODE_MAX = 8 * 64 + 7;   // cache code of the grouped shapes: 8 * chain cpw + fg
static bool in_group(const ffsat_plan *pl, const Bin &b)
{
    if (in_group64(b)) return true;
    if (b.uc || group_variant(b.ct, b.cls, b.seg, b.L) < 0) return false;
    return b.cls == CLASS_DFT || pl->mode == MODE_GROUP_ALL;
}
// Sets the group values (c: transform-free constraints per wave, all-bin
// group only; f: root-of-unity frequency split, 1 or 4) or, with 0, gives
// those bins back their per-bin shapes; the objective rows follow.  While no
// group value is set the bins hold their per-bin shapes, which are recorded
// when one is set.
static void set_group_shapes(ffsat_plan *pl, int c, int f)
{
    std::vector<Bin> &bins = pl->bins[IO_F32];
    if (c == pl->group_real_cpw && f == pl->group_dft_fg) return;
    if (pl->group_real_cpw == 0 && pl->group_dft_fg == 0) {
        pl->solo_cpw.resize(bins.size());
        pl->solo_fg.resize(bins.size());
        for (size_t i = 0; i < bins.size(); ++i) {
            pl->solo_cpw[i] = bins[i].cpw;
            pl->solo_fg[i] = bins[i].fg;
        }
    }
    for (size_t i = 0; i < bins.size(); ++i) {
        Bin &b = bins[i];
        const bool g = pl->grouped && in_group(pl, b);
        if (b.cls == CLASS_REAL)
            b.cpw = g && c > 0 ? std::max(1, std::min({c, real_cpw_cap(b), b.count})) : pl->solo_cpw[i];
        else
            b.fg = g && f > 0 ? f : pl->solo_fg[i];
    }
    pl->group_real_cpw = c;
    pl->group_dft_fg = f;
    pl->fpart_rows[IO_F32] = fpart_rows_of(bins);
}

// Constraints per wave: enough waves per bin to cover the chip (the
// autotuner refines this).  Root-of-unity bins keep one constraint per wave.
static void default_shapes(ffsat_plan *pl)
{
    for (int io = 0; io < 2; ++io) {
        for (Bin &b : pl->bins[io]) {
            b.wpb = 4;
            b.fg = 1;
            if (b.cls == CLASS_DFT) {
                // one constraint per unit; split the frequencies over up to 4
                // waves until the bin alone has about 3 waves per SIMD
                b.cpw = 1;
                if (pl->grouped) {
                    // the grouped launch fills the chip anyway: split the
                    // frequencies of long constraints only (fg 1 or 4)
                    b.fg = b.maxk >= 32 ? 4 : 1;
                } else {
                    const int64_t units = (int64_t)b.count * ((pl->B + (64 / b.L) - 1) / (64 / b.L));
                    while (b.fg < 4 && units * b.fg < 3072) b.fg *= 2;
                }
                continue;
            }
            const int cap = real_cpw_cap(b);
            const int64_t n_rb = (pl->B + (64 / b.L) - 1) / (64 / b.L);
            const int64_t target = 4096;   // waves
            int64_t cpw = ((int64_t)b.count * n_rb) / target;
            b.cpw = (int)std::max<int64_t>(1, std::min<int64_t>(cap, cpw));
        }
        pl->fpart_rows[io] = fpart_rows_of(pl->bins[io]);
    }
    pl->group_real_cpw = 0;
    pl->group_dft_fg = 0;
    if (pl->grouped) set_group_shapes(pl, pl->mode == MODE_GROUP_ALL ? GROUP_REAL_CPW : 0, GROUP_DFT_FG);
}

// Destroys every cached executable graph, each after its latest launch has
// finished (a replay may still be in flight on the caller's stream).
static void clear_graphs(ffsat_plan *pl)
{
    for (auto &kv : pl->graphs) {
        if (kv.second.done) {
            (void)hipEventSynchronize(kv.second.done);
            (void)hipEventDestroy(kv.second.done);
        }
        (void)hipGraphExecDestroy(kv.second.exec);
    }
    pl->graphs.clear();
}

template <typename IO>
static ffsat_status run_eval(ffsat_plan *pl, const IO *x, IO *F, IO *grad, IO *con_val, int32_t *n_sat,
                             uint32_t *unsat_bits, int32_t *U, bool do_value, float *x_step, float eta,
                             hipStream_t s, const float *eta_dev = nullptr, const int32_t *skip = nullptr,
                             float *x_next = nullptr);

// Switches the pull path to class c (PULL_OFF, PULL_LE7, PULL_LE3): builds
// the problem's entry lists for c on first use and the plan's second point
// buffer.  A class without pullable bins, or the grouped launch of every
// bin (which holds the transform-free bins), turns it off; PULL_LE7 without
// constraints of length 4..7 is PULL_LE3.  Changing the class drops the
// cached graphs.
static ffsat_status set_pull(ffsat_plan *pl, int c)
{
    if (c == PULL_LE7) {
        bool mid = false;
        for (const Bin &b : pl->bins[IO_F32]) mid = mid || b.pk == PULL_LE7;
        if (!mid) c = PULL_LE3;
    }
    if (c != PULL_OFF) {
        bool any = false;
        for (const Bin &b : pl->bins[IO_F32]) any = any || b.pk >= c;
        // k_pull's gathers are buffer loads with 31-bit offsets into x
        const bool fits = (int64_t)pl->p->n * pl->B * 4 <= 0x7fffffffll;
        if (!any || !fits || pl->mode == MODE_GROUP_ALL) c = PULL_OFF;
    }
    if (c != PULL_OFF) {
        ffsat_status st = build_pull(pl->p, c);
        if (st != FFSAT_OK) return st;
        if (!pl->d_xalt) {
            const size_t bytes = sizeof(float) * (size_t)pl->p->n * (size_t)pl->B;
            HIPCHK(hipMalloc(&pl->d_xalt, bytes));
            pl->device_bytes += (int64_t)bytes;
        }
    }
    if (c != pl->pull) clear_graphs(pl);
    pl->pull = c;
    return FFSAT_OK;
}

static hipError_t enqueue_iters(ffsat_plan *pl, float *x, int T, bool erwa, float *F, int32_t *n_sat, int32_t *U,
                                hipStream_t s);
static hipError_t enqueue_iters_overlapped(ffsat_plan *pl, float *x, int T, bool erwa, float *F,
                                           int32_t *n_sat, int32_t *U, hipStream_t s);
// Time of one fused iteration (objective, exact check, projected step) under
// the plan's current launch structure and pull class, as the step loops run
// it (side-stream overlap of consecutive iterations included): TUNE_ITERS
// iterations on the tuner's scratch points with step size 0 from the plan's
// device scalar and no weight update, enqueued eagerly (no graph) once to
// warm up and then TUNE_REPS times under events.
static ffsat_status time_iterations(ffsat_plan *pl, hipStream_t s, hipEvent_t e0, hipEvent_t e1, float *ms)
{
    constexpr int TUNE_ITERS = 4, TUNE_REPS = 3;
    if (!pl->d_tune_u) {
        HIPCHK(hipMalloc(&pl->d_tune_u, sizeof(int32_t) * (size_t)pl->p->m));
        pl->device_bytes += (int64_t)(sizeof(int32_t) * (size_t)pl->p->m);
    }
    HIPCHK(launch_set_f32x2(pl->d_hyper, 0.f, 0.f, s));
    auto run = [&]() {
        return pl->iter_side
                   ? enqueue_iters_overlapped(pl, pl->d_scratch_x, TUNE_ITERS, false, nullptr, nullptr, pl->d_tune_u, s)
                   : enqueue_iters(pl, pl->d_scratch_x, TUNE_ITERS, false, nullptr, nullptr, pl->d_tune_u, s);
    };
    HIPCHK(run());
    HIPCHK(hipEventRecord(e0, s));
    for (int r = 0; r < TUNE_REPS; ++r) HIPCHK(run());
    HIPCHK(hipEventRecord(e1, s));
    HIPCHK(hipEventSynchronize(e1));
    float t = 0.f;
    HIPCHK(hipEventElapsedTime(&t, e0, e1));
    *ms = t / (TUNE_REPS * TUNE_ITERS);
    return FFSAT_OK;
}

// With MODE_AUTO (or an automatic pull choice), times the fused iteration
// (time_iterations) under each launch structure and pull class and keeps the
// fastest; the choice is cached with the shapes.
static ffsat_status tune_mode(ffsat_plan *pl, std::map<std::string, Shape> &cache, hipStream_t s)
{
    // a fixed structure and pull class leave nothing to time but the shapes
    // inside a grouped launch
    if (!pl->mode_auto && !pl->pull_auto && pl->mode == MODE_PER_BIN) return FFSAT_OK;
    char kb[200];
    snprintf(kb, sizeof kb, "gfx950|mode|B%d|n%d|m%d|nnz%lld|bins%zu|%s%d", pl->B, pl->p->n, pl->p->m,
             (long long)pl->p->nnz, pl->bins[IO_F32].size(), pl->mode_auto ? "a" : "f", pl->mode);
    const std::string key = pl->pull_auto ? std::string(kb) + "|pull" : std::string(kb) + "|p" + std::to_string(pl->pull);
    auto hit = cache.find(key);
    int best_mode = pl->mode, best_pull = pl->pull, best_gc = 0, best_gf = 0;
    if (hit != cache.end() && hit->second.cpw >= MODE_PER_BIN && hit->second.cpw <= MODE_GROUP_DFT &&
        hit->second.wpb >= PULL_OFF && hit->second.wpb <= PULL_LE3 && hit->second.fg >= 0 &&
        hit->second.fg <= GROUP_CODE_MAX) {
        best_mode = hit->second.cpw;
        best_pull = hit->second.wpb;
        best_gc = best_mode == MODE_GROUP_ALL ? hit->second.fg / 8 : 0;
        best_gf = best_mode != MODE_PER_BIN ? hit->second.fg % 8 : 0;
    } else {
        hipEvent_t e0, e1;
        HIPCHK(hipEventCreate(&e0));
        HIPCHK(hipEventCreate(&e1));
        std::vector<int> modes = pl->mode_auto ? std::vector<int>{MODE_GROUP_DFT, MODE_GROUP_ALL, MODE_PER_BIN}
                                               : std::vector<int>{pl->mode};
        std::vector<int> pulls = pl->pull_auto ? std::vector<int>{PULL_OFF, PULL_LE3, PULL_LE7}
                                               : std::vector<int>{pl->pull};
        // distinct (launch structure, pull class, grouped shapes) candidates
        // after normalisation; grouped launches are timed with their own
        // shapes (the per-bin shapes, timed alone, do not carry over): the
        // root-of-unity frequency split 1 or 4, and in the all-bin group the
        // transform-free bins at 4, 8 or 16 constraints per wave
        struct Cand {
            int mode, pull, gc, gf;
            bool operator==(const Cand &o) const
            {
                return mode == o.mode && pull == o.pull && gc == o.gc && gf == o.gf;
            }
        };
        std::vector<Cand> cands;
        for (int m : modes)
            for (int c : pulls) {
                pl->mode = m;
                ffsat_status st = set_pull(pl, c);
                if (st != FFSAT_OK) return st;
                std::vector<std::pair<int, int>> shapes;
                if (m == MODE_GROUP_ALL)
                    shapes = {{GROUP_REAL_CPW, GROUP_DFT_FG}, {4, 1}, {16, 1}, {GROUP_REAL_CPW, 4}};
                else if (m == MODE_GROUP_DFT)
                    shapes = {{0, GROUP_DFT_FG}, {0, 4}};
                else
                    shapes = {{0, 0}};
                for (const auto &sh : shapes) {
                    const Cand cand{m, pl->pull, sh.first, sh.second};
                    if (std::find(cands.begin(), cands.end(), cand) == cands.end()) cands.push_back(cand);
                }
            }
        // two sweeps over the candidates; a candidate's time is its faster
        // sweep, so that a slow moment of the device does not decide the choice
        std::vector<float> tbest(cands.size(), 1e30f);
        for (int sweep = 0; sweep < 2; ++sweep) {
            for (size_t i = 0; i < cands.size(); ++i) {
                pl->mode = cands[i].mode;
                pl->grouped = pl->mode != MODE_PER_BIN;
                set_group_shapes(pl, cands[i].gc, cands[i].gf);
                ffsat_status st = set_pull(pl, cands[i].pull);
                if (st != FFSAT_OK) return st;
                if ((st = build_groups(pl)) != FFSAT_OK) return st;
                float ms = 0.f;
                if ((st = time_iterations(pl, s, e0, e1, &ms)) != FFSAT_OK) return st;
                tbest[i] = std::min(tbest[i], ms);
            }
        }
        // the fastest; an earlier candidate keeps the choice within 2 %
        size_t bi = 0;
        for (size_t i = 1; i < cands.size(); ++i)
            if (tbest[i] < tbest[bi] * 0.98f) bi = i;
        best_mode = cands[bi].mode;
        best_pull = cands[bi].pull;
        best_gc = cands[bi].gc;
        best_gf = cands[bi].gf;
        std::ostringstream lg;
        for (size_t i = 0; i < cands.size(); ++i)
            lg << (i ? ", " : "") << "[" << cands[i].mode << ", " << PULL_K[cands[i].pull] << ", " << cands[i].gc
               << ", " << cands[i].gf << ", " << tbest[i] << "]";
        pl->tune_log = lg.str();
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        // structure in the cpw field, pull class in wpb, grouped shapes
        // (8 * chain cpw + frequency split) in fg
        cache[key] = Shape{best_mode, best_pull, 8 * best_gc + best_gf};
    }
    pl->mode = best_mode;
    pl->grouped = best_mode != MODE_PER_BIN;
    set_group_shapes(pl, best_gc, best_gf);
    clear_graphs(pl);
    return set_pull(pl, best_pull);
}

extern "C" ffsat_status ffsat_plan_tune(ffsat_plan *pl, void *stream)
{
    if (!pl) return fail(FFSAT_E_INVALID_ARG, "NULL plan");
    hipStream_t s = (hipStream_t)stream;
    ffsat_status st = ensure_workspace(pl, IO_F32);
    if (st != FFSAT_OK) return st;
    const ffsat_problem *p = pl->p;
    if (!pl->d_scratch_x) {
        HIPCHK(hipMalloc(&pl->d_scratch_x, sizeof(float) * (size_t)p->n * (size_t)pl->B));
        pl->device_bytes += (int64_t)(sizeof(float) * (size_t)p->n * (size_t)pl->B);
        HIPCHK(launch_scratch_points(pl->d_scratch_x, (int64_t)p->n * pl->B, 12345u, s));
    }
    std::map<std::string, Shape> cache;
    if (!pl->tune_cache.empty()) cache = read_cache(pl->tune_cache);
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    EvalArgs<float> a = base_args<float>(pl, IO_F32, pl->d_scratch_x, nullptr, true);
    a.want_check = 1;
    const Layout &Ly = p->lay[IO_F32];
    bool dirty = false;
    set_group_shapes(pl, 0, 0);   // per-bin shapes are timed bin by bin
    for (Bin &b : pl->bins[IO_F32]) {
        const std::string key = bin_key(pl, b, IO_F32);
        auto hit = cache.find(key);
        if (hit != cache.end()) {
            b.cpw = hit->second.cpw;
            b.wpb = hit->second.wpb;
            b.fg = b.cls == CLASS_DFT ? hit->second.fg : 1;
            continue;
        }
        a.first = b.first;
        a.count = b.count;
        a.n_rb = (pl->B + (64 / b.L) - 1) / (64 / b.L);
        a.fpart_row0 = 0;
        a.types = b.ct == CT_F32 ? (const void *)Ly.d_t32 : (const void *)Ly.d_t64;
        a.freqs = b.ct == CT_F32 ? (const void *)Ly.d_f32 : (const void *)Ly.d_f64;
        float best = 1e30f;
        Shape bs{b.cpw, b.wpb, b.fg};
        std::vector<Shape> cands;
        if (b.cls == CLASS_DFT) {
            for (int fg : {1, 2, 4})
                for (int cpw : {1, 2, 4}) {
                    if (pl->grouped && fg == 2) break;   // grouped blocks take fg 1 or 4
                    if (cpw > 1 && cpw > b.count) break;
                    if (fg == 1) {
                        for (int wpb : {1, 2, 4}) cands.push_back({cpw, wpb, 1});
                    } else {
                        cands.push_back({cpw, fg, fg});
                    }
                }
        } else {
            for (int cpw : {1, 2, 4, 8, 16, 32, 64}) {
                if (cpw > 1 && cpw > b.count) break;
                for (int wpb : {1, 2, 4}) cands.push_back({cpw, wpb, 1});
            }
        }
        for (const Shape &c : cands) {
            Bin t = b;
            t.cpw = c.cpw;
            t.wpb = c.wpb;
            t.fg = c.fg;
            a.cpw = c.cpw;
            a.fg = c.fg;
            HIPCHK(launch_eval_bin_f32(t, a, s));
            HIPCHK(hipEventRecord(e0, s));
            const int reps = 3;
            for (int r = 0; r < reps; ++r) HIPCHK(launch_eval_bin_f32(t, a, s));
            HIPCHK(hipEventRecord(e1, s));
            HIPCHK(hipEventSynchronize(e1));
            float ms = 0.f;
            HIPCHK(hipEventElapsedTime(&ms, e0, e1));
            ms /= reps;
            if (ms < best * 0.97f) { best = ms; bs = c; }
        }
        b.cpw = bs.cpw;
        b.wpb = bs.wpb;
        b.fg = bs.fg;
        cache[key] = bs;
        dirty = true;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    pl->fpart_rows[IO_F32] = fpart_rows_of(pl->bins[IO_F32]);
    // cached graphs baked the old shapes
    clear_graphs(pl);
    pl->tuned = true;
    const size_t n_cached = cache.size();
    if ((st = tune_mode(pl, cache, s)) != FFSAT_OK) return st;
    if ((st = build_groups(pl)) != FFSAT_OK) return st;
    if ((dirty || cache.size() != n_cached) && !pl->tune_cache.empty()) write_cache(pl->tune_cache, cache);
    return FFSAT_OK;
}

extern "C" ffsat_status ffsat_plan_create(ffsat_problem *p, int32_t B, const ffsat_plan_opts *opts, ffsat_plan **out)
{
    if (!p || !out) return fail(FFSAT_E_INVALID_ARG, "NULL argument");
    if (B < 1) return fail(FFSAT_E_INVALID_ARG, "B must be >= 1 (got %d)", B);
    if ((int64_t)B * (int64_t)std::max<int64_t>(p->nnz, p->m) > ((int64_t)1 << 40))
        return fail(FFSAT_E_UNSUPPORTED, "nnz * B too large");
    ffsat_plan *pl = new ffsat_plan();
    pl->p = p;
    pl->B = B;
    pl->bins[0] = split_bins(p->lay[0].bins, p->lay[0].cost_prefix, p->lay[0].k2_prefix, p->lay[0].alg_prefix);
    pl->bins[1] = split_bins(p->lay[1].bins, p->lay[1].cost_prefix, p->lay[1].k2_prefix, p->lay[1].alg_prefix);
    const int req = opts ? opts->reserved[1] : MODE_AUTO;
    if (req < MODE_AUTO || req > MODE_GROUP_DFT) {
        delete pl;
        return fail(FFSAT_E_INVALID_ARG, "reserved[1] (evaluation mode) must be in 0..3");
    }
    pl->mode_auto = req == MODE_AUTO;
    const int preq = opts ? opts->reserved[2] : 0;
    // an automatic choice before (or without) the tuner: one grouped launch
    // of every bin, fewest launches per step; the root-of-unity group with the
    // transform-free bins beside it when the pulled gradient is asked for,
    // which the all-bin group excludes
    pl->mode = !pl->mode_auto ? req : (preq == 2 || preq == 3 ? MODE_GROUP_DFT : MODE_GROUP_ALL);
    pl->grouped = pl->mode != MODE_PER_BIN;
    const int vc = opts ? opts->reserved[3] : 0;
    const int persist = opts ? opts->reserved[4] : 0;
    if (preq < 0 || preq > 3 || vc < 0 || vc > PULL_VC_MAX || persist < 0 || persist > 1 ||
        (opts && (opts->reserved[5] || opts->reserved[6] || opts->reserved[7]))) {
        delete pl;
        return fail(FFSAT_E_INVALID_ARG, "reserved[2] (pull) must be in 0..3, reserved[3] (variables per wave) in "
                                         "0..8, reserved[4] (persistent step loop) in 0..1, reserved[5..7] must be 0");
    }
    pl->persistent = persist == 1;
    pl->pull_auto = preq == 0;
    pl->pull_vc = vc > 0 ? vc : 8;
    default_shapes(pl);
    pl->use_graphs = opts ? opts->use_graphs != 0 : true;
    if (opts && opts->tune_cache) pl->tune_cache = opts->tune_cache;
    ffsat_status st = ensure_workspace(pl, IO_F32);
    if (st == FFSAT_OK) {
        hipError_t e = hipMalloc(&pl->d_flag, sizeof(int32_t));
        if (e == hipSuccess) e = hipMalloc(&pl->d_umax, 1024 * sizeof(int32_t));
        if (e == hipSuccess) e = hipMalloc(&pl->d_hyper, 2 * sizeof(float));
        if (e != hipSuccess) st = fail(FFSAT_E_NOMEM, "hipMalloc flag: %s", hipGetErrorString(e));
    }
    if (st == FFSAT_OK && !(opts && opts->reserved[0] == 1)) {
        // side streams (default priority) for concurrent bins; reserved[0] == 1 disables them
        hipError_t e = hipEventCreateWithFlags(&pl->ev_fork, hipEventDisableTiming);
        for (int q = 0; q < ffsat_plan::N_SIDE && e == hipSuccess; ++q) {
            e = hipStreamCreateWithFlags(&pl->side[q], hipStreamNonBlocking);
            if (e == hipSuccess) e = hipEventCreateWithFlags(&pl->ev_join[q], hipEventDisableTiming);
        }
        if (e == hipSuccess) e = hipStreamCreateWithFlags(&pl->iter_side, hipStreamNonBlocking);
        for (hipEvent_t *ev : {&pl->ev_eval, &pl->ev_red, &pl->ev_aux, &pl->ev_sum})
            if (e == hipSuccess) e = hipEventCreateWithFlags(ev, hipEventDisableTiming);
        if (e != hipSuccess) st = fail(FFSAT_E_HIP, "side streams: %s", hipGetErrorString(e));
    }
    if (st == FFSAT_OK && !pl->pull_auto) st = set_pull(pl, preq == 1 ? PULL_OFF : (preq == 2 ? PULL_LE7 : PULL_LE3));
    if (st == FFSAT_OK && pl->persistent) {
        // eligible: every constraint pulled (transform-free, length <= 7) and
        // the points, the per-pair gradient terms and the lists fit in LDS
        int cmin = PULL_LE3;
        bool all = !pl->bins[IO_F32].empty();
        for (const Bin &b : pl->bins[IO_F32]) {
            all = all && b.pk >= PULL_LE7;
            cmin = std::min(cmin, b.pk);
        }
        if (all && (int64_t)8 * p->n * B + (int64_t)4 * p->m * B + (int64_t)8 * p->m <= ITERS_SMALL_LDS) {
            st = build_pull(p, cmin);
            if (st == FFSAT_OK &&
                iters_small_lds(PULL_E[cmin], p->n, B, p->m, p->lay[IO_F32].pull[cmin].n_ent) <= ITERS_SMALL_LDS)
                pl->persistent_class = cmin;
        }
    }
    if (st == FFSAT_OK) st = build_groups(pl);
    if (st == FFSAT_OK && opts && opts->autotune) {
        st = ffsat_plan_tune(pl, nullptr);
        if (st == FFSAT_OK) {
            hipError_t e = hipDeviceSynchronize();
            if (e != hipSuccess) st = fail(FFSAT_E_HIP, "sync after tuning: %s", hipGetErrorString(e));
        }
    }
    if (st != FFSAT_OK) {
        ffsat_plan_destroy(pl);
        return st;
    }
    *out = pl;
    return FFSAT_OK;
}

extern "C" ffsat_status ffsat_plan_profile(ffsat_plan *pl, int32_t on)
{
    if (!pl) return fail(FFSAT_E_INVALID_ARG, "NULL plan");
    pl->profiling = on != 0;
    return FFSAT_OK;
}

extern "C" ffsat_status ffsat_plan_profile_read(ffsat_plan *pl, int32_t reset, char *buf, size_t len)
{
    if (!pl || !buf || len == 0) return fail(FFSAT_E_INVALID_ARG, "NULL argument");
    for (ProfRec &r : pl->prof_pending) {
        HIPCHK(hipEventSynchronize(r.e1));
        float ms = 0.f;
        HIPCHK(hipEventElapsedTime(&ms, r.e0, r.e1));
        auto &acc = pl->prof_acc[{r.io, r.bin}];
        acc.first += ms;
        acc.second += 1;
        pl->prof_pool.push_back(r.e0);
        pl->prof_pool.push_back(r.e1);
    }
    pl->prof_pending.clear();
    std::ostringstream o;
    o << "{\"kernels\": [";
    size_t q = 0;
    for (const auto &kv : pl->prof_acc) {
        o << (q++ ? ", " : "") << "{\"io\": \"" << (kv.first.first ? "f64" : "f32") << "\", \"bin\": " << kv.first.second
          << ", \"launches\": " << kv.second.second << ", \"total_ms\": " << kv.second.first
          << ", \"avg_ms\": " << (kv.second.second ? kv.second.first / (double)kv.second.second : 0.0) << "}";
    }
    o << "]}";
    if (reset) pl->prof_acc.clear();
    const std::string str = o.str();
    const size_t nb = std::min(len - 1, str.size());
    memcpy(buf, str.data(), nb);
    buf[nb] = 0;
    return FFSAT_OK;
}

extern "C" ffsat_status ffsat_plan_destroy(ffsat_plan *pl)
{
    if (!pl) return FFSAT_OK;
    for (ProfRec &r : pl->prof_pending) {
        (void)hipEventDestroy(r.e0);
        (void)hipEventDestroy(r.e1);
    }
    for (hipEvent_t e : pl->prof_pool) (void)hipEventDestroy(e);
    clear_graphs(pl);
    (void)hipFree(pl->d_hyper);
    (void)hipFree(pl->d_xalt);
    (void)hipFree(pl->d_tune_u);
    (void)hipFree(pl->d_gent);
    (void)hipFree(pl->d_gblk);
    (void)hipFree(pl->d_gent64);
    (void)hipFree(pl->d_gblk64);
    for (int io = 0; io < 2; ++io) {
        (void)hipFree(pl->d_slot[io]);
        (void)hipFree(pl->d_fpart[io]);
        (void)hipFree(pl->d_ftmp[io]);
    }
    (void)hipFree(pl->d_flag);
    (void)hipFree(pl->d_umax);
    (void)hipFree(pl->d_cpart);
    (void)hipFree(pl->d_ctmp);
    (void)hipFree(pl->d_scratch_x);
    (void)hipFree(pl->d_fz);
    (void)hipFree(pl->d_fg);
    (void)hipFree(pl->d_fFy);
    (void)hipFree(pl->d_fFz);
    (void)hipFree(pl->d_fpartial);
    (void)hipFree(pl->d_fcoef);
    (void)hipFree(pl->d_fflags);
    (void)hipFree(pl->d_fpending);
    if (pl->cap) (void)hipStreamDestroy(pl->cap);
    for (int q = 0; q < ffsat_plan::N_SIDE; ++q) {
        if (pl->side[q]) (void)hipStreamDestroy(pl->side[q]);
        if (pl->ev_join[q]) (void)hipEventDestroy(pl->ev_join[q]);
    }
    if (pl->ev_fork) (void)hipEventDestroy(pl->ev_fork);
    if (pl->iter_side) (void)hipStreamDestroy(pl->iter_side);
    for (hipEvent_t ev : {pl->ev_eval, pl->ev_red, pl->ev_aux, pl->ev_sum})
        if (ev) (void)hipEventDestroy(ev);
    delete pl;
    return FFSAT_OK;
}

static int eval_rows(const ffsat_plan *pl, int io, int pull);

extern "C" ffsat_status ffsat_plan_describe(const ffsat_plan *pl, char *buf, size_t len)
{
    if (!pl || !buf || len == 0) return fail(FFSAT_E_INVALID_ARG, "NULL argument");
    std::ostringstream o;
    static const char *mode_names[] = {"auto", "per_bin", "group_all", "group_dft"};
    o << "{\"B\": " << pl->B << ", \"tuned\": " << (pl->tuned ? "true" : "false") << ", \"mode\": \""
      << mode_names[pl->mode] << "\"" << ", \"mode_auto\": " << (pl->mode_auto ? "true" : "false")
      << ", \"grouped\": " << (pl->grouped && pl->gblocks > 0 ? "true" : "false") << ", \"group_blocks\": " << pl->gblocks
      << ", \"group64_blocks\": " << pl->gblocks64 << ", \"solo_bins\": " << pl->gsolo.size() << ", \"graphs_cached\": " << pl->graphs.size()
      << ", \"graph_captures\": " << pl->captures << ", \"pull\": " << PULL_K[pl->pull]
      << ", \"pull_auto\": " << (pl->pull_auto ? "true" : "false") << ", \"pull_vc\": " << pl->pull_vc
      << ", \"pull_entries\": " << (pl->pull ? pl->p->lay[IO_F32].pull[pl->pull].n_ent : 0)
      << ", \"pull_entry_bytes\": " << (pl->pull ? 4 * PULL_E[pl->pull] : 0)
      << ", \"pull_gathers_per_restart\": " << (pl->pull ? pl->p->lay[IO_F32].pull[pl->pull].n_gather : 0)
      << ", \"pull_other_slots\": " << (pl->pull ? pl->p->lay[IO_F32].pull[pl->pull].n_rest : 0)
      << ", \"pull_chunks\": " << (pl->pull ? (pl->p->n + pl->pull_vc - 1) / pl->pull_vc : 0)
      << ", \"objective_rows\": " << eval_rows(pl, IO_F32, pl->pull)
      << ", \"group_real_cpw\": " << pl->group_real_cpw << ", \"group_dft_fg\": " << pl->group_dft_fg
      << ", \"tuned_modes\": [" << pl->tune_log << "], \"persistent_steps\": "
      << (pl->persistent_class ? "true" : "false") << ", \"bins\": {";
    for (int io = 0; io < 2; ++io) {
        o << (io ? ", " : "") << "\"" << (io ? "f64" : "f32") << "\": [";
        for (size_t i = 0; i < pl->bins[io].size(); ++i) {
            const Bin &b = pl->bins[io][i];
            o << (i ? ", " : "") << "{\"class\": \"" << (b.cls == CLASS_DFT ? (b.uc ? "dft_uc" : "dft") : "real") << "\", \"ct\": \""
              << (b.ct == CT_F32 ? "f32" : "f64") << "\", \"seg\": " << b.seg << ", \"L\": " << b.L
              << ", \"first\": " << b.first << ", \"count\": " << b.count << ", \"maxk\": " << b.maxk
              << ", \"lits\": " << b.lits << ", \"cost\": " << b.cost << ", \"flops_per_restart\": " << b.flops
              << ", \"bytes_per_restart\": " << b.bytes << ", \"positions_per_restart\": " << b.exec_pos
              << ", \"k2_per_restart\": " << b.k2 << ", \"alg_flops_per_restart\": " << b.alg
              << ", \"pull_class\": " << b.pk << ", \"pulled\": " << (io == IO_F32 && pl->pull && b.pk >= pl->pull ? "true" : "false")
              << ", \"cpw\": " << b.cpw
              << ", \"wpb\": " << b.wpb << ", \"fg\": " << b.fg;
            // the grouped launch that evaluates the bin, if any
            const bool g64 = io == IO_F32 && pl->grouped && pl->gblocks64 > 0 && in_group64(b) && (b.fg == 1 || b.fg == 4);
            const bool g32 = io == IO_F32 && pl->grouped && pl->gblocks > 0 && !g64 &&
                             std::find(pl->gsolo.begin(), pl->gsolo.end(), (int)i) == pl->gsolo.end();
            o << ", \"in_group\": " << (g32 ? "true" : "false") << ", \"in_group64\": " << (g64 ? "true" : "false")
              << "}";
        }
        o << "]";
    }
    o << "}}";
    const std::string s = o.str();
    const size_t nb = std::min(len - 1, s.size());
    memcpy(buf, s.data(), nb);
    buf[nb] = 0;
    return FFSAT_OK;
}

// ------------------------------------------------------------------ evaluation

template <typename IO>
static ffsat_status check_finite(ffsat_plan *pl, const IO *x, hipStream_t s)
{
    if (!(pl->p->flags & FFSAT_FLAG_DEBUG_CHECKS)) return FFSAT_OK;
    HIPCHK(launch_fill_i32(pl->d_flag, 1, 0, s));
    const int64_t tot = (int64_t)pl->p->n * pl->B;
    if constexpr (sizeof(IO) == 4) HIPCHK(launch_nonfinite_f32(tot, (const float *)x, pl->d_flag, s));
    else HIPCHK(launch_nonfinite_f64(tot, (const double *)x, pl->d_flag, s));
    int32_t h = 0;
    HIPCHK(hipMemcpyAsync(&h, pl->d_flag, sizeof h, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (h) return fail(FFSAT_E_NONFINITE, "input point contains NaN or Inf");
    return FFSAT_OK;
}

// The pull path serves an FP32 evaluation that produces a gradient or a step
// and no per-constraint values.
static bool pull_on(const ffsat_plan *pl, int io, bool do_value, const void *con_val, bool grad_or_step)
{
    return io == IO_F32 && pl->pull > 0 && do_value && con_val == nullptr && grad_or_step;
}

// Objective / count rows an evaluation writes: the launched bins' rows (the
// first rows), then with the pull path one row per variable chunk.
static int eval_rows(const ffsat_plan *pl, int io, int pull)
{
    int rows = 0;
    for (const Bin &b : pl->bins[io])
        if (!pull || b.pk < pull) rows += (b.count + b.cpw - 1) / b.cpw;
    if (pull) rows += (pl->p->n + pl->pull_vc - 1) / pl->pull_vc;
    return rows;
}

// k_pull: the gradient (grad) or the projected step (x_out != x), the
// objective and check rows of the pulled constraints, and the gradient
// share of every other constraint from its slots.
static hipError_t enqueue_pull(ffsat_plan *pl, const float *x, float *grad, float *x_out, float eta,
                               const float *eta_dev, uint32_t *unsat_bits, int32_t *U, bool want_check,
                               const int32_t *skip, hipStream_t s)
{
    const ffsat_problem *p = pl->p;
    const PullLayout &P = p->lay[IO_F32].pull[pl->pull];
    if (!P.built) return hipErrorNotReady;
    PullArgs a{};
    a.x = x;
    a.x_out = x_out;
    a.grad = grad;
    a.slot = (const float *)pl->d_slot[IO_F32];
    a.vptr = P.d_vptr;
    a.vslot = P.d_vslot;
    a.pptr = P.d_pptr;
    a.pent = P.d_pent;
    a.w = p->d_w;
    a.fpart = (float *)pl->d_fpart[IO_F32];
    a.cpart = pl->d_cpart;
    a.unsat_bits = unsat_bits;
    a.U = U;
    a.eta_dev = eta_dev;
    a.skip = skip;
    a.eta = eta;
    a.n = p->n;
    a.B = pl->B;
    a.vc = pl->pull_vc;
    a.row0 = eval_rows(pl, IO_F32, pl->pull) - (p->n + pl->pull_vc - 1) / pl->pull_vc;
    a.wm = (p->m + 31) / 32;
    a.want_check = want_check ? 1 : 0;
    a.rk = P.d_rk;
    a.x_bytes = (int64_t)p->n * pl->B * (int64_t)sizeof(float);
    return launch_pull(PULL_E[pl->pull], a, s);
}

template <typename IO>
static ReduceArgs<IO> reduce_args(ffsat_plan *pl, int io, IO *grad, float *x_step, float eta, const float *eta_dev,
                                  const int32_t *skip, IO *F, int32_t *n_sat, int pull)
{
    const ffsat_problem *p = pl->p;
    const Layout &Ly = p->lay[io];
    ReduceArgs<IO> r{};
    r.n = p->n;
    r.B = pl->B;
    r.m = p->m;
    r.vptr = Ly.d_vptr;
    r.vslot = Ly.d_vslot;
    r.slot = (const IO *)pl->d_slot[io];
    r.grad = pull ? nullptr : grad;
    r.x_step = pull ? nullptr : x_step;
    r.eta = eta;
    r.eta_dev = eta_dev;
    r.skip = skip;
    r.fpart = (const IO *)pl->d_fpart[io];
    r.cpart = pl->d_cpart;
    r.rows = eval_rows(pl, io, pull);
    r.ftmp = (IO *)pl->d_ftmp[io];
    r.ctmp = pl->d_ctmp;
    r.F = F;
    r.n_sat = n_sat;
    return r;
}

// One evaluation pass: optional value/gradient/objective outputs, optional
// exact check of the same point, optional fused projected step (in place
// into x_step; with the pull path, into x_next when given, else through
// the plan's second point buffer and a copy back).
template <typename IO>
static ffsat_status run_eval(ffsat_plan *pl, const IO *x, IO *F, IO *grad, IO *con_val, int32_t *n_sat,
                             uint32_t *unsat_bits, int32_t *U, bool do_value, float *x_step, float eta,
                             hipStream_t s, const float *eta_dev, const int32_t *skip, float *x_next)
{
    const int io = sizeof(IO) == 4 ? IO_F32 : IO_F64;
    const ffsat_problem *p = pl->p;
    const bool want_check = n_sat || unsat_bits || U;
    if (!do_value && !want_check) return FFSAT_OK;
    if (U) HIPCHK(launch_fill_i32(U, p->m, 0, s));
    if (unsat_bits) HIPCHK(launch_fill_i32((int32_t *)unsat_bits, (int64_t)((p->m + 31) / 32) * pl->B, 0, s));
    const bool grad_slots = do_value && (grad != nullptr || x_step != nullptr);
    const int pull = pull_on(pl, io, do_value, con_val, grad_slots) ? pl->pull : 0;
    EvalArgs<IO> a = base_args<IO>(pl, io, x, do_value ? con_val : nullptr, grad_slots);
    a.do_value = do_value ? 1 : 0;
    a.want_check = want_check ? 1 : 0;
    a.unsat_bits = unsat_bits;
    a.U = U;
    a.skip = skip;
    HIPCHK(enqueue_bins<IO>(pl, io, a, s, pull ? pull : 3));
    ReduceArgs<IO> r = reduce_args<IO>(pl, io, do_value ? grad : nullptr, do_value ? x_step : nullptr, eta, eta_dev,
                                       skip, do_value ? F : nullptr, n_sat, pull);
    // profile records: -3 the pulled gradient, -1 the reduction (with the
    // pull path only the objective / count sums)
    ProfRec rec;
    hipError_t e = hipSuccess;
    if constexpr (sizeof(IO) == 4) {
        if (pull) {
            float *out = nullptr;
            if (x_step) out = x_next ? x_next : pl->d_xalt;
            prof_begin(pl, s, prof_active(pl, s), rec, io, -3);
            e = enqueue_pull(pl, (const float *)x, x_step ? nullptr : (float *)grad, out, eta, eta_dev, unsat_bits, U,
                             want_check, skip, s);
            prof_end(pl, s, rec);
            if (e == hipSuccess && x_step && !x_next)
                e = launch_copy_f32(x_step, pl->d_xalt, (int64_t)p->n * pl->B, s);
        }
        prof_begin(pl, s, prof_active(pl, s), rec, io, -1);
        if (e == hipSuccess) e = launch_reduce_f32(r, s);
    } else {
        prof_begin(pl, s, prof_active(pl, s), rec, io, -1);
        e = launch_reduce_f64(r, s);
    }
    prof_end(pl, s, rec);
    HIPCHK(e);
    return FFSAT_OK;
}

extern "C" ffsat_status ffsat_eval(ffsat_plan *pl, const float *x, float *F, float *grad, float *con_val, void *stream)
{
    if (!pl || !x) return fail(FFSAT_E_INVALID_ARG, "NULL plan or x");
    hipStream_t s = (hipStream_t)stream;
    ffsat_status st = ensure_workspace(pl, IO_F32);
    if (st != FFSAT_OK) return st;
    if ((st = check_finite<float>(pl, x, s)) != FFSAT_OK) return st;
    if (!F && !grad && !con_val) return FFSAT_OK;
    return run_eval<float>(pl, x, F, grad, con_val, nullptr, nullptr, nullptr, true, nullptr, 0.f, s);
}

extern "C" ffsat_status ffsat_eval_check(ffsat_plan *pl, const float *x, float *F, float *grad, float *con_val,
                                         int32_t *n_sat, uint32_t *unsat_bits, int32_t *U, void *stream)
{
    if (!pl || !x) return fail(FFSAT_E_INVALID_ARG, "NULL plan or x");
    hipStream_t s = (hipStream_t)stream;
    ffsat_status st = ensure_workspace(pl, IO_F32);
    if (st != FFSAT_OK) return st;
    if ((st = check_finite<float>(pl, x, s)) != FFSAT_OK) return st;
    const bool value = F || grad || con_val;
    return run_eval<float>(pl, x, F, grad, con_val, n_sat, unsat_bits, U, value, nullptr, 0.f, s);
}

extern "C" ffsat_status ffsat_eval_step(ffsat_plan *pl, float *x, float eta, float *F, int32_t *n_sat, int32_t *U,
                                        void *stream)
{
    if (!pl || !x) return fail(FFSAT_E_INVALID_ARG, "NULL plan or x");
    hipStream_t s = (hipStream_t)stream;
    ffsat_status st = ensure_workspace(pl, IO_F32);
    if (st != FFSAT_OK) return st;
    if ((st = check_finite<float>(pl, x, s)) != FFSAT_OK) return st;
    return run_eval<float>(pl, x, F, nullptr, nullptr, n_sat, nullptr, U, true, x, eta, s);
}

extern "C" ffsat_status ffsat_eval_f64(ffsat_plan *pl, const double *x, double *F, double *grad, double *con_val,
                                       void *stream)
{
    if (!pl || !x) return fail(FFSAT_E_INVALID_ARG, "NULL plan or x");
    hipStream_t s = (hipStream_t)stream;
    ffsat_status st = ensure_workspace(pl, IO_F64);
    if (st != FFSAT_OK) return st;
    if ((st = check_finite<double>(pl, x, s)) != FFSAT_OK) return st;
    if (!F && !grad && !con_val) return FFSAT_OK;
    return run_eval<double>(pl, x, F, grad, con_val, nullptr, nullptr, nullptr, true, nullptr, 0.f, s);
}

extern "C" ffsat_status ffsat_step(ffsat_plan *pl, float *x, const float *grad, const float *eta_B, float eta,
                                   void *stream)
{
    if (!pl || !x || !grad) return fail(FFSAT_E_INVALID_ARG, "NULL argument");
    HIPCHK(launch_step_f32((int64_t)pl->p->n * pl->B, pl->B, x, grad, eta_B, eta, (hipStream_t)stream));
    return FFSAT_OK;
}

extern "C" ffsat_status ffsat_step_f64(ffsat_plan *pl, double *x, const double *grad, const double *eta_B,
                                       double eta, void *stream)
{
    if (!pl || !x || !grad) return fail(FFSAT_E_INVALID_ARG, "NULL argument");
    HIPCHK(launch_step_f64((int64_t)pl->p->n * pl->B, pl->B, x, grad, eta_B, eta, (hipStream_t)stream));
    return FFSAT_OK;
}

// Before a capture ends, every side stream of the plan that joined it must
// have been joined back into the capturing stream: each node at a side
// stream's tail must either be a dependency of the capturing stream's next
// node or have a dependent node of its own.  An unjoined stream is reported
// here, and the capture abandoned, instead of being left to the runtime.
static hipError_t check_joined(const ffsat_plan *pl, hipStream_t origin, int *unjoined)
{
    *unjoined = -1;
    hipStreamCaptureStatus st = hipStreamCaptureStatusNone;
    unsigned long long id = 0;
    const hipGraphNode_t *deps = nullptr;
    size_t nd = 0;
    hipError_t e = hipStreamGetCaptureInfo_v2(origin, &st, &id, nullptr, &deps, &nd);
    if (e != hipSuccess || st != hipStreamCaptureStatusActive) return e;
    const std::vector<hipGraphNode_t> od(deps, deps + nd);
    const hipStream_t sides[] = {pl->side[0], pl->side[1], pl->side[2], pl->iter_side};
    for (int i = 0; i < 4; ++i) {
        if (!sides[i]) continue;
        hipStreamCaptureStatus s2 = hipStreamCaptureStatusNone;
        unsigned long long id2 = 0;
        const hipGraphNode_t *d2 = nullptr;
        size_t n2 = 0;
        if ((e = hipStreamGetCaptureInfo_v2(sides[i], &s2, &id2, nullptr, &d2, &n2)) != hipSuccess) return e;
        if (s2 != hipStreamCaptureStatusActive || id2 != id) continue;
        for (size_t j = 0; j < n2; ++j) {
            if (std::find(od.begin(), od.end(), d2[j]) != od.end()) continue;
            size_t ndep = 0;
            if ((e = hipGraphNodeGetDependentNodes(d2[j], nullptr, &ndep)) != hipSuccess) return e;
            if (ndep == 0) {
                *unjoined = i;
                return hipSuccess;
            }
        }
    }
    return hipSuccess;
}

// The executable graph of a launch sequence, captured once per key on the
// plan's capture stream (side-stream bins become parallel branches) and kept
// (at most 16 per plan; beyond that all are dropped, each after its latest
// launch has finished).  launch_graph replays it on s and records its
// completion event.
template <typename Body>
static ffsat_status cached_graph(ffsat_plan *pl, const GraphKey &key, Body body, GraphEntry **out)
{
    auto it = pl->graphs.find(key);
    if (it == pl->graphs.end()) {
        if (!pl->cap) HIPCHK(hipStreamCreateWithFlags(&pl->cap, hipStreamNonBlocking));
        HIPCHK(hipStreamBeginCapture(pl->cap, hipStreamCaptureModeThreadLocal));
        hipError_t e = body(pl->cap);
        int unjoined = -1;
        if (e == hipSuccess) e = check_joined(pl, pl->cap, &unjoined);
        hipGraph_t g = nullptr;
        const hipError_t e2 = hipStreamEndCapture(pl->cap, &g);
        if (e != hipSuccess || e2 != hipSuccess || unjoined >= 0) {
            if (g) (void)hipGraphDestroy(g);
            if (unjoined >= 0) return fail(FFSAT_E_HIP, "graph capture: side stream %d was not joined back", unjoined);
            return fail(FFSAT_E_HIP, "graph capture failed: %s", hipGetErrorString(e != hipSuccess ? e : e2));
        }
        GraphEntry ent;
        const hipError_t e3 = hipGraphInstantiate(&ent.exec, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (e3 != hipSuccess) return fail(FFSAT_E_HIP, "graph instantiate failed: %s", hipGetErrorString(e3));
        const hipError_t e4 = hipEventCreateWithFlags(&ent.done, hipEventDisableTiming);
        if (e4 != hipSuccess) {
            (void)hipGraphExecDestroy(ent.exec);
            return fail(FFSAT_E_HIP, "graph event: %s", hipGetErrorString(e4));
        }
        if (pl->graphs.size() >= 16) clear_graphs(pl);
        it = pl->graphs.emplace(key, ent).first;
        ++pl->captures;
    }
    *out = &it->second;
    return FFSAT_OK;
}

static ffsat_status launch_graph(GraphEntry *g, hipStream_t s)
{
    HIPCHK(hipGraphLaunch(g->exec, s));
    HIPCHK(hipEventRecord(g->done, s));
    return FFSAT_OK;
}

// T projected steps.  With the pull path the steps alternate between x and
// the plan's second point buffer (k_pull never writes the point it reads);
// an odd count ends with a copy back into x.
static hipError_t enqueue_steps(ffsat_plan *pl, float *x, int T, float *F_last, hipStream_t s)
{
    const bool pp = pl->pull > 0;
    float *cur = x, *nxt = pl->d_xalt;
    for (int t = 0; t < T; ++t) {
        if (run_eval<float>(pl, cur, t == T - 1 ? F_last : nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, true,
                            cur, 0.f, s, pl->d_hyper, nullptr, pp ? nxt : nullptr) != FFSAT_OK)
            return hipErrorUnknown;
        if (pp) std::swap(cur, nxt);
    }
    if (cur != x) return launch_copy_f32(x, cur, (int64_t)pl->p->n * pl->B, s);
    return hipSuccess;
}

// The persistent loop of a small all-pulled problem (plan option): step size
// and weight-update rate from the plan's device scalars.
static hipError_t enqueue_iters_small(ffsat_plan *pl, float *x, int T, float *F, int32_t *n_sat, int32_t *U, bool erwa,
                                      hipStream_t s)
{
    const PullLayout &P = pl->p->lay[IO_F32].pull[pl->persistent_class];
    PullArgs a{};
    a.x = x;
    a.pptr = P.d_pptr;
    a.pent = P.d_pent;
    a.rk = P.d_rk;
    a.eta_dev = pl->d_hyper;
    a.n = pl->p->n;
    a.B = pl->B;
    return launch_iters_small(PULL_E[pl->persistent_class], a, pl->p->m, P.n_ent, T, F, n_sat, U, pl->p->d_w, erwa,
                              pl->d_hyper + 1, s);
}

extern "C" ffsat_status ffsat_run_steps(ffsat_plan *pl, float *x, int32_t T, float eta, float *F_last, void *stream)
{
    if (!pl || !x) return fail(FFSAT_E_INVALID_ARG, "NULL argument");
    if (T < 0) return fail(FFSAT_E_INVALID_ARG, "T must be >= 0");
    if (T == 0) return FFSAT_OK;
    hipStream_t s = (hipStream_t)stream;
    ffsat_status st = ensure_workspace(pl, IO_F32);
    if (st != FFSAT_OK) return st;
    if ((st = check_finite<float>(pl, x, s)) != FFSAT_OK) return st;
    // the step size goes to device memory ahead of the (captured) steps
    HIPCHK(launch_set_f32x2(pl->d_hyper, eta, 0.f, s));
    if (pl->persistent_class) {
        // one launch: all T steps in one workgroup
        HIPCHK(enqueue_iters_small(pl, x, T, F_last, nullptr, nullptr, false, s));
        return FFSAT_OK;
    }
    if (!pl->use_graphs) {
        HIPCHK(enqueue_steps(pl, x, T, F_last, s));
        return FFSAT_OK;
    }
    GraphKey key{};
    key.kind = 0;
    key.x = x;
    key.T = T;
    key.F = F_last;
    GraphEntry *g = nullptr;
    if ((st = cached_graph(pl, key, [&](hipStream_t cs) { return enqueue_steps(pl, x, T, F_last, cs); }, &g)) !=
        FFSAT_OK)
        return st;
    return launch_graph(g, s);
}

// T fused iterations: objective, exact check and projected step of x_t, then
// the adaptive weights from that iteration's violation counts (alpha > 0).
// With the pull path the iterates alternate between x and the plan's second
// point buffer, and an odd count ends with a copy back into x.
static hipError_t enqueue_iters(ffsat_plan *pl, float *x, int T, bool erwa, float *F, int32_t *n_sat, int32_t *U,
                                hipStream_t s)
{
    const bool pp = pl->pull > 0;
    float *cur = x, *nxt = pl->d_xalt;
    for (int t = 0; t < T; ++t) {
        if (run_eval<float>(pl, cur, F, nullptr, nullptr, n_sat, nullptr, U, true, cur, 0.f, s, pl->d_hyper, nullptr,
                            pp ? nxt : nullptr) != FFSAT_OK)
            return hipErrorUnknown;
        if (erwa) {
            const hipError_t e = launch_erwa(pl->p->m, U, pl->p->d_w, 0.f, pl->d_hyper + 1, pl->d_umax, s);
            if (e != hipSuccess) return e;
        }
        if (pp) std::swap(cur, nxt);
    }
    if (cur != x) return launch_copy_f32(x, cur, (int64_t)pl->p->n * pl->B, s);
    return hipSuccess;
}

// The same T iterations with the work that only needs iteration t's counts
// or level-1 sums moved to a side stream: after the counts of iteration t
// are complete (the evaluation, and with the pull path k_pull, which checks
// the pulled constraints), the adaptive weights and the reset of U for t+1
// run beside the rest of the reduction; after reduction t, the level-2 sums
// (F, n_sat of x_t) run beside evaluation t+1.  Evaluation t+1 waits for the
// weights and the reset; reduction t+1 (which rewrites the level-1 sums)
// waits for the level-2 sums of t; the caller's stream waits for the side
// stream at the end.
static hipError_t enqueue_iters_overlapped(ffsat_plan *pl, float *x, int T, bool erwa, float *F,
                                           int32_t *n_sat, int32_t *U, hipStream_t s)
{
    const ffsat_problem *p = pl->p;
    hipStream_t q = pl->iter_side;
    const int pull = pl->pull;
    const bool want_check = n_sat || U;
    hipError_t e;
#define ITER_CHK(call) \
    if ((e = (call)) != hipSuccess) return e
    float *cur = x, *nxt = pl->d_xalt;
    if (U) ITER_CHK(launch_fill_i32(U, p->m, 0, s));
    for (int t = 0; t < T; ++t) {
        EvalArgs<float> a = base_args<float>(pl, IO_F32, cur, nullptr, true);
        a.do_value = 1;
        a.want_check = want_check ? 1 : 0;
        a.unsat_bits = nullptr;
        a.U = U;
        if (t > 0) ITER_CHK(hipStreamWaitEvent(s, pl->ev_aux, 0));   // weights and reset of t-1
        ITER_CHK(enqueue_bins<float>(pl, IO_F32, a, s, pull ? pull : 3));
        if (pull) ITER_CHK(enqueue_pull(pl, cur, nullptr, nxt, 0.f, pl->d_hyper, nullptr, U, want_check, nullptr, s));
        ITER_CHK(hipEventRecord(pl->ev_eval, s));
        ITER_CHK(hipStreamWaitEvent(q, pl->ev_eval, 0));
        if (erwa) ITER_CHK(launch_erwa(p->m, U, p->d_w, 0.f, pl->d_hyper + 1, pl->d_umax, q));
        if (U && t < T - 1) ITER_CHK(launch_fill_i32(U, p->m, 0, q));
        ITER_CHK(hipEventRecord(pl->ev_aux, q));
        if (t > 0) ITER_CHK(hipStreamWaitEvent(s, pl->ev_sum, 0));   // level-2 sums of t-1 read the level-1 rows
        const ReduceArgs<float> r = reduce_args<float>(pl, IO_F32, nullptr, cur, 0.f, pl->d_hyper, nullptr, F, n_sat, pull);
        ITER_CHK(launch_reduce_part_f32(r, 1, s));
        ITER_CHK(hipEventRecord(pl->ev_red, s));
        ITER_CHK(hipStreamWaitEvent(q, pl->ev_red, 0));
        ITER_CHK(launch_reduce_part_f32(r, 2, q));
        ITER_CHK(hipEventRecord(pl->ev_sum, q));
        if (pull) std::swap(cur, nxt);
    }
    ITER_CHK(hipStreamWaitEvent(s, pl->ev_sum, 0));
    if (cur != x) ITER_CHK(launch_copy_f32(x, cur, (int64_t)p->n * pl->B, s));
#undef ITER_CHK
    return hipSuccess;
}

extern "C" ffsat_status ffsat_run_iters(ffsat_plan *pl, float *x, int32_t T, float eta, float alpha, float *F,
                                        int32_t *n_sat, int32_t *U, void *stream)
{
    if (!pl || !x) return fail(FFSAT_E_INVALID_ARG, "NULL argument");
    if (T < 0) return fail(FFSAT_E_INVALID_ARG, "T must be >= 0");
    if (!(alpha >= 0.f && alpha <= 1.f)) return fail(FFSAT_E_INVALID_ARG, "alpha must be in [0, 1]");
    if (alpha > 0.f && !U) return fail(FFSAT_E_INVALID_ARG, "U is required when alpha > 0");
    if (T == 0) return FFSAT_OK;
    hipStream_t s = (hipStream_t)stream;
    ffsat_status st = ensure_workspace(pl, IO_F32);
    if (st != FFSAT_OK) return st;
    if ((st = check_finite<float>(pl, x, s)) != FFSAT_OK) return st;
    const bool erwa = alpha > 0.f;
    // step size and rate go to device memory ahead of the (captured) iterations
    HIPCHK(launch_set_f32x2(pl->d_hyper, eta, alpha, s));
    if (pl->persistent_class) {
        // one launch: all T iterations in one workgroup
        HIPCHK(enqueue_iters_small(pl, x, T, F, n_sat, U, erwa, s));
        return FFSAT_OK;
    }
    auto body = [&](hipStream_t cs) {
        if (pl->iter_side) return enqueue_iters_overlapped(pl, x, T, erwa, F, n_sat, U, cs);
        return enqueue_iters(pl, x, T, erwa, F, n_sat, U, cs);
    };
    if (!pl->use_graphs) {
        HIPCHK(body(s));
        return FFSAT_OK;
    }
    GraphKey key{};
    key.kind = 1;
    key.x = x;
    key.T = T;
    key.opt = erwa ? 1 : 0;
    key.F = F;
    key.n_sat = n_sat;
    key.U = U;
    GraphEntry *g = nullptr;
    if ((st = cached_graph(pl, key, body, &g)) != FFSAT_OK) return st;
    return launch_graph(g, s);
}

// ------------------------------------------------------------------ check, weights

extern "C" ffsat_status ffsat_round_check(ffsat_plan *pl, const float *x, uint32_t *assign_bits, int32_t *n_sat,
                                          uint32_t *unsat_bits, int32_t *U, void *stream)
{
    if (!pl || !x) return fail(FFSAT_E_INVALID_ARG, "NULL plan or x");
    hipStream_t s = (hipStream_t)stream;
    ffsat_status st = ensure_workspace(pl, IO_F32);
    if (st != FFSAT_OK) return st;
    if ((st = run_eval<float>(pl, x, nullptr, nullptr, nullptr, n_sat, unsat_bits, U, false, nullptr, 0.f, s)) !=
        FFSAT_OK)
        return st;
    if (assign_bits) HIPCHK(launch_assign_bits_f32(pl->p->n, pl->B, x, assign_bits, s));
    return FFSAT_OK;
}

extern "C" ffsat_status ffsat_round_check_f64(ffsat_plan *pl, const double *x, uint32_t *assign_bits,
                                              int32_t *n_sat, uint32_t *unsat_bits, int32_t *U, void *stream)
{
    if (!pl || !x) return fail(FFSAT_E_INVALID_ARG, "NULL plan or x");
    hipStream_t s = (hipStream_t)stream;
    ffsat_status st = ensure_workspace(pl, IO_F64);
    if (st != FFSAT_OK) return st;
    if ((st = run_eval<double>(pl, x, nullptr, nullptr, nullptr, n_sat, unsat_bits, U, false, nullptr, 0.f, s)) !=
        FFSAT_OK)
        return st;
    if (assign_bits) HIPCHK(launch_assign_bits_f64(pl->p->n, pl->B, x, assign_bits, s));
    return FFSAT_OK;
}

extern "C" ffsat_status ffsat_sat_weight(ffsat_plan *pl, const uint32_t *unsat_bits, const float *w, double *score,
                                         void *stream)
{
    if (!pl || !unsat_bits || !score) return fail(FFSAT_E_INVALID_ARG, "NULL argument");
    HIPCHK(launch_sat_weight(pl->p->m, pl->B, unsat_bits, w, score, (hipStream_t)stream));
    return FFSAT_OK;
}

extern "C" ffsat_status ffsat_erwa_update(ffsat_plan *pl, const int32_t *U, float alpha, void *stream)
{
    if (!pl || !U) return fail(FFSAT_E_INVALID_ARG, "NULL argument");
    if (!(alpha >= 0.f && alpha <= 1.f)) return fail(FFSAT_E_INVALID_ARG, "alpha must be in [0, 1]");
    HIPCHK(launch_erwa(pl->p->m, U, pl->p->d_w, alpha, nullptr, pl->d_umax, (hipStream_t)stream));
    return FFSAT_OK;
}

static constexpr int FISTA_MAX_LS = 64;

// FISTA workspace of a plan (first use)
static ffsat_status ensure_fista(ffsat_plan *pl)
{
    if (pl->d_fz) return FFSAT_OK;
    const size_t nb = (size_t)pl->p->n * (size_t)pl->B, B = (size_t)pl->B;
    const int rows = fista_rows(pl->p->n, pl->B);
    const size_t chunks = (size_t)((pl->p->n + rows - 1) / rows);
    HIPCHK(hipMalloc(&pl->d_fz, nb * sizeof(float)));
    HIPCHK(hipMalloc(&pl->d_fg, nb * sizeof(float)));
    HIPCHK(hipMalloc(&pl->d_fFy, B * sizeof(float)));
    HIPCHK(hipMalloc(&pl->d_fFz, B * sizeof(float)));
    HIPCHK(hipMalloc(&pl->d_fpartial, 2 * chunks * B * sizeof(float)));
    HIPCHK(hipMalloc(&pl->d_fcoef, B * sizeof(float)));
    HIPCHK(hipMalloc(&pl->d_fflags, 2 * B * sizeof(int32_t)));
    HIPCHK(hipMalloc(&pl->d_fpending, (FISTA_MAX_LS + 1) * sizeof(int32_t)));
    pl->device_bytes += (int64_t)((2 * nb + 2 * chunks * B + 3 * B) * sizeof(float) + 2 * B * sizeof(int32_t) +
                                  (FISTA_MAX_LS + 1) * sizeof(int32_t));
    return FFSAT_OK;
}

// One FISTA iteration per restart (Alg. 5 with backtracking): gradient at y,
// then max_ls trial slots.  A trial runs only while some restart is still
// searching: its kernels read the count of searching restarts left by the
// previous slot (pending[q]) and return at once when it is 0, so the
// sequence is fixed (graph-capturable, no host read-back) and the trials
// that are not needed cost only their launches.
static hipError_t enqueue_fista_iter(ffsat_plan *pl, float *x, float *y, float *eta, float *t, int max_ls, float *F,
                                     hipStream_t s)
{
    const int n = pl->p->n, B = pl->B;
    int32_t *active = pl->d_fflags, *searching = pl->d_fflags + B;
    int32_t *pending = pl->d_fpending;   // [max_ls + 1]: [0] active restarts, [q + 1] searching after trial q
    hipError_t e;
    if ((e = launch_fill_i32(pending, max_ls + 1, 0, s)) != hipSuccess) return e;
    if ((e = launch_fista_begin(B, eta, active, searching, pending, s)) != hipSuccess) return e;
    if (run_eval<float>(pl, y, pl->d_fFy, pl->d_fg, nullptr, nullptr, nullptr, nullptr, true, nullptr, 0.f, s, nullptr,
                        pending) != FFSAT_OK)
        return hipErrorUnknown;
    for (int q = 0; q < max_ls; ++q) {
        if ((e = launch_fista_trial(n, B, y, pl->d_fg, eta, searching, pl->d_fz, pl->d_fpartial, pending + q, s)) !=
            hipSuccess)
            return e;
        if (run_eval<float>(pl, pl->d_fz, pl->d_fFz, nullptr, nullptr, nullptr, nullptr, nullptr, true, nullptr, 0.f, s,
                            nullptr, pending + q) != FFSAT_OK)
            return hipErrorUnknown;
        if ((e = launch_fista_accept(n, B, pl->d_fpartial, pl->d_fFy, pl->d_fFz, eta, searching, F,
                                     q == max_ls - 1 ? 1 : 0, pending + q + 1, pending + q, s)) != hipSuccess)
            return e;
    }
    return launch_fista_finish(n, B, active, t, pl->d_fcoef, pl->d_fz, x, y, s);
}

extern "C" ffsat_status ffsat_fista(ffsat_plan *pl, float *x, float *y, float *eta, float *t, int32_t T,
                                    int32_t max_ls, float *F, void *stream)
{
    if (!pl || !x || !y || !eta || !t) return fail(FFSAT_E_INVALID_ARG, "NULL argument");
    if (T < 0) return fail(FFSAT_E_INVALID_ARG, "T must be >= 0 (got %d)", T);
    if (max_ls < 1 || max_ls > FISTA_MAX_LS)
        return fail(FFSAT_E_INVALID_ARG, "max_ls must be in [1, %d] (got %d)", FISTA_MAX_LS, max_ls);
    if (T == 0) return FFSAT_OK;
    hipStream_t s = (hipStream_t)stream;
    ffsat_status st = ensure_workspace(pl, IO_F32);
    if (st != FFSAT_OK) return st;
    if ((st = ensure_fista(pl)) != FFSAT_OK) return st;
    auto body = [&](hipStream_t cs) {
        hipError_t e = hipSuccess;
        for (int it = 0; it < T && e == hipSuccess; ++it) e = enqueue_fista_iter(pl, x, y, eta, t, max_ls, F, cs);
        return e;
    };
    if (!pl->use_graphs) {
        HIPCHK(body(s));
        return FFSAT_OK;
    }
    GraphKey key{};
    key.kind = 2;
    key.x = x;
    key.T = T;
    key.opt = max_ls;
    key.F = F;
    key.y = y;
    key.eta = eta;
    key.t = t;
    GraphEntry *g = nullptr;
    if ((st = cached_graph(pl, key, body, &g)) != FFSAT_OK) return st;
    return launch_graph(g, s);
}

extern "C" ffsat_status ffsat_weight_grad(ffsat_plan *pl, const float *con_val, const float *gF, float *gw,
                                          void *stream)
{
    if (!pl || !con_val || !gF || !gw) return fail(FFSAT_E_INVALID_ARG, "NULL argument");
    HIPCHK(launch_wgrad(pl->p->m, pl->B, con_val, gF, gw, (hipStream_t)stream));
    return FFSAT_OK;
}

// ------------------------------------------------------------------ autograd, restarts

extern "C" ffsat_status ffsat_vjp(ffsat_plan *pl, const float *grad, const float *con_val, const float *gF, float *gx,
                                  float *gw, void *stream)
{
    if (!pl || !gF) return fail(FFSAT_E_INVALID_ARG, "NULL argument");
    hipStream_t s = (hipStream_t)stream;
    if (gx) {
        if (!grad) return fail(FFSAT_E_INVALID_ARG, "gx needs grad");
        HIPCHK(launch_scale_restarts((int64_t)pl->p->n * pl->B, pl->B, grad, gF, gx, s));
    }
    if (gw) {
        if (!con_val) return fail(FFSAT_E_INVALID_ARG, "gw needs con_val");
        HIPCHK(launch_wgrad(pl->p->m, pl->B, con_val, gF, gw, s));
    }
    return FFSAT_OK;
}

extern "C" ffsat_status ffsat_rephase(ffsat_plan *pl, float *x, int32_t mode, uint64_t seed, const int32_t *mask,
                                      void *stream)
{
    if (!pl || !x) return fail(FFSAT_E_INVALID_ARG, "NULL argument");
    if (mode < 0 || mode > 2) return fail(FFSAT_E_INVALID_ARG, "mode must be 0 (original), 1 (flipped) or 2 (random)");
    HIPCHK(launch_rephase((int64_t)pl->p->n * pl->B, pl->B, x, mode, seed, mask, (hipStream_t)stream));
    return FFSAT_OK;
}
