/*
 * Plain FP64 CPU oracle for the Walsh-expansion objective of a hybrid
 * formula and its gradient.
 *
 * TEST INFRASTRUCTURE ONLY. Nothing in the library's product path may
 * include, link or call this file; only the test suite, the smoke check and
 * the benchmark's CPU-baseline leg use it. It shares no code, header, table
 * or helper with the HIP library.
 *
 * What it computes (paper: Thm. 1 for the Walsh expansion, Def. 3 for the
 * objective, Thm. 2 for the certificate, Prop. 3 for the adaptive weights,
 * App. A.3 / Alg. 5 for the projected step):
 *
 *   For a symmetric constraint c over literal values l_1..l_k in [-1, 1]
 *   (literal +v has value x_v, literal -v has value -x_v; -1 means True),
 *   with truth table f(c) in {-1 (True), +1 (False)} as a function of the
 *   number of true literals, WE_c(l) is the unique multilinear polynomial
 *   that equals f on {-1,1}^k.  Written in the Lagrange basis of the cube,
 *
 *       WE_c(l) = sum_{a in {-1,1}^k} f(a) prod_i (1 + a_i l_i) / 2,
 *
 *   i.e. the expectation of f when literal i is independently True with
 *   probability p_i = (1 - l_i)/2 (the randomised rounding of the GradSAT
 *   appendix).  Three independent routes compute it:
 *
 *   R2 (authority at every length): the count-lattice recursion.  Fwd_i(c)
 *      is the probability that c of the first i literals are true; Bwd_i(c)
 *      is the expected f given c trues among the first i literals.  This is
 *      the symmetric special case of the top-down / bottom-up messages of the
 *      GradSAT appendix (Alg. 4): WE = Bwd_0(0) and
 *      dWE/dl_i = 1/2 sum_c Fwd_{i-1}(c) (Bwd_i(c) - Bwd_i(c+1)).
 *   R1 (the paper's own definition, Eq. effi_eval with Def. 2): WE =
 *      sum_j fhat_j e_j(l), with e_j the elementary symmetric polynomials
 *      (O(k^2) recurrence) and fhat_j the Walsh coefficient of any subset of
 *      size j, computed exactly from the truth table by counting
 *      (Thm. 1): fhat_j = 2^-k sum_c f(c) sum_q (-1)^q C(j,q) C(k-j,c-q).
 *      Its gradient is the explicit FourierSAT form (Alg. 3): the ESPs of
 *      the other k-1 literals dotted with fhat shifted by one.  Exact
 *      coefficients need k <= 62 here; the route is ill-conditioned for long
 *      cardinality constraints (cancellation between large ESP terms), so
 *      tests use it for OR/XOR at any k and cardinality only for short k.
 *   R3 closed forms: OR: WE = -1 + 2 prod (1+l_i)/2 (the footnote of the
 *      transform-free appendix); XOR with parity p: WE = (2p-1) prod l_i
 *      (Cor. 3); at-least-t with t <= 0 is constant -1, with t > k constant
 *      +1, with t = 1 it is OR, with t = k it is AND: 1 - 2 prod (1-l_i)/2.
 *
 * Everything is double precision, loops are plain, and parallelism is only
 * over restarts (OpenMP), so the result of each (constraint, restart) pair
 * does not depend on the thread count.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

enum { ORC_OR = 0, ORC_XOR = 1, ORC_CARD = 2 };
enum { ORC_ROUTE_AUTH = 0, ORC_ROUTE_DP = 1, ORC_ROUTE_ESP = 2, ORC_ROUTE_CLOSED = 3 };

/* f(c): -1 if the constraint is satisfied with c true literals, +1 if not. */
double orc_truth(int kind, int param, int k, int c)
{
    (void)k;
    switch (kind) {
    case ORC_OR:   return c >= 1 ? -1.0 : 1.0;
    case ORC_XOR:  return (c % 2) == (param & 1) ? -1.0 : 1.0;
    case ORC_CARD: return c >= param ? -1.0 : 1.0;
    default:       return 0.0;
    }
}

/* ---------------------------------------------------------------------- */
/* R2: count-lattice recursion                                             */
/* ---------------------------------------------------------------------- */

/* fv[0..k] truth table; dl (may be NULL) receives dWE/dl_i. */
double orc_we_dp(int k, const double *l, const double *fv, double *dl)
{
    /* Fwd[i][c], c = 0..i, stored row by row: row i starts at i(i+1)/2. */
    size_t tri = (size_t)(k + 1) * (size_t)(k + 2) / 2;
    double *fwd = (double *)malloc(tri * sizeof(double));
    double *bwd = (double *)malloc((size_t)(k + 1) * (size_t)(k + 2) * sizeof(double));
#define FWD(i, c) fwd[(size_t)(i) * ((i) + 1) / 2 + (c)]
#define BWD(i, c) bwd[(size_t)(i) * (size_t)(k + 2) + (c)]
    FWD(0, 0) = 1.0;
    for (int i = 1; i <= k; ++i) {
        double p = 0.5 * (1.0 - l[i - 1]);   /* P[literal i true]  */
        double q = 0.5 * (1.0 + l[i - 1]);   /* P[literal i false] */
        for (int c = 0; c <= i; ++c) {
            double stay = (c <= i - 1) ? FWD(i - 1, c) * q : 0.0;
            double move = (c >= 1) ? FWD(i - 1, c - 1) * p : 0.0;
            FWD(i, c) = stay + move;
        }
    }
    for (int c = 0; c <= k; ++c) BWD(k, c) = fv[c];
    for (int i = k - 1; i >= 0; --i) {
        double p = 0.5 * (1.0 - l[i]);
        double q = 0.5 * (1.0 + l[i]);
        for (int c = 0; c <= i; ++c) BWD(i, c) = q * BWD(i + 1, c) + p * BWD(i + 1, c + 1);
    }
    double we = BWD(0, 0);
    if (dl) {
        for (int i = 1; i <= k; ++i) {
            double s = 0.0;
            for (int c = 0; c <= i - 1; ++c) s += FWD(i - 1, c) * (BWD(i, c) - BWD(i, c + 1));
            dl[i - 1] = 0.5 * s;
        }
    }
#undef FWD
#undef BWD
    free(fwd);
    free(bwd);
    return we;
}

/* Probability that at least t of the k literals are true (forward messages
 * only); used for the GradSAT worked example. */
double orc_prob_at_least(int k, const double *l, int t)
{
    double *cur = (double *)calloc((size_t)k + 2, sizeof(double));
    cur[0] = 1.0;
    for (int i = 1; i <= k; ++i) {
        double p = 0.5 * (1.0 - l[i - 1]), q = 0.5 * (1.0 + l[i - 1]);
        for (int c = i; c >= 0; --c) cur[c] = cur[c] * q + (c ? cur[c - 1] * p : 0.0);
    }
    double s = 0.0;
    for (int c = (t < 0 ? 0 : t); c <= k; ++c) s += cur[c];
    free(cur);
    return s;
}

/* ---------------------------------------------------------------------- */
/* R1: Walsh coefficients and elementary symmetric polynomials             */
/* ---------------------------------------------------------------------- */

static __int128 binom128(int n, int r)
{
    if (r < 0 || r > n) return 0;
    if (r > n - r) r = n - r;
    __int128 b = 1;
    for (int i = 1; i <= r; ++i) b = b * (n - r + i) / i;
    return b;
}

/* fhat[j], j = 0..k: Walsh coefficient of every subset of size j.
 * Returns 0 on success, -1 if k is too long for exact integer counting. */
int orc_walsh_coeffs(int k, const double *fv, double *fhat)
{
    if (k > 62) return -1;
    for (int j = 0; j <= k; ++j) {
        __int128 acc = 0;
        for (int c = 0; c <= k; ++c) {
            __int128 cnt = 0;   /* sum over cube points with c trues of prod_{i in S} x_i */
            for (int q = 0; q <= j && q <= c; ++q) {
                __int128 t = binom128(j, q) * binom128(k - j, c - q);
                cnt += (q & 1) ? -t : t;
            }
            int fc = (int)fv[c];
            acc += fc * cnt;
        }
        fhat[j] = ldexpl((long double)acc, -k);
    }
    return 0;
}

/* e[0..k] of the k values l. */
void orc_esp(int k, const double *l, double *e)
{
    e[0] = 1.0;
    for (int j = 1; j <= k; ++j) e[j] = 0.0;
    for (int i = 0; i < k; ++i)
        for (int j = i + 1; j >= 1; --j) e[j] += l[i] * e[j - 1];
}

double orc_we_esp(int k, const double *l, const double *fhat, double *dl)
{
    double *e = (double *)malloc(sizeof(double) * (size_t)(k + 1));
    orc_esp(k, l, e);
    double we = 0.0;
    for (int j = 0; j <= k; ++j) we += fhat[j] * e[j];
    if (dl) {
        double *rest = (double *)malloc(sizeof(double) * (size_t)k);
        for (int i = 0; i < k; ++i) {
            int r = 0;
            for (int t = 0; t < k; ++t) if (t != i) rest[r++] = l[t];
            orc_esp(k - 1, rest, e);
            double s = 0.0;
            for (int j = 1; j <= k; ++j) s += fhat[j] * e[j - 1];
            dl[i] = s;
        }
        free(rest);
    }
    free(e);
    return we;
}

/* ---------------------------------------------------------------------- */
/* R3: closed forms                                                         */
/* ---------------------------------------------------------------------- */

/* returns 0 if a closed form exists for this (kind, k, param), else -1 */
int orc_we_closed(int kind, int param, int k, const double *l, double *we_out, double *dl)
{
    double sgn_prod = 0.0;   /* coefficient of the product form */
    int mode;                /* 0 prod of (1+l)/2 ; 1 prod of l ; 2 prod of (1-l)/2 ; 3 constant */
    double cst = 0.0, scale = 0.0;
    if (kind == ORC_OR || (kind == ORC_CARD && param == 1 && k >= 1)) {
        mode = 0; cst = -1.0; scale = 2.0;                 /* -1 + 2 prod q */
    } else if (kind == ORC_XOR) {
        mode = 1; cst = 0.0; scale = (param & 1) ? 1.0 : -1.0;
    } else if (kind == ORC_CARD && param <= 0) {
        mode = 3; cst = -1.0;
    } else if (kind == ORC_CARD && param > k) {
        mode = 3; cst = 1.0;
    } else if (kind == ORC_CARD && param == k) {
        mode = 2; cst = 1.0; scale = -2.0;                 /* 1 - 2 prod p */
    } else {
        return -1;
    }
    (void)sgn_prod;
    if (mode == 3) {
        *we_out = cst;
        if (dl) for (int i = 0; i < k; ++i) dl[i] = 0.0;
        return 0;
    }
    double prod = 1.0;
    for (int i = 0; i < k; ++i) {
        double f = mode == 0 ? 0.5 * (1.0 + l[i]) : mode == 1 ? l[i] : 0.5 * (1.0 - l[i]);
        prod *= f;
    }
    *we_out = cst + scale * prod;
    if (dl) {
        double dfac = mode == 0 ? 0.5 : mode == 1 ? 1.0 : -0.5;   /* d factor / d l */
        for (int i = 0; i < k; ++i) {
            double rest = 1.0;
            for (int t = 0; t < k; ++t) {
                if (t == i) continue;
                rest *= mode == 0 ? 0.5 * (1.0 + l[t]) : mode == 1 ? l[t] : 0.5 * (1.0 - l[t]);
            }
            dl[i] = scale * dfac * rest;
        }
    }
    return 0;
}

/* ---------------------------------------------------------------------- */
/* one constraint, one restart                                              */
/* ---------------------------------------------------------------------- */

/* Value of constraint c at literal values l, with dWE/dl in dl (may be NULL).
 * route: AUTH = closed form for OR/XOR and the degenerate cardinality cases,
 *        count DP otherwise; DP = count DP always; ESP = R1 always (returns
 *        NAN if k is too long); CLOSED = closed form (NAN if none). */
double orc_constraint(int kind, int param, int k, const double *l, double *dl, int route)
{
    double we = NAN;
    if (route == ORC_ROUTE_CLOSED || route == ORC_ROUTE_AUTH) {
        if (orc_we_closed(kind, param, k, l, &we, dl) == 0) return we;
        if (route == ORC_ROUTE_CLOSED) return NAN;
    }
    double *fv = (double *)malloc(sizeof(double) * (size_t)(k + 1));
    for (int c = 0; c <= k; ++c) fv[c] = orc_truth(kind, param, k, c);
    if (route == ORC_ROUTE_ESP) {
        double *fh = (double *)malloc(sizeof(double) * (size_t)(k + 1));
        if (orc_walsh_coeffs(k, fv, fh) == 0) we = orc_we_esp(k, l, fh, dl);
        free(fh);
    } else {
        we = orc_we_dp(k, l, fv, dl);
    }
    free(fv);
    return we;
}

/* ---------------------------------------------------------------------- */
/* whole formula over a batch of restarts                                   */
/* ---------------------------------------------------------------------- */

static int max_len(int m, const int64_t *con_ptr)
{
    int mx = 0;
    for (int c = 0; c < m; ++c) {
        int k = (int)(con_ptr[c + 1] - con_ptr[c]);
        if (k > mx) mx = k;
    }
    return mx;
}

static int set_threads(int nthreads)
{
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
    return omp_get_max_threads();
#else
    (void)nthreads;
    return 1;
#endif
}

/* x[n][B]. Outputs (each optional):
 *   F[B]           = sum_c w_c WE_c(x_b)                (Def. 3)
 *   g[n][B]        = dF/dx
 *   con_val[m][B]  = WE_c(x_b)
 *   lit_grad[nnz][B] = dWE_c/dl_i for literal slot i (unweighted, unsigned)
 * w may be NULL (all ones). Returns the number of threads used. */
int orc_eval(int n, int m, const int64_t *con_ptr, const int32_t *lits, const int32_t *kinds,
             const int32_t *params, const double *w, int B, const double *x,
             double *F, double *g, double *con_val, double *lit_grad, int route, int nthreads)
{
    int used = set_threads(nthreads);
    int kmax = max_len(m, con_ptr);
    if (g) memset(g, 0, sizeof(double) * (size_t)n * (size_t)B);
#pragma omp parallel
    {
        double *l = (double *)malloc(sizeof(double) * (size_t)(kmax + 1));
        double *dl = (double *)malloc(sizeof(double) * (size_t)(kmax + 1));
#pragma omp for schedule(dynamic, 1)
        for (int b = 0; b < B; ++b) {
            double Fb = 0.0;
            for (int c = 0; c < m; ++c) {
                int64_t a0 = con_ptr[c];
                int k = (int)(con_ptr[c + 1] - a0);
                for (int i = 0; i < k; ++i) {
                    int32_t lit = lits[a0 + i];
                    int v = (lit > 0 ? lit : -lit) - 1;
                    double xv = x[(size_t)v * B + b];
                    l[i] = lit > 0 ? xv : -xv;
                }
                int need_grad = (g != NULL) || (lit_grad != NULL);
                double we = orc_constraint(kinds[c], params[c], k, l, need_grad ? dl : NULL, route);
                double wc = w ? w[c] : 1.0;
                Fb += wc * we;
                if (con_val) con_val[(size_t)c * B + b] = we;
                for (int i = 0; i < k && need_grad; ++i) {
                    int32_t lit = lits[a0 + i];
                    int v = (lit > 0 ? lit : -lit) - 1;
                    if (lit_grad) lit_grad[(size_t)(a0 + i) * B + b] = dl[i];
                    /* each restart b is owned by one thread: no race on g[.][b] */
                    if (g) g[(size_t)v * B + b] += wc * (lit > 0 ? dl[i] : -dl[i]);
                }
            }
            if (F) F[b] = Fb;
        }
        free(l);
        free(dl);
    }
    return used;
}

/* Central finite differences of F at sampled (variable, restart) pairs,
 * using only the constraints incident to the variable.  var_ptr/var_cons is
 * the variable -> constraint incidence (CSR over variables, 0-based). */
void orc_fd_grad(int n, const int64_t *con_ptr, const int32_t *lits, const int32_t *kinds,
                 const int32_t *params, const double *w, const int64_t *var_ptr,
                 const int32_t *var_cons, int B, const double *x, int n_samples,
                 const int32_t *sample_var, const int32_t *sample_b, double h, double *out)
{
    (void)n;
    int kmax = 1;
    for (int s = 0; s < n_samples; ++s) {
        int v = sample_var[s];
        for (int64_t e = var_ptr[v]; e < var_ptr[v + 1]; ++e) {
            int c = var_cons[e];
            int k = (int)(con_ptr[c + 1] - con_ptr[c]);
            if (k > kmax) kmax = k;
        }
    }
    double *l = (double *)malloc(sizeof(double) * (size_t)kmax);
    for (int s = 0; s < n_samples; ++s) {
        int v = sample_var[s], b = sample_b[s];
        double acc[2] = {0.0, 0.0};
        for (int side = 0; side < 2; ++side) {
            double shift = side == 0 ? h : -h;
            for (int64_t e = var_ptr[v]; e < var_ptr[v + 1]; ++e) {
                int c = var_cons[e];
                int64_t a0 = con_ptr[c];
                int k = (int)(con_ptr[c + 1] - a0);
                for (int i = 0; i < k; ++i) {
                    int32_t lit = lits[a0 + i];
                    int u = (lit > 0 ? lit : -lit) - 1;
                    double xv = x[(size_t)u * B + b] + (u == v ? shift : 0.0);
                    l[i] = lit > 0 ? xv : -xv;
                }
                double we = orc_constraint(kinds[c], params[c], k, l, NULL, ORC_ROUTE_DP);
                acc[side] += (w ? w[c] : 1.0) * we;
            }
        }
        out[s] = (acc[0] - acc[1]) / (2.0 * h);
    }
    free(l);
}

/* ---------------------------------------------------------------------- */
/* rounding and the exact checker (Alg. 1 line "F(sgn x) = -sum w")          */
/* ---------------------------------------------------------------------- */

/* Variable v is True iff x_v < 0 (so +0, -0 and NaN are False).
 * Outputs (each optional): assign_bits[B][ceil(n/32)] (bit set = True),
 * n_sat[B], unsat_bits[B][ceil(m/32)], U[m] (restarts violating c). */
void orc_check(int n, int m, const int64_t *con_ptr, const int32_t *lits, const int32_t *kinds,
               const int32_t *params, int B, const double *x, uint32_t *assign_bits,
               int32_t *n_sat, uint32_t *unsat_bits, int32_t *U)
{
    int wn = (n + 31) / 32, wm = (m + 31) / 32;
    if (assign_bits) memset(assign_bits, 0, sizeof(uint32_t) * (size_t)wn * (size_t)B);
    if (unsat_bits) memset(unsat_bits, 0, sizeof(uint32_t) * (size_t)wm * (size_t)B);
    if (U) memset(U, 0, sizeof(int32_t) * (size_t)m);
    for (int b = 0; b < B; ++b) {
        if (assign_bits)
            for (int v = 0; v < n; ++v)
                if (x[(size_t)v * B + b] < 0.0) assign_bits[(size_t)b * wn + v / 32] |= 1u << (v % 32);
        int sat_count = 0;
        for (int c = 0; c < m; ++c) {
            int ntrue = 0;
            int k = (int)(con_ptr[c + 1] - con_ptr[c]);
            for (int i = 0; i < k; ++i) {
                int32_t lit = lits[con_ptr[c] + i];
                int v = (lit > 0 ? lit : -lit) - 1;
                int var_true = x[(size_t)v * B + b] < 0.0;
                int lit_true = lit > 0 ? var_true : !var_true;
                ntrue += lit_true;
            }
            int sat;
            if (kinds[c] == ORC_OR) sat = ntrue >= 1;
            else if (kinds[c] == ORC_XOR) sat = (ntrue % 2) == (params[c] & 1);
            else sat = ntrue >= params[c];
            sat_count += sat;
            if (!sat) {
                if (unsat_bits) unsat_bits[(size_t)b * wm + c / 32] |= 1u << (c % 32);
                if (U) U[c] += 1;
            }
        }
        if (n_sat) n_sat[b] = sat_count;
    }
}

/* ---------------------------------------------------------------------- */
/* projected step, adaptive weights, weight gradient                        */
/* ---------------------------------------------------------------------- */

/* x <- clip(x - eta g, -1, 1) in FP32, with one fused multiply-add, the
 * same contraction the projected-gradient step is defined with. eta_b may
 * be NULL (scalar eta). */
void orc_step_f32(int n, int B, float *x, const float *g, const float *eta_b, float eta)
{
    for (int v = 0; v < n; ++v)
        for (int b = 0; b < B; ++b) {
            size_t i = (size_t)v * B + b;
            float e = eta_b ? eta_b[b] : eta;
            float y = fmaf(-e, g[i], x[i]);
            x[i] = fminf(fmaxf(y, -1.0f), 1.0f);
        }
}

void orc_step_f64(int n, int B, double *x, const double *g, const double *eta_b, double eta)
{
    for (int v = 0; v < n; ++v)
        for (int b = 0; b < B; ++b) {
            size_t i = (size_t)v * B + b;
            double e = eta_b ? eta_b[b] : eta;
            double y = fma(-e, g[i], x[i]);
            x[i] = fmin(fmax(y, -1.0), 1.0);
        }
}

/* Prop. 3: w <- (1 - alpha) w + alpha r, r_c = U_c / max U (r = 0 when
 * max U = 0). */
void orc_erwa(int m, const int32_t *U, double *w, double alpha)
{
    int32_t mx = 0;
    for (int c = 0; c < m; ++c) if (U[c] > mx) mx = U[c];
    for (int c = 0; c < m; ++c) {
        double r = mx > 0 ? (double)U[c] / (double)mx : 0.0;
        w[c] = (1.0 - alpha) * w[c] + alpha * r;
    }
}

/* gw[c] = sum_b gF[b] * con_val[c][b]: the gradient of sum_b gF_b F_b with
 * respect to w_c, since F is linear in w (Def. 3). */
void orc_wgrad(int m, int B, const double *con_val, const double *gF, double *gw)
{
    for (int c = 0; c < m; ++c) {
        double s = 0.0;
        for (int b = 0; b < B; ++b) s += gF[b] * con_val[(size_t)c * B + b];
        gw[c] = s;
    }
}
