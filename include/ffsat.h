/*
 * ffsat.h -- C ABI of the MI355X library that evaluates the Walsh-expansion
 * objective of a hybrid SAT formula (OR, XOR and at-least-t constraints) and
 * its gradient for a batch of restarts, by evaluating elementary symmetric
 * polynomials at roots of unity, plus the projected step, the exact
 * round-and-check, the adaptive weights and the weight gradient.
 *
 * Paper: "Massively Parallel Continuous Local Search for Hybrid SAT Solving
 * on GPUs" (Cen, Zhang, Fong, AAAI-24).
 *
 * Conventions used by every call
 *   - Truth values: -1 is True, +1 is False (Sec. "Walsh Expansions of
 *     Boolean Constraints").  A literal +v has value x_v, a literal -v has
 *     value -x_v.
 *   - Points are stored variable-major and restart-contiguous: x[v * B + b]
 *     for variable v in [0, n) and restart b in [0, B).  The same layout is
 *     used for the gradient; per-constraint values are con_val[c * B + b].
 *   - Device buffers are plain device pointers owned by the caller (for
 *     example torch tensors); the library never frees them.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *     Every call that takes a stream only enqueues work on it and returns
 *     without synchronising; kernel faults surface at the caller's next
 *     synchronisation, as usual for HIP.
 *   - Every call returns an ffsat_status; 0 is success.  On failure no
 *     output argument is written and ffsat_last_error() gives a message
 *     (thread-local).  No C++ exception crosses this interface.
 *   - A problem is immutable after creation except for its weights.  A plan
 *     must be used from one host thread and one stream at a time; calls
 *     that overlap on the device race on the plan's workspace.
 */
#ifndef FFSAT_H
#define FFSAT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t ffsat_status;

#define FFSAT_OK                  0
#define FFSAT_E_INVALID_ARG      -1  /* null pointer, bad size, bad option */
#define FFSAT_E_VAR_RANGE        -2  /* a literal is 0 or |lit| > n_vars */
#define FFSAT_E_DUP_VAR          -3  /* a variable appears twice in one constraint */
#define FFSAT_E_EMPTY_CONSTRAINT -4  /* a constraint with no literal */
#define FFSAT_E_BAD_KIND         -5  /* kind not in {OR, XOR, CARD_GE} */
#define FFSAT_E_DEVICE_MISMATCH  -6  /* device index invalid or not current */
#define FFSAT_E_NOMEM            -7  /* device or host allocation failed */
#define FFSAT_E_HIP              -8  /* a HIP runtime call failed */
#define FFSAT_E_NONFINITE        -9  /* debug checks: NaN/Inf in an input point */
#define FFSAT_E_UNSUPPORTED     -10  /* e.g. a constraint longer than the maximum */

/* constraint kinds */
#define FFSAT_KIND_OR       0   /* clause: at least one literal true            */
#define FFSAT_KIND_XOR      1   /* parity: #true literals odd (param 1) / even (0) */
#define FFSAT_KIND_CARD_GE  2   /* at least `param` literals true               */

/* problem flags */
#define FFSAT_FLAG_FORCE_DFT     1u  /* route OR/XOR through the root-of-unity path too */
#define FFSAT_FLAG_DEBUG_CHECKS  4u  /* check inputs for NaN/Inf (synchronises) */
/* Evaluate the root-of-unity constraints in the paper's own unit-circle form
 * (Alg. 2 with Eq. forward, reduction and inverse as printed: factors
 * omega^a + l_i, unscaled running products, conjugated Walsh coefficients
 * f~ = f^ W^-1) instead of the bounded basis.  An ablation: it reproduces on
 * the device the precision loss the paper reports for long constraints
 * (Sec. Experiments, the need for high bit precision); the FP64 evaluation
 * (ffsat_eval_f64, or fp64_min_len = 1) is its intended use.  Same entry
 * points, outputs and layouts; the grouped launch is not used for these
 * bins.  Results for long constraints near the corners of the box are
 * expected to be inaccurate, in FP32 also non-finite. */
#define FFSAT_FLAG_UNIT_CIRCLE   8u

/* Longest constraint accepted. */
#define FFSAT_MAX_CONSTRAINT_LEN 512

typedef struct ffsat_problem ffsat_problem;
typedef struct ffsat_plan ffsat_plan;

/* Host-side description of a constraint set.  All arrays are host memory
 * and are copied by ffsat_problem_create; the caller may free them on
 * return. */
typedef struct {
    int32_t n_vars;          /* number of variables n >= 1 */
    int32_t n_cons;          /* number of constraints m >= 1 */
    const int64_t *con_ptr;  /* [m+1], con_ptr[0] = 0, non-decreasing: literals of
                                constraint c are lits[con_ptr[c] .. con_ptr[c+1]) */
    const int32_t *lits;     /* [nnz] signed 1-based literals (DIMACS style) */
    const int32_t *kinds;    /* [m] FFSAT_KIND_* */
    const int32_t *params;   /* [m] XOR parity bit / CARD threshold t / ignored for OR.
                                t <= 0 makes the constraint always true, t > k never. */
    const float *weights;    /* [m] initial weights w_c, or NULL for all ones */
    int32_t device;          /* HIP device index; must be the current device */
    int32_t fp64_min_len;    /* root-of-unity products of constraints with at least
                                this many literals run in FP64 in ffsat_eval
                                (0 = default 128: from there the FP64
                                polynomial form is faster than FP32 running
                                products, and more precise) */
    uint32_t flags;          /* FFSAT_FLAG_* */
} ffsat_problem_desc;

typedef struct {
    int32_t n_vars, n_cons;
    int64_t nnz;
    int32_t max_len;
    int32_t n_bins_f32;      /* kernel bins of the FP32 evaluation */
    int32_t n_bins_f64;      /* kernel bins of the FP64 evaluation */
    int32_t device;
    int64_t device_bytes;    /* device memory held by the problem */
} ffsat_problem_info;

typedef struct {
    int32_t autotune;        /* 1: time tile shapes per bin at plan creation */
    int32_t use_graphs;      /* 1: ffsat_run_steps replays a captured hipGraph */
    const char *tune_cache;  /* JSON file for tuned shapes (NULL = in memory only) */
    int32_t reserved[8];     /* reserved[0] = 1: launch all bins on the caller's stream
                                (no internal side streams); reserved[1]: launch
                                structure of the FP32 evaluation, 0 automatic (the
                                autotuner times the others and keeps the fastest;
                                without it 2, or 3 when reserved[2] is 2 or 3;
                                the bins inside a grouped launch then take 8
                                transform-free constraints per wave and one wave
                                per root-of-unity unit),
                                1 one launch per bin, 2 one grouped launch for all
                                bins, 3 a grouped launch for the root-of-unity bins
                                with the others beside it; reserved[2]: gradient of
                                the transform-free constraints of length <= 7
                                (OR, AND, XOR, constants), 0 automatic (the
                                autotuner decides; off without it), 1 through
                                per-literal slots and the slot reduction, 2 gathered
                                per variable for lengths <= 7, 3 for lengths <= 3
                                (the pulled gradient; never with launch structure 2,
                                never for n * B above 2^29); reserved[3]:
                                variables per wave of the pulled gradient, 0..8
                                (0 = 8); reserved[4] = 1: ffsat_run_steps and
                                ffsat_run_iters run all T iterations in one
                                persistent launch of one workgroup (points,
                                per-occurrence gradient terms, constraint values,
                                weights, counts and the per-variable constraint
                                lists in LDS) when every constraint is
                                transform-free of length <= 7 and 8 n B + 4 e B +
                                4 m B + 8 m + 4 B + 4 (n + 1) + 4 e + 4 E e <=
                                65024 bytes (e literal occurrences, E = 4 if
                                every constraint has at most 3 literals, else 8),
                                else as usual; others must be 0 */
} ffsat_plan_opts;

/* ---- errors ------------------------------------------------------------- */

/* Static string for a status code. */
const char *ffsat_status_string(ffsat_status s);
/* Message of the last failing call on this host thread ("" if none). */
const char *ffsat_last_error(void);
/* Library version string. */
const char *ffsat_version(void);

/* ---- problem: "load constraint set" (Def. 3's constraint set C) ---------- */

/* Validates and copies a constraint set to the device: CSR of literals,
 * variable-major transpose, length/kind bins, and the conjugated
 * coefficients of every distinct (kind, length, param) computed in FP64
 * (Eq. inverse, step iii preprocessing).  Validation errors (VAR_RANGE,
 * DUP_VAR, EMPTY_CONSTRAINT, BAD_KIND, UNSUPPORTED, INVALID_ARG) are
 * reported before any device call.  *out is written only on success. */
ffsat_status ffsat_problem_create(const ffsat_problem_desc *d, ffsat_problem **out);
/* Frees the problem (NULL is allowed).  The caller must have synchronised
 * work that uses it. */
ffsat_status ffsat_problem_destroy(ffsat_problem *p);
ffsat_status ffsat_problem_info_get(const ffsat_problem *p, ffsat_problem_info *info);

/* Weights w_c of Def. 3, original constraint order, [m] floats.  on_device
 * selects whether `w` is a device or a host pointer.  Enqueued on stream. */
ffsat_status ffsat_set_weights(ffsat_problem *p, const float *w, int32_t on_device, void *stream);
ffsat_status ffsat_get_weights(const ffsat_problem *p, float *w, int32_t on_device, void *stream);

/* ---- plan: a batch size B and its workspace ------------------------------ */

/* Binds the batch size B >= 1 and allocates the workspace (per-literal slot
 * buffer of nnz*B values, objective partials).  opts may be NULL (no
 * autotuning, graphs on).  *out is written only on success. */
ffsat_status ffsat_plan_create(ffsat_problem *p, int32_t B, const ffsat_plan_opts *opts,
                               ffsat_plan **out);
ffsat_status ffsat_plan_destroy(ffsat_plan *plan);
/* Runs the tile-shape autotuner now (synchronises the stream): per bin,
 * constraints per wave, waves per block and frequency split, each bin timed
 * in launches of its own; then, timed over four fused iterations, the
 * launch structure (when automatic), the pull class (when automatic) and the
 * shapes of the bins inside a grouped launch (transform-free constraints per
 * wave 4, 8 or 16 in the all-bin group; root-of-unity frequency split 1 or
 * 4), which replace the per-bin shapes of those bins.  Results go to the
 * plan's tune cache (in memory, and the JSON file when one is named). */
ffsat_status ffsat_plan_tune(ffsat_plan *plan, void *stream);
/* Writes a JSON description of the bins and their tile shapes into buf
 * (truncated to len-1 characters, always NUL-terminated). */
ffsat_status ffsat_plan_describe(const ffsat_plan *plan, char *buf, size_t len);

/* Kernel timing: while on, every evaluation-kernel launch and every
 * reduction launch made by ffsat_eval / ffsat_eval_f64 / ffsat_run_steps
 * (eager, not graph replays) is bracketed by HIP events on the caller's
 * stream, and the bins run one after another on that stream (no side
 * streams), so that each launch's time is its own.  ffsat_plan_profile_read synchronises on those events and writes
 * JSON {"kernels": [{"io", "bin", "launches", "total_ms", "avg_ms"}]} into
 * buf (truncated to len-1, NUL-terminated); reset != 0 clears the sums. */
ffsat_status ffsat_plan_profile(ffsat_plan *plan, int32_t on);
ffsat_status ffsat_plan_profile_read(ffsat_plan *plan, int32_t reset, char *buf, size_t len);

/* ---- objective and gradient at a batch of points (Def. 3, Alg. 2) ------- */

/* For every restart b with x_b = x[. * B + b] in [-1,1]^n (device, [n][B]):
 *   F[b]           = sum_c w_c WE_c(x_b)          (optional, device [B])
 *   grad[v*B+b]    = dF/dx_v at x_b               (optional, device [n][B])
 *   con_val[c*B+b] = WE_c(x_b), unweighted        (optional, device [m][B])
 * WE_c is evaluated by the three steps of Alg. 2 (affine factors at the
 * roots of unity, product over literals, dot with the conjugated
 * coefficients) and differentiated by leave-one-out prefix/suffix products
 * (Eq. chain); OR and XOR use the transform-free products (App. B).
 * Computation is FP32 except the root-of-unity products of constraints at
 * least fp64_min_len long, which run in FP64; there each lane's segment
 * product at a root is evaluated from the segment's elementary symmetric
 * polynomials and the leave-one-out products through per-degree moments
 * (the same quantities in another rounding order).  Results are deterministic
 * (no floating-point atomics).  Points outside [-1,1] are evaluated as
 * given (the polynomial is defined everywhere). */
ffsat_status ffsat_eval(ffsat_plan *plan, const float *x, float *F, float *grad,
                        float *con_val, void *stream);
/* ffsat_eval plus the exact check of the same point (see ffsat_round_check
 * for the outputs n_sat, unsat_bits, U), in the same kernels: each literal
 * is gathered once for both.  With F, grad and con_val all NULL only the
 * check runs. */
ffsat_status ffsat_eval_check(ffsat_plan *plan, const float *x, float *F, float *grad,
                              float *con_val, int32_t *n_sat, uint32_t *unsat_bits, int32_t *U,
                              void *stream);
/* One projected-gradient iteration with the check of its starting point,
 * in one pass: at x_t (device [n][B], updated in place) computes F[b]
 * (optional), the exact check outputs n_sat / U (optional, as in
 * ffsat_round_check, for x_t), and x_{t+1} = clip(x_t - eta grad, -1, 1)
 * with the gradient rounded to FP32 exactly as ffsat_eval returns it; the
 * gradient itself is not stored. */
ffsat_status ffsat_eval_step(ffsat_plan *plan, float *x, float eta, float *F, int32_t *n_sat,
                             int32_t *U, void *stream);
/* Same as ffsat_eval with double buffers and FP64 computation throughout. */
ffsat_status ffsat_eval_f64(ffsat_plan *plan, const double *x, double *F, double *grad,
                            double *con_val, void *stream);
/* ffsat_eval's F and grad for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): no plan, no allocation and no allocating library call.  The
 * per-literal slots, objective rows and their partial sums live in a fixed
 * 64 MiB device array of the library (one per device, held until the
 * process ends), so 4 * (nnz * B + rows * B + ceil(rows / 64) * B) bytes,
 * each term rounded up to 256, must fit (rows <= the number of
 * constraints); larger calls return FFSAT_E_UNSUPPORTED before any launch.
 * x, F ([B], optional) and grad ([n][B], optional) are device buffers of the
 * problem's device, which must be current.  Bins run one after another on
 * `stream` in the problem's default tile shapes; results equal ffsat_eval's
 * up to the grouping of the FP32 sums.  Every call on a device uses the
 * same array: calls that overlap on one device race. */
ffsat_status ffsat_eval_noalloc(const ffsat_problem *problem, int32_t B, const float *x, float *F,
                                float *grad, void *stream);

/* ---- projected step (App. A.3, Alg. 5, clip to [-1,1]) ------------------- */

/* In place, elementwise: x <- min(max(fma(-eta_b, grad, x), -1), 1) with
 * eta_b = eta_B[b] if eta_B != NULL else eta.  x, grad: device [n][B];
 * eta_B: device [B] or NULL. */
ffsat_status ffsat_step(ffsat_plan *plan, float *x, const float *grad, const float *eta_B,
                        float eta, void *stream);
ffsat_status ffsat_step_f64(ffsat_plan *plan, double *x, const double *grad,
                            const double *eta_B, double eta, void *stream);

/* T fused iterations of (evaluate gradient, projected step with scalar eta)
 * on x (device [n][B], in place), replayed from a captured hipGraph when the
 * plan uses graphs.  F_last (device [B] or NULL) receives the objective at
 * the point the last step started from.  eta is written to plan-owned
 * device memory (in stream order) before the steps, so one captured graph
 * per (x, T, F_last) serves every step size. */
ffsat_status ffsat_run_steps(ffsat_plan *plan, float *x, int32_t T, float eta, float *F_last,
                             void *stream);

/* ---- round and check (Alg. 1, the certificate test of Thm. 2) ------------ */

/* Rounds every variable (x_v < 0 means True; +0, -0 and NaN mean False) and
 * checks every constraint exactly in integers.  All outputs are optional
 * device buffers:
 *   assign_bits[b * ceil(n/32) + v/32] bit v%32 = variable v is True
 *   n_sat[b]    = number of satisfied constraints of restart b
 *   unsat_bits[b * ceil(m/32) + c/32] bit c%32 = constraint c is violated
 *   U[c]        = number of restarts violating c (the ERWA count U_c). */
ffsat_status ffsat_round_check(ffsat_plan *plan, const float *x, uint32_t *assign_bits,
                               int32_t *n_sat, uint32_t *unsat_bits, int32_t *U, void *stream);
ffsat_status ffsat_round_check_f64(ffsat_plan *plan, const double *x, uint32_t *assign_bits,
                                   int32_t *n_sat, uint32_t *unsat_bits, int32_t *U, void *stream);

/* ---- adaptive weights (Prop. 3) and the weight gradient ------------------ */

/* In place on the problem's weights: r_c = U_c / max_c U_c (r = 0 when the
 * maximum is 0) and w_c <- (1 - alpha) w_c + alpha r_c.  U: device [m]. */
ffsat_status ffsat_erwa_update(ffsat_plan *plan, const int32_t *U, float alpha, void *stream);

/* gw[c] = sum_b gF[b] * con_val[c * B + b]: the gradient of sum_b gF_b F_b
 * with respect to w_c (F is linear in w, Def. 3).  Device buffers. */
ffsat_status ffsat_weight_grad(ffsat_plan *plan, const float *con_val, const float *gF,
                               float *gw, void *stream);

/* Optimisation mode (the paper's MaxSAT-style experiments, where not every
 * constraint can hold): score[b] = sum of w_c over the constraints that
 * restart b's rounded point satisfies, from the unsat bits of
 * ffsat_round_check ([B][ceil(m/32)]).  w: device [m] (e.g. the original
 * weights; the problem's weights may have been adapted), or NULL for all
 * ones.  score: device [B] FP64, accumulated in a fixed order. */
ffsat_status ffsat_sat_weight(ffsat_plan *plan, const uint32_t *unsat_bits, const float *w, double *score,
                              void *stream);

/* ---- differentiation of the objective (Def. 3) --------------------------- */

/* Vector-Jacobian product of F (per restart) for an upstream gradient gF[B]:
 *   gx[v*B+b] = gF[b] * grad[v*B+b]     (grad from ffsat_eval; optional)
 *   gw[c]     = sum_b gF[b] * con_val[c*B+b]   (con_val from ffsat_eval; optional)
 * Device buffers; gx may alias grad. */
ffsat_status ffsat_vjp(ffsat_plan *plan, const float *grad, const float *con_val, const float *gF,
                       float *gx, float *gw, void *stream);

/* T fused iterations on device data (Alg. 1's inner loop with the paper's
 * certificate check every step): each evaluates F, checks the rounded point
 * exactly and takes the projected step of x_t (as ffsat_eval_step), then,
 * when alpha > 0, updates the weights from that iteration's violation counts
 * (as ffsat_erwa_update).  F [B], n_sat [B], U [m] receive the last
 * iteration's values (each optional; U required when alpha > 0).  With
 * graphs enabled the sequence is captured once per (x, T, alpha > 0, F,
 * n_sat, U) and replayed; eta and alpha are read from plan-owned device
 * memory written before each replay.  Errors as ffsat_eval_step. */
ffsat_status ffsat_run_iters(ffsat_plan *plan, float *x, int32_t T, float eta, float alpha, float *F,
                             int32_t *n_sat, int32_t *U, void *stream);

/* ---- accelerated projected gradient (Alg. 5 and the line search it names) */

/* T iterations of FISTA with backtracking for every restart b, on device
 * state x[v*B+b], y[v*B+b] (the extrapolated point), eta[b] (step size),
 * t[b] (momentum; start with y = x, t = 1, eta = the initial step):
 *   restarts with eta < 1e-12 have stopped (Alg. 5) and are left unchanged;
 *   g = gradient of F at y;
 *   up to max_ls trials: z = clip(y - eta g, -1, 1); accept when
 *     F(z) <= F(y) + <g, z - y> + |z - y|^2 / (2 eta), else eta /= 2
 *     (after the last trial z is taken with the halved eta);
 *   t' = (1 + sqrt(1 + 4 t^2)) / 2, y' = z + ((t - 1)/t') (z - x), x' = z.
 * F (optional, [B]) receives F(x') of every restart that moved.  max_ls in
 * [1, 64].  Nothing is read back to the host: every iteration enqueues a
 * fixed sequence (the gradient at y and max_ls trial slots); the kernels of
 * a slot return at once when no restart is still searching, so unneeded
 * trials cost only their launches.  With graphs enabled the T iterations
 * are captured once per argument set (buffers, T, max_ls) and replayed.
 * The workspace (two [n][B] arrays and per-restart scalars) is allocated
 * on first use. */
ffsat_status ffsat_fista(ffsat_plan *plan, float *x, float *y, float *eta, float *t, int32_t T,
                         int32_t max_ls, float *F, void *stream);

/* ---- restarts (App. "Restart Heuristics", rephasing) --------------------- */

/* For every restart b with mask[b] != 0 (mask: device [B] int32, or NULL for
 * all): mode 0 keeps x (original phase), 1 sets x <- -x (flipped phase),
 * 2 draws x uniformly in [-1, 1) (random phase) from SplitMix64 applied to
 * seed + (i+1) * 0x9e3779b97f4a7c15 for element i = v*B + b. */
ffsat_status ffsat_rephase(ffsat_plan *plan, float *x, int32_t mode, uint64_t seed,
                           const int32_t *mask, void *stream);

/* ---- learned initialiser (proposal of restart points) -------------------- */

/* A message-passing network over the clause-variable incidence graph that
 * proposes restart points (the paper notes that the initial point matters,
 * Sec. "Restart Heuristics"; the network itself is an addition).  Features:
 * 8 per variable [1, P/8, N/8, (P-N)/(P+N+1), 0...] with P/N its positive /
 * negative occurrences, 8 per constraint [1, is_or, is_xor, is_card, k/64,
 * thr, parity, 0] with thr = t/k (t clipped to [0, k+1]) for at-least-t,
 * 1/k for OR, 0 for XOR.  Layers (W stored [K][H], row-major FP32):
 *   hv = relu(fv Ev + ev), hc = relu(fc Ec + ec)
 *   per round: hc = relu([hc, mean+ hv, mean- hv] Wc + bc)   (mean over the
 *              constraint's positive / negative literals, divided by k)
 *              hv = relu([hv, mean+ hc, mean- hc] Wv + bv)   (divided by the
 *              variable's occurrence count)
 *   mu_v = tanh(hv . wo + bo)
 * Parameters, flat FP32 in the order Ev[8][H], ev[H], Ec[8][H], ec[H], then
 * per round Wc[3H][H], bc[H], Wv[3H][H], bv[H], then wo[H], bo[1].  Matrix
 * products round both operands to bfloat16 (nearest even) and accumulate
 * in FP32 on the matrix cores; everything else is FP32.  Loss: mean over
 * variables of (mu_v - target_v)^2. */
typedef struct ffsat_mpnn ffsat_mpnn;
typedef struct {
    int32_t hidden;     /* H: multiple of 32 in [32, 256] */
    int32_t rounds;     /* R in [1, 8] */
    int32_t device;     /* must be the current device */
    int32_t reserved;   /* 0 */
    uint64_t seed;      /* Glorot-uniform weights and head from SplitMix64; zero biases */
} ffsat_mpnn_desc;

ffsat_status ffsat_mpnn_create(const ffsat_mpnn_desc *d, ffsat_mpnn **out);
ffsat_status ffsat_mpnn_destroy(ffsat_mpnn *net);
ffsat_status ffsat_mpnn_num_params(const ffsat_mpnn *net, int64_t *n);
/* Copies the parameters (which = 0) or the last gradients (which = 1,
 * read only) between the network and buf (num_params floats, host memory
 * unless on_device).  to_net = 1 loads parameters and resets Adam's moments
 * and step count.  Host copies complete before return. */
ffsat_status ffsat_mpnn_params(ffsat_mpnn *net, float *buf, int32_t which, int32_t to_net,
                               int32_t on_device, void *stream);
/* mu[n_vars] (device, optional) = the network's output on the problem's
 * graph (built on first use and kept with the problem). */
ffsat_status ffsat_mpnn_forward(ffsat_mpnn *net, ffsat_problem *p, float *mu, void *stream);
/* Forward, loss against target[n_vars] (device) into *loss (device float,
 * optional) and the gradient of the loss with respect to every parameter
 * (read with ffsat_mpnn_params which = 1).  Split sums run in a fixed order:
 * results are deterministic. */
ffsat_status ffsat_mpnn_backward(ffsat_mpnn *net, ffsat_problem *p, const float *target, float *loss,
                                 void *stream);
/* One Adam step (bias-corrected) with the last gradients. */
ffsat_status ffsat_mpnn_adam(ffsat_mpnn *net, float lr, float beta1, float beta2, float eps, void *stream);
/* Restart points x[v*B+b] (device): the first round(frac_learned * B)
 * restarts get clip(mu_v + sigma*u, -1, 1), the rest u, with u uniform in
 * [-1, 1) from SplitMix64 of seed + (i+1) * 0x9e3779b97f4a7c15, i = v*B+b. */
ffsat_status ffsat_mpnn_propose(ffsat_plan *plan, const float *mu, float *x, float frac_learned,
                                float sigma, uint64_t seed, void *stream);

/* ---- host-only helper ---------------------------------------------------- */

/* Conjugated coefficients of one symmetric constraint in the bounded
 * root-of-unity basis: h[a] = (1/(k+1)) sum_c f(c) exp(-2 pi i a c/(k+1)),
 * a = 0..floor((k+1)/2), with f(c) = -1 if the constraint holds with c true
 * literals and +1 otherwise (Eq. inverse, with the Poisson-binomial basis of
 * this library).  Writes 2*(floor((k+1)/2)+1) doubles (re, im interleaved).
 * Pure host code: no device call. */
ffsat_status ffsat_coefficients(int32_t kind, int32_t k, int32_t param, double *h_out);

/* Walsh coefficients of one symmetric constraint: f_out[j] = the coefficient
 * of the elementary symmetric polynomial e_j (j = 0..k) in the constraint's
 * Walsh expansion (Def. 2, Eq. effi_eval; f = -1 on satisfying inputs,
 * literal value -1 = True).  Computed exactly in integers (Krawtchouk values)
 * and rounded once.  Writes k+1 doubles.  Pure host code: no device call. */
ffsat_status ffsat_walsh_coefficients(int32_t kind, int32_t k, int32_t param, double *f_out);

/* Conjugated Walsh coefficients of the unit-circle form (Eq. inverse):
 * ft[a] = (1/(k+1)) sum_j fhat_{k-j} omega^(-j a), a = 0..k, omega =
 * exp(-2 pi i/(k+1)), the ESP sequence ordered e_k .. e_0, so that
 * WE = sum_a ft[a] prod_i (omega^a + l_i).  Writes 2*(k+1) doubles (re, im
 * interleaved).  Used by FFSAT_FLAG_UNIT_CIRCLE.  Pure host code. */
ffsat_status ffsat_unit_circle_coefficients(int32_t kind, int32_t k, int32_t param, double *ft_out);

#ifdef __cplusplus
}
#endif
#endif /* FFSAT_H */
