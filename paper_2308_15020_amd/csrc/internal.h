// Internal types of the ffsat HIP library (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <map>
#include <string>
#include <tuple>
#include <vector>

#include "ffsat.h"

namespace ffsat {

// Kernel classes: REAL = transform-free product chains (OR, XOR, AND,
// constants; the Nyquist term of the root-of-unity path is the same chain);
// DFT = root-of-unity frequencies (complex chains) + optional real chain.
enum { CLASS_REAL = 0, CLASS_DFT = 1 };
enum { CT_F32 = 0, CT_F64 = 1 };
enum { IO_F32 = 0, IO_F64 = 1 };

// Per distinct constraint type.  WE = cst + sum over complex frequencies of
// Re(c0 * prod psi) + c0r * prod (alpha + beta l); gradients likewise with
// c1 / c1r and leave-one-out products.
template <typename T>
struct TypeT {
    T cst, alpha, beta, c0r, c1r, pad;
    int32_t n1, n2, has_real, tab;
};
// One complex frequency.  Form 1 (first n1 entries of a type): factor
// psi = 1 - i*tk*l.  Form 2 (next n2 entries): psi = tk - i*l.  Each lane
// starts its segment product at `init` (an exact power of two that centres
// the magnitude range); c0/c1 fold in the scaling.
template <typename T>
struct FreqT {
    T tk, init, c0re, c0im, c1re, c1im, p0, p1;
};
// The same entry for the FP64 polynomial form (root-of-unity types with FP64
// arithmetic, unit-circle form excepted): with tau = tk, sg = -tau^2,
// isg = 1 / sg, itau = init tau, c1i = c1 init, c1t = c1 init tau.  The value
// coefficient c0 = i c1 / tau is not needed: Re(c0 T) follows from the
// moments' coefficients and the segment polynomial.
struct FreqPoly {
    double sg, isg, init, itau, c1ire, c1iim, c1tre, c1tim;
};
static_assert(sizeof(FreqPoly) == sizeof(FreqT<double>), "one table for both layouts");
using TypeF32 = TypeT<float>;
using TypeF64 = TypeT<double>;
using FreqF32 = FreqT<float>;
using FreqF64 = FreqT<double>;

struct ConDesc {
    int32_t off;   // first literal slot (binned literal order)
    int32_t k;     // length
    int32_t type;  // index into the type tables
    int32_t orig;  // original constraint index
    int32_t chk;   // exact check: >= 0: satisfied iff #true >= chk;
                   // -1: iff #true even; -2: iff #true odd
    int32_t pad0, pad1, pad2;
};

struct Bin {
    int cls = CLASS_REAL;
    int ct = CT_F32;
    int seg = 8, L = 1;
    int first = 0, count = 0;   // constraint range in binned order
    int maxk = 0;
    double cost = 0;            // estimated VALU work per restart
    int64_t lits = 0;           // literal slots in the bin
    double flops = 0;           // algorithmic FLOPs per restart (value + gradient)
    double bytes = 0;           // algorithmic HBM bytes per restart (gathers + slot writes)
    double exec_pos = 0;        // literal positions executed per restart (with padding)
    double k2 = 0;              // sum of k^2 over the bin's root-of-unity constraints
    double alg = 0;             // roofline FLOPs per restart: 10 k^2 per root-of-unity constraint,
                                // the polynomial form's own count in FP64 (poly_flops)
    int cpw = 1, wpb = 4;       // tile shape: constraints per wave, waves per block
    int fg = 1;                 // root-of-unity bins: waves splitting one unit's frequencies
    bool uc = false;            // root-of-unity bin in the unit-circle form (ablation)
    int pk = 0;                 // pull class: 2 = transform-free, length <= 3; 1 = transform-free,
                                // length 4..7; 0 = other (bins are ordered by pk, then cost)
};

// Pull classes: the gradient of the transform-free constraints of a class
// >= the plan's pull threshold is gathered per variable (k_pull) instead of
// written to slots and reduced.  PULL_K[c] is the longest constraint of
// class c, PULL_E[c] the entry width in int32: {constraint, meta, the other
// PULL_K - 1 literals}.
enum { PULL_OFF = 0, PULL_LE7 = 1, PULL_LE3 = 2 };
constexpr int PULL_K[3] = {0, 7, 3};
constexpr int PULL_E[3] = {0, 8, 4};
constexpr int PULL_VC_MAX = 8;   // variables per wave of k_pull (its LDS holds their sums and points)

// Pulled occurrences of the constraints of pull class >= c, per variable.
struct PullLayout {
    bool built = false;
    int64_t n_ent = 0;           // pulled (literal occurrence) entries
    int64_t n_gather = 0;        // other literals over all entries (gathers per restart)
    int64_t n_rest = 0;          // slots of the other constraints
    int32_t *d_pptr = nullptr;   // [n+1] variable -> first entry
    int32_t *d_pent = nullptr;   // [n_ent][PULL_E[c]]
    int32_t *d_vptr = nullptr;   // [n+1] variable-major transpose of the remaining slots
    int32_t *d_vslot = nullptr;  // ascending slot order per variable
    float *d_rk = nullptr;       // [RK_TABLE] coefficients of the transform-free kinds
};

struct ProfRec {
    int io, bin;                // bin = -1: gradient / objective reduction
    hipEvent_t e0, e1;
};

struct Layout {
    int io = IO_F32;
    std::vector<Bin> bins;
    std::vector<double> cost_prefix;   // [m+1] prefix sums of per-constraint cost (binned order)
    std::vector<double> k2_prefix;     // [m+1] prefix sums of k^2 of root-of-unity constraints (binned order)
    std::vector<double> alg_prefix;    // [m+1] prefix sums of the constraints' roofline FLOPs (Bin::alg)
    ConDesc *d_con = nullptr;
    int32_t *d_lit = nullptr;    // var | (negated << 31), binned order
    int32_t *d_vptr = nullptr;   // [n+1] variable -> slot CSR
    int32_t *d_vslot = nullptr;  // [nnz]
    int32_t *d_pos = nullptr;    // [m] original index -> binned position
    TypeF32 *d_t32 = nullptr;
    TypeF64 *d_t64 = nullptr;
    FreqF32 *d_f32 = nullptr;
    FreqF64 *d_f64 = nullptr;
    int n_types = 0;
    int64_t n_freqs = 0;
    // host copies of the binned descriptors and literals (FP32 layout: the
    // pulled-occurrence lists are built from them on first use)
    std::vector<ConDesc> h_con;
    std::vector<int32_t> h_lit;
    std::vector<int8_t> h_rk;    // [m] binned order: transform-free kind (RKIND_*) or -1
    PullLayout pull[3];          // by pull threshold class (index 1, 2)
};

// Transform-free kinds of the pull path: OR, AND, odd / even XOR, and the
// constants -1 / +1 (thresholds outside [1, k]).
enum { RKIND_OR = 0, RKIND_AND = 1, RKIND_XOR_ODD = 2, RKIND_XOR_EVEN = 3, RKIND_TRUE = 4, RKIND_FALSE = 5,
       RKIND_N = 6 };

}  // namespace ffsat

struct ffsat_problem {
    int32_t n = 0, m = 0;
    int64_t nnz = 0;
    int32_t maxk = 0;
    int32_t device = 0;
    int32_t fp64_min_len = 128;
    uint32_t flags = 0;
    float *d_w = nullptr;        // weights, original order
    int32_t *d_kind = nullptr;   // original order
    int32_t *d_param = nullptr;
    ffsat::Layout lay[2];
    int64_t device_bytes = 0;
    // host copy of the constraint set (original order)
    std::vector<int64_t> h_con_ptr;
    std::vector<int32_t> h_lits, h_kinds, h_params;
    void *mpnn_graph = nullptr;   // incidence graph of the learned initialiser, built on first use
};

namespace ffsat {

template <typename IO>
struct EvalArgs {
    const IO *x;
    IO *slot;
    IO *fpart;
    IO *con_val;
    int32_t *cpart;        // violated-constraint count rows (with fpart's row layout)
    uint32_t *unsat_bits;  // [B][wm] or null (pre-zeroed)
    int32_t *U;            // [m] or null (pre-zeroed)
    const ConDesc *con;
    const int32_t *lit;
    const float *w;
    const void *types;
    const void *freqs;
    int B, first, count, cpw, n_rb, fpart_row0;
    int want_grad, do_value, want_check, wm;
    int fg;                // root-of-unity bins: waves sharing one unit's frequencies (1, 2 or 4)
    const int32_t *skip;   // if set and *skip == 0, every wave returns at once (nothing to evaluate)
};

// A wave's constraint range and tiling (one bin, or one entry of a grouped launch).
struct Span {
    int first, count, cpw, n_rb, fpart_row0;
};

// One bin of a grouped evaluation launch: its kernel variant and tiling.
struct GroupEntry {
    int32_t variant, first, count, cpw, n_rb, fpart_row0, fg, pad;
};

// Launch structure of the FP32 evaluation.
enum { MODE_AUTO = 0, MODE_PER_BIN = 1, MODE_GROUP_ALL = 2, MODE_GROUP_DFT = 3 };

// A captured launch sequence is keyed by its buffers and shape only: step
// size and weight-update rate are read from device memory (written before
// each replay), so one graph serves every value.
struct GraphKey {
    int32_t kind;          // 0: ffsat_run_steps, 1: ffsat_run_iters, 2: ffsat_fista
    const void *x;
    int32_t T;
    int32_t opt;           // run_iters: weights updated (alpha > 0); fista: trials per iteration
    const void *F, *n_sat, *U;
    const void *y, *eta, *t;
    bool operator<(const GraphKey &o) const {
        return std::tie(kind, x, T, opt, F, n_sat, U, y, eta, t) <
               std::tie(o.kind, o.x, o.T, o.opt, o.F, o.n_sat, o.U, o.y, o.eta, o.t);
    }
};
// An executable graph and the event recorded after its latest launch (waited
// on before the executable is destroyed).
struct GraphEntry {
    hipGraphExec_t exec = nullptr;
    hipEvent_t done = nullptr;
};

}  // namespace ffsat

// Records msg as the thread's last error and returns st (for sources other
// than the one holding the problem / plan entry points).
ffsat_status ffsat_fail_external(ffsat_status st, const char *msg);
// Frees the learned initialiser's incidence graph kept with a problem.
void ffsat_free_mpnn_graph(void *g);

struct ffsat_plan {
    ffsat_problem *p = nullptr;
    int32_t B = 0;
    std::vector<ffsat::Bin> bins[2];   // tuned copies of the problem's bins
    void *d_slot[2] = {nullptr, nullptr};
    void *d_fpart[2] = {nullptr, nullptr};
    void *d_ftmp[2] = {nullptr, nullptr};
    int32_t *d_cpart = nullptr;      // violated-count rows (shared by both precisions)
    int32_t *d_ctmp = nullptr;
    int fpart_rows[2] = {0, 0};
    int32_t *d_flag = nullptr;       // debug non-finite flag
    int32_t *d_umax = nullptr;       // [1024] partial maxima of the weight update
    float *d_scratch_x = nullptr;    // autotuner input
    // FISTA workspace (allocated on first use): trial point, gradient at y,
    // objective at y and at the trial, partial sums, flags, momentum, counter
    float *d_fz = nullptr, *d_fg = nullptr, *d_fFy = nullptr, *d_fFz = nullptr, *d_fpartial = nullptr;
    float *d_fcoef = nullptr;
    int32_t *d_fflags = nullptr, *d_fpending = nullptr;
    hipStream_t cap = nullptr;       // capture stream for graphs
    // grouped FP32 evaluation: one launch over a block table (entries =
    // bins); bins without a grouped variant are launched one by one
    bool grouped = true;             // mode GROUP_ALL or GROUP_DFT
    int mode = 0;                    // MODE_* (evaluation launch structure)
    bool mode_auto = false;          // chosen by the tuner
    ffsat::GroupEntry *d_gent = nullptr;
    int2 *d_gblk = nullptr;
    int gblocks = 0;
    size_t glds = 0;
    ffsat::GroupEntry *d_gent64 = nullptr;   // the FP64 root-of-unity group (grouped structures)
    int2 *d_gblk64 = nullptr;
    int gblocks64 = 0;
    size_t glds64 = 0;
    std::vector<int> gsolo;          // bin indices launched on their own
    // three side streams: with the caller's stream, one per hardware queue
    // of HIP's default of four per process
    static constexpr int N_SIDE = 3;
    hipStream_t side[N_SIDE] = {};   // bins run concurrently on these (fork/join)
    hipEvent_t ev_fork = nullptr;
    hipEvent_t ev_join[N_SIDE] = {};
    // fused iterations: adaptive weights, counter reset and level-2 sums of
    // iteration t run here beside the gradient reduction and the next evaluation
    hipStream_t iter_side = nullptr;
    hipEvent_t ev_eval = nullptr, ev_red = nullptr, ev_aux = nullptr, ev_sum = nullptr;
    bool use_graphs = true;
    bool tuned = false;
    std::string tune_cache;
    std::map<ffsat::GraphKey, ffsat::GraphEntry> graphs;
    float *d_hyper = nullptr;        // [2] step size and weight-update rate read by captured graphs
    // pulled gradient of the short transform-free constraints (PULL_*;
    // chosen by the tuner unless fixed by the options)
    int pull = 0;
    bool pull_auto = false;
    int pull_vc = 8;                 // variables per wave of k_pull
    bool persistent = false;         // ffsat_run_steps as one persistent launch (small all-pulled problems)
    int persistent_class = 0;        // the pull class whose entry lists it reads (0: not eligible)
    float *d_xalt = nullptr;         // [n][B] second point buffer of in-place pulled steps
    std::string tune_log;            // [launch structure, pull length, grouped chain cpw, grouped fg,
                                     //  ms per fused iteration] per tuned candidate
    // shapes of the bins inside a grouped launch, timed there (0: the bins'
    // own per-bin shapes): constraints per wave of the transform-free bins
    // (all-bin group only) and the frequency split of the root-of-unity bins
    int group_real_cpw = 0;
    int group_dft_fg = 0;
    std::vector<int> solo_cpw, solo_fg;   // the per-bin shapes, restored when the group values are cleared
    int32_t *d_tune_u = nullptr;     // [m] violation counts of the tuner's timed iterations
    int64_t captures = 0;            // graphs captured over the plan's life
    int64_t device_bytes = 0;
    bool profiling = false;
    std::vector<ffsat::ProfRec> prof_pending;
    std::vector<hipEvent_t> prof_pool;
    std::map<std::pair<int, int>, std::pair<double, int64_t>> prof_acc;   // (io, bin) -> (ms, launches)
};

namespace ffsat {

// kernels (eval.hip / aux.hip)
hipError_t launch_eval_bin_f32(const Bin &bin, const EvalArgs<float> &a, hipStream_t s);
hipError_t launch_eval_bin_f64(const Bin &bin, const EvalArgs<double> &a, hipStream_t s);
int group_variant(int ct, int cls, int seg, int L);
hipError_t launch_eval_group_f32(const EvalArgs<float> &a, const GroupEntry *ent, const int2 *blk, int nblk,
                                 size_t lds, hipStream_t s);
// the long FP64-arithmetic root-of-unity bins of the FP32 evaluation
int group_variant64(int seg, int L);
hipError_t launch_eval_group64_f32(const EvalArgs<float> &a, const GroupEntry *ent, const int2 *blk, int nblk,
                                   size_t lds, hipStream_t s);
bool eval_variant_exists(int io, int ct, int cls, int seg, int L, bool uc);

// Reduction after the evaluation kernels: gradient (or fused projected step
// when x_step != null) over the variable-major transpose, objective rows into
// F, violated-count rows into n_sat = m - sum.
template <typename IO>
struct ReduceArgs {
    int n, B, m;
    const int32_t *vptr, *vslot;
    const IO *slot;
    IO *grad;
    float *x_step;
    float eta;
    const float *eta_dev;   // if set, the step size is read here instead of eta
    const IO *fpart;
    const int32_t *cpart;
    int rows;
    IO *ftmp;
    int32_t *ctmp;
    IO *F;
    int32_t *n_sat;
    const int32_t *skip;   // if set and *skip == 0, the reduction does nothing
};
hipError_t launch_reduce_f32(const ReduceArgs<float> &r, hipStream_t s);

// Pulled gradient (k_pull): for every variable of a chunk of vc variables
// and 64 restarts, the remaining constraints' slots (ascending slot order)
// plus the pulled occurrences' terms (entry order), summed in FP64; then
// either the gradient or the projected step into x_out (never x).  The
// objective term and the exact check of every pulled constraint are taken
// at the entry of its first literal; one objective / count row per chunk.
struct PullArgs {
    const float *x;
    float *x_out;             // projected step (x_out != x), or null
    float *grad;              // gradient, or null (exactly one of x_out, grad)
    const float *slot;
    const int32_t *vptr, *vslot;
    const int32_t *pptr, *pent;
    const float *w;
    float *fpart;
    int32_t *cpart;
    uint32_t *unsat_bits;
    int32_t *U;
    const float *eta_dev;
    const int32_t *skip;
    float eta;
    // per transform-free kind r: factor alpha + beta l, value coefficient c0,
    // gradient coefficient c1 and constant at rk[r], rk[8 + r], rk[16 + r],
    // rk[24 + r], rk[32 + r]
    const float *rk;
    int64_t x_bytes;               // size of x (buffer-load bound, < 2^31)
    int n, B, vc, row0, wm, want_check;
};
constexpr int RK_TABLE = 40;
hipError_t launch_pull(int E, const PullArgs &a, hipStream_t s);
// Persistent loop of T fused iterations of a small problem whose constraints
// are all pulled: one workgroup; x, the per-(entry, restart) gradient terms,
// the constraint values, the weights, U and the entry lists in LDS
// (iters_small_lds bytes <= ITERS_SMALL_LDS).  Optional outputs of the last
// iteration's point: F, n_sat, U; with erwa, the weight update after every
// iteration.
constexpr int ITERS_SMALL_LDS = 65536 - 512;   // leaves room for the kernel's own small arrays
size_t iters_small_lds(int E, int n, int B, int m, int64_t n_ent);
hipError_t launch_iters_small(int E, const PullArgs &a, int m, int64_t n_ent, int T, float *F, int32_t *n_sat,
                              int32_t *U, float *w, bool erwa, const float *alpha_dev, hipStream_t s);

// Maximum over a block of up to 1024 threads (values >= 0); every thread
// gets it.  Uses red[16] and one barrier.
__device__ __forceinline__ int32_t block_max_1024(int32_t v, int32_t *red)
{
#pragma unroll
    for (int d = 32; d > 0; d >>= 1) v = max(v, __shfl_xor(v, d, 64));
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (lane == 0) red[wave] = v;
    __syncthreads();
    // every lane of every wave ends with the block maximum (counts are >= 0)
    v = lane < (int)(blockDim.x >> 6) ? red[lane] : 0;
#pragma unroll
    for (int d = 32; d > 0; d >>= 1) v = max(v, __shfl_xor(v, d, 64));
    return v;
}

// The adaptive weight of a constraint violated by u of the batch's restarts
// (Prop. 3 with r = u / max U, r = 0 when nothing is violated); one
// expression for every kernel that updates weights.
__device__ __forceinline__ float erwa_weight(float w, int32_t u, int32_t umax, float inv, float alpha)
{
    const float r = umax > 0 ? (float)u * inv : 0.0f;
    return (1.0f - alpha) * w + alpha * r;
}
hipError_t launch_copy_f32(float *dst, const float *src, int64_t n, hipStream_t s);
hipError_t launch_reduce_f64(const ReduceArgs<double> &r, hipStream_t s);
// parts: 1 = gradient / step and level 1 of the sums, 2 = level 2, 3 = both
hipError_t launch_reduce_part_f32(const ReduceArgs<float> &r, int parts, hipStream_t s);
hipError_t launch_step_f32(int64_t total, int B, float *x, const float *g, const float *eta_b,
                           float eta, hipStream_t s);
hipError_t launch_step_f64(int64_t total, int B, double *x, const double *g,
                           const double *eta_b, double eta, hipStream_t s);
hipError_t launch_assign_bits_f32(int n, int B, const float *x, uint32_t *bits, hipStream_t s);
hipError_t launch_assign_bits_f64(int n, int B, const double *x, uint32_t *bits, hipStream_t s);
hipError_t launch_erwa(int m, const int32_t *U, float *w, float alpha, const float *alpha_dev, int32_t *part,
                       hipStream_t s);
hipError_t launch_set_f32x2(float *p, float a, float b, hipStream_t s);
hipError_t launch_wgrad(int m, int B, const float *con_val, const float *gF, float *gw,
                        hipStream_t s);
hipError_t launch_scale_restarts(int64_t total, int B, const float *grad, const float *gF, float *gx,
                                 hipStream_t s);
hipError_t launch_rephase(int64_t total, int B, float *x, int mode, uint64_t seed, const int32_t *mask,
                          hipStream_t s);
hipError_t launch_nonfinite_f32(int64_t total, const float *x, int32_t *flag, hipStream_t s);
hipError_t launch_nonfinite_f64(int64_t total, const double *x, int32_t *flag, hipStream_t s);
hipError_t launch_fill_i32(int32_t *p, int64_t n, int32_t v, hipStream_t s);
hipError_t launch_scratch_points(float *x, int64_t total, uint32_t seed, hipStream_t s);
hipError_t launch_sat_weight(int m, int B, const uint32_t *bits, const float *w, double *score, hipStream_t s);
int fista_rows(int n, int B);
hipError_t launch_fista_begin(int B, const float *eta, int32_t *active, int32_t *searching, int32_t *n_active,
                              hipStream_t s);
hipError_t launch_fista_trial(int n, int B, const float *y, const float *g, const float *eta, const int32_t *searching,
                              float *z, float *part, const int32_t *skip, hipStream_t s);
hipError_t launch_fista_accept(int n, int B, const float *part, const float *Fy, const float *Fz, float *eta,
                               int32_t *searching, float *Fout, int last, int32_t *pending, const int32_t *skip,
                               hipStream_t s);
hipError_t launch_fista_finish(int n, int B, const int32_t *active, float *t, float *coef, const float *z, float *x,
                               float *y, hipStream_t s);

// number of F-partial rows of a bin list
int fpart_rows_of(const std::vector<Bin> &bins);
int f_splits(int rows);

}  // namespace ffsat
