// ffsat_eval_noalloc: the objective and gradient of ffsat_eval without a plan
// and without any device allocation.  The evaluation kernels' per-literal
// slots, objective rows and their partial sums live in one file-scope device
// array of NOALLOC_SCRATCH_BYTES; each device that calls the entry point
// holds its own copy of that array until the process ends.  Bins are
// launched one after another on the caller's stream with the problem's
// default tile shapes; the gradient reduction follows in the fixed slot
// order, as in ffsat_eval.  Calls that overlap on one device share the
// array and race.
#include <mutex>

#include "internal.h"

namespace ffsat {

static constexpr size_t NOALLOC_SCRATCH_BYTES = (size_t)64 << 20;
static constexpr int NOALLOC_MAX_DEVICES = 64;

static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];

// per device: the device address of `scratch` (its host-side name is only a
// stand-in for the symbol and is never passed to a kernel)
static std::mutex g_scratch_mu;
static void *g_scratch_ptr[NOALLOC_MAX_DEVICES];

static hipError_t scratch_ptr(int dev, void **out)
{
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return hipSuccess;
}

static size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

}  // namespace ffsat

using namespace ffsat;

extern "C" ffsat_status ffsat_eval_noalloc(const ffsat_problem *p, int32_t B, const float *x, float *F, float *grad,
                                           void *stream)
{
    if (!p || !x) return ffsat_fail_external(FFSAT_E_INVALID_ARG, "NULL problem or x");
    if (B < 1) return ffsat_fail_external(FFSAT_E_INVALID_ARG, "B must be >= 1");
    if (!F && !grad) return FFSAT_OK;
    const Layout &Ly = p->lay[IO_F32];
    int rows = 0;
    for (const Bin &b : Ly.bins) rows += (b.count + b.cpw - 1) / b.cpw;
    const size_t nb = (size_t)B;
    const size_t slot_bytes = align256((size_t)p->nnz * nb * sizeof(float));
    const size_t fpart_bytes = align256((size_t)rows * nb * sizeof(float));
    const size_t ftmp_bytes = align256((size_t)f_splits(rows) * nb * sizeof(float));
    const size_t need = slot_bytes + fpart_bytes + ftmp_bytes;
    if (need > NOALLOC_SCRATCH_BYTES) {
        char msg[200];
        snprintf(msg, sizeof msg, "ffsat_eval_noalloc: needs %zu bytes of scratch (nnz * B * 4 + objective rows), "
                                  "more than its fixed %zu", need, NOALLOC_SCRATCH_BYTES);
        return ffsat_fail_external(FFSAT_E_UNSUPPORTED, msg);
    }
    int cur = -1;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return ffsat_fail_external(FFSAT_E_HIP, hipGetErrorString(e));
    if (cur != p->device) return ffsat_fail_external(FFSAT_E_DEVICE_MISMATCH, "current device is not the problem's");
    if (cur < 0 || cur >= NOALLOC_MAX_DEVICES) return ffsat_fail_external(FFSAT_E_UNSUPPORTED, "device index too large");
    void *base = nullptr;
    if ((e = scratch_ptr(cur, &base)) != hipSuccess) return ffsat_fail_external(FFSAT_E_HIP, hipGetErrorString(e));
    float *slot = (float *)base;
    float *fpart = (float *)((char *)base + slot_bytes);
    float *ftmp = (float *)((char *)base + slot_bytes + fpart_bytes);
    hipStream_t s = (hipStream_t)stream;

    EvalArgs<float> a{};
    a.x = x;
    a.slot = slot;
    a.fpart = fpart;
    a.con = Ly.d_con;
    a.lit = Ly.d_lit;
    a.w = p->d_w;
    a.B = B;
    a.wm = (p->m + 31) / 32;
    a.want_grad = grad ? 1 : 0;
    a.do_value = 1;
    int row0 = 0;
    for (const Bin &b : Ly.bins) {
        a.first = b.first;
        a.count = b.count;
        a.cpw = b.cpw;
        a.fg = 1;
        a.n_rb = (B + (64 / b.L) - 1) / (64 / b.L);
        a.fpart_row0 = row0;
        a.types = b.ct == CT_F32 ? (const void *)Ly.d_t32 : (const void *)Ly.d_t64;
        a.freqs = b.ct == CT_F32 ? (const void *)Ly.d_f32 : (const void *)Ly.d_f64;
        Bin t = b;
        t.fg = 1;
        if ((e = launch_eval_bin_f32(t, a, s)) != hipSuccess) return ffsat_fail_external(FFSAT_E_HIP, hipGetErrorString(e));
        row0 += (b.count + b.cpw - 1) / b.cpw;
    }
    ReduceArgs<float> r{};
    r.n = p->n;
    r.B = B;
    r.m = p->m;
    r.vptr = Ly.d_vptr;
    r.vslot = Ly.d_vslot;
    r.slot = slot;
    r.grad = grad;
    r.fpart = fpart;
    r.rows = rows;
    r.ftmp = ftmp;
    r.F = F;
    if ((e = launch_reduce_f32(r, s)) != hipSuccess) return ffsat_fail_external(FFSAT_E_HIP, hipGetErrorString(e));
    return FFSAT_OK;
}
