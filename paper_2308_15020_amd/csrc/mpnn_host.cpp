// Host side of the message-passing initialiser: incidence graph of a
// problem, parameters (FP32 masters, products in BF16 on the matrix cores),
// forward pass, backward pass, Adam, and proposals of restart points.
// Network: see ffsat_mpnn_create in include/ffsat.h.
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "mpnn_internal.h"

using namespace ffsat;

#define MCHK(call)                                                                                   \
    do {                                                                                             \
        hipError_t e_ = (call);                                                                      \
        if (e_ != hipSuccess) {                                                                      \
            char b_[256];                                                                            \
            snprintf(b_, sizeof b_, "%s failed: %s", #call, hipGetErrorString(e_));                  \
            return ffsat_fail_external(e_ == hipErrorOutOfMemory ? FFSAT_E_NOMEM : FFSAT_E_HIP, b_); \
        }                                                                                            \
    } while (0)

struct ffsat_mpnn {
    int H = 64, R = 3, device = 0;
    int64_t P = 0;
    std::vector<int64_t> off;   // parameter offsets in the order of the layout
    float *w = nullptr, *g = nullptr, *m1 = nullptr, *m2 = nullptr;
    int step = 0;
    // workspace, sized for the largest graph seen
    int cap_n = 0, cap_m = 0;
    std::vector<float *> bufs;
    float *hv0 = nullptr, *hc0 = nullptr;
    std::vector<float *> Xc, Hc, Xv, Hv;
    float *mu = nullptr, *dz = nullptr, *lterm = nullptr, *dHv = nullptr, *dHc = nullptr;
    float *dXv = nullptr, *dXc = nullptr, *part = nullptr, *cpart = nullptr;
    size_t part_len = 0;
};

namespace {

enum { P_EV = 0, P_EVB, P_EC, P_ECB };   // then per round Wc, bc, Wv, bv, then wo, bo
inline int p_wc(int r) { return 4 + 4 * r; }
inline int p_bc(int r) { return 5 + 4 * r; }
inline int p_wv(int r) { return 6 + 4 * r; }
inline int p_bv(int r) { return 7 + 4 * r; }
inline int p_wo(int R) { return 4 + 4 * R; }

void layout(ffsat_mpnn *net, std::vector<std::pair<int64_t, int64_t>> *shapes)
{
    const int H = net->H;
    std::vector<std::pair<int64_t, int64_t>> sh = {{8, H}, {1, H}, {8, H}, {1, H}};
    for (int r = 0; r < net->R; ++r) {
        sh.push_back({3 * H, H});
        sh.push_back({1, H});
        sh.push_back({3 * H, H});
        sh.push_back({1, H});
    }
    sh.push_back({1, H});
    sh.push_back({1, 1});
    net->off.clear();
    int64_t o = 0;
    for (auto &s : sh) {
        net->off.push_back(o);
        o += s.first * s.second;
    }
    net->P = o;
    if (shapes) *shapes = sh;
}

uint64_t splitmix(uint64_t &state)
{
    uint64_t z = (state += 0x9e3779b97f4a7c15ull);
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

void free_ws(ffsat_mpnn *net)
{
    for (float *b : net->bufs) (void)hipFree(b);
    net->bufs.clear();
    net->Xc.clear(); net->Hc.clear(); net->Xv.clear(); net->Hv.clear();
    net->cap_n = net->cap_m = 0;
}

ffsat_status ensure_ws(ffsat_mpnn *net, int n, int m)
{
    if (n <= net->cap_n && m <= net->cap_m) return FFSAT_OK;
    // grow with a quarter of headroom, so that a stream of similar instances
    // (a test set, training batches) does not reallocate on every larger one
    n = std::max(n, net->cap_n);
    m = std::max(m, net->cap_m);
    n += n / 4;
    m += m / 4;
    free_ws(net);
    const int H = net->H;
    auto get = [&](size_t count, float **dst) -> ffsat_status {
        float *p = nullptr;
        MCHK(hipMalloc(&p, std::max<size_t>(count, 1) * sizeof(float)));
        net->bufs.push_back(p);
        *dst = p;
        return FFSAT_OK;
    };
    ffsat_status st;
    const size_t N = (size_t)n, Mc = (size_t)m;
    if ((st = get(N * H, &net->hv0)) || (st = get(Mc * H, &net->hc0))) return st;
    net->Xc.resize(net->R); net->Hc.resize(net->R); net->Xv.resize(net->R); net->Hv.resize(net->R);
    for (int r = 0; r < net->R; ++r) {
        if ((st = get(Mc * 3 * H, &net->Xc[r])) || (st = get(Mc * H, &net->Hc[r])) ||
            (st = get(N * 3 * H, &net->Xv[r])) || (st = get(N * H, &net->Hv[r])))
            return st;
    }
    if ((st = get(N, &net->mu)) || (st = get(N, &net->dz)) || (st = get(N, &net->lterm)) ||
        (st = get(N * H, &net->dHv)) || (st = get(Mc * H, &net->dHc)) || (st = get(N * 3 * H, &net->dXv)) ||
        (st = get(Mc * 3 * H, &net->dXc)))
        return st;
    net->part_len = (size_t)64 * 3 * H * H;
    if ((st = get(net->part_len, &net->part)) || (st = get((size_t)1024 * (H + 1), &net->cpart))) return st;
    net->cap_n = n;
    net->cap_m = m;
    return FFSAT_OK;
}

// The graph's arrays packed into one host staging buffer at 256-byte
// aligned offsets, then one allocation and one copy to the device (ten
// separate allocations and blocking copies cost ~0.5 ms per problem).
struct Packer {
    std::vector<char> host;
    std::vector<std::pair<void **, size_t>> fix;   // pointer to set, offset
    template <typename T>
    void add(T **dst, const std::vector<T> &v)
    {
        const size_t off = (host.size() + 255) & ~(size_t)255;
        host.resize(off + std::max<size_t>(v.size(), 1) * sizeof(T), 0);
        if (!v.empty()) memcpy(host.data() + off, v.data(), v.size() * sizeof(T));
        fix.push_back({(void **)dst, off});
    }
    ffsat_status upload(void **buf)
    {
        MCHK(hipMalloc(buf, std::max<size_t>(host.size(), 1)));
        MCHK(hipMemcpy(*buf, host.data(), host.size(), hipMemcpyHostToDevice));
        for (auto &f : fix) *f.first = (char *)*buf + f.second;
        return FFSAT_OK;
    }
};

// Incidence graph and node features (original constraint order).
ffsat_status graph_of(ffsat_problem *p, MpnnGraph **out)
{
    if (p->mpnn_graph) {
        *out = (MpnnGraph *)p->mpnn_graph;
        return FFSAT_OK;
    }
    const int n = p->n, m = p->m;
    const int nnz = (int)p->nnz;
    std::vector<int32_t> cptr(m + 1), lit(nnz), vof(nnz), cof(nnz), vptr(n + 1, 0), vsl(nnz);
    std::vector<float> wk(nnz), wd(nnz), fv((size_t)n * 8, 0.f), fc((size_t)m * 8, 0.f);
    std::vector<int> P(n, 0), Nn(n, 0);
    for (int c = 0; c <= m; ++c) cptr[c] = (int32_t)p->h_con_ptr[c];
    for (int c = 0; c < m; ++c) {
        const int k = cptr[c + 1] - cptr[c];
        for (int e = cptr[c]; e < cptr[c + 1]; ++e) {
            const int32_t l = p->h_lits[e];
            const int v = (l > 0 ? l : -l) - 1;
            lit[e] = v | (l < 0 ? (int32_t)0x80000000u : 0);
            vof[e] = v;
            cof[e] = c;
            wk[e] = 1.0f / (float)k;
            if (l > 0) P[v]++; else Nn[v]++;
            vptr[v + 1]++;
        }
        const int kind = p->h_kinds[c], prm = p->h_params[c];
        float *f = &fc[(size_t)c * 8];
        f[0] = 1.f;
        f[1] = kind == FFSAT_KIND_OR;
        f[2] = kind == FFSAT_KIND_XOR;
        f[3] = kind == FFSAT_KIND_CARD_GE;
        f[4] = (float)k / 64.f;
        const double t = std::min<double>(std::max<double>(prm, 0.0), k + 1.0);
        f[5] = kind == FFSAT_KIND_CARD_GE ? (float)(t / k) : (kind == FFSAT_KIND_OR ? 1.f / (float)k : 0.f);
        f[6] = kind == FFSAT_KIND_XOR ? (float)(prm & 1) : 0.f;
    }
    for (int v = 0; v < n; ++v) vptr[v + 1] += vptr[v];
    {
        std::vector<int32_t> fill(vptr.begin(), vptr.end() - 1);
        for (int e = 0; e < nnz; ++e) vsl[fill[vof[e]]++] = e;
    }
    for (int e = 0; e < nnz; ++e) {
        const int v = vof[e];
        wd[e] = 1.0f / (float)std::max(1, P[v] + Nn[v]);
    }
    for (int v = 0; v < n; ++v) {
        float *f = &fv[(size_t)v * 8];
        f[0] = 1.f;
        f[1] = (float)P[v] / 8.f;
        f[2] = (float)Nn[v] / 8.f;
        f[3] = (float)(P[v] - Nn[v]) / (float)(P[v] + Nn[v] + 1);
    }
    MpnnGraph *g = new MpnnGraph();
    g->n = n; g->m = m; g->nnz = nnz;
    Packer pk;
    pk.add(&g->con_ptr, cptr); pk.add(&g->lit, lit); pk.add(&g->var_of, vof); pk.add(&g->con_of, cof);
    pk.add(&g->vptr, vptr); pk.add(&g->vslots, vsl); pk.add(&g->wk, wk); pk.add(&g->wd, wd);
    pk.add(&g->fv, fv); pk.add(&g->fc, fc);
    const ffsat_status st = pk.upload(&g->buf);
    if (st != FFSAT_OK) {
        ffsat_free_mpnn_graph(g);   // nothing half-built stays attached to the problem
        return st;
    }
    p->mpnn_graph = g;   // freed with the problem
    *out = g;
    return FFSAT_OK;
}

int splits_for(int K) { return std::max(1, std::min(64, (K + 511) / 512)); }

// dW (K x H) = X^T dZ over `rows` rows, split over the rows, fixed-order sum
hipError_t weight_grad(ffsat_mpnn *net, int rows, int K, const float *X, int ldx, const float *dZ, float *out,
                       hipStream_t s)
{
    const int H = net->H;
    int S = splits_for(rows);
    while ((size_t)S * K * H > net->part_len && S > 1) S /= 2;
    hipError_t e = gemm(true, false, 0, K, H, rows, X, ldx, dZ, H, net->part, H, nullptr, S, (size_t)K * H, s);
    if (e != hipSuccess) return e;
    // exactly the slices the product wrote
    return sum_slices((int64_t)K * H, gemm_slices(rows, S), net->part, (size_t)K * H, out, false, s);
}

ffsat_status forward(ffsat_mpnn *net, MpnnGraph *g, hipStream_t s)
{
    const int H = net->H, n = g->n, m = g->m;
    const float *W = net->w;
    const auto &o = net->off;
    MCHK(gemm(false, false, 1, n, H, 8, g->fv, 8, W + o[P_EV], H, net->hv0, H, W + o[P_EVB], 1, 0, s));
    MCHK(gemm(false, false, 1, m, H, 8, g->fc, 8, W + o[P_EC], H, net->hc0, H, W + o[P_ECB], 1, 0, s));
    const float *hv = net->hv0, *hc = net->hc0;
    for (int r = 0; r < net->R; ++r) {
        // messages into columns H..3H of X, the constraint's own state into 0..H
        MCHK(gather(m, H, g->con_ptr, nullptr, g->var_of, g->lit, g->wk, hv, H, 0, 0, net->Xc[r], 3 * H, H, 2 * H, 0, s,
                    hc));
        MCHK(gemm(false, false, 1, m, H, 3 * H, net->Xc[r], 3 * H, W + o[p_wc(r)], H, net->Hc[r], H, W + o[p_bc(r)], 1,
                  0, s));
        hc = net->Hc[r];
        MCHK(gather(n, H, g->vptr, g->vslots, g->con_of, g->lit, g->wd, hc, H, 0, 0, net->Xv[r], 3 * H, H, 2 * H, 0, s,
                    hv));
        MCHK(gemm(false, false, 1, n, H, 3 * H, net->Xv[r], 3 * H, W + o[p_wv(r)], H, net->Hv[r], H, W + o[p_bv(r)], 1,
                  0, s));
        hv = net->Hv[r];
    }
    MCHK(head(n, H, hv, W + o[p_wo(net->R)], W + o[p_wo(net->R) + 1], net->mu, s));
    return FFSAT_OK;
}

ffsat_status backward(ffsat_mpnn *net, MpnnGraph *g, const float *target, float *loss, hipStream_t s)
{
    const int H = net->H, n = g->n, m = g->m, R = net->R;
    const float *W = net->w;
    float *G = net->g;
    const auto &o = net->off;
    MCHK(head_back(n, H, net->mu, target, W + o[p_wo(R)], net->dz, net->lterm, net->dHv, s));
    MCHK(dwo(n, H, net->dz, net->Hv[R - 1], net->cpart, 1024, G + o[p_wo(R)], s));   // wo then bo
    if (loss) MCHK(colsum(n, 1, net->lterm, net->cpart, 1024, loss, s));
    MCHK(fill_f32((int64_t)m * H, net->dHc, 0.f, s));
    for (int r = R - 1; r >= 0; --r) {
        MCHK(relu_back(n, H, net->dHv, net->Hv[r], nullptr, 0, s));
        MCHK(weight_grad(net, n, 3 * H, net->Xv[r], 3 * H, net->dHv, G + o[p_wv(r)], s));
        MCHK(colsum(n, H, net->dHv, net->cpart, 1024, G + o[p_bv(r)], s));
        MCHK(gemm(false, true, 0, n, 3 * H, H, net->dHv, H, W + o[p_wv(r)], H, net->dXv, 3 * H, nullptr, 1, 0, s));
        MCHK(take_cols(n, H, net->dXv, 3 * H, net->dHv, s));
        MCHK(gather(m, H, g->con_ptr, nullptr, g->var_of, g->lit, g->wd, net->dXv, 3 * H, H, 2 * H, net->dHc, H, 0, 0,
                    1, s));
        MCHK(relu_back(m, H, net->dHc, net->Hc[r], nullptr, 0, s));
        MCHK(weight_grad(net, m, 3 * H, net->Xc[r], 3 * H, net->dHc, G + o[p_wc(r)], s));
        MCHK(colsum(m, H, net->dHc, net->cpart, 1024, G + o[p_bc(r)], s));
        MCHK(gemm(false, true, 0, m, 3 * H, H, net->dHc, H, W + o[p_wc(r)], H, net->dXc, 3 * H, nullptr, 1, 0, s));
        MCHK(take_cols(m, H, net->dXc, 3 * H, net->dHc, s));
        MCHK(gather(n, H, g->vptr, g->vslots, g->con_of, g->lit, g->wk, net->dXc, 3 * H, H, 2 * H, net->dHv, H, 0, 0,
                    1, s));
    }
    MCHK(relu_back(n, H, net->dHv, net->hv0, nullptr, 0, s));
    MCHK(weight_grad(net, n, 8, g->fv, 8, net->dHv, G + o[P_EV], s));
    MCHK(colsum(n, H, net->dHv, net->cpart, 1024, G + o[P_EVB], s));
    MCHK(relu_back(m, H, net->dHc, net->hc0, nullptr, 0, s));
    MCHK(weight_grad(net, m, 8, g->fc, 8, net->dHc, G + o[P_EC], s));
    MCHK(colsum(m, H, net->dHc, net->cpart, 1024, G + o[P_ECB], s));
    return FFSAT_OK;
}

}  // namespace

void ffsat_free_mpnn_graph(void *gp)
{
    MpnnGraph *g = (MpnnGraph *)gp;
    if (!g) return;
    (void)hipFree(g->buf);
    delete g;
}

extern "C" ffsat_status ffsat_mpnn_create(const ffsat_mpnn_desc *d, ffsat_mpnn **out)
{
    if (!d || !out) return ffsat_fail_external(FFSAT_E_INVALID_ARG, "NULL argument");
    if (d->hidden < 32 || d->hidden % 32 != 0 || d->hidden > 256)
        return ffsat_fail_external(FFSAT_E_INVALID_ARG, "hidden must be a multiple of 32 in [32, 256]");
    if (d->reserved != 0) return ffsat_fail_external(FFSAT_E_INVALID_ARG, "reserved must be 0");
    if (d->rounds < 1 || d->rounds > 8) return ffsat_fail_external(FFSAT_E_INVALID_ARG, "rounds must be in [1, 8]");
    int cur = -1;
    MCHK(hipGetDevice(&cur));
    if (cur != d->device) return ffsat_fail_external(FFSAT_E_DEVICE_MISMATCH, "device is not the current device");
    ffsat_mpnn *net = new ffsat_mpnn();
    net->H = d->hidden;
    net->R = d->rounds;
    net->device = d->device;
    std::vector<std::pair<int64_t, int64_t>> shapes;
    layout(net, &shapes);
    // Glorot-uniform matrices and head vector, zero biases
    std::vector<float> w((size_t)net->P, 0.f);
    uint64_t st = d->seed;
    for (size_t q = 0; q < shapes.size(); ++q) {
        const int64_t rows = shapes[q].first, cols = shapes[q].second;
        const bool is_bias = rows == 1 && q != (size_t)p_wo(net->R);
        if (is_bias) continue;
        const double fan = q == (size_t)p_wo(net->R) ? (double)(cols + 1) : (double)(rows + cols);
        const double lim = std::sqrt(6.0 / fan);
        for (int64_t i = 0; i < rows * cols; ++i) {
            const double u = (double)(splitmix(st) >> 11) * (1.0 / 9007199254740992.0);
            w[(size_t)(net->off[q] + i)] = (float)((2.0 * u - 1.0) * lim);
        }
    }
    auto fail_free = [&](ffsat_status s) {
        (void)hipFree(net->w); (void)hipFree(net->g); (void)hipFree(net->m1); (void)hipFree(net->m2);
        delete net;
        return s;
    };
    const size_t bytes = (size_t)net->P * sizeof(float);
    if (hipMalloc(&net->w, bytes) != hipSuccess || hipMalloc(&net->g, bytes) != hipSuccess ||
        hipMalloc(&net->m1, bytes) != hipSuccess || hipMalloc(&net->m2, bytes) != hipSuccess)
        return fail_free(ffsat_fail_external(FFSAT_E_NOMEM, "mpnn parameters"));
    if (hipMemcpy(net->w, w.data(), bytes, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemset(net->g, 0, bytes) != hipSuccess || hipMemset(net->m1, 0, bytes) != hipSuccess ||
        hipMemset(net->m2, 0, bytes) != hipSuccess)
        return fail_free(ffsat_fail_external(FFSAT_E_HIP, "mpnn parameter upload"));
    *out = net;
    return FFSAT_OK;
}

extern "C" ffsat_status ffsat_mpnn_destroy(ffsat_mpnn *net)
{
    if (!net) return FFSAT_OK;
    free_ws(net);
    (void)hipFree(net->w); (void)hipFree(net->g); (void)hipFree(net->m1); (void)hipFree(net->m2);
    delete net;
    return FFSAT_OK;
}

extern "C" ffsat_status ffsat_mpnn_num_params(const ffsat_mpnn *net, int64_t *n)
{
    if (!net || !n) return ffsat_fail_external(FFSAT_E_INVALID_ARG, "NULL argument");
    *n = net->P;
    return FFSAT_OK;
}

extern "C" ffsat_status ffsat_mpnn_params(ffsat_mpnn *net, float *buf, int32_t which, int32_t to_net,
                                          int32_t on_device, void *stream)
{
    if (!net || !buf) return ffsat_fail_external(FFSAT_E_INVALID_ARG, "NULL argument");
    if (which < 0 || which > 1 || (which == 1 && to_net))
        return ffsat_fail_external(FFSAT_E_INVALID_ARG, "which: 0 parameters, 1 gradients (read only)");
    float *dev = which == 0 ? net->w : net->g;
    const size_t bytes = (size_t)net->P * sizeof(float);
    hipStream_t s = (hipStream_t)stream;
    hipMemcpyKind k = to_net ? (on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice)
                             : (on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost);
    MCHK(hipMemcpyAsync(to_net ? (void *)dev : (void *)buf, to_net ? (const void *)buf : (const void *)dev, bytes, k,
                        s));
    if (!on_device) MCHK(hipStreamSynchronize(s));
    if (to_net) {
        // a new parameter vector restarts the optimiser
        MCHK(fill_f32(net->P, net->m1, 0.f, s));
        MCHK(fill_f32(net->P, net->m2, 0.f, s));
        net->step = 0;
    }
    return FFSAT_OK;
}

extern "C" ffsat_status ffsat_mpnn_forward(ffsat_mpnn *net, ffsat_problem *p, float *mu, void *stream)
{
    if (!net || !p) return ffsat_fail_external(FFSAT_E_INVALID_ARG, "NULL argument");
    hipStream_t s = (hipStream_t)stream;
    MpnnGraph *g = nullptr;
    ffsat_status st;
    if ((st = graph_of(p, &g)) != FFSAT_OK) return st;
    if ((st = ensure_ws(net, g->n, g->m)) != FFSAT_OK) return st;
    if ((st = forward(net, g, s)) != FFSAT_OK) return st;
    if (mu) MCHK(hipMemcpyAsync(mu, net->mu, sizeof(float) * (size_t)g->n, hipMemcpyDeviceToDevice, s));
    return FFSAT_OK;
}

extern "C" ffsat_status ffsat_mpnn_backward(ffsat_mpnn *net, ffsat_problem *p, const float *target, float *loss,
                                            void *stream)
{
    if (!net || !p || !target) return ffsat_fail_external(FFSAT_E_INVALID_ARG, "NULL argument");
    hipStream_t s = (hipStream_t)stream;
    MpnnGraph *g = nullptr;
    ffsat_status st;
    if ((st = graph_of(p, &g)) != FFSAT_OK) return st;
    if ((st = ensure_ws(net, g->n, g->m)) != FFSAT_OK) return st;
    if ((st = forward(net, g, s)) != FFSAT_OK) return st;
    return backward(net, g, target, loss, s);
}

extern "C" ffsat_status ffsat_mpnn_adam(ffsat_mpnn *net, float lr, float beta1, float beta2, float eps, void *stream)
{
    if (!net) return ffsat_fail_external(FFSAT_E_INVALID_ARG, "NULL argument");
    if (!(lr > 0.f) || !(beta1 >= 0.f && beta1 < 1.f) || !(beta2 >= 0.f && beta2 < 1.f) || !(eps > 0.f))
        return ffsat_fail_external(FFSAT_E_INVALID_ARG, "bad Adam hyper-parameters");
    net->step += 1;
    MCHK(adam(net->P, net->w, net->g, net->m1, net->m2, lr, beta1, beta2, eps, net->step, (hipStream_t)stream));
    return FFSAT_OK;
}

extern "C" ffsat_status ffsat_mpnn_propose(ffsat_plan *plan, const float *mu, float *x, float frac_learned,
                                           float sigma, uint64_t seed, void *stream)
{
    if (!plan || !mu || !x) return ffsat_fail_external(FFSAT_E_INVALID_ARG, "NULL argument");
    if (!(frac_learned >= 0.f && frac_learned <= 1.f))
        return ffsat_fail_external(FFSAT_E_INVALID_ARG, "frac_learned must be in [0, 1]");
    const int B = plan->B;
    const int nl = (int)std::floor(frac_learned * (float)B + 0.5f);
    MCHK(propose((int64_t)plan->p->n * B, B, nl, mu, sigma, seed, x, (hipStream_t)stream));
    return FFSAT_OK;
}
