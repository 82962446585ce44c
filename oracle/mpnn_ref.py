"""FP64 reference of the message-passing initialiser (test infrastructure only).

The network the library trains and runs on the GPU, written out plainly in
numpy so that its forward pass, loss and parameter gradients can be checked
(and this reference itself is checked against central finite differences).

Graph: the clause-variable incidence of a hybrid formula; literal (c, v, s)
with sign s = +1 for +v and -1 for -v.  d_v = occurrences of v, k_c = length.

Features (8 per node):
  variable:   [1, P_v/8, N_v/8, (P_v - N_v)/(P_v + N_v + 1), 0, 0, 0, 0]
  constraint: [1, is_or, is_xor, is_card, k_c/64, thr, par, 0]
with P_v / N_v the positive / negative occurrences, thr = t/k for at-least-t
(t clipped to [0, k+1]), 1/k for OR, 0 for XOR, par = the XOR parity bit.

Layers (H = hidden width, R rounds, W stored as [K][H]):
  hv = relu(fv Ev + ev),  hc = relu(fc Ec + ec)
  round r:  a+_c = (1/k_c) sum_{(c,v,+)} hv_v,  a-_c likewise over negative literals
            hc = relu([hc, a+_c, a-_c] Wc_r + bc_r)
            a+_v = (1/max(d_v,1)) sum_{(c,v,+)} hc_c,  a-_v likewise
            hv = relu([hv, a+_v, a-_v] Wv_r + bv_r)
  mu_v = tanh(hv . wo + bo)
Loss: mean over variables of (mu_v - t_v)^2.

`bf16=True` rounds both operands of every matrix product (not the head) to
bfloat16 (round to nearest even) before multiplying, the operand precision
of the device's matrix cores.
"""
from __future__ import annotations

import numpy as np


def bf16_round(a):
    a = np.asarray(a, dtype=np.float32)
    u = a.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def features(inst):
    n, m = inst.n_vars, inst.m
    lits = inst.lits.astype(np.int64)
    v = np.abs(lits) - 1
    P = np.bincount(v[lits > 0], minlength=n).astype(np.float64)
    N = np.bincount(v[lits < 0], minlength=n).astype(np.float64)
    fv = np.zeros((n, 8))
    fv[:, 0] = 1.0
    fv[:, 1] = P / 8.0
    fv[:, 2] = N / 8.0
    fv[:, 3] = (P - N) / (P + N + 1.0)
    k = np.diff(inst.con_ptr).astype(np.float64)
    fc = np.zeros((m, 8))
    fc[:, 0] = 1.0
    kinds = inst.kinds
    fc[:, 1] = kinds == 0
    fc[:, 2] = kinds == 1
    fc[:, 3] = kinds == 2
    fc[:, 4] = k / 64.0
    t = np.clip(inst.params.astype(np.float64), 0, k + 1)
    fc[:, 5] = np.where(kinds == 2, t / k, np.where(kinds == 0, 1.0 / k, 0.0))
    fc[:, 6] = np.where(kinds == 1, inst.params & 1, 0)
    return fv, fc


def param_shapes(H=64, R=3):
    shapes = [("Ev", (8, H)), ("ev", (H,)), ("Ec", (8, H)), ("ec", (H,))]
    for r in range(R):
        shapes += [(f"Wc{r}", (3 * H, H)), (f"bc{r}", (H,)), (f"Wv{r}", (3 * H, H)), (f"bv{r}", (H,))]
    shapes += [("wo", (H,)), ("bo", (1,))]
    return shapes


def unflatten(flat, H=64, R=3):
    out, o = {}, 0
    for name, shp in param_shapes(H, R):
        sz = int(np.prod(shp))
        out[name] = np.asarray(flat[o:o + sz], dtype=np.float64).reshape(shp)
        o += sz
    assert o == len(flat)
    return out


def flatten(d, H=64, R=3):
    return np.concatenate([np.asarray(d[name]).ravel() for name, _ in param_shapes(H, R)])


class Graph:
    def __init__(self, inst):
        self.n, self.m = inst.n_vars, inst.m
        lens = np.diff(inst.con_ptr)
        self.c_of = np.repeat(np.arange(self.m), lens)
        self.v_of = np.abs(inst.lits).astype(np.int64) - 1
        self.pos = inst.lits > 0
        self.k = lens.astype(np.float64)
        self.d = np.maximum(np.bincount(self.v_of, minlength=self.n), 1).astype(np.float64)
        self.fv, self.fc = features(inst)


def _mm(a, b, bf16):
    if bf16:
        return bf16_round(a) @ bf16_round(b)
    return a @ b


def forward(g: Graph, p: dict, R=3, bf16=False, keep=False):
    H = p["ev"].shape[0]
    relu = lambda z: np.maximum(z, 0.0)  # noqa: E731
    cache = {}
    hv = relu(_mm(g.fv, p["Ev"], bf16) + p["ev"])
    hc = relu(_mm(g.fc, p["Ec"], bf16) + p["ec"])
    cache["hv0"], cache["hc0"] = hv, hc
    for r in range(R):
        ap = np.zeros((g.m, H))
        an = np.zeros((g.m, H))
        np.add.at(ap, g.c_of[g.pos], hv[g.v_of[g.pos]])
        np.add.at(an, g.c_of[~g.pos], hv[g.v_of[~g.pos]])
        Xc = np.concatenate([hc, ap / g.k[:, None], an / g.k[:, None]], axis=1)
        hc = relu(_mm(Xc, p[f"Wc{r}"], bf16) + p[f"bc{r}"])
        bp = np.zeros((g.n, H))
        bn = np.zeros((g.n, H))
        np.add.at(bp, g.v_of[g.pos], hc[g.c_of[g.pos]])
        np.add.at(bn, g.v_of[~g.pos], hc[g.c_of[~g.pos]])
        Xv = np.concatenate([hv, bp / g.d[:, None], bn / g.d[:, None]], axis=1)
        hv = relu(_mm(Xv, p[f"Wv{r}"], bf16) + p[f"bv{r}"])
        cache[f"Xc{r}"], cache[f"hc{r + 1}"] = Xc, hc
        cache[f"Xv{r}"], cache[f"hv{r + 1}"] = Xv, hv
    z = hv @ p["wo"] + p["bo"][0]
    mu = np.tanh(z)
    cache["mu"] = mu
    return (mu, cache) if keep else mu


def loss(mu, target):
    return float(np.mean((mu - target) ** 2))


def backward(g: Graph, p: dict, target, R=3, bf16=False):
    """Returns (loss, grads dict) by the chain rule through every layer."""
    H = p["ev"].shape[0]
    mu, c = forward(g, p, R, bf16, keep=True)
    n = g.n
    gr = {}
    dmu = 2.0 * (mu - target) / n
    dz = dmu * (1.0 - mu * mu)
    hv = c[f"hv{R}"]
    gr["wo"] = hv.T @ dz
    gr["bo"] = np.array([dz.sum()])
    dhv = np.outer(dz, p["wo"])
    dhc = np.zeros((g.m, H))
    for r in reversed(range(R)):
        dZv = dhv * (c[f"hv{r + 1}"] > 0)
        Xv = c[f"Xv{r}"]
        gr[f"Wv{r}"] = _mm(Xv.T, dZv, bf16)
        gr[f"bv{r}"] = dZv.sum(0)
        dXv = _mm(dZv, p[f"Wv{r}"].T, bf16)
        dhv = dXv[:, :H].copy()
        dbp = dXv[:, H:2 * H] / g.d[:, None]
        dbn = dXv[:, 2 * H:] / g.d[:, None]
        dhc = dhc.copy()
        np.add.at(dhc, g.c_of[g.pos], dbp[g.v_of[g.pos]])
        np.add.at(dhc, g.c_of[~g.pos], dbn[g.v_of[~g.pos]])
        dZc = dhc * (c[f"hc{r + 1}"] > 0)
        Xc = c[f"Xc{r}"]
        gr[f"Wc{r}"] = _mm(Xc.T, dZc, bf16)
        gr[f"bc{r}"] = dZc.sum(0)
        dXc = _mm(dZc, p[f"Wc{r}"].T, bf16)
        dhc = dXc[:, :H].copy()
        dap = dXc[:, H:2 * H] / g.k[:, None]
        dan = dXc[:, 2 * H:] / g.k[:, None]
        np.add.at(dhv, g.v_of[g.pos], dap[g.c_of[g.pos]])
        np.add.at(dhv, g.v_of[~g.pos], dan[g.c_of[~g.pos]])
    dZv0 = dhv * (c["hv0"] > 0)
    gr["Ev"] = _mm(g.fv.T, dZv0, bf16)
    gr["ev"] = dZv0.sum(0)
    dZc0 = dhc * (c["hc0"] > 0)
    gr["Ec"] = _mm(g.fc.T, dZc0, bf16)
    gr["ec"] = dZc0.sum(0)
    return loss(mu, target), gr


def init_params(H=64, R=3, seed=0):
    """Glorot-uniform weights, zero biases (the library initialises the same
    way from its own generator; tests pass explicit parameters)."""
    rng = np.random.default_rng(seed)
    p = {}
    for name, shp in param_shapes(H, R):
        if len(shp) == 2:
            lim = np.sqrt(6.0 / (shp[0] + shp[1]))
            p[name] = rng.uniform(-lim, lim, shp)
        elif name == "wo":
            lim = np.sqrt(6.0 / (H + 1))
            p[name] = rng.uniform(-lim, lim, shp)
        else:
            p[name] = np.zeros(shp)
    return p
