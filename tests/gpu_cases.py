"""Shared helpers for the GPU parity tests: instances that exercise every
kernel bin, natural-scale error measures and the oracle comparisons."""
import numpy as np

import workloads
from workloads import assemble, random_hybrid

# Tolerances (natural scale): |dWE_c| <= 1, |dWE_c/dl_i| <= 1, so a
# per-constraint value is compared absolutely, the objective relative to
# sum_c |w_c| and the gradient of variable v relative to
# S_v = sum_{c containing v} |w_c|.  FP32 target 1e-5; FP64 target 1e-12.
TOL32 = 1e-5
TOL64 = 1e-12


def every_bin_instance(seed=11, n=700):
    """Short and long constraints of every kind: all segment counts of the
    FP32 and FP64 kernels (FP64 root-of-unity shapes 14..32 positions over
    16 lanes, 16..32 over 8), thresholds outside [1, k], length-1
    constraints."""
    base = random_hybrid(n, seed, n_or=150, or_len=(1, 9), n_xor=60, xor_len=(1, 40),
                         n_card=70, card_len=(1, 140), card_t=(0, 70), weights="uniform")
    rng = np.random.default_rng(seed + 1)
    extra = []
    for kind, k, t in [(2, 512, 200), (2, 400, 133), (2, 300, 299), (2, 257, 128), (2, 256, 100),
                       (2, 255, 7), (2, 200, 100), (0, 512, 0), (1, 511, 1), (1, 300, 0),
                       (2, 64, 64), (2, 65, 1), (2, 33, 34), (0, 17, 0), (1, 64, 1),
                       (2, 340, 170), (2, 384, 1), (2, 449, 224), (2, 180, 90), (2, 47, 20), (1, 46, 1),
                       (2, 430, 215), (2, 441, 100), (2, 470, 235), (2, 490, 17), (2, 128, 64),
                       (2, 150, 75), (2, 161, 3), (2, 206, 50), (2, 220, 110), (2, 230, 5), (2, 240, 120),
                       (2, 248, 124)]:
        v = rng.choice(n, size=k, replace=False) + 1
        sg = np.where(rng.random(k) < 0.5, -1, 1)
        extra.append((kind, [t], [(v * sg).astype(np.int32)]))
    groups = []
    for c in range(base.m):
        kd, pr, li = base.constraint(c)
        groups.append((kd, [pr], [li.copy()]))
    groups += extra
    inst = assemble(n, groups)
    inst.weights = rng.uniform(0.5, 1.5, inst.m).astype(np.float32)
    return inst


def var_scale(inst):
    w = np.abs(inst.weights_or_ones().astype(np.float64))
    lens = np.diff(inst.con_ptr)
    con_of_slot = np.repeat(np.arange(inst.m), lens)
    S = np.zeros(inst.n_vars)
    np.add.at(S, np.abs(inst.lits) - 1, w[con_of_slot])
    return np.maximum(S, 1e-30)


def errors(inst, gpu, ref, cols=None):
    """max natural-scale errors of F, grad, con_val (cols: restart subset of gpu)."""
    sel = (lambda a: a) if cols is None else (lambda a: a[..., cols])
    out = {}
    wsum = float(np.abs(inst.weights_or_ones().astype(np.float64)).sum())
    if "F" in gpu:
        out["F"] = float(np.max(np.abs(sel(gpu["F"]) - ref["F"])) / wsum)
    if "grad" in gpu:
        S = var_scale(inst)[:, None]
        out["grad"] = float(np.max(np.abs(sel(gpu["grad"]) - ref["g"]) / S))
    if "con_val" in gpu and ref.get("con_val") is not None:
        out["con_val"] = float(np.max(np.abs(sel(gpu["con_val"]) - ref["con_val"])))
    return out


def to_np(d):
    return {k: v.detach().cpu().numpy() for k, v in d.items()}


def points(inst, B, seed, dist):
    x = workloads.points(inst.n_vars, B, seed, dist=dist)
    if dist == "mixed_edge":
        x[0, :] = -0.0
        x[1, ::2] = 0.0
    return x
