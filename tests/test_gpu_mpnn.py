"""Learned initialiser on the GPU against the FP64 reference network.

The device runs matrix products with bfloat16 operands and FP32
accumulation; the reference emulates that operand rounding (bf16=True) in
FP64.  Residual differences come from FP32 accumulation and from the rare
activation whose FP32 and FP64 values round to different bfloat16 neighbours
(one bfloat16 ulp, 2^-8 relative, on one product term).  Tolerances:
  mu:            max abs difference <= 2e-3 (mu in [-1, 1])
  loss:          relative <= 1e-3
  each gradient: max abs difference <= 2e-2 * max |reference gradient|
and against the unrounded FP64 network (the bfloat16 rounding error itself,
about sqrt(K) * 2^-9 relative for K-term products) 10x looser.
"""
import numpy as np
import pytest

import workloads
from oracle import mpnn_ref

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
DEV = "cuda:0"
H, R = 64, 3


@pytest.fixture(scope="module")
def ffs():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2308_15020_amd as P
    P.lib()
    return P


def _instance(seed=3):
    return workloads.random_hybrid(300, seed, n_or=700, or_len=(3, 7), n_xor=60, xor_len=(3, 12),
                                   n_card=30, card_len=(10, 40))


def _setup(ffs, inst, seed=5):
    from paper_2308_15020_amd.mpnn import Mpnn
    prob = ffs.Problem(inst, device=0)
    net = Mpnn(H, R, device=0, seed=1)
    p = mpnn_ref.init_params(H, R, seed=seed)
    # non-zero biases exercise the bias paths
    rng = np.random.default_rng(seed + 1)
    for name, shp in mpnn_ref.param_shapes(H, R):
        if len(shp) == 1 and name != "wo":
            p[name] = rng.uniform(-0.1, 0.1, shp)
    flat = mpnn_ref.flatten(p, H, R).astype(np.float32)
    net.set_params(flat)
    pref = mpnn_ref.unflatten(flat.astype(np.float64), H, R)
    return prob, net, pref


def _grad_errs(g_dev, gref, scale=1.0):
    out = {}
    o = 0
    for name, shp in mpnn_ref.param_shapes(H, R):
        sz = int(np.prod(shp))
        got = g_dev[o:o + sz].astype(np.float64).reshape(shp)
        ref = np.asarray(gref[name]).reshape(shp)
        den = max(np.abs(ref).max(), 1e-30)
        out[name] = float(np.abs(got - ref).max() / den)
        o += sz
    assert o == g_dev.size
    return out


def test_forward_backward_parity(ffs):
    inst = _instance()
    prob, net, pref = _setup(ffs, inst)
    g = mpnn_ref.Graph(inst)
    mu = net.forward(prob).cpu().numpy().astype(np.float64)
    mu_bf = mpnn_ref.forward(g, pref, R, bf16=True)
    mu_64 = mpnn_ref.forward(g, pref, R, bf16=False)
    assert np.abs(mu - mu_bf).max() <= 2e-3, np.abs(mu - mu_bf).max()
    assert np.abs(mu - mu_64).max() <= 2e-2
    tgt = np.where(np.random.default_rng(0).random(inst.n_vars) < 0.5, -1.0, 1.0) * 0.8
    loss = float(net.backward(prob, torch.from_numpy(tgt.astype(np.float32)).to(DEV)).item())
    gd = net.grads()
    l_bf, gr_bf = mpnn_ref.backward(g, pref, tgt.astype(np.float32).astype(np.float64), R, bf16=True)
    l_64, gr_64 = mpnn_ref.backward(g, pref, tgt.astype(np.float32).astype(np.float64), R, bf16=False)
    assert abs(loss - l_bf) <= 1e-3 * l_bf
    e_bf = _grad_errs(gd, gr_bf)
    e_64 = _grad_errs(gd, gr_64)
    print("bf16-emulated:", {k: f"{v:.1e}" for k, v in e_bf.items()})
    print("fp64:", {k: f"{v:.1e}" for k, v in e_64.items()})
    assert max(e_bf.values()) <= 2e-2, e_bf
    assert max(e_64.values()) <= 2e-1, e_64


def test_backward_deterministic_and_adam(ffs):
    inst = _instance(4)
    prob, net, pref = _setup(ffs, inst, seed=7)
    tgt = torch.from_numpy(np.linspace(-0.9, 0.9, inst.n_vars).astype(np.float32)).to(DEV)
    l1 = net.backward(prob, tgt).item()
    g1 = net.grads()
    l2 = net.backward(prob, tgt).item()
    g2 = net.grads()
    assert l1 == l2 and np.array_equal(g1, g2)
    p0 = net.get_params()
    lr, b1, b2, eps = 1e-2, 0.9, 0.999, 1e-8
    net.adam(lr, b1, b2, eps)
    p1 = net.get_params()
    # first step: m_hat = g, v_hat = g^2 -> p - lr g / (|g| + eps)
    g = g2.astype(np.float64)
    m = (1 - np.float32(b1)) * g2
    v = (1 - np.float32(b2)) * g2 * g2
    want = p0.astype(np.float64) - lr * (m / (1 - b1)) / (np.sqrt(v / (1 - b2)) + eps)
    assert np.allclose(p1, want, rtol=1e-5, atol=1e-7), np.abs(p1 - want).max()
    assert np.all(np.abs(p1 - p0) <= lr * 1.0001 + 1e-7) and g.size == p0.size


def _splitmix64(z):
    msk = (1 << 64) - 1
    z &= msk
    z = ((z ^ (z >> 30)) * 0xbf58476d1ce4e5b9) & msk
    z = ((z ^ (z >> 27)) * 0x94d049bb133111eb) & msk
    return z ^ (z >> 31)


def test_propose(ffs):
    from paper_2308_15020_amd.mpnn import Mpnn
    inst = workloads.random_hybrid(23, 1, n_or=15, or_len=(2, 4))
    prob = ffs.Problem(inst, device=0)
    B = 10
    plan = ffs.Plan(prob, B)
    net = Mpnn(32, 1, device=0, seed=3)
    mu = torch.from_numpy(np.linspace(-1, 1, 23).astype(np.float32)).to(DEV)
    seed, sigma = 987654321, 0.25
    x = net.propose(plan, mu, frac_learned=0.6, sigma=sigma, seed=seed).cpu().numpy()
    mun = mu.cpu().numpy()
    for v in range(23):
        for b in range(B):
            i = v * B + b
            r = _splitmix64(seed + (i + 1) * 0x9e3779b97f4a7c15)
            u = np.float32((r >> 40) * (2.0 / 16777216.0) - 1.0)
            if b < 6:
                want = min(max(float(mun[v]) + sigma * float(u), -1.0), 1.0)
                assert abs(x[v, b] - want) <= 1.2e-7, (v, b)
            else:
                assert x[v, b] == u, (v, b)


def test_training_lowers_loss(ffs):
    from paper_2308_15020_amd.mpnn import Mpnn, fit
    insts = [workloads.planted_hybrid(200, s, n_or=700, or_len=(3, 4), n_xor=8, xor_len=(2, 3),
                                      n_card=8, card_len=(5, 15)) for s in range(3)]
    probs = [ffs.Problem(i, device=0) for i, _ in insts]
    tg = [torch.from_numpy(np.where(h, -1.0, 1.0).astype(np.float32)).to(DEV) for _, h in insts]
    net = Mpnn(H, R, device=0, seed=11)
    hist = fit(net, probs, tg, epochs=25, lr=3e-3)
    assert np.all(np.isfinite(hist))
    assert hist[-1] < 0.9 * hist[0], hist
