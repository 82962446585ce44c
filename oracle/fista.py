"""FP64 reference of the projected-gradient optimiser with the line search
the paper's Alg. 5 names (test infrastructure only).

Alg. 5 calls a line search (FISTA, accelerated proximal gradient, in the
library the paper uses) and clips to [-1, 1]; it stops once the step size
drops below 1e-12.  For each restart independently, with state
(x, y, eta, t) and F, G the objective and gradient of Def. 3:

  if eta < 1e-12: nothing changes (the restart has stopped).
  g = G(y)
  repeat up to max_ls times:
      z = clip(y - eta g, -1, 1)                       (projection = prox)
      accept if F(z) <= F(y) + <g, z - y> + |z - y|^2 / (2 eta)
      otherwise eta <- eta / 2
  (after max_ls rejections the last z is taken, with the halved eta)
  t' = (1 + sqrt(1 + 4 t^2)) / 2
  y' = z + ((t - 1) / t') (z - x),   x' = z

Everything here is plain numpy over ``oracle.eval_batch`` (FP64).
"""
from __future__ import annotations

import numpy as np

from . import eval_batch

ETA_MIN = 1e-12


def iterate(inst, x, y, eta, t, w=None, max_ls=15):
    """One iteration for every restart (columns of x[n][B]).  Returns
    (x', y', eta', t', F(y), F(x'), trials[B], margin[B]) where margin is
    the smallest |slack| of the sufficient-decrease tests the restart ran
    (how close a decision came to going the other way at another precision)."""
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    eta = np.asarray(eta, dtype=np.float64).copy()
    t = np.asarray(t, dtype=np.float64).copy()
    n, B = x.shape
    r = eval_batch(inst, y, w=w, want_g=True)
    Fy, g = r["F"], r["g"]
    z = y.copy()
    Fz = Fy.copy()
    active = eta >= ETA_MIN
    searching = active.copy()
    trials = np.zeros(B, dtype=np.int64)
    margin = np.full(B, np.inf)
    for _ in range(max_ls):
        if not searching.any():
            break
        cols = np.nonzero(searching)[0]
        zc = np.clip(y[:, cols] - eta[cols] * g[:, cols], -1.0, 1.0)
        Fc = eval_batch(inst, np.ascontiguousarray(zc), w=w, want_g=False)["F"]
        d = zc - y[:, cols]
        bound = Fy[cols] + np.sum(g[:, cols] * d, axis=0) + np.sum(d * d, axis=0) / (2.0 * eta[cols])
        ok = Fc <= bound
        z[:, cols] = zc
        Fz[cols] = Fc
        trials[cols] += 1
        margin[cols] = np.minimum(margin[cols], np.abs(bound - Fc))
        for q, c in enumerate(cols):
            if ok[q]:
                searching[c] = False
            else:
                eta[c] *= 0.5
    tn = np.where(active, (1.0 + np.sqrt(1.0 + 4.0 * t * t)) / 2.0, t)
    coef = np.where(active, (t - 1.0) / tn, 0.0)
    xn = np.where(active[None, :], z, x)
    yn = np.where(active[None, :], z + coef[None, :] * (z - x), y)
    return xn, yn, eta, tn, Fy, np.where(active, Fz, np.nan), trials, margin


def run(inst, x0, eta0, T, w=None, max_ls=15):
    """T iterations from x0 (y = x0, t = 1, eta = eta0 for every restart)."""
    x = np.asarray(x0, dtype=np.float64).copy()
    y = x.copy()
    B = x.shape[1]
    eta = np.full(B, float(eta0))
    t = np.ones(B)
    for _ in range(T):
        x, y, eta, t, *_ = iterate(inst, x, y, eta, t, w=w, max_ls=max_ls)
    return x, y, eta, t
