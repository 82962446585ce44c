"""Seeded synthetic hybrid-SAT instances and evaluation points.

This module only draws random structure and random points. It holds none of
the method's arithmetic, so both the HIP library's tests and the CPU oracle
can take their inputs from it.

Conventions (as in the paper's Preliminaries and its restart examples):
  * literals are DIMACS-style signed 1-based integers: ``+v`` is x_v and
    ``-v`` is its negation, whose value in [-1, 1] is ``-x_v``;
  * kinds: 0 = OR (CNF clause), 1 = XOR, 2 = at-least-t cardinality;
  * params: XOR parity bit p (1 = an odd number of true literals is
    required), cardinality threshold t, ignored for OR;
  * points are stored variable-major, ``x[n][B]``, restarts contiguous.

Workload shapes follow the random formulas of the paper's benchmark
appendix (random cardinality formulas: literals all positive or all
negative with probability 1/2; the RQ1 gradient-timing formulas) and the
configurations this library is measured on (random 3-SAT at ratio 4.26, a
mixed OR/XOR/cardinality instance, and a large mixed instance).
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Optional

import numpy as np

KIND_OR, KIND_XOR, KIND_CARD = 0, 1, 2
KIND_NAMES = {KIND_OR: "or", KIND_XOR: "xor", KIND_CARD: "card"}


@dataclass
class Instance:
    n_vars: int
    con_ptr: np.ndarray            # int64 [m+1]
    lits: np.ndarray               # int32 [nnz], signed 1-based
    kinds: np.ndarray              # int32 [m]
    params: np.ndarray             # int32 [m]
    weights: Optional[np.ndarray] = None   # float32 [m] or None (all ones)
    name: str = ""
    meta: dict = field(default_factory=dict)

    @property
    def m(self) -> int:
        return int(self.kinds.shape[0])

    @property
    def nnz(self) -> int:
        return int(self.lits.shape[0])

    def lengths(self) -> np.ndarray:
        return np.diff(self.con_ptr).astype(np.int64)

    def constraint(self, c: int):
        a, b = int(self.con_ptr[c]), int(self.con_ptr[c + 1])
        return int(self.kinds[c]), int(self.params[c]), self.lits[a:b]

    def weights_or_ones(self) -> np.ndarray:
        if self.weights is None:
            return np.ones(self.m, dtype=np.float32)
        return np.asarray(self.weights, dtype=np.float32)

    def save(self, path: str) -> None:
        np.savez(path, n_vars=np.int64(self.n_vars), con_ptr=self.con_ptr,
                 lits=self.lits, kinds=self.kinds, params=self.params,
                 weights=(self.weights if self.weights is not None
                          else np.zeros(0, np.float32)))

    @staticmethod
    def load(path: str) -> "Instance":
        z = np.load(path, allow_pickle=False)
        w = z["weights"]
        return Instance(int(z["n_vars"]), z["con_ptr"], z["lits"], z["kinds"],
                        z["params"], w if w.size else None)


# --------------------------------------------------------------------------
# building blocks
# --------------------------------------------------------------------------

def _distinct_rows(rng: np.random.Generator, n: int, rows: int, k: int) -> np.ndarray:
    """rows x k matrix of variable indices in [0, n), distinct within a row
    (repeated entries of a row are redrawn until the row has none)."""
    if k > n:
        raise ValueError(f"cannot draw {k} distinct variables out of {n}")
    out = rng.integers(0, n, size=(rows, k), dtype=np.int64)
    if k == 1:
        return out
    s = np.sort(out, axis=1)
    bad = np.nonzero((s[:, 1:] == s[:, :-1]).any(axis=1))[0]
    for r in bad:
        row = out[r]
        while True:
            _, first = np.unique(row, return_index=True)
            dup = np.ones(k, dtype=bool)
            dup[first] = False
            if not dup.any():
                break
            row[dup] = rng.integers(0, n, size=int(dup.sum()), dtype=np.int64)
        out[r] = row
    return out


def _draw_group(rng, n, count, kmin, kmax, sign_mode):
    """Draw `count` constraints with lengths U{kmin..kmax}.

    sign_mode: 'bernoulli' (each literal negated with prob. 1/2),
               'positive' (no negations),
               'uniform_block' (all literals of a constraint share one sign,
                                negative with prob. 1/2).
    Returns (lengths[count], list of signed-literal arrays in draw order).
    """
    lens = rng.integers(kmin, kmax + 1, size=count)
    rows = [None] * count
    for k in np.unique(lens):
        idx = np.nonzero(lens == k)[0]
        vars_ = _distinct_rows(rng, n, idx.size, int(k)) + 1
        if sign_mode == "bernoulli":
            neg = rng.random(vars_.shape) < 0.5
        elif sign_mode == "positive":
            neg = np.zeros(vars_.shape, dtype=bool)
        elif sign_mode == "uniform_block":
            neg = np.repeat(rng.random((idx.size, 1)) < 0.5, int(k), axis=1)
        else:
            raise ValueError(sign_mode)
        signed = np.where(neg, -vars_, vars_).astype(np.int32)
        for r, c in enumerate(idx):
            rows[c] = signed[r]
    return lens, rows


def assemble(n_vars: int, groups, name: str = "", weights=None, meta=None) -> Instance:
    """groups: list of (kind, params[count], rows list). Constraints keep the order given."""
    kinds, params, rows = [], [], []
    for kind, prm, rws in groups:
        kinds.append(np.full(len(rws), kind, dtype=np.int32))
        params.append(np.asarray(prm, dtype=np.int32))
        rows.extend(rws)
    lens = np.array([len(r) for r in rows], dtype=np.int64)
    con_ptr = np.zeros(len(rows) + 1, dtype=np.int64)
    np.cumsum(lens, out=con_ptr[1:])
    lits = (np.concatenate(rows).astype(np.int32) if rows else np.zeros(0, np.int32))
    return Instance(n_vars, con_ptr, lits, np.concatenate(kinds) if kinds else
                    np.zeros(0, np.int32), np.concatenate(params) if params else
                    np.zeros(0, np.int32), weights, name, meta or {})


def random_hybrid(n: int, seed: int, *, n_or=0, or_len=(3, 3), or_signs="bernoulli",
                  n_xor=0, xor_len=(3, 3), xor_signs="positive",
                  n_card=0, card_len=(10, 10), card_signs="uniform_block",
                  card_t="half", weights=None, name="") -> Instance:
    """Random hybrid formula: OR, XOR and at-least-t groups, in that order.

    card_t: 'half' -> t ~ U{1..floor(len/2)}; 'exact_half' -> t = len // 2;
            an int -> that threshold for every constraint;
            a (lo, hi) tuple -> t ~ U{lo..hi} (may leave [1, len]).
    weights: None, 'uniform' (U[0.5, 1.5]) or an array.
    """
    rng = np.random.default_rng(seed)
    groups = []
    if n_or:
        _, rows = _draw_group(rng, n, n_or, or_len[0], or_len[1], or_signs)
        groups.append((KIND_OR, np.zeros(n_or, np.int32), rows))
    if n_xor:
        _, rows = _draw_group(rng, n, n_xor, xor_len[0], xor_len[1], xor_signs)
        par = rng.integers(0, 2, size=n_xor)
        groups.append((KIND_XOR, par, rows))
    if n_card:
        lens, rows = _draw_group(rng, n, n_card, card_len[0], card_len[1], card_signs)
        if card_t == "half":
            t = np.array([rng.integers(1, max(1, L // 2) + 1) for L in lens])
        elif card_t == "exact_half":
            t = np.maximum(1, lens // 2)
        elif isinstance(card_t, tuple):
            t = rng.integers(card_t[0], card_t[1] + 1, size=n_card)
        else:
            t = np.full(n_card, int(card_t))
        groups.append((KIND_CARD, t, rows))
    inst = assemble(n, groups, name=name)
    m = inst.m
    if isinstance(weights, str) and weights == "uniform":
        inst.weights = rng.uniform(0.5, 1.5, size=m).astype(np.float32)
    elif weights is not None:
        inst.weights = np.asarray(weights, dtype=np.float32)
    return inst


# --------------------------------------------------------------------------
# named workloads
# --------------------------------------------------------------------------

def instance_seed(config: int, i: int = 0) -> int:
    return 1000 * config + i


def point_seed(inst_seed: int) -> int:
    return inst_seed + 500000


def config1(seed: int = 1000) -> Instance:
    """Random 3-SAT, n = 50, m = 213 (clause/variable ratio 4.26)."""
    return random_hybrid(50, seed, n_or=213, or_len=(3, 3), name="3sat-n50-m213")


def config2(seed: int = 2000, weights=None) -> Instance:
    """Mixed: n = 2000; 8000 OR (len 3..7), 500 XOR (len 3..20, positive
    literals, random parity), 200 at-least-t (len 10..100, t ~ U{1..len/2},
    literals all positive or all negative)."""
    return random_hybrid(2000, seed, n_or=8000, or_len=(3, 7), n_xor=500,
                         xor_len=(3, 20), n_card=200, card_len=(10, 100),
                         weights=weights, name="mixed-n2000-m8700")


def config3(seed: int = 3000) -> Instance:
    """Large mixed: n = 100000; 420000 3-SAT + 10000 XOR (len 8..64) +
    2000 at-least-t (len 128..512, t ~ U{1..len/2})."""
    return random_hybrid(100000, seed, n_or=420000, or_len=(3, 3), n_xor=10000,
                         xor_len=(8, 64), n_card=2000, card_len=(128, 512),
                         name="mixed-n100000-m432000")


def config3a(seed: int = 3000) -> Instance:
    """The 3-SAT part of the large instance alone (n = 100000, m = 420000)."""
    return random_hybrid(100000, seed, n_or=420000, or_len=(3, 3),
                         name="3sat-n100000-m420000")


def config4(seed: int = 4000) -> Instance:
    """The mixed n = 2000 shape with weights w ~ U[0.5, 1.5]."""
    return config2(seed, weights="uniform")


RQ1_SHAPES = {
    # name: (n_xor, xor_len, n_card, card_len)
    "xor+card": (800, 8, 1, 32),
    "xor1": (200, 8, 0, 0),
    "xor2": (400, 16, 0, 0),
    "xor3": (800, 32, 0, 0),
    "card1": (0, 0, 50, 8),
    "card2": (0, 0, 100, 16),
    "card3": (0, 0, 200, 32),
}


def rq1(name: str, seed: int = 6000, n: int = 1000) -> Instance:
    """The paper's RQ1 formula shapes (counts and lengths); n and the
    cardinality thresholds are not given there: n = 1000 and t = len/2."""
    nx, lx, nc, lc = RQ1_SHAPES[name]
    return random_hybrid(n, seed, n_xor=nx, xor_len=(lx, lx), n_card=nc,
                         card_len=(lc, lc), card_t="exact_half", name=name)


def points(n: int, B: int, seed: int, dist: str = "uniform",
           dtype=np.float32) -> np.ndarray:
    """x[n][B] in [-1, 1].

    dist: 'uniform'      U[-1, 1];
          'near_corner'  +-0.99 with random signs;
          'corner'       exact +-1;
          'mixed_edge'   uniform with 10% exact +-1, 5% exact 0, 5% +-0.99.
    """
    rng = np.random.default_rng(seed)
    if dist == "uniform":
        x = rng.uniform(-1.0, 1.0, size=(n, B))
    elif dist == "near_corner":
        x = np.where(rng.random((n, B)) < 0.5, -0.99, 0.99)
    elif dist == "corner":
        x = np.where(rng.random((n, B)) < 0.5, -1.0, 1.0)
    elif dist == "mixed_edge":
        x = rng.uniform(-1.0, 1.0, size=(n, B))
        u = rng.random((n, B))
        sgn = np.where(rng.random((n, B)) < 0.5, -1.0, 1.0)
        x = np.where(u < 0.10, sgn, x)
        x = np.where((u >= 0.10) & (u < 0.15), 0.0, x)
        x = np.where((u >= 0.15) & (u < 0.20), 0.99 * sgn, x)
    else:
        raise ValueError(dist)
    return np.ascontiguousarray(x.astype(dtype))


def planted_hybrid(n: int, seed: int, *, n_or=0, or_len=(3, 3), n_xor=0, xor_len=(3, 3),
                   n_card=0, card_len=(10, 10), name="") -> tuple:
    """A hybrid formula satisfied by a hidden assignment (returned with it).

    OR clauses with Bernoulli(1/2) signs are redrawn until the hidden
    assignment satisfies them; XOR constraints take the parity of the hidden
    assignment; at-least-t constraints take the all-positive or all-negative
    sign that the hidden assignment makes more often true, and t ~ U{1..that
    count} (so they hold).  Returns (Instance, hidden bool[n], True = True)."""
    rng = np.random.default_rng(seed)
    hidden = rng.random(n) < 0.5
    groups = []

    def lit_true(lits):
        v = np.abs(lits) - 1
        return np.where(lits > 0, hidden[v], ~hidden[v])

    if n_or:
        _, rows = _draw_group(rng, n, n_or, or_len[0], or_len[1], "bernoulli")
        for i, r in enumerate(rows):
            while not lit_true(r).any():
                r = np.where(rng.random(r.size) < 0.5, -np.abs(r), np.abs(r)).astype(np.int32)
            rows[i] = r
        groups.append((KIND_OR, np.zeros(n_or, np.int32), rows))
    if n_xor:
        _, rows = _draw_group(rng, n, n_xor, xor_len[0], xor_len[1], "positive")
        par = np.array([int(lit_true(r).sum() % 2) for r in rows])
        groups.append((KIND_XOR, par, rows))
    if n_card:
        lens, rows = _draw_group(rng, n, n_card, card_len[0], card_len[1], "positive")
        ts = []
        for i, r in enumerate(rows):
            pos = int(lit_true(np.abs(r)).sum())
            neg = r.size - pos
            if neg > pos:
                rows[i] = (-np.abs(r)).astype(np.int32)
                cnt = neg
            else:
                cnt = pos
            ts.append(int(rng.integers(1, max(1, cnt) + 1)))
        groups.append((KIND_CARD, np.array(ts), rows))
    return assemble(n, groups, name=name or f"planted-n{n}"), hidden


def hidden2_ksat(n: int, seed: int, ratio: float = 4.26, k: int = 3, name="") -> tuple:
    """Satisfiable random k-SAT with two hidden assignments (sigma and its
    complement), the "2-hidden" generator of Achlioptas, Jia and Moore (2005):
    clauses over k distinct variables with Bernoulli(1/2) signs are drawn
    uniformly and kept only if both sigma and not-sigma satisfy them (at least
    one literal true and one false under sigma).  Every variable then occurs
    as often positive as negative in expectation, so, unlike a one-sided
    planted formula, the literal counts say nothing about sigma.
    m = round(ratio * n).  Returns (Instance, sigma bool[n], True = True)."""
    rng = np.random.default_rng(seed)
    sigma = rng.random(n) < 0.5
    m = int(round(ratio * n))
    rows = []
    while len(rows) < m:
        v = rng.choice(n, size=k, replace=False)
        neg = rng.random(k) < 0.5
        true_under_sigma = np.where(neg, ~sigma[v], sigma[v])
        if true_under_sigma.any() and not true_under_sigma.all():
            rows.append(np.where(neg, -(v + 1), v + 1).astype(np.int32))
    return assemble(n, [(KIND_OR, np.zeros(m, np.int32), rows)], name=name or f"hidden2-{k}sat-n{n}"), sigma


def hidden2_hybrid(n: int, seed: int, *, n_or=0, or_len=(3, 3), n_xor=0, xor_len=(3, 3),
                   n_card=0, card_len=(10, 10), name="") -> tuple:
    """A hybrid formula satisfied by a hidden assignment sigma whose literal
    counts carry no hint of sigma (the 2-hidden idea of hidden2_ksat carried
    over to mixed formulas):
      * OR clauses with Bernoulli(1/2) signs are kept only if both sigma and
        its complement satisfy them (some literal true and some false);
      * XOR constraints over positive literals take the parity of sigma;
      * at-least-t constraints have all-positive or all-negative literals
        with probability 1/2 each, drawn independently of sigma, and
        t ~ U{1..floor(len/2)} redrawn from U{1..c} when sigma makes only
        c < t of its literals true (c = 0: the sign is redrawn).
    Returns (Instance, sigma bool[n], True = True)."""
    rng = np.random.default_rng(seed)
    sigma = rng.random(n) < 0.5
    groups = []

    def lit_true(lits):
        v = np.abs(lits) - 1
        return np.where(lits > 0, sigma[v], ~sigma[v])

    if n_or:
        lens = rng.integers(or_len[0], or_len[1] + 1, size=n_or)
        rows = []
        for k in lens:
            while True:
                v = rng.choice(n, size=int(k), replace=False)
                neg = rng.random(int(k)) < 0.5
                r = np.where(neg, -(v + 1), v + 1).astype(np.int32)
                tr = lit_true(r)
                if tr.any() and not tr.all():
                    rows.append(r)
                    break
        groups.append((KIND_OR, np.zeros(n_or, np.int32), rows))
    if n_xor:
        _, rows = _draw_group(rng, n, n_xor, xor_len[0], xor_len[1], "positive")
        par = np.array([int(lit_true(r).sum() % 2) for r in rows])
        groups.append((KIND_XOR, par, rows))
    if n_card:
        lens, rows = _draw_group(rng, n, n_card, card_len[0], card_len[1], "uniform_block")
        ts = []
        for i, r in enumerate(rows):
            cnt = int(lit_true(r).sum())
            while cnt == 0:
                r = -r
                rows[i] = r
                cnt = int(lit_true(r).sum())
            t = int(rng.integers(1, max(1, r.size // 2) + 1))
            if t > cnt:
                t = int(rng.integers(1, cnt + 1))
            ts.append(t)
        groups.append((KIND_CARD, np.array(ts), rows))
    return assemble(n, groups, name=name or f"hidden2-hybrid-n{n}"), sigma


def maxcut_planted(n: int, seed: int, p_in: float = 0.1, p_out: float = 0.3, w_in: float = 1.0,
                   w_out: float = 2.0) -> Instance:
    """Weighted Max-Cut on a planted two-part graph as weighted 2-XOR: edge
    (u, v) is cut iff exactly one endpoint is True, i.e. XOR(u, v) with odd
    parity.  Edges appear with probability p_in inside a part and p_out
    across; weight w_in inside, w_out across (the paper's weighted Max-Cut
    experiments use MaxSAT-evaluation graphs, which are not available: this
    generator stands in for them).  meta["part"] holds the planted parts."""
    rng = np.random.default_rng(seed)
    part = rng.random(n) < 0.5
    rows, wts = [], []
    for u in range(n):
        for v in range(u + 1, n):
            same = part[u] == part[v]
            if rng.random() < (p_in if same else p_out):
                rows.append(np.array([u + 1, v + 1], np.int32))
                wts.append(w_in if same else w_out)
    inst = assemble(n, [(1, np.ones(len(rows), np.int32), rows)], name=f"maxcut_n{n}_s{seed}",
                    weights=np.asarray(wts, np.float32), meta={"part": part})
    return inst


def parity_learning(n: int, seed: int, m: Optional[int] = None, noise: float = 0.25) -> Instance:
    """Learning parity with noise as XOR constraints: a hidden secret s in
    {0,1}^n; m (default 2n) random subsets a (each variable with probability
    1/2, at least one), each an XOR over a whose parity is <a, s> flipped with
    probability `noise`.  Not all constraints can hold; the optimum is the
    assignment satisfying the most.  meta["secret"] (bool, True = True)."""
    rng = np.random.default_rng(seed)
    m = 2 * n if m is None else m
    secret = rng.random(n) < 0.5
    rows, par = [], []
    for _ in range(m):
        a = np.nonzero(rng.random(n) < 0.5)[0]
        if a.size == 0:
            a = np.array([rng.integers(0, n)])
        p = int(secret[a].sum() % 2) ^ int(rng.random() < noise)
        rows.append((a + 1).astype(np.int32))
        par.append(p)
    return assemble(n, [(1, np.asarray(par, np.int32), rows)], name=f"lpn_n{n}_s{seed}",
                    meta={"secret": secret})
