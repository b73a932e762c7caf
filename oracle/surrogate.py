"""Learned fitness surrogate that pre-screens over-generated offspring
(oracle side; test infrastructure only).

A variant of the generation of Algorithm 1 (section 3.1) that spends
cheap predictions instead of evaluations:

* the n_E elites are kept as usual; k * (P - n_E) candidate children are
  made instead of P - n_E: the first k * n_C by crossover, the rest by
  mutation, each with its parents and random draws taken from slot P + c
  of the generation's streams (candidate c), with the paper's selection
  and operators (sections 3.1, 3.2);
* every candidate gets features: a fixed random projection of its genome
  (256 rows of +-1 signs, the genome rounded to bfloat16, times 1/sqrt(g)
  for g genes), its parents' adjusted fitness, and its distance to parent 1
  (Euclidean, times 1/sqrt(g));
* the MLP sees every feature standardised over the generation's candidates
  (minus its mean over them, divided by its standard deviation; a feature
  that does not vary is 0): the projections of children of similar parents
  differ from each other far less than from zero, and the parents' fitness
  drifts from generation to generation, so raw values would leave the MLP
  chasing a moving offset;
* a two-layer MLP (259 -> 64 ReLU -> 1) predicts each candidate's
  standardised fitness; the P - n_E best predictions (descending, ties by
  candidate index, NaN last) fill the non-elite slots in that order;
* the new population is evaluated as usual (its fitness judges the
  surrogate), and the MLP takes full-batch gradient steps on the mean
  squared error between its predictions and those fitness values
  standardised over the kept candidates (a ranking is all the screen uses,
  and it does not change under that affine map);
* until the MLP has trained for `warmup` generations and its Kendall tau
  (tau-a) between predicted and evaluated fitness in the previous
  generation reaches tau_min, the pre-screening is off and the first n_C
  crossover and first n_M mutation candidates are kept (plain LEEA's mix).

Everything here is float64 except what the genetic operators and the
stored parameters fix in float32.
"""

import math

import numpy as np

from . import leea as L
from . import philox
from .precision import round_bf16

F32 = np.float32
FEATURES = 256
HIDDEN = 64
INPUTS = FEATURES + 3


def projection_signs(genes, seed, run=0, rows=FEATURES):
    """R[r][i] = +1 or -1: bit (i mod 32) of word (i >> 5) mod 4 of Philox
    block (SURR, generation 0, slot r, i >> 7); a set bit gives -1."""
    R = np.empty((rows, genes), dtype=np.int8)
    i = np.arange(genes)
    blocks = (genes + 127) // 128
    for r in range(rows):
        w = np.array([philox.draw(seed, philox.SURR, 0, r, blk, run) for blk in range(blocks)],
                     dtype=np.uint64)                         # [blocks][4]
        words = w[i >> 7, (i >> 5) & 3]
        bits = (words >> (i & 31).astype(np.uint64)) & np.uint64(1)
        R[r] = np.where(bits == 1, -1, 1)
    return R


def scale(genes):
    """The float32 constant 1/sqrt(g) applied to projections and distances."""
    return F32(1.0 / math.sqrt(genes))


def features(children, parents1, f_p1, f_p2, R):
    """[n][259] features (float64): projection of the bfloat16-rounded child
    genome, the parents' adjusted fitness, and the scaled distance to
    parent 1."""
    children = np.asarray(children, dtype=F32)
    g = children.shape[1]
    s = float(scale(g))
    proj = (round_bf16(children).astype(np.float64) @ R.T.astype(np.float64)) * s
    d = children.astype(np.float64) - np.asarray(parents1, dtype=F32).astype(np.float64)
    nu = np.sqrt(np.sum(d * d, axis=1)) * s
    return np.concatenate([proj, np.asarray(f_p1, dtype=np.float64)[:, None],
                           np.asarray(f_p2, dtype=np.float64)[:, None], nu[:, None]], axis=1)


def standardize(X):
    """Each column minus its mean over the rows, divided by its standard
    deviation (over the rows, no Bessel correction); a column whose standard
    deviation is 0 becomes 0 (float64)."""
    X = np.asarray(X, dtype=np.float64)
    mu = X.mean(axis=0)
    sd = np.sqrt(((X - mu) ** 2).mean(axis=0))
    safe = np.where(sd > 0, sd, 1.0)
    return np.where(sd > 0, (X - mu) / safe, 0.0)


def mlp_inputs(X):
    """The MLP's inputs: every feature standardised over the generation's
    candidates (`standardize`), then the FEATURES projection columns scaled
    by 1/sqrt(FEATURES) = 2^-4, so that the projection block weighs as much
    as one scalar feature (its mean squared norm per candidate is 1, where
    every projection varies).  The factor is a power of two, so the scaling
    is exact."""
    Z = standardize(X)
    Z[:, :FEATURES] *= 1.0 / math.sqrt(FEATURES)
    return Z


def standardize_targets(y):
    """Training targets: the finite entries minus their mean, divided by their
    standard deviation (1 if it is 0); non-finite entries stay as they are
    (the gradient step leaves them out)."""
    y = np.asarray(y, dtype=np.float64)
    ok = np.isfinite(y)
    if not ok.any():
        return y.copy()
    mu = y[ok].mean()
    sd = math.sqrt(((y[ok] - mu) ** 2).mean())
    sd = sd if sd > 0 else 1.0
    return np.where(ok, (y - mu) / sd, y)


def init_mlp(seed, run=0):
    """Glorot-uniform first and second layers from Philox (SURR, generation
    1, slot h: input weights of hidden unit h; generation 2, slot 0: output
    weights), zero biases; every weight fl32(fl32(2u - 1) * a) with
    u = (w >> 8) 2^-24 as in the population's initialisation (section 4.1)."""
    a1 = F32(math.sqrt(6.0 / (INPUTS + HIDDEN)))
    a2 = F32(math.sqrt(6.0 / (HIDDEN + 1)))

    def u(word):
        return F32(int(word) >> 8) * F32(2.0 ** -24)

    W1 = np.empty((HIDDEN, INPUTS), dtype=F32)
    for h in range(HIDDEN):
        for d in range(INPUTS):
            w = philox.draw(seed, philox.SURR, 1, h, d >> 2, run)[d & 3]
            W1[h, d] = (F32(2.0) * u(w) - F32(1.0)) * a1
    w2 = np.empty(HIDDEN, dtype=F32)
    for h in range(HIDDEN):
        w = philox.draw(seed, philox.SURR, 2, 0, h >> 2, run)[h & 3]
        w2[h] = (F32(2.0) * u(w) - F32(1.0)) * a2
    return dict(W1=W1, b1=np.zeros(HIDDEN, dtype=F32), w2=w2, b2=F32(0.0))


def mlp_forward(params, X):
    """Predictions (float64) and the hidden pre-activations."""
    X = np.asarray(X, dtype=np.float64)
    pre = X @ params["W1"].astype(np.float64).T + params["b1"].astype(np.float64)
    h = np.maximum(pre, 0.0)
    return h @ params["w2"].astype(np.float64) + float(params["b2"]), pre


def mlp_gradient_step(params, X, y, lr):
    """One full-batch gradient step on mean((pred - y)^2) over the rows
    whose target is a number; returns new float64 parameters."""
    X = np.asarray(X, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    ok = np.isfinite(y)
    X, y = X[ok], y[ok]
    n = len(y)
    p = {k: np.asarray(v, dtype=np.float64) for k, v in params.items()}
    if n == 0:
        return p
    pred, pre = mlp_forward(p, X)
    h = np.maximum(pre, 0.0)
    e = (2.0 / n) * (pred - y)                      # dL/dpred
    g_w2 = h.T @ e
    g_b2 = e.sum()
    dh = np.outer(e, p["w2"]) * (pre > 0)
    g_W1 = dh.T @ X
    g_b1 = dh.sum(axis=0)
    return dict(W1=p["W1"] - lr * g_W1, b1=p["b1"] - lr * g_b1, w2=p["w2"] - lr * g_w2,
                b2=p["b2"] - lr * g_b2)


def kendall_tau_a(a, b):
    """(concordant - discordant) / (n (n - 1) / 2) over all pairs; a pair
    tied in either list counts as neither; pairs with a non-number are
    left out of both counts (the denominator counts every pair)."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    n = len(a)
    if n < 2:
        return 0.0
    da = np.sign(a[:, None] - a[None, :])
    db = np.sign(b[:, None] - b[None, :])
    prod = np.nan_to_num(da * db, nan=0.0)
    s = np.triu(prod, 1).sum()
    return float(s) / (n * (n - 1) / 2)


def candidate_plan(order, f_adj, cfg, gen, k):
    """Operators, parents and inherited fitness of the k (P - n_E)
    candidates (slot P + c of the selection stream for candidate c)."""
    n_e, n_c, n_m, n_rho = L.counts(cfg.pop, cfg.p_elite, cfg.p_cross, cfg.p_mut, cfg.rho)
    P = cfg.pop
    M = k * (P - n_e)
    order = np.asarray(order)
    f_adj = np.asarray(f_adj, dtype=F32)
    ops = np.empty(M, dtype=np.int32)
    p1 = np.empty(M, dtype=np.int64)
    p2 = np.empty(M, dtype=np.int64)
    f_inh = np.empty(M, dtype=F32)
    for c in range(M):
        slot = P + c
        if c < k * n_c:
            ops[c] = L.CROSS
            p1[c] = order[L._parent_rank(cfg, n_rho, gen, slot, 0)]
            p2[c] = order[L._parent_rank(cfg, n_rho, gen, slot, 1)]
            f_inh[c] = (f_adj[p1[c]] + f_adj[p2[c]]) * F32(0.5)
        else:
            ops[c] = L.MUT
            p1[c] = p2[c] = order[L._parent_rank(cfg, n_rho, gen, slot, 0)]
            f_inh[c] = f_adj[p1[c]]
    return ops, p1, p2, f_inh


def candidates(pop, ops, p1, p2, cfg, gen):
    """The candidate genomes (random draws of candidate c from slot P + c)."""
    threshold = L.mutation_threshold(cfg.p_gene)
    sigma = F32(cfg.sigma)
    P, g = pop.shape
    out = np.empty((len(ops), g), dtype=F32)
    for c in range(len(ops)):
        out[c] = L._child(pop, ops, p1, p2, cfg, gen, sigma, threshold, c, g, slot=P + c)
    return out


def screen(pred, n_keep, use, k, n_c, n_m):
    """Indices of the kept candidates, in slot order."""
    if not use:
        return np.concatenate([np.arange(n_c), k * n_c + np.arange(n_m)]).astype(np.int64)
    order = L.rank(np.asarray(pred, dtype=F32))        # descending, ties by index, NaN last
    return order[:n_keep].astype(np.int64)
