"""The limited-evaluation EA of the paper, step by step (oracle side).

Follows Algorithm 1 (section 3.1) in its own order:
  initialise lambda networks; then per generation draw a batch, sort the
  population by fitness (descending), take the elites, draw crossover parent
  pairs and mutation parents from the top rho*lambda by truncation selection,
  apply crossover and mutation, form the new population and evaluate it.

Readings of points the paper leaves open (each is also listed in the design
notes):
* The sort needs fitness before any evaluation exists, so the initial
  population is evaluated once on a generation-0 batch; every generation
  then ranks on the previous fitness and evaluates the new population on
  its own batch.
* Fractions p*lambda are rounded half up; mutation takes the remainder.
* Parent pairs are two independent uniform draws from the top n_rho (with
  replacement, both may be the same network).
* Inherited fitness uses the parents' adjusted fitness; elites inherit their
  own.
* Ties in the sort are broken by slot index; -0 equals +0; NaN ranks last.
* Fitness is the left-hand side of Eq. 1 (mean log-likelihood of the true
  class); the right-hand side differs by the constant factor 1/d.
* Biases start at zero; only weights are Glorot-uniform.

Nothing here is fast.  Forward pass and fitness are float64; the genetic
operators are float32 op by op (see ``normal32``) so that they can be
compared bit for bit.
"""

from dataclasses import dataclass, field
from fractions import Fraction
import math

import numpy as np

from . import philox
from .normal32 import exp32, normal_pair, normals4

F32 = np.float32

ELITE, CROSS, MUT = 0, 1, 2


# ---------------------------------------------------------------- config ---

@dataclass
class Config:
    """Hyperparameters of one EA run (section 4 lists the paper defaults)."""
    widths: tuple                 # (n0, n1, ..., nL): input dim ... classes
    pop: int = 1000               # lambda
    p_elite: float = 0.05
    p_cross: float = 0.50
    p_mut: float = 0.45
    rho: float = 0.50             # truncation selection proportion
    selection: str = "truncation"  # or "tournament" (not in the paper)
    tournament_k: int = 2
    crossover: str = "uniform"    # or "arithmetic"
    sigma: float = 0.001
    p_gene: float = 1.0           # per-gene mutation probability (1 = paper)
    alpha: float = 1.0            # fitness-inheritance weight (1 = off)
    sigma_mode: str = "constant"  # "constant", "decay" or "self_adaptive" (section 3.2)
    sigma_decay_k: float = 1.0    # k of sigma_i = sigma * 0.99**(i/k)
    tau: float = 0.0              # self-adaptation rate (0 -> 1/sqrt(c))
    pool: int = 0                 # 2: 2x2 max-pool of square image inputs (section 4.1)
    seed: int = 0
    run: int = 0
    extra: dict = field(default_factory=dict)


def counts(pop, p_elite, p_cross, p_mut, rho):
    """Integer numbers of elites, crossover and mutation offspring, and n_rho.

    Algorithm 1 takes p_E*lambda elites, p_C*lambda pairs and p_M*lambda
    mutants from the top rho*lambda.  Products are rounded half up, the
    mutants take the remainder so the three always sum to lambda.
    """
    if pop < 1:
        raise ValueError("population must be positive")
    if abs(p_elite + p_cross + p_mut - 1.0) > 1e-9:
        raise ValueError("p_E + p_C + p_M must equal 1")
    n_e = int(math.floor(p_elite * pop + 0.5))
    n_c = int(math.floor(p_cross * pop + 0.5))
    n_m = pop - n_e - n_c
    if n_e < 0 or n_c < 0 or n_m < 0:
        raise ValueError("counts do not fit the population")
    n_rho = min(max(int(math.floor(rho * pop + 0.5)), 1), pop)
    return n_e, n_c, n_m, n_rho


def mutation_threshold(p_gene):
    """Gene is mutated iff its 32-bit draw is below floor(p * 2**32)."""
    if not 0.0 <= p_gene <= 1.0:
        raise ValueError("p_gene must be in [0, 1]")
    return min(1 << 32, int(math.floor(Fraction(p_gene) * (1 << 32))))


# ---------------------------------------------------------------- layout ---

def layer_slices(widths):
    """Gene index ranges of every layer's weight matrix and bias vector.

    Layer l (1-based) holds W_l with shape [n_l, n_{l-1}] row-major, then
    b_l with n_l entries; layers follow each other in order.
    """
    out = []
    off = 0
    for l in range(1, len(widths)):
        n_in, n_out = widths[l - 1], widths[l]
        w = (off, off + n_in * n_out)
        off = w[1]
        b = (off, off + n_out)
        off = b[1]
        out.append((w, b))
    return out


def param_count(widths):
    """Total number of parameters c of one directly encoded network."""
    return sum(widths[l - 1] * widths[l] + widths[l] for l in range(1, len(widths)))


def unpack(genome, widths):
    """List of (W_l, b_l) views of one genome."""
    layers = []
    for l, ((w0, w1), (b0, b1)) in enumerate(layer_slices(widths), start=1):
        W = genome[w0:w1].reshape(widths[l], widths[l - 1])
        layers.append((W, genome[b0:b1]))
    return layers


def glorot_bound(n_in, n_out):
    """Glorot-uniform limit sqrt(6 / (fan_in + fan_out)) (section 4.1)."""
    return F32(math.sqrt(6.0 / (n_in + n_out)))


# ------------------------------------------------------------------ init ---

def init_population(cfg, slots=None):
    """lambda networks with independent Glorot-uniform weights, zero biases.

    Gene i of slot j draws word (i & 3) of Philox block (INIT, gen 0, slot j,
    block i >> 2); u = (word >> 8) * 2**-24 in [0, 1) and the weight is
    (2u - 1) * a_l in float32.  ``slots`` restricts the output to those
    slots (rows in the given order).
    """
    widths = tuple(cfg.widths)
    c = param_count(widths)
    slots = range(cfg.pop) if slots is None else list(slots)
    pop = np.zeros((len(slots), c), dtype=F32)
    genes = np.arange(c, dtype=np.int64)
    for row, j in enumerate(slots):
        words = philox.draw(cfg.seed, philox.INIT, 0, j, genes >> 2, cfg.run)
        w = words[genes, genes & 3]
        u = (w >> np.uint32(8)).astype(F32) * F32(2.0 ** -24)
        t = F32(2.0) * u
        t = t - F32(1.0)
        for l, ((w0, w1), _b) in enumerate(layer_slices(widths), start=1):
            a = glorot_bound(widths[l - 1], widths[l])
            pop[row, w0:w1] = t[w0:w1] * a
    return pop


# --------------------------------------------------------------- forward ---

def forward(genome, widths, x):
    """Logits of one network on a batch, float64.

    h_0 = x; h_l = ReLU(h_{l-1} W_l^T + b_l) for every layer but the last,
    which has no ReLU (section 4.1; softmax is part of the fitness).
    """
    h = np.asarray(x, dtype=np.float64)
    layers = unpack(np.asarray(genome), widths)
    for l, (W, b) in enumerate(layers):
        h = h @ W.astype(np.float64).T + b.astype(np.float64)
        if l < len(layers) - 1:
            h = np.maximum(h, 0.0)
    return h


def fitness_from_logits(z, y):
    """Negative mean cross-entropy (Eq. 1, left-hand side) and accuracy.

    ll_i = (z_{i,y_i} - m_i) - log sum_k exp(z_ik - m_i) with m_i = max_k z_ik;
    fitness = mean_i ll_i.  Accuracy counts argmax_k z_ik == y_i with the
    lowest class index winning ties.
    """
    z = np.asarray(z, dtype=np.float64)
    y = np.asarray(y, dtype=np.int64)
    n = z.shape[0]
    if n == 0:
        raise ValueError("empty batch")
    m = z.max(axis=1)
    lse = np.log(np.exp(z - m[:, None]).sum(axis=1))
    ll = (z[np.arange(n), y] - m) - lse
    f = ll.sum() / n
    acc = float(np.count_nonzero(np.argmax(z, axis=1) == y)) / n
    return f, acc


def fitness_rhs_scale(f, d):
    """Eq. 1 printed right-hand side: the same quantity divided by d."""
    return f / d


def evaluate(pop, widths, x, y):
    """Raw fitness and accuracy of every network on batch (x, y), float64."""
    P = pop.shape[0]
    f = np.empty(P, dtype=np.float64)
    acc = np.empty(P, dtype=np.float64)
    for j in range(P):
        f[j], acc[j] = fitness_from_logits(forward(pop[j], widths, x), y)
    return f, acc


def evaluate_logits(pop, widths, x):
    """All logits [P, b, d] (float64), for per-sample checks."""
    return np.stack([forward(pop[j], widths, x) for j in range(pop.shape[0])])


# ----------------------------------------------------------- inheritance ---

def inherit(f_raw, f_inh, alpha, has_inh=True):
    """f_adj = (1 - alpha) * f_inh + alpha * fitness (section 3.1).

    alpha = 1 disables inheritance (f_adj = fitness); before the first
    selection there is nothing to inherit and f_adj = fitness.
    """
    f_raw = np.asarray(f_raw, dtype=np.float64)
    if not has_inh or alpha == 1.0:
        return f_raw.copy()
    return (1.0 - alpha) * np.asarray(f_inh, dtype=np.float64) + alpha * f_raw


def inherit_f32(f_raw, f_inh, alpha, has_inh=True):
    """The same weighted sum in float32 with a fixed operation order:
    fl(fl(fl(1 - alpha) * f_inh) + fl(alpha * fitness))."""
    f_raw = np.asarray(f_raw, dtype=F32)
    a = F32(alpha)
    if not has_inh or a == F32(1.0):
        return f_raw.copy()
    oma = F32(1.0) - a
    return (oma * np.asarray(f_inh, dtype=F32) + a * f_raw).astype(F32)


# ------------------------------------------------------------------ rank ---

def rank(f_adj):
    """Slots ordered by fitness, best first (Algorithm 1, the sort).

    Ties keep slot order; -0 and +0 tie; NaN ranks after every number.
    """
    f = np.asarray(f_adj)
    nan = np.isnan(f)
    negf = np.where(nan, 0.0, -f.astype(np.float64))
    idx = np.arange(f.shape[0])
    return np.lexsort((idx, negf, nan)).astype(np.int64)


# ------------------------------------------------------------------ plan ---

def _word(seed, gen, slot, widx, run):
    """32-bit selection word number ``widx`` for slot ``slot``."""
    blk = philox.draw(seed, philox.SEL, gen, slot, widx >> 2, run)
    return int(blk[widx & 3])


def _parent_rank(cfg, n_rho, gen, slot, p):
    """Rank (0 = best) of parent p (0 or 1) of offspring ``slot``."""
    if cfg.selection == "truncation":
        w = _word(cfg.seed, gen, slot, p, cfg.run)
        return (w * n_rho) >> 32
    if cfg.selection == "tournament":
        k = cfg.tournament_k
        ranks = [(_word(cfg.seed, gen, slot, p * k + c, cfg.run) * cfg.pop) >> 32
                 for c in range(k)]
        return min(ranks)
    raise ValueError(cfg.selection)


def plan(order, f_adj, cfg, gen):
    """Operator and parents of every offspring slot, and its inherited fitness.

    Slots [0, n_E) are elites (slot j copies rank j), the next n_C slots are
    crossover children, the rest mutants (Algorithm 1).  Truncation selection
    draws a rank uniformly from [0, n_rho) as floor(word * n_rho / 2**32).
    Tournament selection (not in the paper) draws k ranks uniformly from the
    whole population and keeps the best.

    Returns (ops, p1, p2, f_inh); if f_adj is float32, f_inh is computed in
    float32 as fl(fl(f1 + f2) * 0.5) for crossover.
    """
    n_e, n_c, n_m, n_rho = counts(cfg.pop, cfg.p_elite, cfg.p_cross, cfg.p_mut, cfg.rho)
    P = cfg.pop
    order = np.asarray(order)
    f_adj = np.asarray(f_adj)
    f32 = f_adj.dtype == F32
    ops = np.empty(P, dtype=np.int32)
    p1 = np.empty(P, dtype=np.int64)
    p2 = np.empty(P, dtype=np.int64)
    f_inh = np.empty(P, dtype=F32 if f32 else np.float64)
    for j in range(P):
        if j < n_e:
            ops[j] = ELITE
            p1[j] = p2[j] = order[j]
            f_inh[j] = f_adj[p1[j]]
        elif j < n_e + n_c:
            ops[j] = CROSS
            p1[j] = order[_parent_rank(cfg, n_rho, gen, j, 0)]
            p2[j] = order[_parent_rank(cfg, n_rho, gen, j, 1)]
            if f32:
                f_inh[j] = (F32(f_adj[p1[j]]) + F32(f_adj[p2[j]])) * F32(0.5)
            else:
                f_inh[j] = 0.5 * (f_adj[p1[j]] + f_adj[p2[j]])
        else:
            ops[j] = MUT
            p1[j] = p2[j] = order[_parent_rank(cfg, n_rho, gen, j, 0)]
            f_inh[j] = f_adj[p1[j]]
    return ops, p1, p2, f_inh


# ------------------------------------------------------------------ vary ---

def uniform_mask(seed, gen, slot, c, run=0):
    """Uniform-crossover choice of every gene (True = take parent 2).

    Gene i = 8192 G + 256 t + 4 q + e (t < 32, q < 64, e < 4) takes bit
    4 (t mod 8) + e of word t // 8 of Philox block (XO, gen, slot, 64 G + q).
    Each gene's bit is a fair coin (section 3.2, uniform crossover).
    """
    i = np.arange(c, dtype=np.int64)
    G = i >> 13
    t = (i >> 8) & 31
    q = (i >> 2) & 63
    e = i & 3
    blocks = np.arange(((c + 8191) >> 13) * 64, dtype=np.int64)
    words = philox.draw(seed, philox.XO, gen, slot, blocks, run)
    w = words[G * 64 + q, t >> 3]
    return ((w >> (4 * (t & 7) + e).astype(np.uint32)) & np.uint32(1)).astype(bool)


def mutation_parts(seed, gen, slot, c, threshold, run=0):
    """Which genes mutate, and their standard normal draws.

    Gene i is mutated iff word (i & 3) of block (MUTMASK, gen, slot, i >> 2)
    is below the threshold (always, at threshold 2**32); its normal is number
    (i & 3) of the four drawn from block (MUTNORM, gen, slot, i >> 2).
    """
    blocks = np.arange((c + 3) >> 2, dtype=np.int64)
    if threshold >= (1 << 32):
        mutated = np.ones(c, dtype=bool)
    else:
        mw = philox.draw(seed, philox.MUTMASK, gen, slot, blocks, run).reshape(-1)[:c]
        mutated = mw.astype(np.uint64) < np.uint64(threshold)
    z = normals4(philox.draw(seed, philox.MUTNORM, gen, slot, blocks, run)).reshape(-1)[:c]
    return mutated, z


def vary(pop, ops, p1, p2, cfg, gen, sigma=None, slots=None):
    """New population from the plan (Algorithm 1: E, C', M' and their union).

    Elites are copied unchanged.  Crossover children are not mutated.
    Uniform crossover takes each gene from one parent by a fair coin;
    arithmetic crossover is fl(fl(t1 + t2) * 0.5); mutation adds
    fl(sigma * z) to each mutated gene (section 3.2).  ``slots`` restricts
    the output to those offspring slots (rows in the given order).
    """
    sigma = F32(cfg.sigma if sigma is None else sigma)
    threshold = mutation_threshold(cfg.p_gene)
    P, c = pop.shape
    slots = range(len(ops)) if slots is None else list(slots)
    out = np.empty((len(slots), c), dtype=pop.dtype)
    for row, j in enumerate(slots):
        out[row] = _child(pop, ops, p1, p2, cfg, gen, sigma, threshold, j, c)
    return out


def _child(pop, ops, p1, p2, cfg, gen, sigma, threshold, j, c, slot=None):
    """Offspring of slot j (one row of ``vary``); its random draws use slot
    ``slot`` (default j) of the generation's streams."""
    s = j if slot is None else slot
    a = pop[p1[j]]
    if ops[j] == ELITE:
        return a.copy()
    if ops[j] == CROSS:
        b = pop[p2[j]]
        if cfg.crossover == "uniform":
            return np.where(uniform_mask(cfg.seed, gen, s, c, cfg.run), b, a)
        if cfg.crossover == "arithmetic":
            return (a + b) * F32(0.5)
        raise ValueError(cfg.crossover)
    mutated, z = mutation_parts(cfg.seed, gen, s, c, threshold, cfg.run)
    noise = sigma * z
    return np.where(mutated, a + noise, a)


# ------------------------------------------------------------ sigma ---

def sigma_decay(sigma, gen, k):
    """Exponentially decaying mutation strength sigma_i = sigma * 0.99**(i/k)
    (section 3.2) for the mutation that creates generation ``gen``.  sigma and
    k are float32 hyperparameters; the product is formed in float64 and
    rounded once to float32."""
    return F32(float(F32(sigma)) * math.pow(0.99, gen / float(F32(k))))


def default_tau(widths):
    """Self-adaptation rate when none is given: 1/sqrt(c), c = genes."""
    return 1.0 / math.sqrt(param_count(widths))


def child_sigmas(sig, ops, p1, p2, cfg, gen):
    """Per-individual sigma genes of the next population (section 3.2,
    self-adaptive control): elites keep theirs; crossover children take the
    mean fl(fl(s1 + s2) * 0.5); mutants take fl(s * exp32(fl(tau * z))) with z
    the first normal of the pair from block (SIGMA, gen, slot, 0)."""
    tau = F32(cfg.tau if cfg.tau > 0 else default_tau(cfg.widths))
    sig = np.asarray(sig, dtype=F32)
    out = np.empty(len(ops), dtype=F32)
    for j in range(len(ops)):
        if ops[j] == ELITE:
            out[j] = sig[p1[j]]
        elif ops[j] == CROSS:
            out[j] = (sig[p1[j]] + sig[p2[j]]) * F32(0.5)
        else:
            w = philox.draw(cfg.seed, philox.SIGMA, gen, j, 0, cfg.run)
            z, _ = normal_pair(w[0], w[1])
            out[j] = sig[p1[j]] * exp32(tau * F32(z))
    return out


def vary_adaptive(pop, sig_new, ops, p1, p2, cfg, gen, slots=None):
    """vary() where each mutant uses its own (already adapted) sigma gene."""
    threshold = mutation_threshold(cfg.p_gene)
    P, c = pop.shape
    slots = range(len(ops)) if slots is None else list(slots)
    out = np.empty((len(slots), c), dtype=pop.dtype)
    for row, j in enumerate(slots):
        out[row] = _child(pop, ops, p1, p2, cfg, gen, F32(sig_new[j]), threshold, j, c)
    return out


# ----------------------------------------------------------- pooling ---

def pool2x2(x, side):
    """2x2 max-pooling of square images x [n][side*side] -> [n][(side/2)**2]
    (section 4.1: the network max-pools its 28x28 inputs first)."""
    x = np.asarray(x)
    n = x.shape[0]
    h = side // 2
    return x.reshape(n, h, 2, h, 2).max(axis=(2, 4)).reshape(n, h * h)


# ----------------------------------------------------------------- batch ---

def batch_indices(seed, gen, b, n_train, run=0):
    """Example k of generation gen's batch: floor(word * N / 2**32) where word
    is number (k & 3) of block (BATCH, gen, slot 0, k >> 2); drawn with
    replacement (Algorithm 1, random batch)."""
    k = np.arange(b, dtype=np.int64)
    words = philox.draw(seed, philox.BATCH, gen, 0, k >> 2, run)
    w = words[k, k & 3].astype(np.uint64)
    return ((w * np.uint64(n_train)) >> np.uint64(32)).astype(np.int64)


# ------------------------------------------------------------------ loop ---

def run(cfg, x_train, y_train, generations, batch, teacher=None, log=None):
    """Run Algorithm 1 for ``generations`` generations after generation 0.

    teacher: optional callable(gen, f_adj_oracle) -> f_adj used for ranking
    (teacher forcing with another implementation's float32 fitness).
    Returns the final population, f_adj and a per-generation history.
    """
    widths = tuple(cfg.widths)
    n_train = x_train.shape[0]
    pop = init_population(cfg)
    idx = batch_indices(cfg.seed, 0, batch, n_train, cfg.run)
    f_raw, acc = evaluate(pop, widths, x_train[idx], y_train[idx])
    f_adj = inherit(f_raw, None, cfg.alpha, has_inh=False)
    hist = [dict(gen=0, f_raw=f_raw, acc=acc, f_adj=f_adj)]
    for g in range(1, generations + 1):
        idx = batch_indices(cfg.seed, g, batch, n_train, cfg.run)
        f_rank = teacher(g - 1, f_adj) if teacher is not None else f_adj
        order = rank(f_rank)
        ops, p1, p2, f_inh = plan(order, f_rank, cfg, g)
        pop = vary(pop, ops, p1, p2, cfg, g)
        f_raw, acc = evaluate(pop, widths, x_train[idx], y_train[idx])
        f_adj = inherit(f_raw, f_inh, cfg.alpha, has_inh=True)
        rec = dict(gen=g, order=order, ops=ops, p1=p1, p2=p2, f_inh=f_inh,
                   f_raw=f_raw, acc=acc, f_adj=f_adj)
        hist.append(rec)
        if log is not None:
            log(rec)
    return pop, f_adj, hist
