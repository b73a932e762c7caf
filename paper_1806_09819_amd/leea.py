"""Thin Python binding of libleea.so (argument marshalling only).

Every step of the EA runs in the library's HIP kernels; PyTorch supplies the
device memory (workspace, batches, outputs) and the stream.  The library
must be built (``python -m paper_1806_09819_amd.build``); importing this
module does not fall back to anything if it is missing.
"""

import ctypes
import os

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libleea.so")

MAX_LAYERS = 8
OK, EINVAL, ENOMEM, EDEVICE, ESTATE = 0, 1, 2, 3, 4
SEL = {"truncation": 0, "tournament": 1}
XO = {"uniform": 0, "arithmetic": 1}
SIGMA_MODES = {"constant": 0, "decay": 1, "self_adaptive": 2}
EVAL_DTYPES = {"f32": 0, "bf16": 1, "fp8": 2}
OP_ELITE, OP_CROSS, OP_MUT = 0, 1, 2


class LeeaError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("leea status %d: %s" % (status, msg))
        self.status = status


class Config(ctypes.Structure):
    _fields_ = [
        ("n_layers", ctypes.c_int32),
        ("widths", ctypes.c_int32 * (MAX_LAYERS + 1)),
        ("pop", ctypes.c_int32),
        ("n_elite", ctypes.c_int32),
        ("n_cross", ctypes.c_int32),
        ("n_mut", ctypes.c_int32),
        ("n_trunc", ctypes.c_int32),
        ("selection", ctypes.c_int32),
        ("tournament_k", ctypes.c_int32),
        ("crossover", ctypes.c_int32),
        ("sigma", ctypes.c_float),
        ("alpha", ctypes.c_float),
        ("mut_threshold", ctypes.c_uint64),
        ("glorot_a", ctypes.c_float * MAX_LAYERS),
        ("seed", ctypes.c_uint64),
        ("run", ctypes.c_uint32),
        ("max_batch", ctypes.c_int32),
        ("sigma_mode", ctypes.c_int32),
        ("sigma_decay_k", ctypes.c_float),
        ("tau", ctypes.c_float),
        ("input_pool", ctypes.c_int32),
        ("eval_dtype", ctypes.c_int32),
    ]


class SurrogateConfig(ctypes.Structure):
    """leea_surrogate_config."""
    _fields_ = [("oversample", ctypes.c_int32), ("steps", ctypes.c_int32),
                ("lr", ctypes.c_float), ("warmup", ctypes.c_int32), ("tau_min", ctypes.c_float)]


_lib = None


def library():
    """Load libleea.so (after torch, so both share torch's HIP runtime)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("libleea.so is not built: run python -m paper_1806_09819_amd.build")
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.c_void_p
    I32, I64, U32, U64, F = ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_float
    CP = ctypes.POINTER(Config)
    sig = {
        "leea_param_count": [CP, ctypes.POINTER(I64), ctypes.POINTER(I64)],
        "leea_config_from_fractions": [CP, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                       ctypes.c_double, ctypes.c_double],
        "leea_workspace_bytes": [CP, ctypes.POINTER(ctypes.c_size_t)],
        "leea_init_population": [CP, P, ctypes.c_size_t, P, ctypes.POINTER(P)],
        "leea_draw_batch": [P, U32, P, P, I64, I32, P, P],
        "leea_evaluate": [P, P, P, I32, P, P, P],
        "leea_score": [P, P, P, I32, P, P],
        "leea_select": [P, P, P, P],
        "leea_crossover_mutate": [P],
        "leea_step": [P, P, P, I32, P, P, P],
        "leea_set_sigma": [P, F],
        "leea_generation": [P, ctypes.POINTER(U32)],
        "leea_population": [P, ctypes.POINTER(P), ctypes.POINTER(I64), ctypes.POINTER(P)],
        "leea_set_state": [P, P, P, P],
        "leea_state_bytes": [P, ctypes.POINTER(ctypes.c_size_t)],
        "leea_save": [P, P, ctypes.c_size_t],
        "leea_load": [P, P, ctypes.c_size_t],
        "leea_set_fused_step": [P, I32],
        "leea_crossover_mutate_evaluate": [P, P, P, I32, P, P, P],
        "leea_sigmas": [P, ctypes.POINTER(P)],
        "leea_set_sigmas": [P, P],
        "leea_pool2x2": [P, I64, I32, P, P],
        "leea_rng_philox": [P, U64, P, I64, P],
        "leea_rng_ln32": [P, P, I64, P],
        "leea_rng_normal_pairs": [P, P, I64, P],
        "leea_score_noalloc": [CP, P, I64, P, P, I32, P, P, P],
    }
    for name, args in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = ctypes.c_int
    lib.leea_last_error.argtypes = [P]
    lib.leea_last_error.restype = ctypes.c_char_p
    lib.leea_destroy.argtypes = [P]
    lib.leea_destroy.restype = None
    runs_sig = {
        "leea_runs_workspace_bytes": [P, I32, ctypes.POINTER(ctypes.c_size_t)],
        "leea_runs_create": [P, I32, P, ctypes.c_size_t, P, ctypes.POINTER(P)],
        "leea_runs_generation": [P, P, P, I64],
        "leea_runs_set_graph": [P, I32],
        "leea_runs_generation_count": [P, ctypes.POINTER(U32)],
        "leea_runs_population": [P, I32, ctypes.POINTER(P), ctypes.POINTER(I64), ctypes.POINTER(P),
                                 ctypes.POINTER(P), ctypes.POINTER(P)],
        "leea_runs_shape": [P, I32, ctypes.POINTER(I32), ctypes.POINTER(I32)],
        "leea_runs_set_shape": [P, I32, I32, I32],
        "leea_runs_autotune": [P, P, P, I64, P, P, P],
    }
    for name, args in runs_sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = ctypes.c_int
    SP = ctypes.POINTER(SurrogateConfig)
    sur_sig = {
        "leea_surrogate_workspace_bytes": [CP, SP, ctypes.POINTER(ctypes.c_size_t)],
        "leea_surrogate_attach": [P, SP, P, ctypes.c_size_t],
        "leea_surrogate_step": [P, P, P, I32, P, P, P, P],
        "leea_surrogate_views": [P] + [ctypes.POINTER(P)] * 8 + [ctypes.POINTER(I32)],
    }
    for name, args in sur_sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = ctypes.c_int
    lib.leea_runs_last_error.argtypes = [P]
    lib.leea_runs_last_error.restype = ctypes.c_char_p
    lib.leea_runs_destroy.argtypes = [P]
    lib.leea_runs_destroy.restype = None
    _lib = lib
    return lib


def _check(st, ctx=None):
    if st != OK:
        msg = library().leea_last_error(ctx)
        raise LeeaError(st, msg.decode() if msg else "")


# ------------------------------------------------------------ host helpers --

def _fractions_config(pop, widths, p_elite, p_cross, p_mut, rho, p_gene):
    """A Config whose counts, mutation threshold and Glorot bounds come from
    the library's leea_config_from_fractions (section 3.1 rounding)."""
    widths = tuple(int(w) for w in widths)
    L = len(widths) - 1
    if not 1 <= L <= MAX_LAYERS:
        raise ValueError("1..8 weight layers")
    c = Config()
    c.n_layers = L
    for i, w in enumerate(widths):
        c.widths[i] = w
    c.pop = pop
    st = library().leea_config_from_fractions(ctypes.byref(c), p_elite, p_cross, p_mut, rho,
                                              p_gene)
    if st != OK:
        raise ValueError(library().leea_last_error(None).decode())
    return c


def counts(pop, p_elite, p_cross, p_mut, rho):
    """(n_elite, n_cross, n_mut, n_trunc) as the library rounds them."""
    c = _fractions_config(pop, (4, 2), p_elite, p_cross, p_mut, rho, 1.0)
    return c.n_elite, c.n_cross, c.n_mut, c.n_trunc


def threshold(p_gene):
    """The library's 32-bit mutation threshold for a per-gene probability."""
    return _fractions_config(1, (4, 2), 0.0, 0.0, 1.0, 1.0, p_gene).mut_threshold


def make_config(widths, pop, p_elite=0.05, p_cross=0.50, p_mut=0.45, rho=0.5,
                selection="truncation", tournament_k=2, crossover="uniform", sigma=0.001,
                p_gene=1.0, alpha=1.0, seed=0, run=0, max_batch=512, sigma_mode="constant",
                sigma_decay_k=1.0, tau=0.0, pool=0, eval_dtype="f32", **_ignored):
    """leea_config from the paper's hyperparameters (fractions); the integer
    counts, the mutation threshold and the Glorot bounds are filled in by the
    library (leea_config_from_fractions)."""
    c = _fractions_config(pop, widths, p_elite, p_cross, p_mut, rho, p_gene)
    c.selection = SEL[selection]
    c.tournament_k = tournament_k
    c.crossover = XO[crossover]
    c.sigma = sigma
    c.alpha = alpha
    c.seed = seed
    c.run = run
    c.max_batch = max_batch
    c.sigma_mode = SIGMA_MODES[sigma_mode]
    c.sigma_decay_k = sigma_decay_k
    c.tau = tau
    c.input_pool = pool
    c.eval_dtype = EVAL_DTYPES[eval_dtype]
    return c


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


# ------------------------------------------------------------------- ctx --

class Leea:
    """One EA run on the current CUDA (HIP) device and stream."""

    def __init__(self, cfg, device="cuda"):
        lib = library()
        self.cfg = cfg
        self.device = torch.device(device)
        nbytes = ctypes.c_size_t()
        _check(lib.leea_workspace_bytes(ctypes.byref(cfg), ctypes.byref(nbytes)))
        genes, stride = ctypes.c_int64(), ctypes.c_int64()
        _check(lib.leea_param_count(ctypes.byref(cfg), ctypes.byref(genes), ctypes.byref(stride)))
        self.genes, self.stride = genes.value, stride.value
        self.pop = cfg.pop
        self.d = cfg.widths[cfg.n_layers]
        self.workspace = torch.empty(nbytes.value, dtype=torch.uint8, device=self.device)
        ctx = ctypes.c_void_p()
        _check(lib.leea_init_population(ctypes.byref(cfg), _ptr(self.workspace), nbytes.value,
                                        _stream(), ctypes.byref(ctx)))
        self._ctx = ctx

    @classmethod
    def from_params(cls, device="cuda", **kw):
        return cls(make_config(**kw), device=device)

    def close(self):
        if getattr(self, "_ctx", None):
            library().leea_destroy(self._ctx)
            self._ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _out(self, dtype=torch.float32, shape=None):
        return torch.empty(shape if shape is not None else (self.pop,), dtype=dtype,
                           device=self.device)

    def evaluate(self, x, y):
        f_adj, f_raw, acc = self._out(), self._out(), self._out()
        _check(library().leea_evaluate(self._ctx, _ptr(x), _ptr(y), x.shape[0], _ptr(f_adj),
                                       _ptr(f_raw), _ptr(acc)), self._ctx)
        return f_adj, f_raw, acc

    def score(self, x, y):
        f_raw, acc = self._out(), self._out()
        _check(library().leea_score(self._ctx, _ptr(x), _ptr(y), x.shape[0], _ptr(f_raw),
                                    _ptr(acc)), self._ctx)
        return f_raw, acc

    def select(self):
        plan = self._out(torch.int32, (self.pop, 4))
        f_inh = self._out()
        order = self._out(torch.int32)
        _check(library().leea_select(self._ctx, _ptr(plan), _ptr(f_inh), _ptr(order)), self._ctx)
        return plan, f_inh, order

    def crossover_mutate(self):
        _check(library().leea_crossover_mutate(self._ctx), self._ctx)

    def crossover_mutate_evaluate(self, x, y):
        f_adj, f_raw, acc = self._out(), self._out(), self._out()
        _check(library().leea_crossover_mutate_evaluate(self._ctx, _ptr(x), _ptr(y), x.shape[0],
                                                        _ptr(f_adj), _ptr(f_raw), _ptr(acc)),
               self._ctx)
        return f_adj, f_raw, acc

    def step(self, x, y, outputs=True):
        if outputs:
            f_adj, f_raw, acc = self._out(), self._out(), self._out()
        else:
            f_adj = f_raw = acc = None
        _check(library().leea_step(self._ctx, _ptr(x), _ptr(y), x.shape[0], _ptr(f_adj),
                                   _ptr(f_raw), _ptr(acc)), self._ctx)
        return f_adj, f_raw, acc

    def draw_batch(self, gen, x_train, y_train, b, x_out=None, y_out=None):
        if x_out is None:
            x_out = torch.empty((b, self.cfg.widths[0]), dtype=torch.float32, device=self.device)
            y_out = torch.empty((b,), dtype=torch.int32, device=self.device)
        _check(library().leea_draw_batch(self._ctx, gen, _ptr(x_train), _ptr(y_train),
                                         x_train.shape[0], b, _ptr(x_out), _ptr(y_out)), self._ctx)
        return x_out, y_out

    def set_fused_step(self, enable):
        _check(library().leea_set_fused_step(self._ctx, 1 if enable else 0), self._ctx)

    def set_sigma(self, sigma):
        _check(library().leea_set_sigma(self._ctx, sigma), self._ctx)

    @property
    def generation(self):
        g = ctypes.c_uint32()
        _check(library().leea_generation(self._ctx, ctypes.byref(g)), self._ctx)
        return g.value

    def _view(self, ptr, nbytes):
        off = ptr - self.workspace.data_ptr()
        assert 0 <= off and off + nbytes <= self.workspace.numel()
        return self.workspace[off:off + nbytes]

    def population(self):
        """(genomes [pop, stride] float32 view, f_adj [pop] view) -- borrowed."""
        g, f = ctypes.c_void_p(), ctypes.c_void_p()
        stride = ctypes.c_int64()
        _check(library().leea_population(self._ctx, ctypes.byref(g), ctypes.byref(stride),
                                         ctypes.byref(f)), self._ctx)
        genomes = self._view(g.value, self.pop * self.stride * 4).view(torch.float32)
        f_adj = self._view(f.value, self.pop * 4).view(torch.float32)
        return genomes.view(self.pop, self.stride), f_adj

    def sigmas(self):
        """Self-adaptive sigma genes [pop] (borrowed view), or None."""
        ptr = ctypes.c_void_p()
        _check(library().leea_sigmas(self._ctx, ctypes.byref(ptr)), self._ctx)
        if not ptr.value:
            return None
        return self._view(ptr.value, self.pop * 4).view(torch.float32)

    def set_sigmas(self, sig):
        _check(library().leea_set_sigmas(self._ctx, _ptr(sig)), self._ctx)

    def set_state(self, genomes=None, f_adj=None, f_inh=None):
        _check(library().leea_set_state(self._ctx, _ptr(genomes), _ptr(f_adj), _ptr(f_inh)),
               self._ctx)

    # --------------------------------------------------- fitness surrogate --

    def attach_surrogate(self, oversample=4, steps=4, lr=0.01, warmup=2, tau_min=0.2):
        lib = library()
        sc = SurrogateConfig(oversample, steps, lr, warmup, tau_min)
        n = ctypes.c_size_t()
        _check(lib.leea_surrogate_workspace_bytes(ctypes.byref(self.cfg), ctypes.byref(sc),
                                                  ctypes.byref(n)))
        self.sur_workspace = torch.empty(n.value, dtype=torch.uint8, device=self.device)
        _check(lib.leea_surrogate_attach(self._ctx, ctypes.byref(sc), _ptr(self.sur_workspace),
                                         n.value), self._ctx)
        self.sur_cfg = sc

    def surrogate_step(self, x, y):
        """One pre-screened generation: (f_adj, f_raw, acc, stats[4])."""
        f_adj, f_raw, acc = self._out(), self._out(), self._out()
        stats = torch.empty(4, dtype=torch.float32, device=self.device)
        _check(library().leea_surrogate_step(self._ctx, _ptr(x), _ptr(y), x.shape[0],
                                             _ptr(f_adj), _ptr(f_raw), _ptr(acc), _ptr(stats)),
               self._ctx)
        return f_adj, f_raw, acc, stats

    def surrogate_views(self):
        """Borrowed views of the last surrogate step: dict of candidates
        [n, stride], plan [n, 4], features [n, 260], inputs (standardised
        features) [n, 260], pred [n], chosen [pop - n_elite], chosen_pred,
        params [16769]."""
        ptrs = [ctypes.c_void_p() for _ in range(8)]
        n = ctypes.c_int32()
        _check(library().leea_surrogate_views(self._ctx, *[ctypes.byref(q) for q in ptrs],
                                              ctypes.byref(n)), self._ctx)
        M = n.value
        N = self.pop - self.cfg.n_elite
        ws = self.sur_workspace

        def view(ptr, count, dtype, esize):
            off = ptr - ws.data_ptr()
            assert 0 <= off and off + count * esize <= ws.numel()
            return ws[off:off + count * esize].view(dtype)

        return dict(
            candidates=view(ptrs[0].value, M * self.stride, torch.float32, 4).view(M, self.stride),
            plan=view(ptrs[1].value, M * 4, torch.int32, 4).view(M, 4),
            features=view(ptrs[2].value, M * 260, torch.float32, 4).view(M, 260),
            inputs=view(ptrs[3].value, M * 260, torch.float32, 4).view(M, 260),
            pred=view(ptrs[4].value, M, torch.float32, 4),
            chosen=view(ptrs[5].value, N, torch.int32, 4),
            chosen_pred=view(ptrs[6].value, N, torch.float32, 4),
            params=view(ptrs[7].value, 64 * 259 + 2 * 64 + 1, torch.float32, 4))

    def save(self):
        n = ctypes.c_size_t()
        _check(library().leea_state_bytes(self._ctx, ctypes.byref(n)), self._ctx)
        buf = np.empty(n.value, dtype=np.uint8)
        _check(library().leea_save(self._ctx, buf.ctypes.data, n.value), self._ctx)
        return buf

    def load(self, buf):
        buf = np.ascontiguousarray(buf, dtype=np.uint8)
        _check(library().leea_load(self._ctx, buf.ctypes.data, buf.size), self._ctx)


def score_noalloc(cfg, genomes, stride, x, y, f_raw=None, acc=None):
    """leea_score_noalloc: fitness and accuracy of the population in genomes
    ([pop, stride] float32 device tensor) on (x, y) without a ctx; partial
    sums in the library's static device scratch (no allocation there)."""
    pop = cfg.pop
    if f_raw is None:
        f_raw = torch.empty(pop, dtype=torch.float32, device=genomes.device)
    if acc is None:
        acc = torch.empty(pop, dtype=torch.float32, device=genomes.device)
    _check(library().leea_score_noalloc(ctypes.byref(cfg), _ptr(genomes), stride, _ptr(x),
                                        _ptr(y), x.shape[0], _ptr(f_raw), _ptr(acc), _stream()))
    return f_raw, acc


# ------------------------------------------------------ generator checks --

def rng_philox(ctr, key):
    """Philox4x32-10 of device uint32 counters [n, 4] under a 64-bit key."""
    out = torch.empty_like(ctr)
    _check(library().leea_rng_philox(_ptr(ctr), key, _ptr(out), ctr.shape[0], _stream()))
    return out


def pool2x2(x, side):
    """2x2 max-pooling of square images x [n, side*side] on the device."""
    h = side // 2
    out = torch.empty((x.shape[0], h * h), dtype=torch.float32, device=x.device)
    _check(library().leea_pool2x2(_ptr(x), x.shape[0], side, _ptr(out), _stream()))
    return out


def rng_ln32(u):
    out = torch.empty_like(u)
    _check(library().leea_rng_ln32(_ptr(u), _ptr(out), u.numel(), _stream()))
    return out


def rng_normal_pairs(ab):
    z = torch.empty(ab.shape, dtype=torch.float32, device=ab.device)
    _check(library().leea_rng_normal_pairs(_ptr(ab), _ptr(z), ab.shape[0], _stream()))
    return z


# ------------------------------------------------------ many runs at once --

def _rcheck(st, m=None):
    if st != OK:
        msg = library().leea_runs_last_error(m)
        raise LeeaError(st, msg.decode() if msg else "")


class Runs:
    """Many independent EA runs (one leea_config each) advanced together by
    grouped launches replayed from a captured HIP graph.  The runs use their
    own (non-default) stream; sync() waits for it."""

    def __init__(self, cfgs, device="cuda"):
        lib = library()
        self.cfgs = list(cfgs)
        self.n = len(self.cfgs)
        arr = (Config * self.n)(*self.cfgs)
        self._arr = arr
        self.device = torch.device(device)
        nbytes = ctypes.c_size_t()
        _rcheck(lib.leea_runs_workspace_bytes(arr, self.n, ctypes.byref(nbytes)))
        self.workspace = torch.empty(nbytes.value, dtype=torch.uint8, device=self.device)
        self.stream = torch.cuda.Stream(device=self.device)
        torch.cuda.current_stream(self.device).synchronize()
        m = ctypes.c_void_p()
        _rcheck(lib.leea_runs_create(arr, self.n, _ptr(self.workspace), nbytes.value,
                                     ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(m)))
        self._m = m

    def close(self):
        if getattr(self, "_m", None):
            self.sync()
            library().leea_runs_destroy(self._m)
            self._m = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def sync(self):
        self.stream.synchronize()

    def generation(self, x_train, y_train):
        """Generation 0 on the first call, then one generation per call."""
        torch.cuda.current_stream(self.device).synchronize()
        _rcheck(library().leea_runs_generation(self._m, _ptr(x_train), _ptr(y_train),
                                               x_train.shape[0]), self._m)

    def set_graph(self, enable):
        _rcheck(library().leea_runs_set_graph(self._m, 1 if enable else 0), self._m)

    @property
    def generation_count(self):
        g = ctypes.c_uint32()
        _rcheck(library().leea_runs_generation_count(self._m, ctypes.byref(g)), self._m)
        return g.value

    def _view(self, ptr, nbytes):
        off = ptr - self.workspace.data_ptr()
        assert 0 <= off and off + nbytes <= self.workspace.numel()
        return self.workspace[off:off + nbytes]

    def population(self, r):
        """(genomes [pop, stride], f_adj, f_raw, acc) of run r -- borrowed
        views, valid until the next generation (call sync() first)."""
        g, fa, fr, ac = (ctypes.c_void_p() for _ in range(4))
        stride = ctypes.c_int64()
        _rcheck(library().leea_runs_population(self._m, r, ctypes.byref(g), ctypes.byref(stride),
                                               ctypes.byref(fa), ctypes.byref(fr),
                                               ctypes.byref(ac)), self._m)
        pop = self.cfgs[r].pop
        genomes = self._view(g.value, pop * stride.value * 4).view(torch.float32)
        f = [self._view(p.value, pop * 4).view(torch.float32) for p in (fa, fr, ac)]
        return (genomes.view(pop, stride.value), *f)

    def shape(self, r):
        k, mw = ctypes.c_int32(), ctypes.c_int32()
        _rcheck(library().leea_runs_shape(self._m, r, ctypes.byref(k), ctypes.byref(mw)), self._m)
        return k.value, mw.value

    def set_shape(self, r, kind, mw):
        _rcheck(library().leea_runs_set_shape(self._m, r, kind, mw), self._m)

    def autotune(self, x_train, y_train):
        """Pick the fastest evaluation shape per (pop, widths, batch, dtype);
        returns (kind[n], mw[n], microseconds[n])."""
        kind = np.zeros(self.n, dtype=np.int32)
        mw = np.zeros(self.n, dtype=np.int32)
        us = np.zeros(self.n, dtype=np.float32)
        torch.cuda.current_stream(self.device).synchronize()
        _rcheck(library().leea_runs_autotune(self._m, _ptr(x_train), _ptr(y_train),
                                             x_train.shape[0], kind.ctypes.data, mw.ctypes.data,
                                             us.ctypes.data), self._m)
        return kind, mw, us
