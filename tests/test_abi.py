"""CPU checks of the C-ABI library: it loads, exports every entry point that
include/leea.h declares, and rejects bad arguments on the host before any
device work (no compute calls here)."""
import ctypes
import os
import re

import pytest

from paper_1806_09819_amd import leea as B
from oracle import leea as O

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(B.LIB_PATH):
        from paper_1806_09819_amd import build
        build.build()
    return B.library()


def declared_functions():
    names = set()
    for h in os.listdir(os.path.join(ROOT, "include")):
        if h.endswith(".h"):
            with open(os.path.join(ROOT, "include", h)) as fh:
                text = fh.read()
            names |= set(re.findall(r"\b(leea_[a-z0-9_]+)\s*\(", text))
    return names


def test_exports_every_declared_symbol(lib):
    names = declared_functions()
    assert {"leea_init_population", "leea_evaluate", "leea_select", "leea_crossover_mutate",
            "leea_step"} <= names
    for n in sorted(names):
        assert hasattr(lib, n), n


def paper_cfg(**kw):
    d = dict(widths=(784, 112, 32, 10), pop=1000, max_batch=512)
    d.update(kw)
    return B.make_config(**d)


def test_param_count_and_workspace(lib):
    g, s = ctypes.c_int64(), ctypes.c_int64()
    for widths, c in (((784, 32, 10), 25450), ((784, 112, 32, 10), 91866),
                      ((196, 256, 128, 64, 10), 92234)):
        cfg = paper_cfg(widths=widths)
        assert lib.leea_param_count(ctypes.byref(cfg), ctypes.byref(g), ctypes.byref(s)) == 0
        assert g.value == c == O.param_count(widths)
        assert s.value % 64 == 0 and 0 <= s.value - c < 64
    n = ctypes.c_size_t()
    cfg = paper_cfg()
    assert lib.leea_workspace_bytes(ctypes.byref(cfg), ctypes.byref(n)) == 0
    assert n.value >= 2 * 1000 * 91904 * 4


def test_host_counts_match_the_paper_settings(lib):
    """leea_config_from_fractions (the library's section 3.1 rounding) against
    the oracle's counts, mutation threshold and Glorot bounds."""
    for args in ((16, 0.05, 0.5, 0.45, 0.25), (1000, 0.05, 0.5, 0.45, 0.5),
                 (2000, 0.05, 0.75, 0.2, 0.5), (7, 0.1, 0.3, 0.6, 0.9)):
        assert B.counts(*args) == O.counts(*args)
    for pop in range(1, 4097, 13):
        for fr in ((0.05, 0.50, 0.45), (0.05, 0.75, 0.20), (0.1, 0.3, 0.6)):
            for rho in (0.01, 0.25, 0.5, 1.0):
                assert B.counts(pop, *fr, rho) == O.counts(pop, *fr, rho)
    for p in (0.0, 0.1, 0.5, 1.0, 0.3333, 1 - 2 ** -40, 2 ** -33):
        assert B.threshold(p) == O.mutation_threshold(p)
    for widths in ((784, 32, 10), (784, 112, 32, 10), (196, 256, 128, 64, 10)):
        cfg = B.make_config(widths, 100)
        for l in range(len(widths) - 1):
            assert cfg.glorot_a[l] == O.glorot_bound(widths[l], widths[l + 1])
        assert all(cfg.glorot_a[l] == 0.0 for l in range(len(widths) - 1, B.MAX_LAYERS))


def test_config_from_fractions_rejects_bad_fractions(lib):
    cfg = B.Config()
    cfg.n_layers = 2
    cfg.widths[0], cfg.widths[1], cfg.widths[2] = 784, 32, 10
    cfg.pop = 16
    before = bytes(cfg)
    for args in ((0.5, 0.5, 0.5, 0.5, 1.0), (0.05, 0.5, 0.45, 1.5, 1.0),
                 (0.05, 0.5, 0.45, 0.5, 1.5), (-0.1, 0.6, 0.5, 0.5, 1.0)):
        assert lib.leea_config_from_fractions(ctypes.byref(cfg), *args) == B.EINVAL
        assert lib.leea_last_error(None)
    assert bytes(cfg) == before
    cfg.pop = 0
    assert lib.leea_config_from_fractions(ctypes.byref(cfg), 0.05, 0.5, 0.45, 0.5, 1.0) == B.EINVAL


@pytest.mark.parametrize("field,value", [
    ("n_layers", 0), ("n_layers", 9), ("pop", 0), ("pop", 8193), ("n_trunc", 0),
    ("n_trunc", 1001), ("selection", 2), ("crossover", 5), ("sigma", -1.0),
    ("alpha", 1.5), ("mut_threshold", (1 << 32) + 1), ("max_batch", 0), ("max_batch", 65537),
    ("n_elite", 51), ("tournament_k", 0),
])
def test_invalid_configs_rejected(lib, field, value):
    cfg = paper_cfg(selection="tournament") if field == "tournament_k" else paper_cfg()
    setattr(cfg, field, value)
    n = ctypes.c_size_t()
    assert lib.leea_workspace_bytes(ctypes.byref(cfg), ctypes.byref(n)) == B.EINVAL
    assert lib.leea_last_error(None)


def test_invalid_widths_rejected(lib):
    n = ctypes.c_size_t()
    for widths in ((783, 10), (784, 257, 10), (784, 0, 10), (784, 1)):
        cfg = paper_cfg(widths=widths)
        assert lib.leea_workspace_bytes(ctypes.byref(cfg), ctypes.byref(n)) == B.EINVAL


def test_init_rejects_bad_workspace_before_device_work(lib):
    cfg = paper_cfg()
    ctx = ctypes.c_void_p()
    n = ctypes.c_size_t()
    lib.leea_workspace_bytes(ctypes.byref(cfg), ctypes.byref(n))
    assert lib.leea_init_population(ctypes.byref(cfg), None, n.value, None, ctypes.byref(ctx)) == B.EINVAL
    assert lib.leea_init_population(ctypes.byref(cfg), ctypes.c_void_p(0x1000 + 16), n.value, None,
                                    ctypes.byref(ctx)) == B.EINVAL
    assert lib.leea_init_population(ctypes.byref(cfg), ctypes.c_void_p(0x100000), n.value - 1,
                                    None, ctypes.byref(ctx)) == B.ENOMEM
    assert ctx.value is None
    assert b"workspace" in lib.leea_last_error(None)


def test_calls_without_ctx_fail_cleanly(lib):
    assert lib.leea_evaluate(None, None, None, 1, None, None, None) == B.EINVAL
    assert lib.leea_select(None, None, None, None) == B.EINVAL
    assert lib.leea_crossover_mutate(None) == B.EINVAL
    assert lib.leea_step(None, None, None, 1, None, None, None) == B.EINVAL
    assert lib.leea_rng_philox(None, 0, None, 1, None) == B.EINVAL
    lib.leea_destroy(None)


def test_runs_workspace_and_validation(lib):
    n = ctypes.c_size_t()
    good = [paper_cfg(widths=(784, h, 10), pop=p, max_batch=b, eval_dtype="bf16")
            for h, p, b in ((16, 32, 8), (256, 2048, 256), (112, 500, 64))]
    arr = (B.Config * 3)(*good)
    assert lib.leea_runs_workspace_bytes(arr, 3, ctypes.byref(n)) == 0
    genomes = 0     # every run keeps two generations of genomes in the group's workspace
    for c in good:
        m = ctypes.c_size_t()
        assert lib.leea_workspace_bytes(ctypes.byref(c), ctypes.byref(m)) == 0
        genes, stride = ctypes.c_int64(), ctypes.c_int64()
        assert lib.leea_param_count(ctypes.byref(c), ctypes.byref(genes), ctypes.byref(stride)) == 0
        genomes += 2 * c.pop * stride.value * 4
        assert m.value >= 2 * c.pop * stride.value * 4
    assert n.value >= genomes
    for bad in (paper_cfg(eval_dtype="fp8"), paper_cfg(sigma_mode="decay", sigma_decay_k=5.0),
                paper_cfg(widths=(783, 10))):
        arr2 = (B.Config * 2)(good[0], bad)
        assert lib.leea_runs_workspace_bytes(arr2, 2, ctypes.byref(n)) == B.EINVAL
    assert lib.leea_runs_workspace_bytes(arr, 0, ctypes.byref(n)) == B.EINVAL
    m = ctypes.c_void_p()
    assert lib.leea_runs_create(arr, 3, None, n.value, None, ctypes.byref(m)) == B.EINVAL
    assert m.value is None
    assert lib.leea_runs_generation(None, None, None, 1) == B.EINVAL
    lib.leea_runs_destroy(None)
