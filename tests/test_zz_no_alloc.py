"""leea_score_noalloc (the entry point for callers that cannot allocate)
against leea_score, whose kernels it shares: bit-identical fitness and
accuracy on two calls in a row, the second with a smaller input, both
through the C ABI, and its host-side limit checks."""
import ctypes

import numpy as np
import pytest
import torch

from gpu_helpers import make_run, say, to_dev, to_np
from paper_1806_09819_amd import datagen
from paper_1806_09819_amd import leea as B
from paper_1806_09819_amd import presets

pytestmark = pytest.mark.gpu


def _noalloc(cfg, genomes, stride, x, y):
    pop = cfg.pop
    f_raw = torch.full((pop,), float("nan"), dtype=torch.float32, device="cuda")
    acc = torch.full((pop,), float("nan"), dtype=torch.float32, device="cuda")
    st = B.library().leea_score_noalloc(ctypes.byref(cfg), B._ptr(genomes), stride, B._ptr(x),
                                        B._ptr(y), x.shape[0], B._ptr(f_raw), B._ptr(acc),
                                        B._stream())
    assert st == B.OK, B.library().leea_last_error(None)
    return f_raw, acc


def _evolved(params, b, gens=2):
    run, _ = make_run(params, max_batch=b)
    x, y = datagen.prototype_data(3000, seed=0)
    xd, yd = to_dev(x), to_dev(y)
    xb, yb = run.draw_batch(0, xd, yd, b)
    run.evaluate(xb, yb)
    for g in range(1, gens + 1):
        xb, yb = run.draw_batch(g, xd, yd, b)
        run.step(xb, yb)
    return run, xd, yd


def test_noalloc_matches_score_on_two_calls():
    params = dict(presets.PAPER)                       # 784-112-32-10, P = 1000
    run, xd, yd = _evolved(params, 512)
    genomes, _ = run.population()
    for n in (512, 8):                                 # second call: smaller input
        say("noalloc call, n =", n)
        x, y = run.draw_batch(100 + n, xd, yd, n)
        f_ref, a_ref = run.score(x, y)
        f_na, a_na = _noalloc(run.cfg, genomes, run.stride, x, y)
        torch.cuda.synchronize()
        assert np.array_equal(to_np(f_na).view(np.uint32), to_np(f_ref).view(np.uint32)), n
        assert np.array_equal(to_np(a_na).view(np.uint32), to_np(a_ref).view(np.uint32)), n
        assert np.isfinite(to_np(f_na)).all()
    run.close()


def test_noalloc_smaller_population_after_larger():
    """A second configuration (fewer networks, 64-row partial groups past
    the first call's) reuses the same scratch; results stay identical."""
    for params, n in ((dict(presets.PAPER, pop=1000), 300),
                      (dict(presets.SMALL, pop=37), 130)):
        say("noalloc population", params["pop"], "n =", n)
        run, xd, yd = _evolved(params, max(n, 64), gens=1)
        genomes, _ = run.population()
        x, y = run.draw_batch(7, xd, yd, n)
        f_ref, a_ref = run.score(x, y)
        f_na, a_na = _noalloc(run.cfg, genomes, run.stride, x, y)
        torch.cuda.synchronize()
        assert np.array_equal(to_np(f_na).view(np.uint32), to_np(f_ref).view(np.uint32))
        assert np.array_equal(to_np(a_na).view(np.uint32), to_np(a_ref).view(np.uint32))
        run.close()


def test_noalloc_rejects_what_it_cannot_hold():
    lib = B.library()
    cfg = B.make_config(**dict(presets.PAPER, max_batch=512))
    g = torch.zeros((cfg.pop, 91904), dtype=torch.float32, device="cuda")
    x = torch.zeros((8385, 784), dtype=torch.float32, device="cuda")
    y = torch.zeros((8385,), dtype=torch.int32, device="cuda")
    out = torch.empty(cfg.pop, dtype=torch.float32, device="cuda")
    P = B._ptr
    # pop * ceil(8385 / 64) = 1000 * 132 partials > 131072
    assert lib.leea_score_noalloc(ctypes.byref(cfg), P(g), 91904, P(x), P(y), 8385, P(out),
                                  P(out), B._stream()) == B.EINVAL
    assert b"scratch" in lib.leea_last_error(None)
    assert lib.leea_score_noalloc(ctypes.byref(cfg), P(g), 91904, P(x), P(y), 8384, P(out),
                                  None, B._stream()) == B.OK
    assert lib.leea_score_noalloc(ctypes.byref(cfg), P(g), 91903, P(x), P(y), 8, P(out),
                                  None, B._stream()) == B.EINVAL
    bf = B.make_config(**dict(presets.PAPER, eval_dtype="bf16", max_batch=16))
    assert lib.leea_score_noalloc(ctypes.byref(bf), P(g), 91904, P(x), P(y), 8, P(out),
                                  None, B._stream()) == B.EINVAL
    torch.cuda.synchronize()
