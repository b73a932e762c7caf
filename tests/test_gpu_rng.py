"""GPU parity of the random streams and the initial population: Philox
blocks, the float32 ln (all 2^24 inputs), Box-Muller pairs (all 2^24 radii
and all 2^24 angles) and Glorot init, bit for bit against the oracle."""
import numpy as np
import pytest
import torch

from gpu_helpers import F32, batch, genomes_np, make_run, say, to_dev, to_np
from oracle import leea as O
from oracle import normal32 as N
from oracle import philox as PH
from paper_1806_09819_amd import leea as B
from paper_1806_09819_amd import presets

pytestmark = pytest.mark.gpu


def test_philox_blocks_bit_exact(golden_dir):
    say("philox: 1M random counters")
    rng = np.random.Generator(np.random.PCG64(1))
    n = 1 << 20
    ctr = rng.integers(0, 2**32, size=(n, 4), dtype=np.uint64).astype(np.uint32)
    key = 0x0123456789ABCDEF
    got = to_np(B.rng_philox(to_dev(ctr), key), np.uint32)
    ref = np.stack(PH.philox4x32_10(ctr[:, 0], ctr[:, 1], ctr[:, 2], ctr[:, 3],
                                    key & 0xFFFFFFFF, key >> 32), axis=1)
    assert np.array_equal(got, ref)
    with open(golden_dir + "/philox_kat.txt") as fh:
        rows = [[int(t, 16) for t in l.split()] for l in fh if l.strip() and l[0] != "#"]
    for r in rows:
        c = np.array([r[:4]], dtype=np.uint32)
        out = to_np(B.rng_philox(to_dev(c), r[4] | (r[5] << 32)), np.uint32)[0]
        assert [int(v) for v in out] == r[6:10]


def test_ln32_all_inputs_bit_exact():
    say("ln32: all 2^24 inputs")
    k = np.arange(1, 2**24 + 1, dtype=np.uint32)
    u = k.astype(F32) * F32(2.0**-24)
    got = to_np(B.rng_ln32(to_dev(u)))
    ref = N.ln32(u)
    bad = np.nonzero(got.view(np.uint32) != ref.view(np.uint32))[0]
    assert bad.size == 0, (bad.size, u[bad[:5]], got[bad[:5]], ref[bad[:5]])


@pytest.mark.parametrize("which", ["radius", "angle"])
def test_normal_pairs_all_radii_and_angles_bit_exact(which):
    say("normal pairs: all 2^24", which)
    rng = np.random.Generator(np.random.PCG64(2 if which == "radius" else 3))
    n = 1 << 24
    k = np.arange(n, dtype=np.uint32)
    other = rng.integers(0, 2**32, size=n, dtype=np.uint64).astype(np.uint32)
    if which == "radius":
        a = (k << np.uint32(8)) | (other & np.uint32(0xFF))
        b = other
    else:
        a = other
        b = (other & np.uint32(0xC000003F)) | (k << np.uint32(6))
    ab = np.stack([a, b], axis=1)
    got = to_np(B.rng_normal_pairs(to_dev(ab)))
    z0, z1 = N.normal_pair(a, b)
    ref = np.stack([z0, z1], axis=1)
    bad = np.nonzero(np.any(got.view(np.uint32) != ref.view(np.uint32), axis=1))[0]
    assert bad.size == 0, (bad.size, ab[bad[:3]], got[bad[:3]], ref[bad[:3]])


@pytest.mark.parametrize("name", ["small", "paper", "paper_net"])
def test_init_population_bit_exact(name):
    params = dict(presets.ALL[name], max_batch=64)
    say("init:", name)
    run, ocfg = make_run(params)
    torch.cuda.synchronize()
    g = to_np(run.population()[0])
    assert np.all(g[:, run.genes:] == 0)
    slots = list(range(run.pop)) if run.pop <= 16 else [0, 1, 2, run.pop // 2, run.pop - 1]
    ref = O.init_population(ocfg, slots=slots)
    for row, j in enumerate(slots):
        assert np.array_equal(g[j, :run.genes].view(np.uint32), ref[row].view(np.uint32)), j


def test_draw_batch_bit_exact():
    say("draw_batch")
    params = dict(presets.SMALL, max_batch=512)
    run, ocfg = make_run(params)
    xt, yt = batch(784, 4999, 10, 7)
    xd, yd = to_dev(xt), to_dev(yt)
    for gen, b in ((0, 1), (3, 32), (11, 509)):
        xb, yb = run.draw_batch(gen, xd, yd, b)
        idx = O.batch_indices(ocfg.seed, gen, b, 4999, ocfg.run)
        assert np.array_equal(to_np(xb), xt[idx]) and np.array_equal(to_np(yb), yt[idx])
