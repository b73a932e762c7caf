"""Philox4x32-10 counter-based generator (oracle side).

Definition: Salmon, Moraes, Dror, Shaw, "Parallel Random Numbers: As Easy as
1, 2, 3", SC'11, section on the Philox family.  A 128-bit counter
(c0, c1, c2, c3) and a 64-bit key (k0, k1) go through ten rounds.  One round
multiplies c0 and c2 by the two round multipliers, producing 64-bit products
(hi, lo), and outputs

    (hi(M1*c2) ^ c1 ^ k0,  lo(M1*c2),  hi(M0*c0) ^ c3 ^ k1,  lo(M0*c0)).

Between rounds the key is bumped by the two Weyl constants (golden ratio and
sqrt(3)-1 scaled to 32 bits).  The first round uses the unbumped key.

The paper (section 3.2) draws uniform and normal random numbers for its
operators but does not name a generator; this counter layout is the reading
that lets the oracle and the device draw identical numbers:

    key     = (seed & 0xffffffff, seed >> 32)
    counter = (block, slot, generation, (run << 8) | purpose)

``block`` is the per-purpose block index (a gene block, a word block of a
selection draw, a batch-index block), ``slot`` the population slot being
produced, ``generation`` the generation whose population is being built, and
``run`` the index of an independent EA run sharing the seed.

Pins: Random123 known-answer vectors (tests/golden/philox_kat.txt) and a
cross-check against rocRAND's open-source Philox engine compiled for the host.
"""

import numpy as np

# round multipliers and Weyl key increments of Philox4x32 (SC'11)
M0 = 0xD2511F53
M1 = 0xCD9E8D57
W0 = 0x9E3779B9
W1 = 0xBB67AE85

# draw purposes (the low byte of the last counter word)
INIT = 0      # initial genome values (Glorot-uniform)
SEL = 1       # parent-selection draws
XO = 2        # uniform-crossover masks
MUTMASK = 3   # per-gene mutation decisions
MUTNORM = 4   # Gaussian mutation noise
SIGMA = 5     # sigma self-adaptation noise (reserved)
BATCH = 6     # minibatch example indices
SURR = 7      # fitness-surrogate projection signs and initial weights

_MASK32 = np.uint64(0xFFFFFFFF)


def philox4x32_10(c0, c1, c2, c3, k0, k1):
    """Ten Philox4x32 rounds on broadcastable uint32 counter words.

    Returns four uint32 arrays (the output words 0..3).
    """
    x0, x1, x2, x3 = np.broadcast_arrays(
        *(np.asarray(c, dtype=np.uint64) & _MASK32 for c in (c0, c1, c2, c3)))
    k0 = int(k0) & 0xFFFFFFFF
    k1 = int(k1) & 0xFFFFFFFF
    m0 = np.uint64(M0)
    m1 = np.uint64(M1)
    for r in range(10):
        if r:
            k0 = (k0 + W0) & 0xFFFFFFFF
            k1 = (k1 + W1) & 0xFFFFFFFF
        p0 = x0 * m0          # exact: both factors < 2**32
        p1 = x2 * m1
        y0 = (p1 >> np.uint64(32)) ^ x1 ^ np.uint64(k0)
        y1 = p1 & _MASK32
        y2 = (p0 >> np.uint64(32)) ^ x3 ^ np.uint64(k1)
        y3 = p0 & _MASK32
        x0, x1, x2, x3 = y0, y1, y2, y3
    return tuple(v.astype(np.uint32) for v in (x0, x1, x2, x3))


def draw(seed, purpose, gen, slot, block, run=0):
    """Four uint32 words for (purpose, generation, slot, block) under ``seed``.

    ``slot`` and ``block`` may be arrays (broadcast together).  Returns a
    uint32 array of shape broadcast(slot, block) + (4,).
    """
    seed = int(seed)
    c3 = ((int(run) << 8) | int(purpose)) & 0xFFFFFFFF
    w = philox4x32_10(block, slot, int(gen) & 0xFFFFFFFF, c3,
                      seed & 0xFFFFFFFF, seed >> 32)
    return np.stack(w, axis=-1)
