"""Plain, slow, obviously correct CPU oracle for the limited-evaluation EA
(Prellberg & Kramer, "Limited Evaluation Evolutionary Optimization of Large
Neural Networks", arXiv 1806.09819).

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the CPU
baseline leg of the benchmark may import this package.  The product path (the
HIP library and its Python binding) never calls into it, and this package
imports nothing from the product path: the two share no code, headers,
constants or tables.  Random numbers are produced on each side by its own
implementation of the same published counter-based generator (Philox4x32-10,
Salmon et al., SC'11).

Arithmetic conventions
* Forward pass and fitness: float64, from float32 genomes and float32 inputs
  (the paper fixes no precision).
* Genetic operators and every step that turns random bits into numbers:
  float32 op by op with numpy (IEEE round-to-nearest, no fused multiply-add),
  because those results must match the device bit for bit.

Modules
* ``philox``   -- Philox4x32-10 and the counter layout used for every draw.
* ``normal32`` -- the float32 Box-Muller normal sampler (ln / sin / cos built
                  from series with +,-,*,/,sqrt only).
* ``leea``     -- Algorithm 1 of the paper step by step: counts, init,
                  forward, fitness (Eq. 1), inheritance, rank, plan, vary,
                  batch draw, and the generation loop.

Pins: every function here is checked by ``tests/test_oracle_*.py`` against
published known-answer vectors, closed forms, library routines, invariants
or brute force.  Functions without such a pin are listed as "parity unpinned"
in their docstrings.
"""

from . import philox, normal32, leea  # noqa: F401
