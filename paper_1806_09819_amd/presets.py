"""Named workloads: network widths, population, batch, generations and EA
hyperparameters as the paper states them (fractions, not counts).

* ``small``: 784-32-10 MLP (25,450 parameters), population 16, batch 32,
  10 generations; teacher-labelled uniform inputs; uniform crossover,
  Gaussian mutation sigma = 0.01 with per-gene probability 0.1, truncation
  selection of the top 25 %; p_E / p_C / p_M are the paper defaults.
* ``paper``: 784-112-32-10 MLP (91,866 parameters, close to the paper's
  92k), population 1000 and the section-4 default hyperparameters
  (uniform crossover, p_E = 0.05, p_C = 0.50, p_M = 0.45, sigma = 0.001,
  rho = 0.5, alpha = 1, batch 512); batches 1, 8, 64 and 512 are measured.
* ``final``: the section-4.5 setting (population 2000, batch 1024,
  p_C = 0.75, p_M = 0.20).
* ``paper_net``: the paper's own network after 2x2 max-pooling of the
  inputs: 196-256-128-64-10 (92,234 parameters).
"""

SMALL = dict(widths=(784, 32, 10), pop=16, batch=32, generations=10,
             p_elite=0.05, p_cross=0.50, p_mut=0.45, rho=0.25,
             selection="truncation", tournament_k=2, crossover="uniform",
             sigma=0.01, p_gene=0.1, alpha=1.0, seed=2, data="teacher")

PAPER = dict(widths=(784, 112, 32, 10), pop=1000, batch=512, generations=1000,
             p_elite=0.05, p_cross=0.50, p_mut=0.45, rho=0.50,
             selection="truncation", tournament_k=2, crossover="uniform",
             sigma=0.001, p_gene=1.0, alpha=1.0, seed=0, data="prototypes")

FINAL = dict(PAPER, pop=2000, batch=1024, p_cross=0.75, p_mut=0.20)

PAPER_NET = dict(PAPER, widths=(196, 256, 128, 64, 10))

PAPER_BATCHES = (1, 8, 64, 512)

ALL = dict(small=SMALL, paper=PAPER, final=FINAL, paper_net=PAPER_NET)
