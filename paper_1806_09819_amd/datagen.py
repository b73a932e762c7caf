"""Seeded synthetic inputs shaped like the paper's MNIST workload.

The paper evaluates on MNIST (section 4: 28x28 grey-scale inputs, d = 10
classes, a 45k / 5k / 10k train / validation / test split).  MNIST is not
available here, so two synthetic stand-ins with the same shapes are used.
This module only makes inputs; it holds none of the EA's arithmetic and is
shared by the oracle-side tests and the device path.

* ``teacher``: x ~ U[0, 1]^784; the label is the argmax of a fixed random
  teacher MLP 784 -> 64 -> 10 (ReLU, Glorot-normal weights) applied to
  x - 0.5, after subtracting each class's mean logit over a fixed reference
  sample of 4096 inputs, which keeps the classes roughly balanced.
* ``prototypes``: ten class prototypes mu_k = 0.5 + s * g_k with
  g_k ~ N(0, I_784); a sample of class y (uniform) is
  clip(mu_y + N(0, 0.3^2 I), 0, 1).  The spread s = 0.042 puts the
  nearest-prototype accuracy near 97-98 %, an MNIST-like difficulty.
"""

import numpy as np

N_IN = 784
N_CLASSES = 10
SPLITS = (45000, 5000, 10000)
PROTO_SPREAD = 0.042
NOISE_STD = 0.3


def teacher_labels(x, seed=1, hidden=64):
    """Labels from a fixed random teacher MLP (input generation only)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    n_in = x.shape[1]
    w1 = rng.normal(0.0, np.sqrt(2.0 / (n_in + hidden)), size=(n_in, hidden))
    w2 = rng.normal(0.0, np.sqrt(2.0 / (hidden + N_CLASSES)), size=(hidden, N_CLASSES))
    ref = rng.random((4096, n_in))

    def logits(v):
        return np.maximum((v.astype(np.float64) - 0.5) @ w1, 0.0) @ w2

    offset = logits(ref).mean(axis=0)
    return np.argmax(logits(x) - offset, axis=1).astype(np.int32)


def teacher_data(n, seed=0, teacher_seed=1):
    """(x [n, 784] float32 in [0, 1), y [n] int32) for the teacher task."""
    rng = np.random.Generator(np.random.PCG64(seed))
    x = rng.random((n, N_IN), dtype=np.float32)
    y = teacher_labels(x, teacher_seed)
    return x, y


def prototypes(seed=0, spread=PROTO_SPREAD):
    rng = np.random.Generator(np.random.PCG64(seed))
    return 0.5 + spread * rng.standard_normal((N_CLASSES, N_IN))


def prototype_data(n, seed=0, sample_seed=None, spread=PROTO_SPREAD):
    """(x [n, 784] float32 in [0, 1], y [n] int32) for the prototype task."""
    mu = prototypes(seed, spread)
    rng = np.random.Generator(np.random.PCG64(
        seed + 1000 if sample_seed is None else sample_seed))
    y = rng.integers(0, N_CLASSES, size=n).astype(np.int32)
    x = mu[y] + NOISE_STD * rng.standard_normal((n, N_IN))
    return np.clip(x, 0.0, 1.0).astype(np.float32), y


def splits(kind, sizes=SPLITS, seed=0):
    """Train / validation / test arrays of one task as a dict."""
    n = sum(sizes)
    if kind == "teacher":
        x, y = teacher_data(n, seed)
    elif kind == "prototypes":
        x, y = prototype_data(n, seed)
    else:
        raise ValueError(kind)
    a, b = sizes[0], sizes[0] + sizes[1]
    return dict(x_train=x[:a], y_train=y[:a], x_val=x[a:b], y_val=y[a:b],
                x_test=x[b:], y_test=y[b:])


def uniform_inputs(shape, seed):
    """Plain U[0, 1) float32 array (for parity cases with arbitrary shapes)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.random(shape, dtype=np.float32)


def labels(n, d, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.integers(0, d, size=n).astype(np.int32)
