"""Seeded test vectors shared by the GPU parity tests (inputs only)."""
import numpy as np


def mixed_vector(n, seed, spread=6.0):
    """Normal values with per-entry magnitude spreads up to `spread` decades,
    exact zeros, -0.0, subnormals and a few powers of two."""
    rng = np.random.default_rng(seed)
    x = rng.standard_normal(n) * 10.0 ** rng.uniform(-spread, 0, n)
    x[rng.random(n) < 0.02] = 0.0
    x[rng.random(n) < 0.01] = -0.0
    sub = rng.random(n) < 0.005
    x[sub] = rng.standard_normal(int(sub.sum())) * 1e-310
    p2 = rng.random(n) < 0.01
    x[p2] = np.ldexp(1.0, rng.integers(-20, 20, int(p2.sum())))
    return x


def adversarial_blocks():
    """Blocks that hit the corner cases of the FRSZ2 steps, 32 values each."""
    B = []
    B.append(np.zeros(32))
    B.append(-np.zeros(32))
    z = np.zeros(32); z[17] = -3.5; B.append(z)
    z = np.full(32, 1e-300); z[0] = 1.0; B.append(z)                 # every k >= l-1
    z = np.linspace(-1, 1, 32) * 2.0 ** 1000; z[3] = 1.7e308; B.append(z)  # top exponent 2046
    B.append(np.arange(32) * 5e-324)                                  # subnormal-only
    B.append(np.ldexp(1.0, np.arange(-31, 1)))                        # every k from 0 to 31
    B.append(-np.ldexp(1.0, np.arange(-31, 1)) * (1 - 2.0 ** -52))
    z = np.ones(32) * (1 - 2.0 ** -53); B.append(z)
    z = np.array([(-1) ** i * (1 + i * 2.0 ** -30) for i in range(32)]); B.append(z)
    return np.concatenate(B)
