"""Seeded synthetic inputs shared by the tests, the benchmark and the smoke check.

This module only draws numbers; it holds none of the method's arithmetic.
Both the oracle and the HIP path receive its arrays as plain inputs.

Layout of block vectors drawn here: (N, P) -- one row per interior node
(x fastest), one column per chaos mode in graded order.
"""

import numpy as np

# Workload presets: cells per side, KL terms m, degree p, sigma, correlation length, and the
# GMRES restart length each workload names.
CONFIGS = {
    "c1": dict(n=32, m=2, p=2, sigma=0.3, corr_len=0.5, restart=30),
    "c2": dict(n=128, m=4, p=3, sigma=0.3, corr_len=0.5, restart=30),
    "c3": dict(n=512, m=6, p=4, sigma=0.4, corr_len=0.5, restart=30),
    "c3_65": dict(n=64, m=6, p=4, sigma=0.4, corr_len=0.5, restart=30),
    "c4": dict(n=1024, m=8, p=3, sigma=0.5, corr_len=0.25, restart=20),
    "c4_129": dict(n=128, m=8, p=3, sigma=0.5, corr_len=0.25, restart=20),
    "c5": dict(n=256, m=5, p=3, sigma=0.3, corr_len=0.5, restart=30),
}


def uniform_block(N, P, seed=1234, dtype=np.float64):
    """i.i.d. U[-1, 1] entries, shape (N, P)."""
    rng = np.random.default_rng(seed)
    return rng.uniform(-1.0, 1.0, size=(N, P)).astype(dtype)


def separable_factors(N, P, rank, seed=4321):
    """Factors v_r (N) and w_r (P) of a rank-`rank` block U = sum_r v_r w_r^T."""
    rng = np.random.default_rng(seed)
    return rng.uniform(-1.0, 1.0, size=(rank, N)), rng.uniform(-1.0, 1.0, size=(rank, P))


def a0_noise_field(n, seed=2024, amplitude=0.1):
    """Nodal mean field a0 = 1 + amplitude * noise on the (n+1)^2 grid, x fastest.

    noise = sum_{i,j=1..4} z_ij sin(i pi x1) sin(j pi x2) / (i^2 + j^2),
    z_ij ~ N(0, 1), scaled so that max |noise| over the vertices is 1.  It
    vanishes on the boundary, so a0 = 1 there.
    """
    rng = np.random.default_rng(seed)
    z = rng.standard_normal((4, 4))
    t = np.linspace(0.0, 1.0, n + 1)
    x1, x2 = np.meshgrid(t, t, indexing="xy")
    noise = np.zeros_like(x1)
    for i in range(1, 5):
        for j in range(1, 5):
            noise += z[i - 1, j - 1] * np.sin(i * np.pi * x1) * np.sin(j * np.pi * x2) / (i * i + j * j)
    noise /= np.max(np.abs(noise))
    return (1.0 + amplitude * noise).ravel()


def unit_directions(count, dim, seed=7):
    """`count` random unit vectors of length `dim` (rows)."""
    rng = np.random.default_rng(seed)
    v = rng.standard_normal((count, dim))
    return v / np.linalg.norm(v, axis=1, keepdims=True)
