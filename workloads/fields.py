"""Seeded smooth fields sampled at mesh nodes (coefficient inputs).

Solution-dependent coefficients are evaluated from the interpolated field
u_h = phi^T u (Section 5, nonlinear FEM); the nodal vector u is the input.
Space-dependent coefficients k(x) = exp(g(x)) are handled the same way with a
nodal sample of g. These generators only draw random numbers and evaluate
sines/cosines at node coordinates; the coefficient maps themselves (1+a u^2,
exp) are applied by whoever assembles.
"""
from __future__ import annotations

import numpy as np


def rng_for(cfg_id: int, stream: int = 0):
    return np.random.default_rng([2204, cfg_id, stream])


def random_sinusoids(coords: np.ndarray, n_terms: int, rng, amplitude: float = 1.0, kmax: int = 3):
    """u(x) = amplitude * sum_j sin(2 pi kappa_j . x + theta_j), kappa_j in {-kmax..kmax}^d minus 0."""
    dim = coords.shape[0]
    out = np.zeros(coords.shape[1], dtype=np.float64)
    for _ in range(n_terms):
        while True:
            kap = rng.integers(-kmax, kmax + 1, size=dim)
            if np.any(kap != 0):
                break
        theta = rng.uniform(0.0, 2.0 * np.pi)
        out += np.sin(2.0 * np.pi * (kap.astype(np.float64) @ coords) + theta)
    return amplitude * out


def gaussian_random_field(coords: np.ndarray, n_features: int, rng, length: float = 0.1):
    """Random Fourier features of a unit-variance squared-exponential field.

    g(x) = sqrt(2/F) * sum_j cos(omega_j . x + theta_j), omega_j ~ N(0, length^-2 I).
    """
    dim = coords.shape[0]
    omega = rng.normal(0.0, 1.0 / length, size=(n_features, dim))
    theta = rng.uniform(0.0, 2.0 * np.pi, size=n_features)
    out = np.zeros(coords.shape[1], dtype=np.float64)
    for j in range(n_features):
        out += np.cos(omega[j] @ coords + theta[j])
    return np.sqrt(2.0 / n_features) * out
