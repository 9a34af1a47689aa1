"""Seeded nodal values and closed-form source terms (input generators only)."""
from __future__ import annotations

import numpy as np


def uniform_values(count: int, seed) -> np.ndarray:
    """``count`` values ~ U[-1, 1] from PCG64 ``default_rng(seed)``.

    Callers draw one value per unique micro-vertex in canonical key order, so
    both sides of a comparison see the same value at the same point.
    """
    return np.random.default_rng(seed).uniform(-1.0, 1.0, size=count)


def sine_solution(xyz: np.ndarray) -> np.ndarray:
    """u(x, y, z) = sin(pi x) sin(pi y) sin(pi z)."""
    x, y, z = xyz[..., 0], xyz[..., 1], xyz[..., 2]
    return np.sin(np.pi * x) * np.sin(np.pi * y) * np.sin(np.pi * z)


def sine_source(xyz: np.ndarray) -> np.ndarray:
    """f = -Laplace(u) = 3 pi^2 sin(pi x) sin(pi y) sin(pi z)."""
    return 3.0 * np.pi ** 2 * sine_solution(xyz)


def smooth_field_params(seed, terms: int = 4):
    """Frequencies, phases and amplitudes of :func:`smooth_field`."""
    rng = np.random.default_rng(seed)
    k = rng.uniform(0.5, 3.0, size=(terms, 3))
    phase = rng.uniform(0.0, 2 * np.pi, size=terms)
    amp = rng.uniform(0.5, 1.0, size=terms)
    return k, phase, amp


def smooth_field(xyz: np.ndarray, seed, terms: int = 4) -> np.ndarray:
    """Sum of a few seeded plane-wave cosines of the physical coordinates.

    A field that any code holding the coordinates can evaluate on its own,
    used where neither side can afford to enumerate every vertex.
    """
    k, phase, amp = smooth_field_params(seed, terms)
    out = np.zeros(xyz.shape[:-1])
    for t in range(terms):
        out += amp[t] * np.cos(xyz @ k[t] + phase[t])
    return out


def coefficient_field(xyz: np.ndarray) -> np.ndarray:
    """Diffusion coefficient k(x, y, z) = 1 + sin(2 pi x) sin(2 pi y)
    sin(2 pi z) / 2, between 1/2 and 3/2."""
    x, y, z = xyz[..., 0], xyz[..., 1], xyz[..., 2]
    return 1.0 + 0.5 * (np.sin(2 * np.pi * x) * np.sin(2 * np.pi * y) *
                        np.sin(2 * np.pi * z))
