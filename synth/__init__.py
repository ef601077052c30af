"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the bench.

This module draws random numbers and lays out vertex arrays; it holds none of
the method's arithmetic (no bases, no quadrature, no operators), so both the
oracle and the HIP path can take their inputs from it without sharing code.

Recipes (stated in the design doc as well):
  * uniform box meshes: vertex (i, j, k) at lo + (hi - lo) * (i, j, k) / N;
  * perturbed meshes: every vertex gets i.i.d. offsets U(-frac*h, frac*h) per
    coordinate from numpy's PCG64 (``default_rng(seed)``); components normal
    to a boundary face are zeroed, so boundary-face vertices slide in their
    face, boundary-edge vertices along their edge, and corners stay fixed;
  * Fourier coefficients and random right-hand sides: i.i.d. N(0, 1) from
    ``default_rng(seed)``.
"""
import numpy as np


def uniform_vertices(nel, lo=None, hi=None):
    """Vertex coordinates (N_1+1, ..., N_d+1, d) of a uniform box mesh."""
    nel = tuple(int(n) for n in nel)
    dim = len(nel)
    lo = np.zeros(dim) if lo is None else np.asarray(lo, float)
    hi = np.ones(dim) if hi is None else np.asarray(hi, float)
    axes = [lo[a] + (hi[a] - lo[a]) * np.arange(nel[a] + 1) / nel[a] for a in range(dim)]
    grid = np.meshgrid(*axes, indexing="ij")
    return np.ascontiguousarray(np.stack(grid, axis=-1))


def perturbed_vertices(nel, frac, seed, lo=None, hi=None):
    """Uniform vertices plus seeded offsets of at most ``frac`` of the cell size."""
    v = uniform_vertices(nel, lo, hi)
    dim = len(nel)
    lo = np.zeros(dim) if lo is None else np.asarray(lo, float)
    hi = np.ones(dim) if hi is None else np.asarray(hi, float)
    h = (hi - lo) / np.asarray(nel, float)
    rng = np.random.default_rng(seed)
    off = rng.uniform(-1.0, 1.0, size=v.shape) * (frac * h)
    for a in range(dim):
        idx = [slice(None)] * dim
        for end in (0, nel[a]):
            idx[a] = end
            off[tuple(idx) + (a,)] = 0.0
    return np.ascontiguousarray(v + off)


def fourier_coeffs(seed, nmodes=8, ncomp=1):
    """N(0, 1) coefficients, shape (nmodes, ncomp)."""
    return np.random.default_rng(seed).standard_normal((nmodes, ncomp))


def random_vector(n, seed, nrhs=1):
    """N(0, 1) vector(s), shape (nrhs, n) flattened row-major."""
    return np.random.default_rng(seed).standard_normal((nrhs, n)).reshape(-1)


def modes_3d():
    """Wave-number triples (a, b, c) in {1, 2}^3, a fastest."""
    return [(a, b, c) for c in (1, 2) for b in (1, 2) for a in (1, 2)]


def modes_2d():
    return [(a, b) for b in (1, 2) for a in (1, 2)]
