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
  * counter-based perturbed meshes (``perturbed_vertices_counter``): the
    same boundary rule with offsets (2u - 1)*frac*h, u = (z >> 11) 2^-53 from
    SplitMix64 word z of index dim*v + a (v the vertex's lexicographic index,
    axis 0 fastest), the definition the C library's mesh constructor uses;
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


def _splitmix64(seed, k):
    """SplitMix64 word k of stream `seed` (Steele, Lea & Flood 2014), vectorised."""
    z = (np.uint64(seed) + (k.astype(np.uint64) + np.uint64(1)) * np.uint64(0x9E3779B97F4A7C15))
    z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
    z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
    return z ^ (z >> np.uint64(31))


def counter_normal(seed, n, first=0):
    """N(0, 1) vector of length n, zero below index `first`, from SplitMix64
    words u = (z >> 11) 2^-53 and Box-Muller: b_i = sqrt(-2 log(1 - u_{2i}))
    cos(2 pi u_{2i+1}) for i = k - first.  The serving loop draws the same
    numbers on the GPU from the same published definitions."""
    out = np.zeros(n)
    m = n - first
    if m <= 0:
        return out
    i = np.arange(m, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z1 = _splitmix64(seed, 2 * i)
        z2 = _splitmix64(seed, 2 * i + np.uint64(1))
    u1 = (z1 >> np.uint64(11)).astype(np.float64) * 2.0 ** -53
    u2 = (z2 >> np.uint64(11)).astype(np.float64) * 2.0 ** -53
    out[first:] = np.sqrt(-2.0 * np.log(1.0 - u1)) * np.cos(2.0 * np.pi * u2)
    return out


def perturbed_vertices_counter(nel, frac, seed, lo=None, hi=None):
    """Uniform vertices plus counter-based offsets: vertex v (lexicographic,
    axis 0 fastest), coordinate a, moves by (2u - 1) * (frac * h_a) with u
    from SplitMix64 word dim*v + a of stream `seed`; no offset along a on the
    faces normal to a."""
    v = uniform_vertices(nel, lo, hi)
    nel = tuple(int(n) for n in nel)
    dim = len(nel)
    lo = np.zeros(dim) if lo is None else np.asarray(lo, float)
    hi = np.ones(dim) if hi is None else np.asarray(hi, float)
    # vertex index with axis 0 fastest, in the (N_1+1, ..., N_d+1) array order
    vid = np.zeros(v.shape[:-1], dtype=np.uint64)
    stride = 1
    for a in range(dim):
        shape = [1] * dim
        shape[a] = nel[a] + 1
        vid = vid + (np.arange(nel[a] + 1, dtype=np.uint64) * np.uint64(stride)).reshape(shape)
        stride *= nel[a] + 1
    off = np.zeros_like(v)
    for a in range(dim):
        h = (hi[a] - lo[a]) / float(nel[a])
        with np.errstate(over="ignore"):
            z = _splitmix64(seed, vid * np.uint64(dim) + np.uint64(a))
        u = (z >> np.uint64(11)).astype(np.float64) * 2.0 ** -53
        off_a = (2.0 * u - 1.0) * (frac * h)
        idx = [slice(None)] * dim
        for end in (0, nel[a]):
            idx[a] = end
            off_a[tuple(idx)] = 0.0
        off[..., a] = off_a
    return np.ascontiguousarray(v + off)
