"""The seeded input generators (synth/): properties of the counter-based
perturbed mesh that the C library's constructor mirrors (the bitwise
comparison with the library runs in test_gpu_boundary.py)."""
import numpy as np

import synth


def test_counter_perturbation_rules():
    nel, frac = (6, 5, 4), 0.15
    v = synth.perturbed_vertices_counter(nel, frac, seed=3)
    u = synth.uniform_vertices(nel)
    off = v - u
    h = 1.0 / np.asarray(nel, float)
    assert np.all(np.abs(off) <= frac * h * (1 + 1e-12))
    for a in range(3):
        idx = [slice(None)] * 3
        for end in (0, nel[a]):
            idx[a] = end
            assert np.all(off[tuple(idx) + (a,)] == 0.0)   # slides within the boundary face
    for corner in np.ndindex(2, 2, 2):
        c = tuple(ci * n for ci, n in zip(corner, nel))
        assert np.array_equal(v[c], u[c])
    # interior offsets fill the allowed range and are seeded
    inner = off[1:-1, 1:-1, 1:-1] / (frac * h)
    assert inner.min() < -0.8 and inner.max() > 0.8
    assert np.array_equal(v, synth.perturbed_vertices_counter(nel, frac, seed=3))
    assert not np.array_equal(v, synth.perturbed_vertices_counter(nel, frac, seed=4))


def test_counter_perturbation_word_index():
    # vertex (i, j, k), coordinate a takes SplitMix64 word 3 v + a with
    # v = i + (nx+1)(j + (ny+1) k): check one interior vertex by hand
    nel, frac, seed = (3, 4, 2), 0.1, 99
    v = synth.perturbed_vertices_counter(nel, frac, seed)
    i, j, k = 2, 1, 1
    vid = i + (nel[0] + 1) * (j + (nel[1] + 1) * k)
    mask = (1 << 64) - 1

    def word(w):
        z = (seed + (w + 1) * 0x9E3779B97F4A7C15) & mask
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & mask
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & mask
        return z ^ (z >> 31)

    for a in range(3):
        u = (word(3 * vid + a) >> 11) * 2.0 ** -53
        x = (i, j, k)[a] / nel[a] + (2.0 * u - 1.0) * (frac / nel[a])
        assert abs(v[i, j, k, a] - x) < 1e-15
