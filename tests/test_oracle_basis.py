"""Pins of the oracle's 1-D tables against closed forms."""
import numpy as np
import pytest

from oracle import basis1d


@pytest.mark.parametrize("r", [1, 2, 3, 4])
def test_edge_functions_are_dual_to_sub_intervals(r):
    nodes = basis1d.gll_nodes(r)
    g, w = basis1d.gauss(12)
    M = np.zeros((r, r))
    for i in range(r):
        h = nodes[i + 1] - nodes[i]
        x = nodes[i] + h * g
        M[i] = (basis1d.edge_values(r, x) * (w * h)[:, None]).sum(0)
    assert np.abs(M - np.eye(r)).max() < 1e-13


@pytest.mark.parametrize("r", [1, 2, 3, 4])
def test_partition_of_unity_and_interpolation(r):
    x = np.linspace(0, 1, 37)
    phi = basis1d.nodal_values(r, x)
    assert np.abs(phi.sum(1) - 1).max() < 1e-13
    nodes = basis1d.gll_nodes(r)
    assert np.abs(basis1d.nodal_values(r, nodes) - np.eye(r + 1)).max() < 1e-13


@pytest.mark.parametrize("r", [1, 2, 3, 4])
def test_derivative_is_the_incidence(r):
    # phi_i' = e_{i-1} - e_i, i.e. the 1-D derivative has entries +-1.
    x = np.linspace(0, 1, 23)
    d = basis1d.nodal_derivatives(r, x)
    e = basis1d.edge_values(r, x)
    ep = np.concatenate([np.zeros((x.size, 1)), e, np.zeros((x.size, 1))], axis=1)
    for i in range(r + 1):
        assert np.abs(d[:, i] - (ep[:, i] - ep[:, i + 1])).max() < 1e-11


def test_derivative_matches_finite_difference():
    r = 3
    x = np.linspace(0.1, 0.9, 9)
    h = 1e-6
    fd = (basis1d.nodal_values(r, x + h) - basis1d.nodal_values(r, x - h)) / (2 * h)
    assert np.abs(fd - basis1d.nodal_derivatives(r, x)).max() < 1e-7


def test_lowest_order_is_whitney():
    # Section 4.1: r = 1 gives phi = (1 - x, x) and a constant edge function.
    x = np.linspace(0, 1, 11)
    assert np.allclose(basis1d.nodal_values(1, x), np.stack([1 - x, x], 1), atol=0, rtol=0)
    assert np.allclose(basis1d.edge_values(1, x), 1.0, atol=1e-15)


def test_gll_nodes_closed_forms():
    assert np.allclose(basis1d.gll_nodes(2), [0, 0.5, 1], atol=1e-15)
    s = 1 / np.sqrt(5)
    assert np.allclose(basis1d.gll_nodes(3), [0, (1 - s) / 2, (1 + s) / 2, 1], atol=1e-15)
    t = np.sqrt(3 / 7)
    assert np.allclose(basis1d.gll_nodes(4), [0, (1 - t) / 2, 0.5, (1 + t) / 2, 1], atol=1e-15)


@pytest.mark.parametrize("q", [1, 2, 3, 5])
def test_gauss_exactness(q):
    x, w = basis1d.gauss(q)
    for k in range(2 * q):
        assert abs((w * x ** k).sum() - 1 / (k + 1)) < 1e-14
    assert abs((w * x ** (2 * q)).sum() - 1 / (2 * q + 1)) > 1e-6
