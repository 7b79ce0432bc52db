"""Pins of the oracle's finite-element tables against closed forms."""
import itertools

import numpy as np
import pytest

from oracle import fe
from oracle import operator as op


@pytest.mark.parametrize("q", [1, 2, 3, 4, 5, 6])
def test_gauss_exact_monomials(q):
    x, w = fe.gauss_legendre_01(q)
    for j in range(2 * q):
        assert abs((w * x ** j).sum() - 1.0 / (j + 1)) < 1e-14


def test_gauss3_textbook_values():
    x, w = fe.gauss_legendre_01(3)
    r = np.sqrt(3.0 / 5.0)
    assert np.allclose(x, [(1 - r) / 2, 0.5, (1 + r) / 2], atol=1e-15)
    assert np.allclose(w, [5 / 18, 8 / 18, 5 / 18], atol=1e-15)


@pytest.mark.parametrize("k", [1, 2, 3, 4])
def test_lagrange_cardinal_and_reproduction(k):
    nodes = fe.lagrange_nodes(k)
    assert np.allclose(fe.lagrange_values(k, nodes), np.eye(k + 1), atol=1e-14)
    x = np.linspace(-0.3, 1.2, 17)
    V, D = fe.lagrange_values(k, x), fe.lagrange_derivs(k, x)
    assert np.allclose(V.sum(1), 1.0, atol=1e-13)
    assert np.allclose(D.sum(1), 0.0, atol=1e-12)
    rng = np.random.default_rng(k)
    c = rng.standard_normal(k + 1)
    f = np.polynomial.Polynomial(c)
    assert np.allclose(V @ f(nodes), f(x), atol=1e-12)
    assert np.allclose(D @ f(nodes), f.deriv()(x), atol=1e-11)


def test_lagrange_derivative_matches_finite_difference():
    k = 4
    x = np.array([0.13, 0.41, 0.77])
    hstep = 1e-6
    fd = (fe.lagrange_values(k, x + hstep) - fe.lagrange_values(k, x - hstep)) / (2 * hstep)
    assert np.allclose(fe.lagrange_derivs(k, x), fd, atol=1e-7)


@pytest.mark.parametrize("dim,k", [(2, 1), (2, 3), (3, 2), (3, 4)])
def test_tensor_basis_partition_of_unity(dim, k):
    tb = fe.TensorBasis(dim, k)
    assert np.allclose(tb.val.sum(1), 1.0, atol=1e-13)
    assert np.allclose(tb.grad.sum(1), 0.0, atol=1e-11)
    assert abs(tb.w.sum() - 1.0) < 1e-14


def test_tensor_basis_is_product_of_1d():
    # N_p(x_q) for a 2D Q2 basis equals l_{p0}(x_{q0}) l_{p1}(x_{q1})
    tb = fe.TensorBasis(2, 2)
    x, _ = fe.gauss_legendre_01(3)
    B = fe.lagrange_values(2, x)
    for q, (q1, q0) in enumerate(itertools.product(range(3), range(3))):
        for p, (p1, p0) in enumerate(itertools.product(range(3), range(3))):
            assert abs(tb.val[q, p] - B[q0, p0] * B[q1, p1]) < 1e-15


@pytest.mark.parametrize("dim,N,k", [(2, 3, 2), (3, 2, 3), (2, 4, 1)])
def test_cells_of_nodes_brute_force(dim, N, k):
    mesh = fe.Mesh(dim, N, k)
    cn = mesh.cell_nodes()
    rng = np.random.default_rng(0)
    nodes = rng.choice(mesh.n_nodes, size=min(20, mesh.n_nodes), replace=False)
    for n in nodes:
        brute = sorted(np.flatnonzero((cn == n).any(1)).tolist())
        assert mesh.cells_of_nodes([n]).tolist() == brute


@pytest.mark.parametrize("k,w1", [(1, [1 / 2, 1 / 2]), (2, [1 / 6, 4 / 6, 1 / 6]),
                                  (3, [1 / 8, 3 / 8, 3 / 8, 1 / 8]),
                                  (4, [7 / 90, 32 / 90, 12 / 90, 32 / 90, 7 / 90])])
def test_lumped_mass_newton_cotes(k, w1):
    # integral of an equispaced Lagrange basis function = closed Newton-Cotes weight
    mesh = fe.Mesh(2, 3, k)
    ML = op.lumped_phi_mass(mesh)
    h = mesh.h
    w1 = np.asarray(w1) * h
    # 1D weights per global node: vertices shared by two cells
    m1 = np.zeros(mesh.M)
    for c in range(mesh.N):
        m1[k * c: k * c + k + 1] += w1
    assert np.allclose(ML, np.kron(m1, m1), rtol=1e-13)
    assert (ML > 0).all() and abs(ML.sum() - 1.0) < 1e-13
