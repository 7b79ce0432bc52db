"""Pins of the oracle's isotropic model (no split, the isotropic case of Section 5) against the
mathematics: Hooke's law in Voigt matrix form, the stress as the derivative of the energy, the
coincidence with the volumetric/deviatoric split in pure tension, and on meshes the
finite-difference Jacobian (no branch to cross), the energy gradient, and rigid-body modes in the
kernel of the undamaged displacement block.
"""
import numpy as np
import pytest

from oracle import fe, material as mat
from oracle import operator as op

LAM, MU = 121.15e3, 80.77e3
MAT = op.Material(lam=LAM, mu=MU, Gc=2.7, eps=0.05, kappa=1e-10, split="none")
CASES = [(2, 4, 1), (2, 3, 2), (3, 2, 1), (3, 2, 2)]


def _voigt_stiffness(d):
    """Isotropic stiffness in Voigt form (engineering shear strains), written out per entry."""
    n = d * (d + 1) // 2
    C = np.zeros((n, n))
    C[:d, :d] = LAM
    for i in range(d):
        C[i, i] = LAM + 2 * MU
    for i in range(d, n):
        C[i, i] = MU
    return C


def _voigt(e):
    d = e.shape[-1]
    if d == 2:
        return np.stack([e[..., 0, 0], e[..., 1, 1], 2 * e[..., 0, 1]], -1)
    return np.stack([e[..., 0, 0], e[..., 1, 1], e[..., 2, 2], 2 * e[..., 0, 1], 2 * e[..., 0, 2],
                     2 * e[..., 1, 2]], -1)


def _voigt_stress(s):
    d = s.shape[-1]
    if d == 2:
        return np.stack([s[..., 0, 0], s[..., 1, 1], s[..., 0, 1]], -1)
    return np.stack([s[..., 0, 0], s[..., 1, 1], s[..., 2, 2], s[..., 0, 1], s[..., 0, 2], s[..., 1, 2]], -1)


def test_hooke_law_and_energy():
    rng = np.random.default_rng(41)
    for d in (2, 3):
        G = rng.standard_normal((200, d, d)) * 1e-2
        s = mat.isotropic_split(G, LAM, MU)
        ev = _voigt(s["e"])
        assert np.allclose(_voigt_stress(s["sig_p"]), ev @ _voigt_stiffness(d).T, rtol=1e-13, atol=1e-9)
        assert np.allclose(s["E_p"], 0.5 * np.einsum("ni,ij,nj->n", ev, _voigt_stiffness(d), ev), rtol=1e-12)
        assert np.all(s["E_m"] == 0) and np.all(s["sig_m"] == 0)
        D = 0.5 * (lambda A: A + np.swapaxes(A, -1, -2))(rng.standard_normal((200, d, d)))
        hs = 1e-7
        fd = (mat.isotropic_split(G + hs * D, LAM, MU)["E_p"] - mat.isotropic_split(G - hs * D, LAM, MU)["E_p"]) / (2 * hs)
        assert np.allclose(fd, np.einsum("nij,nij->n", s["sig_p"], D), rtol=1e-6, atol=1e-6)


def test_equals_volumetric_deviatoric_split_in_tension():
    rng = np.random.default_rng(42)
    for d in (2, 3):
        G = rng.standard_normal((300, d, d)) * 1e-2
        iso, amor = mat.isotropic_split(G, LAM, MU), mat.amor_split(G, LAM, MU)
        t = amor["t"] >= 0
        assert 50 < t.sum() < 250
        for key in ("sig_p", "E_p"):
            assert np.allclose(iso[key][t], amor[key][t], rtol=1e-12, atol=1e-9), key
        # and always the sum of the two branches of that split
        assert np.allclose(iso["E_p"], amor["E_p"] + amor["E_m"], rtol=1e-12)
        assert np.allclose(iso["sig_p"], amor["sig_p"] + amor["sig_m"], rtol=1e-12, atol=1e-9)


def _state(dim, N, k, seed):
    mesh = fe.Mesh(dim, N, k)
    rng = np.random.default_rng(seed)
    u = 1e-2 * rng.standard_normal((dim, mesh.n_nodes))
    phi = rng.uniform(0.1, 1.0, mesh.n_nodes)
    phit = rng.uniform(0.1, 1.0, mesh.n_nodes)
    return mesh, u, phi, phit


@pytest.mark.parametrize("dim,N,k", CASES)
def test_jacobian_matches_central_difference_of_residual(dim, N, k):
    mesh, u, phi, phit = _state(dim, N, k, 43)
    G = op.assemble_jacobian(mesh, MAT, u, phi, phit)
    rng = np.random.default_rng(44)
    nu = dim * mesh.n_nodes
    V = rng.standard_normal(nu + mesh.n_nodes)
    V[:nu] *= 1e-2
    hs = 1e-6

    def R(U):
        return op.residual(mesh, MAT, U[:nu].reshape(dim, -1), U[nu:], phit)
    U = np.concatenate([u.ravel(), phi])
    fd = (R(U + hs * V) - R(U - hs * V)) / (2 * hs)
    GV = G @ V
    assert np.linalg.norm(fd - GV) <= 1e-7 * np.linalg.norm(GV)


@pytest.mark.parametrize("dim,N,k", CASES)
def test_residual_is_energy_gradient_and_rigid_modes(dim, N, k):
    mesh, u, phi, _ = _state(dim, N, k, 45)
    nu = dim * mesh.n_nodes
    R = op.residual(mesh, MAT, u, phi, phi)
    rng = np.random.default_rng(46)
    U = np.concatenate([u.ravel(), phi])
    for _ in range(3):
        V = rng.standard_normal(U.size)
        V[:nu] *= 1e-2
        hs = 1e-6
        Ep = op.energy(mesh, MAT, (U + hs * V)[:nu].reshape(dim, -1), (U + hs * V)[nu:])
        Em = op.energy(mesh, MAT, (U - hs * V)[:nu].reshape(dim, -1), (U - hs * V)[nu:])
        assert abs((Ep - Em) / (2 * hs) - R @ V) <= 1e-7 * abs(R @ V) + 1e-10
    # undamaged body (phi~ = 1): translations and the infinitesimal rotations span the kernel of G_uu
    ones = np.ones(mesh.n_nodes)
    Guu = op.assemble_jacobian(mesh, MAT, u, ones, ones).tocsr()[:nu, :nu]
    X = np.stack(np.meshgrid(*[np.arange(mesh.M) / (mesh.M - 1)] * dim, indexing="ij"), -1)
    X = X.transpose(*range(dim - 1, -1, -1), dim).reshape(-1, dim)  # lexicographic, axis 0 fastest
    modes = [np.concatenate([ones * (c == a) for c in range(dim)]) for a in range(dim)]
    for a in range(dim):
        for b in range(a + 1, dim):
            w = np.zeros((dim, mesh.n_nodes))
            w[a], w[b] = -X[:, b], X[:, a]
            modes.append(w.ravel())
    scale = abs(Guu).max()
    for w in modes:
        assert np.abs(Guu @ w).max() <= 1e-9 * scale
