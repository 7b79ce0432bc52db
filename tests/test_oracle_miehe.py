"""Pins of the oracle's spectral (Miehe) split of Section 2.1 and of its
tangent (Section 3.5) against the mathematics.

Independent of the oracle's formulas: the energy identity E^+ + E^- = E_s,
central differences of the energies (stress) and of the stress (tangent),
Algorithm 2 written out step by step here (on distinct eigenvalues), the
closed-form special cases (pure tension, pure compression, isotropic
strain, a 2x2 strain with one positive and one negative eigenvalue), the
coincidence with the volumetric/deviatoric split in pure tension, and, on
meshes, the finite-difference Jacobian, the energy gradient and the block
symmetry of eq. (G).
"""
import numpy as np
import pytest

from oracle import fe, material as mat
from oracle import operator as op

LAM, MU = 121.15e3, 80.77e3
MAT = op.Material(lam=LAM, mu=MU, Gc=2.7, eps=0.05, kappa=1e-10, split="miehe")
CASES = [(2, 4, 1), (2, 3, 2), (3, 2, 1), (3, 2, 2)]


def _sym(A):
    return 0.5 * (A + np.swapaxes(A, -1, -2))


def _strains(rng, n, d, scale=1e-2):
    return _sym(rng.standard_normal((n, d, d)) * scale)


def _algorithm_2(A, dA):
    """Derivative of A^+ in direction dA for one symmetric A with distinct
    eigenvalues, following the steps of Algorithm 2."""
    lam_, V = np.linalg.eigh(A)
    d = A.shape[0]
    dV = np.zeros((d, d))
    dlp = np.zeros(d)
    for i in range(d):
        Ddag = np.array([0.0 if j == i else 1.0 / (lam_[j] - lam_[i]) for j in range(d)])
        Ldag = V @ np.diag(Ddag) @ V.T
        vi = V[:, i]
        dV[:, i] = -Ldag @ dA @ vi
        dli = vi @ dA @ vi
        dlp[i] = 0.0 if lam_[i] < 0 else dli
    Dp = np.diag(np.maximum(lam_, 0.0))
    return dV @ Dp @ V.T + V @ np.diag(dlp) @ V.T + V @ Dp @ dV.T


def test_energy_sum_and_stress_is_energy_derivative():
    rng = np.random.default_rng(11)
    for d in (2, 3):
        A = rng.standard_normal((300, d, d)) * 1e-2
        s = mat.miehe_split(A, LAM, MU)
        e, t = s["e"], s["t"]
        Es = 0.5 * LAM * t ** 2 + MU * np.einsum("nij,nij->n", e, e)
        assert np.allclose(s["E_p"] + s["E_m"], Es, rtol=1e-13, atol=0)
        assert np.allclose(s["sig_p"] + s["sig_m"], LAM * t[:, None, None] * np.eye(d) + 2 * MU * e, rtol=1e-13,
                           atol=1e-12)
        D = _strains(rng, 300, d, 1.0)
        hs = 1e-7
        sp_, sm_ = mat.miehe_split(A + hs * D, LAM, MU), mat.miehe_split(A - hs * D, LAM, MU)
        fdp = (sp_["E_p"] - sm_["E_p"]) / (2 * hs)
        fdm = (sp_["E_m"] - sm_["E_m"]) / (2 * hs)
        # E^+ and E^- are C^1: their differences match the stresses everywhere
        assert np.allclose(fdp, np.einsum("nij,nij->n", s["sig_p"], D), rtol=1e-6, atol=1e-6)
        assert np.allclose(fdm, np.einsum("nij,nij->n", s["sig_m"], D), rtol=1e-6, atol=1e-6)


def test_tangent_matches_difference_of_stress():
    rng = np.random.default_rng(12)
    for d in (2, 3):
        A = rng.standard_normal((400, d, d)) * 1e-2
        s = mat.miehe_split(A, LAM, MU)
        D = _strains(rng, 400, d, 1.0)
        hs = 1e-8
        sp_, sm_ = mat.miehe_split(A + hs * D, LAM, MU), mat.miehe_split(A - hs * D, LAM, MU)
        # only points where neither the trace nor any eigenvalue changes sign
        ok = (np.sign(sp_["t"]) == np.sign(sm_["t"])) & np.all(np.sign(sp_["ev"]) == np.sign(sm_["ev"]), axis=-1)
        assert ok.sum() > 350
        gt = rng.uniform(0, 1, 400)
        st = lambda S: gt[:, None, None] * S["sig_p"] + S["sig_m"]
        fd = (st(sp_) - st(sm_)) / (2 * hs)
        ds = mat.dsigma_miehe(D, s, gt, LAM, MU)
        scale = np.abs(ds).max()
        assert np.abs(fd[ok] - ds[ok]).max() <= 1e-6 * scale


def test_positive_part_derivative_is_algorithm_2_on_distinct_eigenvalues():
    rng = np.random.default_rng(13)
    for d in (2, 3):
        for _ in range(200):
            A = _sym(rng.standard_normal((d, d)))
            lam_ = np.linalg.eigvalsh(A)
            if np.min(np.diff(lam_)) < 1e-3 or np.min(np.abs(lam_)) < 1e-3:
                continue
            dA = _sym(rng.standard_normal((d, d)))
            ev, V = np.linalg.eigh(A)
            ours = mat.dpositive_part(ev, V, dA)
            assert np.allclose(ours, _algorithm_2(A, dA), rtol=1e-10, atol=1e-12)


def test_positive_part_derivative_special_cases():
    rng = np.random.default_rng(14)
    for d in (2, 3):
        dA = _sym(rng.standard_normal((d, d)))
        Q, _ = np.linalg.qr(rng.standard_normal((d, d)))
        # pure tension: e^+ = e, derivative is the identity map; pure compression: zero
        for sign, expect in ((1.0, dA), (-1.0, np.zeros((d, d)))):
            A = Q @ np.diag(sign * rng.uniform(0.5, 2.0, d)) @ Q.T
            ev, V = np.linalg.eigh(A)
            assert np.allclose(mat.dpositive_part(ev, V, dA), expect, atol=1e-13)
        # isotropic strain alpha I: any orthonormal basis is an eigenbasis; the result must not
        # depend on it
        for alpha, expect in ((0.7, dA), (-0.7, np.zeros((d, d)))):
            for _ in range(3):
                B, _ = np.linalg.qr(rng.standard_normal((d, d)))
                assert np.allclose(mat.dpositive_part(np.full(d, alpha), B, dA), expect, atol=1e-13)
    # e = diag(a, -b): the off-diagonal entry of d e^+ is a / (a + b) times that of de
    a, b = 0.3, 0.5
    dA = np.array([[0.2, 1.0], [1.0, -0.4]])
    got = mat.dpositive_part(np.array([-b, a]), np.array([[0.0, 1.0], [1.0, 0.0]]), dA)
    assert np.allclose(got, [[0.2, a / (a + b)], [a / (a + b), 0.0]], atol=1e-15)


def test_coincides_with_volumetric_deviatoric_split_in_pure_tension():
    rng = np.random.default_rng(15)
    for d in (2, 3):
        Q, _ = np.linalg.qr(rng.standard_normal((50, d, d)))
        e = np.einsum("nik,nk,njk->nij", Q, rng.uniform(1e-3, 1e-2, (50, d)), Q)
        sm, sa = mat.miehe_split(e, LAM, MU), mat.amor_split(e, LAM, MU)
        for key in ("sig_p", "sig_m", "E_p", "E_m"):
            assert np.allclose(sm[key], sa[key], rtol=1e-12, atol=1e-9), key
        D = _strains(rng, 50, d, 1.0)
        gt = rng.uniform(0, 1, 50)
        assert np.allclose(mat.dsigma_miehe(D, sm, gt, LAM, MU), mat.dsigma(D, sa["H"], gt, sa["K"], MU), rtol=1e-12,
                           atol=1e-6)


# ---------------------------------------------------------------- on meshes
def _state(dim, N, k, seed, amp=1e-2):
    mesh = fe.Mesh(dim, N, k)
    rng = np.random.default_rng(seed)
    u = amp * rng.standard_normal((dim, mesh.n_nodes))
    phi = rng.uniform(0.1, 1.0, mesh.n_nodes)
    phit = rng.uniform(0.1, 1.0, mesh.n_nodes)
    return mesh, u, phi, phit


def _split_U(U, mesh):
    d, nn = mesh.dim, mesh.n_nodes
    return U[: d * nn].reshape(d, nn), U[d * nn:]


def _branches(mesh, u, phi, phit):
    tb = fe.TensorBasis(mesh.dim, mesh.k)
    cd = op.CellData(mesh, tb, MAT, u, phi, phit, np.arange(mesh.n_cells))
    return np.sign(cd.split["t"]), np.sign(cd.split["ev"])


@pytest.mark.parametrize("dim,N,k", CASES)
def test_jacobian_matches_central_difference_of_residual(dim, N, k):
    mesh, u, phi, phit = _state(dim, N, k, seed=22)
    G = op.assemble_jacobian(mesh, MAT, u, phi, phit)
    rng = np.random.default_rng(23)
    U = np.concatenate([u.ravel(), phi])
    V = rng.standard_normal(U.size)
    V[: dim * mesh.n_nodes] *= 1e-2
    hs = 1e-7
    Up, Um = U + hs * V, U - hs * V
    tp, ep = _branches(mesh, *_split_U(Up, mesh), phit)
    tm, em = _branches(mesh, *_split_U(Um, mesh), phit)
    assert int((tp != tm).sum()) == 0 and int((ep != em).sum()) == 0
    fd = (op.residual(mesh, MAT, *_split_U(Up, mesh), phit) - op.residual(mesh, MAT, *_split_U(Um, mesh), phit)) / (2 * hs)
    GV = G @ V
    assert np.linalg.norm(fd - GV) <= 1e-6 * np.linalg.norm(GV)


@pytest.mark.parametrize("dim,N,k", CASES)
def test_residual_is_energy_gradient(dim, N, k):
    mesh, u, phi, _ = _state(dim, N, k, seed=24)
    R = op.residual(mesh, MAT, u, phi, phi)
    rng = np.random.default_rng(25)
    U = np.concatenate([u.ravel(), phi])
    for _ in range(3):
        V = rng.standard_normal(U.size)
        V[: dim * mesh.n_nodes] *= 1e-2
        hs = 1e-6
        Ep = op.energy(mesh, MAT, *_split_U(U + hs * V, mesh))
        Em = op.energy(mesh, MAT, *_split_U(U - hs * V, mesh))
        assert abs((Ep - Em) / (2 * hs) - R @ V) <= 1e-7 * abs(R @ V) + 1e-10


@pytest.mark.parametrize("dim,N,k", CASES)
def test_block_structure_and_symmetry(dim, N, k):
    mesh, u, phi, phit = _state(dim, N, k, seed=26)
    G = op.assemble_jacobian(mesh, MAT, u, phi, phit).tocsr()
    nu = dim * mesh.n_nodes
    Guu, Gup = G[:nu, :nu], G[:nu, nu:]
    assert Gup.count_nonzero() == 0
    assert abs(Guu - Guu.T).max() <= 1e-13 * abs(Guu).max()
