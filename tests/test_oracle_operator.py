"""Pins of the oracle's residual and Jacobian against the mathematics.

Each check is independent of the oracle's own element loops: finite
differences of the residual and of the discrete energy, exact 1D
polynomial integrals assembled by Kronecker products, rigid-body modes,
a patch test, and the structural facts the paper states (symmetric
diagonal blocks, G_{u phi} = 0 because phi~ is frozen, Section 3.2/3.3).
"""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle import fe, material as mat
from oracle import operator as op

CASES = [(2, 4, 1), (2, 3, 2), (3, 2, 1), (3, 2, 2)]
MAT = op.Material(lam=121.15e3, mu=80.77e3, Gc=2.7, eps=0.05, kappa=1e-10)


def _state(dim, N, k, seed=0, amp=1e-2):
    mesh = fe.Mesh(dim, N, k)
    rng = np.random.default_rng(seed)
    u = amp * rng.standard_normal((dim, mesh.n_nodes))
    phi = rng.uniform(0.1, 1.0, mesh.n_nodes)
    phit = rng.uniform(0.1, 1.0, mesh.n_nodes)
    return mesh, u, phi, phit


def _split(U, mesh):
    d, nn = mesh.dim, mesh.n_nodes
    return U[: d * nn].reshape(d, nn), U[d * nn:]


def _traces(mesh, u, phi, phit):
    tb = fe.TensorBasis(mesh.dim, mesh.k)
    cd = op.CellData(mesh, tb, MAT, u, phi, phit, np.arange(mesh.n_cells))
    return cd.split["t"]


# ---------------------------------------------------------------- split
def test_split_energy_sum_and_stress_derivatives():
    rng = np.random.default_rng(1)
    for d in (2, 3):
        A = rng.standard_normal((200, d, d)) * 1e-2
        s = mat.amor_split(A, MAT.lam, MAT.mu)
        e, t = s["e"], s["t"]
        Es = 0.5 * MAT.lam * t ** 2 + MAT.mu * np.einsum("nij,nij->n", e, e)
        assert np.allclose(s["E_p"] + s["E_m"], Es, rtol=1e-13, atol=0)
        # sigma^+ = dE^+/de and sigma^- = dE^-/de by central differences
        D = rng.standard_normal((200, d, d))
        D = 0.5 * (D + np.swapaxes(D, 1, 2))
        hs = 1e-7
        sp_, sm_ = mat.amor_split(A + hs * D, MAT.lam, MAT.mu), mat.amor_split(A - hs * D, MAT.lam, MAT.mu)
        ok = np.sign(sp_["t"]) == np.sign(sm_["t"])
        fdp = (sp_["E_p"] - sm_["E_p"]) / (2 * hs)
        fdm = (sp_["E_m"] - sm_["E_m"]) / (2 * hs)
        assert np.allclose(fdp[ok], np.einsum("nij,nij->n", s["sig_p"], D)[ok], rtol=1e-6, atol=1e-6)
        assert np.allclose(fdm[ok], np.einsum("nij,nij->n", s["sig_m"], D)[ok], rtol=1e-6, atol=1e-6)
        # tangent of g sigma^+ + sigma^-
        gt = rng.uniform(0, 1, 200)
        st = lambda S: gt[:, None, None] * S["sig_p"] + S["sig_m"]
        fd = (st(sp_) - st(sm_)) / (2 * hs)
        ds = mat.dsigma(D, s["H"], gt, s["K"], MAT.mu)
        assert np.allclose(fd[ok], ds[ok], rtol=1e-6, atol=1e-3)


def test_heaviside_at_zero_is_one():
    s = mat.amor_split(np.zeros((1, 2, 2)), MAT.lam, MAT.mu)
    assert s["H"][0] == 1.0


# ---------------------------------------------------------------- Jacobian
@pytest.mark.parametrize("dim,N,k", CASES)
def test_jacobian_matches_central_difference_of_residual(dim, N, k):
    mesh, u, phi, phit = _state(dim, N, k, seed=2)
    G = op.assemble_jacobian(mesh, MAT, u, phi, phit)
    rng = np.random.default_rng(3)
    U = np.concatenate([u.ravel(), phi])
    V = rng.standard_normal(U.size)
    V[: dim * mesh.n_nodes] *= 1e-2
    hs = 1e-6
    Up, Um = U + hs * V, U - hs * V
    # no quadrature point may change its tension/compression branch
    tp, tm = _traces(mesh, *_split(Up, mesh), phit), _traces(mesh, *_split(Um, mesh), phit)
    assert int((np.sign(tp) != np.sign(tm)).sum()) == 0
    Rp = op.residual(mesh, MAT, *_split(Up, mesh), phit)
    Rm = op.residual(mesh, MAT, *_split(Um, mesh), phit)
    fd = (Rp - Rm) / (2 * hs)
    GV = G @ V
    assert np.linalg.norm(fd - GV) <= 1e-7 * np.linalg.norm(GV)


@pytest.mark.parametrize("dim,N,k", CASES)
def test_residual_is_energy_gradient(dim, N, k):
    mesh, u, phi, _ = _state(dim, N, k, seed=4)
    R = op.residual(mesh, MAT, u, phi, phi)           # phi~ = phi
    rng = np.random.default_rng(5)
    U = np.concatenate([u.ravel(), phi])
    for _ in range(3):
        V = rng.standard_normal(U.size)
        V[: dim * mesh.n_nodes] *= 1e-2
        hs = 1e-6
        Ep = op.energy(mesh, MAT, *_split(U + hs * V, mesh))
        Em = op.energy(mesh, MAT, *_split(U - hs * V, mesh))
        fd = (Ep - Em) / (2 * hs)
        assert abs(fd - R @ V) <= 1e-7 * abs(R @ V) + 1e-10


@pytest.mark.parametrize("dim,N,k", CASES)
def test_block_structure_and_symmetry(dim, N, k):
    mesh, u, phi, phit = _state(dim, N, k, seed=6)
    G = op.assemble_jacobian(mesh, MAT, u, phi, phit).tocsr()
    nu = dim * mesh.n_nodes
    Guu, Gpp, Gup = G[:nu, :nu], G[nu:, nu:], G[:nu, nu:]
    assert Gup.count_nonzero() == 0
    assert abs(Guu - Guu.T).max() <= 1e-14 * abs(Guu).max()
    assert abs(Gpp - Gpp.T).max() <= 1e-14 * abs(Gpp).max()
    # both diagonal blocks positive definite on the free dofs (smallest eig of a small case)
    if mesh.n_dofs < 800:
        p = op.free_vector(mesh, np.zeros(mesh.n_nodes), True)
        A = op.constrain(G, p).toarray()
        assert np.linalg.eigvalsh(0.5 * (A[:nu, :nu] + A[:nu, :nu].T)).min() > 0
        assert np.linalg.eigvalsh(A[nu:, nu:]).min() > 0


def _exact_1d(k, h):
    """Exact 1D element matrices by polynomial integration of the Lagrange
    polynomials built from a Vandermonde solve (independent of quadrature)."""
    nodes = np.arange(k + 1) / k
    V = np.vander(nodes, k + 1, increasing=True)
    C = np.linalg.solve(V, np.eye(k + 1))            # column i: coefficients of l_i
    polys = [np.polynomial.Polynomial(C[:, i]) for i in range(k + 1)]
    def integ(p):
        P = p.integ()
        return P(1.0) - P(0.0)
    M = np.array([[integ(a * b) for b in polys] for a in polys]) * h
    K = np.array([[integ(a.deriv() * b.deriv()) for b in polys] for a in polys]) / h
    Cm = np.array([[integ(a.deriv() * b) for b in polys] for a in polys])   # test derivative on rows
    return M, K, Cm


def _global_1d(E, N, k):
    M = k * N + 1
    out = np.zeros((M, M))
    for c in range(N):
        out[k * c: k * c + k + 1, k * c: k * c + k + 1] += E
    return out


def test_q1_exact_1d_matrices_closed_form():
    M, K, _ = _exact_1d(1, 0.25)
    assert np.allclose(M, 0.25 / 6 * np.array([[2, 1], [1, 2]]), atol=1e-15)
    assert np.allclose(K, 4.0 * np.array([[1, -1], [-1, 1]]), atol=1e-14)


def _kron_all(mats):
    out = mats[0]
    for m_ in mats[1:]:
        out = np.kron(m_, out)      # axis 0 is the fastest node index
    return out


@pytest.mark.parametrize("dim,N,k", CASES)
def test_phase_block_at_zero_displacement_is_kronecker(dim, N, k):
    # u = 0: E^+ = 0, so G_phiphi = Gc (M/eps + eps K) with M, K Kronecker products
    mesh, _, phi, phit = _state(dim, N, k, seed=7)
    u = np.zeros((dim, mesh.n_nodes))
    G = op.assemble_jacobian(mesh, MAT, u, phi, phit).tocsr()
    nu = dim * mesh.n_nodes
    M1e, K1e, _ = _exact_1d(k, mesh.h)
    M1, K1 = _global_1d(M1e, N, k), _global_1d(K1e, N, k)
    Mg = _kron_all([M1] * dim)
    Kg = sum(_kron_all([K1 if a == b else M1 for b in range(dim)]) for a in range(dim))
    ref = MAT.Gc * (Mg / MAT.eps + MAT.eps * Kg)
    got = G[nu:, nu:].toarray()
    assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()
    # G_phi u vanishes at u = 0 (sigma^+(0) = 0)
    assert abs(G[nu:, :nu]).max() == 0.0


@pytest.mark.parametrize("dim,N,k", CASES)
def test_displacement_block_at_intact_state_is_linear_elasticity(dim, N, k):
    # phi~ = 1: g = 1, delta sigma = lambda tr(de) I + 2 mu de for either branch
    mesh, u, phi, _ = _state(dim, N, k, seed=8)
    phit = np.ones(mesh.n_nodes)
    G = op.assemble_jacobian(mesh, MAT, u, phi, phit).tocsr()
    nu, nn = dim * mesh.n_nodes, mesh.n_nodes
    M1e, K1e, C1e = _exact_1d(k, mesh.h)
    M1, K1, C1 = _global_1d(M1e, N, k), _global_1d(K1e, N, k), _global_1d(C1e, N, k)

    def S(a, b):  # integral of d_a N_p (test) d_b N_q (trial)
        mats = []
        for m_ in range(dim):
            if m_ == a and m_ == b:
                mats.append(K1)
            elif m_ == a:
                mats.append(C1)
            elif m_ == b:
                mats.append(C1.T)
            else:
                mats.append(M1)
        return _kron_all(mats)

    ref = np.zeros((nu, nu))
    lap = sum(S(a, a) for a in range(dim))
    for c in range(dim):
        for cp in range(dim):
            blk = MAT.lam * S(c, cp) + MAT.mu * S(cp, c)
            if c == cp:
                blk = blk + MAT.mu * lap
            ref[c * nn:(c + 1) * nn, cp * nn:(cp + 1) * nn] = blk
    got = G[:nu, :nu].toarray()
    assert np.abs(got - ref).max() <= 1e-11 * np.abs(ref).max()


@pytest.mark.parametrize("dim,N,k", CASES)
def test_rigid_body_modes_in_kernel(dim, N, k):
    mesh, u, phi, phit = _state(dim, N, k, seed=9)
    G = op.assemble_jacobian(mesh, MAT, u, phi, phit).tocsr()
    X = fe.Mesh(dim, N, k)
    from synth import node_coords
    xy = node_coords(dim, N, k)
    nn = mesh.n_nodes
    modes = []
    for c in range(dim):
        r = np.zeros((dim, nn)); r[c] = 1.0; modes.append(r)
    pairs = [(0, 1)] if dim == 2 else [(0, 1), (0, 2), (1, 2)]
    for a, b in pairs:
        r = np.zeros((dim, nn)); r[a] = -xy[:, b]; r[b] = xy[:, a]; modes.append(r)
    scale = abs(G).max()
    for r in modes:
        V = np.concatenate([r.ravel(), np.zeros(nn)])
        assert np.abs(G @ V).max() <= 1e-11 * scale


@pytest.mark.parametrize("dim,N,k", [(2, 4, 1), (2, 3, 2), (3, 3, 2)])
def test_patch_test_linear_field(dim, N, k):
    # all-boundary Dirichlet data of a linear field: the solve reproduces it
    mesh, u, phi, _ = _state(dim, N, k, seed=10)
    phit = np.ones(mesh.n_nodes)
    G = op.assemble_jacobian(mesh, MAT, u, phi, phit).tocsr()
    nn, nu = mesh.n_nodes, dim * mesh.n_nodes
    from synth import node_coords
    X = node_coords(dim, N, k)
    rng = np.random.default_rng(11)
    A, c0 = rng.standard_normal((dim, dim)), rng.standard_normal(dim)
    ulin = (X @ A.T + c0).T.ravel()
    bnd = np.zeros(nn, bool)
    for a in range(dim):
        bnd |= mesh.boundary_nodes(a)
    fixed = np.concatenate([bnd] * dim)
    Guu = G[:nu, :nu].tocsr()
    free = ~fixed
    rhs = -Guu[free][:, fixed] @ ulin[fixed]
    sol = spla.spsolve(Guu[free][:, free].tocsc(), rhs)
    assert np.abs(sol - ulin[free]).max() <= 1e-10 * np.abs(ulin).max()
    # and the interior residual rows of a linear field vanish at constant phi~
    R = op.residual(mesh, MAT, ulin.reshape(dim, nn), phi, phit)
    assert np.abs(R[:nu][free]).max() <= 1e-9 * np.abs(R[:nu]).max()


def test_constraints_identity_rows_and_columns():
    mesh, u, phi, phit = _state(2, 3, 2, seed=12)
    G = op.assemble_jacobian(mesh, MAT, u, phi, phit)
    act = (np.random.default_rng(0).random(mesh.n_nodes) < 0.3).astype(np.uint8)
    p = op.free_vector(mesh, act, True)
    A = op.constrain(G, p).toarray()
    for i in np.flatnonzero(p == 0):
        e = np.zeros(mesh.n_dofs); e[i] = 1.0
        assert np.array_equal(A[i], e) and np.array_equal(A[:, i], e)
    free = p == 1
    assert np.array_equal(A[np.ix_(free, free)], G.toarray()[np.ix_(free, free)])


@pytest.mark.parametrize("dim,N,k", [(2, 4, 2), (3, 3, 2)])
def test_sampled_rows_agree_with_assembly(dim, N, k):
    mesh, u, phi, phit = _state(dim, N, k, seed=13)
    G = op.assemble_jacobian(mesh, MAT, u, phi, phit)
    act = (np.random.default_rng(1).random(mesh.n_nodes) < 0.2).astype(np.uint8)
    p = op.free_vector(mesh, act, True)
    A = op.constrain(G, p)
    x = np.random.default_rng(2).standard_normal(mesh.n_dofs)
    nodes = np.random.default_rng(3).choice(mesh.n_nodes, 15, replace=False)
    rows = np.stack([c * mesh.n_nodes + nodes for c in range(dim + 1)])
    assert np.allclose(op.apply_rows(mesh, MAT, u, phi, phit, p, x, nodes), (A @ x)[rows], rtol=1e-13, atol=1e-9)
    assert np.allclose(op.apply_rows(mesh, MAT, u, phi, phit, p, x, nodes, transpose=True),
                       (A.T @ x)[rows], rtol=1e-13, atol=1e-9)
    assert np.allclose(op.diag_rows(mesh, MAT, u, phi, phit, p, nodes), A.diagonal()[rows], rtol=1e-14)
    R = op.residual(mesh, MAT, u, phi, phit)
    assert np.allclose(op.residual_rows(mesh, MAT, u, phi, phit, nodes), R[rows], rtol=1e-13, atol=1e-9)


@pytest.mark.parametrize("dim,N,k", [(2, 4, 2), (3, 2, 2)])
def test_parameter_vjp_against_differences(dim, N, k):
    mesh, u, phi, phit = _state(dim, N, k, seed=14)
    v = np.random.default_rng(15).standard_normal(mesh.n_dofs)
    dGc, deps = op.param_vjp(mesh, MAT, u, phi, phit, v)
    # R is affine in Gc: any step gives the exact derivative
    m1 = op.Material(MAT.lam, MAT.mu, MAT.Gc + 0.5, MAT.eps, MAT.kappa)
    m0 = op.Material(MAT.lam, MAT.mu, MAT.Gc - 0.5, MAT.eps, MAT.kappa)
    fd = v @ (op.residual(mesh, m1, u, phi, phit) - op.residual(mesh, m0, u, phi, phit)) / 1.0
    assert abs(fd - dGc) <= 1e-12 * (abs(dGc) + 1)
    he = 1e-4 * MAT.eps   # truncation ~ (he/eps)^2 ~ 1e-8, large enough to beat rounding in R
    m1 = op.Material(MAT.lam, MAT.mu, MAT.Gc, MAT.eps + he, MAT.kappa)
    m0 = op.Material(MAT.lam, MAT.mu, MAT.Gc, MAT.eps - he, MAT.kappa)
    fd = v @ (op.residual(mesh, m1, u, phi, phit) - op.residual(mesh, m0, u, phi, phit)) / (2 * he)
    assert abs(fd - deps) <= 1e-7 * abs(deps)


def test_fd_gap_with_branch_crossing_cells_excluded():
    """The crossing-cell exclusion used by the full-size autograd check, run on the oracle itself:
    with a step large enough that many points change branch, the central difference misses the
    tangent by far more than rounding, and taking the crossing cells out of both sides brings the
    gap down to rounding.  A step so small that no point crosses changes nothing."""
    import fdcheck
    from synth import CONFIGS, make_inputs
    Mesh = fe.Mesh
    cfg = CONFIGS["C5"].with_(N=6)
    inp = make_inputs(cfg, ("cotangent", "directions"))
    mesh = Mesh(cfg.dim, cfg.N, cfg.k)
    m = op.material_of(cfg)
    d, nn = cfg.dim, cfg.n_nodes
    U = np.concatenate([inp["u"].ravel(), inp["phi"]])
    pt, v = inp["phi_tilde"], inp["cotangent"]
    G = op.assemble_jacobian(mesh, m, inp["u"], inp["phi"], pt)
    gT = G.T @ v
    # displacement-only directions: on a fixed branch R is then at most quadratic along the line,
    # so the central difference is exact up to rounding at any step
    dirs = inp["directions"][:6].copy()
    dirs[:, d * nn:] = 0.0

    def full_sums(h):
        fd, ad = [], []
        for dv in dirs:
            Rp = op.residual(mesh, m, (U + h * dv)[: d * nn].reshape(d, nn), (U + h * dv)[d * nn:], pt)
            Rm = op.residual(mesh, m, (U - h * dv)[: d * nn].reshape(d, nn), (U - h * dv)[d * nn:], pt)
            fd.append(float(v @ (Rp - Rm)) / (2 * h))
            ad.append(float(gT @ dv))
        return fd, ad

    h = 2e-3   # moves u by ~2e-6 per node: about 100 of the 5,832 points change branch
    res = fdcheck.excluded_gaps(mesh, m, U, pt, v, dirs, h, *full_sums(h))
    assert all(r[0] > 0 and r[1] < mesh.n_cells // 2 for r in res)
    assert min(r[2] for r in res) > 1e-3                       # crossings spoil the difference
    assert max(r[3] for r in res) <= 1e-11                     # and nothing else does
    res = fdcheck.excluded_gaps(mesh, m, U, pt, v, dirs, 1e-6, *full_sums(1e-6))
    assert all(r[0] == 0 and r[3] == r[2] and r[2] <= 1e-8 for r in res)
