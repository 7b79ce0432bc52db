"""Pins of the oracle's multigrid, Krylov and Newton pieces."""
import os

import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from oracle import fe, krylov, multigrid as mg, newton
from oracle import operator as op
from oracle.splitmix import mix64, GAMMA, uniform_pm1
from synth import CONFIGS, level_list, make_inputs, node_coords

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ------------------------------------------------------------- SplitMix64
def test_splitmix_published_vector():
    ref = [int(l) for l in open(os.path.join(GOLDEN, "splitmix64_seed1234567.txt")) if l.strip() and l[0] != "#"]
    s = np.uint64(1234567)
    with np.errstate(over="ignore"):
        got = [int(mix64(s + np.uint64(n) * GAMMA)) for n in range(1, 6)]
    assert got == ref


def test_uniform_range_and_streams():
    a = uniform_pm1(7, 0, 100000)
    b = uniform_pm1(7, 1, 100000)
    assert a.min() >= -1 and a.max() < 1 and abs(a.mean()) < 0.01
    assert not np.array_equal(a[:10], b[:10])


# ------------------------------------------------------------- transfers
@pytest.mark.parametrize("fine,coarse", [((8, 2), (4, 2)), ((4, 4), (4, 2)), ((4, 2), (4, 1)),
                                         ((6, 3), (3, 3)), ((4, 4), (4, 1))])
def test_prolongation_reproduces_coarse_polynomials(fine, coarse):
    mf, mc = fe.Mesh(1, *fine), fe.Mesh(1, *coarse)
    P1 = mg.prolongation_1d(mf, mc)
    xf = np.arange(mf.M) / (mf.k * mf.N)
    xc = np.arange(mc.M) / (mc.k * mc.N)
    rng = np.random.default_rng(0)
    for deg in range(mc.k + 1):
        f = np.polynomial.Polynomial(rng.standard_normal(deg + 1))
        assert np.allclose(P1 @ f(xc), f(xf), atol=1e-12)
    # injection: coarse node positions are fine node positions
    idx = mg.injection_index(fe.Mesh(2, *fine), fe.Mesh(2, *coarse))
    Xf, Xc = node_coords(2, *fine), node_coords(2, *coarse)
    assert np.allclose(Xf[idx], Xc, atol=0)


def test_restriction_is_adjoint_and_masked():
    cfg = CONFIGS["C2"].with_(N=8, n_h_levels=2)
    inp = make_inputs(cfg)
    H = mg.Hierarchy(cfg, level_list(cfg), inp["u"], inp["phi"], inp["phi_tilde"], inp["active"])
    P = H.P[1]
    f, c = H.levels[1], H.levels[0]
    rng = np.random.default_rng(1)
    x, y = rng.standard_normal(f.mesh.n_dofs), rng.standard_normal(c.mesh.n_dofs)
    assert abs((P.T @ x) @ y - x @ (P @ y)) <= 1e-12 * np.linalg.norm(x) * np.linalg.norm(y)
    assert np.all((P @ y)[f.pvec == 0] == 0) and np.all((P.T @ x)[c.pvec == 0] == 0)


# ------------------------------------------------------------- Chebyshev
def test_chebyshev_residual_polynomial_closed_form():
    # diag(lam), D = I: 1 - lam p(lam) = T_s((theta - lam)/delta) / T_s(theta/delta)
    class L:
        pass
    n, nu = 40, 25
    lam = np.linspace(0.05, 2.0, n)
    lev = L()
    lev.nu, lev.D = nu, np.ones(n)
    lev.Ablk = sp.diags(lam)
    lmax = (2.0, 2.0)
    for s in (1, 2, 4, 5, 7):
        x = mg.chebyshev_block(lev, lmax, np.ones(n), s, 0.24, 1.2)
        lo, hi = 0.24 * 2.0, 1.2 * 2.0
        th, de = (hi + lo) / 2, (hi - lo) / 2
        T = np.polynomial.chebyshev.Chebyshev.basis(s)
        assert np.allclose(1 - lam * x, T((th - lam) / de) / T(th / de), atol=1e-13)


# ------------------------------------------------------------- Lanczos
def test_cg_lanczos_full_space_gives_exact_spectrum_top():
    rng = np.random.default_rng(2)
    n = 12
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    A = Q @ np.diag(np.linspace(1, 50, n)) @ Q.T
    D = np.diag(A).copy()
    al, be = mg.cg_lanczos(A, D, rng.standard_normal(n), n)
    ref = sla.eigh(A, np.diag(D), eigvals_only=True)[-1]
    assert abs(mg.lanczos_ritz_max(al, be) - ref) <= 1e-8 * ref


def test_lanczos_bounds_on_c1_blocks():
    cfg = CONFIGS["C1"]
    inp = make_inputs(cfg)
    H = mg.Hierarchy(cfg, level_list(cfg), inp["u"], inp["phi"], inp["phi_tilde"], inp["active"])
    lev = H.levels[1]
    nu = lev.nu
    for b, sl in ((0, slice(0, nu)), (1, slice(nu, None))):
        A = lev.A[sl, sl].toarray()
        ev = sla.eigh(A, np.diag(lev.D[sl]), eigvals_only=True)[-1]
        est = H.lam[1][b]
        assert est <= ev * (1 + 1e-12) and est >= 0.95 * ev


def test_lanczos_fully_masked_block_is_one():
    al, be = mg.cg_lanczos(np.eye(3), np.ones(3), np.zeros(3), 15)
    assert al == [] and mg.lanczos_ritz_max(al, be) == 1.0


# ------------------------------------------------------------- V-cycle / coarse
def test_single_level_cycle_is_exact_solve():
    cfg = CONFIGS["C2"].with_(N=4, n_h_levels=1)
    inp = make_inputs(cfg, ("rhs",))
    H = mg.Hierarchy(cfg, level_list(cfg), inp["u"], inp["phi"], inp["phi_tilde"], inp["active"])
    A = H.levels[0].A
    b = inp["rhs"]
    assert np.allclose(H.vcycle(b), spla.spsolve(A.tocsc(), b), rtol=1e-10, atol=1e-14)


@pytest.mark.parametrize("name,kw", [("C1", dict(N=16)), ("C2", dict(N=8, n_h_levels=2)),
                                     ("C3", dict(N=4, n_h_levels=2)), ("C4", dict(dim=2, N=8, n_h_levels=2))])
def test_two_grid_error_operator_contracts(name, kw):
    # intact material (phi = phi~ = 1), the workload's displacement, no active set:
    # the two-grid error operator of the V-cycle must contract (power iteration)
    cfg = CONFIGS[name].with_(**kw)
    inp = make_inputs(cfg)
    lv = level_list(cfg)[-2:]
    one = np.ones(cfg.n_nodes)
    H = mg.Hierarchy(cfg, lv, inp["u"], one, one, np.zeros(cfg.n_nodes, np.uint8))
    A = H.levels[-1].A
    rng = np.random.default_rng(3)
    e = rng.standard_normal(A.shape[0])
    rho = 0.0
    for _ in range(25):
        e_new = e - H.vcycle(A @ e)
        rho = np.linalg.norm(e_new) / np.linalg.norm(e)
        e = e_new / np.linalg.norm(e_new)
    assert rho < 0.8


@pytest.mark.parametrize("name,kw,split", [("C2", dict(N=4, n_h_levels=1, p_coarse=()), "amor"),
                                           ("C2", dict(N=4, n_h_levels=1, p_coarse=()), "miehe"),
                                           ("C3", dict(N=2, n_h_levels=1, p_coarse=()), "amor"),
                                           ("C3", dict(N=2, n_h_levels=1, p_coarse=()), "miehe")])
def test_coarse_blocks_are_positive_semidefinite(name, kw, split):
    # the premise of the Cholesky-only coarse solve: on a random state, with phi~ outside [0, 1]
    # (linear extrapolation can leave it) and no Dirichlet rows, both diagonal blocks of G are
    # symmetric with no eigenvalue below -1e-12 of the largest (g >= 0, convex energies in e)
    cfg = CONFIGS[name].with_(split=split, dirichlet=False, **kw)
    inp = make_inputs(cfg)
    rng = np.random.default_rng(11)
    pt = rng.uniform(-0.3, 1.3, cfg.n_nodes)
    u = rng.standard_normal((cfg.dim, cfg.n_nodes)) * 1e-3
    mesh = fe.Mesh(cfg.dim, cfg.N, cfg.k)
    A = op.assemble_jacobian(mesh, op.material_of(cfg), u, inp["phi"], pt).toarray()
    nu = cfg.dim * mesh.n_nodes
    for B in (A[:nu, :nu], A[nu:, nu:]):
        assert np.abs(B - B.T).max() <= 1e-13 * np.abs(B).max()
        ev = np.linalg.eigvalsh(B)
        assert ev.min() >= -1e-12 * ev.max()


def test_singular_coarse_block_is_rejected():
    # kappa = 0 and phi = phi~ = 0 at u = 0: g = 0 and tr e = 0 (tension branch), so every free
    # displacement row of G is zero; the coarse solve reports it instead of returning inf/NaN
    cfg = CONFIGS["C1"].with_(N=4, n_h_levels=1, p_coarse=(), kappa=0.0)
    z = np.zeros(cfg.n_nodes)
    with pytest.raises(np.linalg.LinAlgError, match="singular"):
        mg.Hierarchy(cfg, [(cfg.N, cfg.k)], np.zeros((cfg.dim, cfg.n_nodes)), z, z, np.zeros(cfg.n_nodes, np.uint8))


def test_indefinite_coarse_block_takes_the_lu_path():
    # kappa < 0 makes g negative where phi is small, so G_uu is indefinite: the Cholesky fails,
    # the LU solves, and the result satisfies the block lower-triangular system exactly
    cfg = CONFIGS["C1"].with_(N=8, n_h_levels=1, p_coarse=(), kappa=-0.5, phi_mode="smooth")
    inp = make_inputs(cfg, ("rhs",))
    H = mg.Hierarchy(cfg, [(cfg.N, cfg.k)], inp["u"], inp["phi"], inp["phi_tilde"], inp["active"])
    cs = H.coarse
    assert cs.fu[0] == "lu" and cs.fp[0] == "chol"
    assert np.linalg.eigvalsh(cs.Auu).min() < 0
    b = inp["rhs"]
    x = cs.solve(b)
    nu = cs.nu
    Lx = np.concatenate([cs.Auu @ x[:nu], cs.Apu @ x[:nu] + cs.App @ x[nu:]])
    assert np.abs(Lx - b).max() <= 1e-10 * np.abs(b).max()


@pytest.mark.parametrize("name,kw", [("C1", dict(N=16, n_h_levels=2)), ("C2", dict(N=8, n_h_levels=2)),
                                     ("C1", dict(dim=3, N=4, n_h_levels=2))])
def test_two_grid_contracts_on_the_slit_mesh(name, kw):
    # intact material on the slit mesh, no active set: the two-grid error operator with the
    # slit-aware transfers contracts like on the uniform mesh
    cfg = CONFIGS[name].with_(slit=True, **kw)
    inp = make_inputs(cfg)
    one = np.ones(cfg.n_nodes)
    H = mg.Hierarchy(cfg, level_list(cfg)[-2:], inp["u"], one, one, np.zeros(cfg.n_nodes, np.uint8))
    A = H.levels[-1].A
    e = np.random.default_rng(3).standard_normal(A.shape[0])
    rho = 0.0
    for _ in range(25):
        e_new = e - H.vcycle(A @ e)
        rho = np.linalg.norm(e_new) / np.linalg.norm(e)
        e = e_new / np.linalg.norm(e_new)
    assert rho < 0.8, rho


# ------------------------------------------------------------- FGMRES
def test_fgmres_against_direct_solve_nonsymmetric():
    rng = np.random.default_rng(4)
    n = 60
    A = np.eye(n) * 4 + rng.standard_normal((n, n)) * 0.3
    b = rng.standard_normal(n)
    Minv = np.linalg.inv(np.diag(np.diag(A)))
    for m in (5, 30):
        x, info = krylov.fgmres(lambda v: A @ v, lambda v: Minv @ v, b, m=m, rtol=1e-10, max_iter=500)
        assert info["converged"]
        assert np.linalg.norm(b - A @ x) <= 1e-10 * np.linalg.norm(b)
        assert np.allclose(x, np.linalg.solve(A, b), rtol=1e-8)


def test_fgmres_reports_nonconvergence():
    rng = np.random.default_rng(5)
    A = np.diag(np.linspace(1, 1e4, 80))
    b = rng.standard_normal(80)
    x, info = krylov.fgmres(lambda v: A @ v, lambda v: v, b, m=5, rtol=1e-12, max_iter=3)
    assert not info["converged"] and info["iterations"] == 3


def test_gmg_fgmres_c1_vs_spsolve():
    cfg = CONFIGS["C1"]
    inp = make_inputs(cfg, ("rhs",))
    H = mg.Hierarchy(cfg, level_list(cfg), inp["u"], inp["phi"], inp["phi_tilde"], inp["active"])
    A = H.levels[-1].A
    b = H.levels[-1].pvec * inp["rhs"]
    x, info = krylov.fgmres(lambda v: A @ v, H.vcycle, b, cfg.restart, cfg.rtol, cfg.max_iter)
    assert info["converged"] and np.linalg.norm(b - A @ x) <= 1e-8 * np.linalg.norm(b)
    xs = spla.spsolve(A.tocsc(), b)
    cond = np.linalg.cond(A.toarray())
    assert np.linalg.norm(x - xs) <= cond * 1e-8 * np.linalg.norm(xs)


# ------------------------------------------------------------- Newton
def test_active_set_sign_convention():
    # phi = phi_old: active exactly where the phase-field residual is negative
    mesh = fe.Mesh(2, 3, 1)
    R = np.zeros(mesh.n_dofs)
    nn = mesh.n_nodes
    R[2 * nn:] = np.linspace(-1, 1, nn)
    act, _ = newton.active_set(mesh, R, np.ones(nn), np.ones(nn))
    assert np.array_equal(act.astype(bool), R[2 * nn:] < 0)
    # phi above phi_old pushes towards active
    act2, _ = newton.active_set(mesh, np.zeros(mesh.n_dofs), np.full(nn, 1.0), np.full(nn, 0.5))
    assert act2.all()


def test_newton_step_solves_linearised_system():
    cfg = CONFIGS["C2"].with_(N=8, n_h_levels=2)
    inp = make_inputs(cfg)
    out = newton.newton_step(cfg, level_list(cfg), inp["u"], inp["phi"], inp["phi_old"], inp["phi_tilde"])
    A = out["hier"].levels[-1].A
    assert out["info"]["converged"]
    assert np.linalg.norm(out["b"] - A @ out["dU"]) <= 1e-8 * np.linalg.norm(out["b"])
    # constrained dofs do not move
    p = out["hier"].levels[-1].pvec
    assert np.all(out["dU"][p == 0] == 0)


@pytest.mark.parametrize("name,kw", [("C1", {}), ("C2", dict(N=16, n_h_levels=3))])
def test_active_set_loop_stops_at_a_fixed_point_with_a_superlinear_tail(name, kw):
    # Algorithm 1 to its stopping test: the final active set is a fixed point of the rule, the
    # free residual is below tol times the first one, and the Newton tail contracts
    # superlinearly (the Jacobian is the derivative of the residual).
    cfg = CONFIGS[name].with_(**kw)
    inp = make_inputs(cfg)
    out = newton.pdas_solve(cfg, level_list(cfg), inp["u"], inp["phi"], inp["phi_old"], inp["phi_tilde"],
                            max_newton=20, tol=1e-8)
    assert out["converged"] and 1 <= out["steps"] <= 20
    mesh = fe.Mesh(cfg.dim, cfg.N, cfg.k)
    m = op.material_of(cfg)
    R = op.residual(mesh, m, out["u"], out["phi"], inp["phi_tilde"])
    act, _ = newton.active_set(mesh, R, out["phi"], inp["phi_old"], cfg.as_c)
    assert np.array_equal(act, out["active"])
    pvec = op.free_vector(mesh, act, cfg.dirichlet)
    assert np.linalg.norm(pvec * R) <= 1e-8 * out["norms"][0]
    r = out["norms"]
    assert r[-1] / r[-2] <= 1e-3 and r[-1] / r[-2] < r[-2] / r[-3]


def test_projected_active_set_loop_reaches_the_kkt_point():
    """With the projected update (phi := phi_old on A_k before the step) the loop ends at a point of
    the variational inequality of the irreversibility constraint phi <= phi_old: phi <= phi_old
    everywhere, phi = phi_old with a multiplier -R_phi > 0 on the active set, and R_phi = 0 (to the
    tolerance) off it; and that point does not depend on how ties of the first active set are
    broken (two starts that differ by 1e-13 in u)."""
    from oracle import loading
    from oracle.fe import Mesh
    from synth.fields import make_phi
    cfg = CONFIGS["C2"].with_(N=8, n_h_levels=2, phi_mode="ones", pdas_project=True)
    levels = level_list(cfg)
    mesh = Mesh(cfg.dim, cfg.N, cfg.k)
    phi0 = make_phi(cfg)
    nn, d = mesh.n_nodes, cfg.dim
    outs = []
    for seed in (1, 2):
        u0 = 1e-13 * np.random.default_rng(seed).standard_normal((d, nn))
        rec = loading.load_step(cfg, levels, u0, phi0, phi0, None, [0.0, 5e-4], tol=1e-10)
        assert rec["converged"]
        act = rec["active"] != 0
        Rp = rec["R"][d * nn:]
        r0 = rec["norms"][0]
        assert np.all(rec["phi"] <= phi0 + 1e-12)
        assert np.array_equal(rec["phi"][act], phi0[act])
        assert np.all(Rp[act] < 0)
        assert np.abs(Rp[~act]).max() <= 1e-8 * r0
        outs.append(rec)
    a, b = outs
    assert np.abs(a["phi"] - b["phi"]).max() <= 1e-8
    assert np.linalg.norm(a["u"] - b["u"]) <= 1e-8 * np.linalg.norm(a["u"])


# ------------------------------------------------------------- V-cycle as composed (Section 3.3)
def _cheb_block_matrix(lev, lam, s, lo_f, hi_f):
    """Dense linear map r -> diag(C_u, C_phi) r from the closed form of the Jacobi-scaled Chebyshev
    polynomial (not from the recurrence): with X = D^-1/2 A_bb D^-1/2 = Q diag(mu) Q^T,
    C_b = D^-1/2 Q diag((1 - T_s((theta - mu)/delta) / T_s(theta/delta)) / mu) Q^T D^-1/2."""
    A = lev.A.toarray()
    n, nu = A.shape[0], lev.nu
    C = np.zeros((n, n))
    T = np.polynomial.chebyshev.Chebyshev.basis(s)
    for sl, lm in ((slice(0, nu), lam[0]), (slice(nu, n), lam[1])):
        Abb = A[sl, sl]
        dh = 1.0 / np.sqrt(lev.D[sl])
        X = dh[:, None] * Abb * dh[None, :]
        mu, Q = np.linalg.eigh(0.5 * (X + X.T))
        lo, hi = lo_f * lm, hi_f * lm
        th, de = 0.5 * (hi + lo), 0.5 * (hi - lo)
        f = (1.0 - T((th - mu) / de) / T(th / de)) / mu
        C[sl, sl] = dh[:, None] * (Q * f) @ Q.T * dh[None, :]
    return C


def _vcycle_error_operator(H, l):
    """E_l = (I - C_l G_l)(I - P_l B_{l-1} P_l^T G_l)(I - C_l G_l) with B_{l-1} = (I - E_{l-1}) G_{l-1}^-1
    and B_0 = G_0^-1 (the exact coarse solve): the textbook error propagation of a V-cycle with one
    pre- and one post-smoothing step, returned together with B_l."""
    lev = H.levels[l]
    A = lev.A.toarray()
    n = A.shape[0]
    if l == 0:
        B = np.linalg.inv(A)
        return np.zeros((n, n)), B
    _, Bc = _vcycle_error_operator(H, l - 1)
    P = H.P[l].toarray()
    C = _cheb_block_matrix(lev, H.lam[l], H.cfg.cheb_degree, H.cfg.cheb_lo, H.cfg.cheb_hi)
    I = np.eye(n)
    S = I - C @ A
    E = S @ (I - P @ Bc @ P.T @ A) @ S
    return E, (I - E) @ np.linalg.inv(A)


def _vcycle_columns(H, vc):
    A = H.levels[-1].A
    n = A.shape[0]
    I = np.eye(n)
    return np.column_stack([I[:, j] - vc(A @ I[:, j]) for j in range(n)])


class _NoPostSmoothing(mg.Hierarchy):
    # planted mistake: the post-smoothing step is dropped
    def vcycle(self, b, l=None):
        l = self.L if l is None else l
        lev = self.levels[l]
        if l == 0:
            return self.coarse.solve(b)
        x = mg.chebyshev_block(lev, self.lam[l], b, self.cfg.cheb_degree, self.cfg.cheb_lo, self.cfg.cheb_hi)
        r = b - lev.A @ x
        return x + self.P[l] @ self.vcycle(self.P[l].T @ r, l - 1)


class _BlockResidual(mg.Hierarchy):
    # planted mistake: the coarse-correction residual uses diag(G_uu, G_phiphi) instead of G
    def vcycle(self, b, l=None):
        l = self.L if l is None else l
        lev = self.levels[l]
        if l == 0:
            return self.coarse.solve(b)
        s, lo, hi = self.cfg.cheb_degree, self.cfg.cheb_lo, self.cfg.cheb_hi
        x = mg.chebyshev_block(lev, self.lam[l], b, s, lo, hi)
        r = b - lev.Ablk @ x
        x = x + self.P[l] @ self.vcycle(self.P[l].T @ r, l - 1)
        r = b - lev.A @ x
        return x + mg.chebyshev_block(lev, self.lam[l], r, s, lo, hi)


VCYCLE_PIN_CASES = {
    # the 2D Q1 workload at full size (32x32, two levels), notch and ~10% active set
    "c1": ("C1", {}, None),
    # 2D Q2, three h-levels (2x2 .. 8x8), smooth phi with the notch, ~5% active set
    "q2_three_levels": ("C2", dict(N=8, n_h_levels=3), None),
    # 2D Q2 with a p-step: 4x4 Q1 -> 4x4 Q2 -> 8x8 Q2
    "q2_pstep": ("C2", dict(N=8, n_h_levels=2, p_coarse=(1,)), None),
    # 3D Q1, two levels (2^3 -> 4^3)
    "3d_q1": ("C3", dict(N=4, k=1, n_h_levels=2, vcycle_prec="f64"), None),
    # the slit mesh of Section 5.1 on every level (slit-aware injection and transfers)
    "slit_q1": ("C1", dict(N=8, n_h_levels=2, slit=True, phi_mode="smooth"), None),
    "slit_q2_pstep": ("C2", dict(N=4, n_h_levels=2, p_coarse=(1,), slit=True), None),
}


@pytest.mark.parametrize("case", list(VCYCLE_PIN_CASES))
def test_vcycle_equals_its_error_propagation_operator(case):
    """The oracle's V-cycle, column by column, against E_l composed densely from its factors: the
    Chebyshev smoother from its closed form, the masked transfers, the exact coarse inverse.  Two
    planted mistakes (no post-smoothing; the block-diagonal operator in the coarse-correction
    residual) must fail the same comparison."""
    name, kw, _ = VCYCLE_PIN_CASES[case]
    cfg = CONFIGS[name].with_(**kw)
    inp = make_inputs(cfg)
    lv = level_list(cfg)
    H = mg.Hierarchy(cfg, lv, inp["u"], inp["phi"], inp["phi_tilde"], inp["active"])
    E, _ = _vcycle_error_operator(H, H.L)
    got = _vcycle_columns(H, H.vcycle)
    scale = np.abs(E).max()
    assert np.abs(got - E).max() <= 1e-12 * max(scale, 1.0)
    if case in ("q2_three_levels", "3d_q1"):
        for bad in (_NoPostSmoothing, _BlockResidual):
            Hb = bad(cfg, lv, inp["u"], inp["phi"], inp["phi_tilde"], inp["active"])
            wrong = _vcycle_columns(Hb, Hb.vcycle)
            assert np.abs(wrong - E).max() > 1e-3 * max(scale, 1.0)
