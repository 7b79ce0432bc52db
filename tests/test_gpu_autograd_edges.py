"""Autograd of the residual against central differences, and the edge cases
and error paths of the C ABI (all forced from the host, no device faults)."""
import numpy as np
import pytest
import torch

from helpers import dev, host, rel_err, say
from oracle import fe, krylov, multigrid as mg
from oracle import operator as op
from synth import CONFIGS, level_list, make_inputs

pytestmark = pytest.mark.gpu


def _ctx(cfg, levels, **kw):
    from paper_2005_00331_amd import Context, problem_from
    return Context(problem_from(cfg, levels, **kw))


def _traces(cfg, U):
    mesh = fe.Mesh(cfg.dim, cfg.N, cfg.k)
    nn = cfg.n_nodes
    cd = op.CellData(mesh, fe.TensorBasis(cfg.dim, cfg.k), op.material_of(cfg), U[: cfg.dim * nn].reshape(cfg.dim, nn),
                     U[cfg.dim * nn:], U[cfg.dim * nn:], np.arange(mesh.n_cells))
    return cd.split["t"]


def _autograd_fd(cfg, hstep, tol, phi_only=False, count_kinks=False):
    """Directional central differences of <v, R> against the hand-written backward."""
    from paper_2005_00331_amd.autograd import residual
    inp = make_inputs(cfg, ("cotangent", "directions"))
    ctx = _ctx(cfg, [(cfg.N, cfg.k)])
    nn = cfg.n_nodes
    u = dev(inp["u"]).requires_grad_(True)
    phi = dev(inp["phi"]).requires_grad_(True)
    Gc = torch.tensor(cfg.Gc, dtype=torch.float64, requires_grad=True)
    eps = torch.tensor(cfg.eps, dtype=torch.float64, requires_grad=True)
    pt = dev(inp["phi_tilde"])
    v = dev(inp["cotangent"])
    R = residual(u, phi, Gc, eps, pt, ctx)
    (R * v).sum().backward()
    g = torch.cat([u.grad, phi.grad]).cpu().numpy()
    U = np.concatenate([inp["u"].ravel(), inp["phi"]])
    worst = 0.0
    kinks = 0
    for dvec in inp["directions"]:
        if phi_only:
            dvec = dvec.copy()
            dvec[: cfg.dim * nn] = 0.0
        Up, Um = U + hstep * dvec, U - hstep * dvec
        if count_kinks:
            kinks += int((np.sign(_traces(cfg, Up)) != np.sign(_traces(cfg, Um))).sum())
        Rp = ctx.residual(dev(Up[: cfg.dim * nn]), dev(Up[cfg.dim * nn:]), pt)
        Rm = ctx.residual(dev(Um[: cfg.dim * nn]), dev(Um[cfg.dim * nn:]), pt)
        fd = float(((Rp - Rm) * v).sum()) / (2 * hstep)
        ad = float(g @ dvec)
        worst = max(worst, abs(fd - ad) / abs(ad))
    say(cfg.name, cfg.N, "phi only" if phi_only else "u and phi", "h", hstep, "worst relative FD gap", worst,
        "branch flips", kinks if count_kinks else "not counted")
    assert worst <= tol
    if count_kinks:
        assert kinks == 0
    return Gc, eps, inp, pt, v


def _param_fd(cfg, Gc, eps, inp, pt, v, eps_tol=1e-7):
    # R is affine in Gc (exact for any step); eps by a central difference (truncation
    # ~ (step/eps)^2 = 1e-8; at full size the cancellation in <v, R> over ~1e6 rows
    # leaves ~1e-7)
    for name, base, step in (("Gc", cfg.Gc, 0.5), ("eps", cfg.eps, 1e-4 * cfg.eps)):
        vals = []
        for sgn in (1, -1):
            c2 = _ctx(cfg.with_(**({"Gc": base + sgn * step} if name == "Gc" else {})),
                      [(cfg.N, cfg.k)], **({"eps": base + sgn * step} if name == "eps" else {}))
            vals.append(float((c2.residual(dev(inp["u"]), dev(inp["phi"]), pt) * v).sum()))
            c2.close()
        fd = (vals[0] - vals[1]) / (2 * step)
        ad = float((Gc if name == "Gc" else eps).grad)
        assert abs(fd - ad) <= (1e-9 if name == "Gc" else eps_tol) * abs(ad), (name, fd, ad)


def test_autograd_reduced_size_exact():
    # 3D Q2 on 6^3 cells, full directions: no quadrature point changes branch (counted)
    cfg = CONFIGS["C5"].with_(N=6)
    _param_fd(cfg, *_autograd_fd(cfg, 1e-6, 1e-6, count_kinks=True))


def _fullsize_gradient_and_differences(cfg, hstep):
    """Backward of <v, R> at the workload state, and per direction the central difference of
    <v, R> (GPU residuals) and <G^T v, d>."""
    from paper_2005_00331_amd.autograd import residual
    inp = make_inputs(cfg, ("cotangent", "directions"))
    ctx = _ctx(cfg, [(cfg.N, cfg.k)])
    nn = cfg.n_nodes
    u = dev(inp["u"]).requires_grad_(True)
    phi = dev(inp["phi"]).requires_grad_(True)
    Gc = torch.tensor(cfg.Gc, dtype=torch.float64)
    eps = torch.tensor(cfg.eps, dtype=torch.float64)
    pt = dev(inp["phi_tilde"])
    v = dev(inp["cotangent"])
    (residual(u, phi, Gc, eps, pt, ctx) * v).sum().backward()
    g = torch.cat([u.grad, phi.grad]).cpu().numpy()
    U = np.concatenate([inp["u"].ravel(), inp["phi"]])
    fd, ad = [], []
    for dvec in inp["directions"]:
        Up, Um = U + hstep * dvec, U - hstep * dvec
        Rp = ctx.residual(dev(Up[: cfg.dim * nn]), dev(Up[cfg.dim * nn:]), pt)
        Rm = ctx.residual(dev(Um[: cfg.dim * nn]), dev(Um[cfg.dim * nn:]), pt)
        fd.append(float(((Rp - Rm) * v).sum()) / (2 * hstep))
        ad.append(float(g @ dvec))
    ctx.close()
    return inp, U, fd, ad


def test_autograd_fullsize_c5():
    # 48^3 Q2 (3,650,692 dofs).
    # phi-only directions leave tr e unchanged and R is linear in phi: exact up to rounding.
    cfg = CONFIGS["C5"]
    _param_fd(cfg, *_autograd_fd(cfg, 1e-6, 1e-8, phi_only=True), eps_tol=1e-6)


def test_autograd_fullsize_c5_full_directions_crossings_excluded():
    """32 full directions at h = 1e-6 (1e-3 N(0,1) on u, N(0,1) on phi).  Every quadrature point
    whose branch (sign of tr e) changes between U +- h d is counted; the oracle's share of those
    points' cells is taken out of both the difference and the tangent; what remains must agree
    to 1e-8.  A point that crosses makes the difference an average of two tangents, an O(1) term
    against a random-sign sum over ~3e6 points, hence the separate bookkeeping."""
    import fdcheck
    cfg = CONFIGS["C5"]
    h = 1e-6
    inp, U, fd, ad = _fullsize_gradient_and_differences(cfg, h)
    mesh = fe.Mesh(cfg.dim, cfg.N, cfg.k)
    res = fdcheck.excluded_gaps(mesh, op.material_of(cfg), U, inp["phi_tilde"], inp["cotangent"],
                                inp["directions"], h, fd, ad)
    for j, (npts, ncells, full, rest) in enumerate(res):
        say("C5 direction", j, "crossing points", npts, "cells", ncells, "gap", f"{full:.2e}",
            "gap without crossing cells", f"{rest:.2e}")
    say("C5 crossing points in total", sum(r[0] for r in res), "worst gap", max(r[2] for r in res),
        "worst gap without crossing cells", max(r[3] for r in res))
    assert max(r[3] for r in res) <= 1e-8
    # secondary: a step 100x smaller leaves few crossings, and the raw gap is already small
    inp, U, fd, ad = _fullsize_gradient_and_differences(cfg, 1e-8)
    assert max(abs(f - a) / abs(a) for f, a in zip(fd, ad)) <= 5e-3


def test_autograd_rejects_a_dirichlet_context():
    # a context with Dirichlet rows (the default of the workloads) would give identity rows in
    # the transposed product, so the u gradient would be wrong there: the forward refuses it
    from paper_2005_00331_amd.autograd import residual
    cfg = CONFIGS["C5"].with_(N=3, dirichlet=True)
    inp = make_inputs(cfg)
    ctx = _ctx(cfg, [(cfg.N, cfg.k)])
    u = dev(inp["u"]).requires_grad_(True)
    Gc = torch.tensor(cfg.Gc, dtype=torch.float64)
    eps = torch.tensor(cfg.eps, dtype=torch.float64)
    with pytest.raises(ValueError, match="dirichlet"):
        residual(u, dev(inp["phi"]), Gc, eps, dev(inp["phi_tilde"]), ctx)
    ctx.close()


@pytest.mark.parametrize("split", ["none", "miehe"])
def test_autograd_reduced_size_other_splits(split):
    # the isotropic model has no branch: full directions are exact; the spectral split has
    # eigenvalue branches, so only phi-only directions (R is linear in phi at fixed u) are exact
    cfg = CONFIGS["C5"].with_(N=6, split=split)
    _param_fd(cfg, *_autograd_fd(cfg, 1e-6, 1e-6, phi_only=(split == "miehe")))


@pytest.mark.parametrize("split", ["amor", "miehe", "none"])
def test_transposed_product_matches_assembled_transpose(split):
    from paper_2005_00331_amd import OP_GT
    cfg = CONFIGS["C5"].with_(N=5, split=split)
    inp = make_inputs(cfg)
    mesh = fe.Mesh(cfg.dim, cfg.N, cfg.k)
    G = op.assemble_jacobian(mesh, op.material_of(cfg), inp["u"], inp["phi"], inp["phi_tilde"])
    ctx = _ctx(cfg, [(cfg.N, cfg.k)])
    ctx.set_point(dev(inp["u"]), dev(inp["phi"]), dev(inp["phi_old"]), dev(np.zeros(cfg.n_nodes, np.uint8)),
                  dev(inp["phi_tilde"]))
    v = np.random.default_rng(5).standard_normal(mesh.n_dofs)
    assert rel_err(host(ctx.apply_jacobian(-1, dev(v), op=OP_GT)), G.T @ v) <= 1e-12


# ------------------------------------------------------------------ edge cases
def test_all_phi_dofs_active():
    cfg = CONFIGS["C1"]
    levels = level_list(cfg)
    inp = make_inputs(cfg, ("rhs",))
    act = np.ones(cfg.n_nodes, np.uint8)
    H = mg.Hierarchy(cfg, levels, inp["u"], inp["phi"], inp["phi_tilde"], act)
    ctx = _ctx(cfg, levels)
    ctx.set_linearization(dev(inp["u"]), dev(inp["phi"]), dev(inp["phi_old"]), dev(act), dev(inp["phi_tilde"]))
    info = ctx.levels[-1]
    assert info.lanczos_steps_phi == 0 and info.lambda_phi == 1.0
    assert H.lam[-1][1] == 1.0
    A = H.levels[-1].A
    b = H.levels[-1].pvec * inp["rhs"]
    x, st = ctx.gmres_solve(dev(b))
    xo, _ = krylov.fgmres(lambda w: A @ w, H.vcycle, b, cfg.restart, cfg.rtol, cfg.max_iter)
    assert st["converged"] == 1 and np.linalg.norm(host(x) - xo) <= 1e-6 * np.linalg.norm(xo)


def test_zero_rhs_and_nonconvergence_and_state_errors():
    from paper_2005_00331_amd import MfpffError
    cfg = CONFIGS["C1"]
    levels = level_list(cfg)
    inp = make_inputs(cfg, ("rhs",))
    ctx = _ctx(cfg, levels, max_iter=1)
    with pytest.raises(MfpffError) as ei:
        ctx.vcycle(dev(inp["rhs"]))
    assert ei.value.status == 2
    with pytest.raises(MfpffError) as ei:
        ctx.apply_jacobian(-1, dev(inp["rhs"]))
    assert ei.value.status == 2
    ctx.set_linearization(dev(inp["u"]), dev(inp["phi"]), dev(inp["phi_old"]), dev(inp["active"]), dev(inp["phi_tilde"]))
    x, st = ctx.gmres_solve(torch.zeros(cfg.n_dofs, dtype=torch.float64, device="cuda"))
    assert st["converged"] == 1 and st["iterations"] == 0 and float(x.abs().max()) == 0.0
    x, st = ctx.gmres_solve(dev(inp["rhs"]), raise_on_noconv=False)
    assert st["converged"] == 0 and st["iterations"] == 1 and st["rel_residual"] > cfg.rtol
    with pytest.raises(MfpffError) as ei:
        ctx.gmres_solve(dev(inp["rhs"]))
    assert ei.value.status == 5


def test_nonfinite_input_rejected():
    from paper_2005_00331_amd import MfpffError
    cfg = CONFIGS["C1"]
    inp = make_inputs(cfg)
    u = inp["u"].copy()
    u[1, 17] = np.nan
    ctx = _ctx(cfg, level_list(cfg))
    with pytest.raises(MfpffError) as ei:
        ctx.set_linearization(dev(u), dev(inp["phi"]), dev(inp["phi_old"]), dev(inp["active"]), dev(inp["phi_tilde"]))
    assert ei.value.status == 6


@pytest.mark.parametrize("dim,N", [(2, 8), (3, 4)])
def test_indefinite_coarse_block_takes_the_lu_path(dim, N):
    # kappa < 0: g < 0 where phi is small, so G_uu is indefinite and its Cholesky fails; the
    # Gauss-Jordan inverse then gives the coarse solve, against the oracle's LU solve
    cfg = CONFIGS["C1"].with_(dim=dim, N=N, n_h_levels=1, p_coarse=(), kappa=-0.5, phi_mode="smooth")
    inp = make_inputs(cfg, ("rhs",))
    H = mg.Hierarchy(cfg, [(cfg.N, cfg.k)], inp["u"], inp["phi"], inp["phi_tilde"], inp["active"])
    assert H.coarse.fu[0] == "lu"
    ctx = _ctx(cfg, [(cfg.N, cfg.k)])
    say("indefinite coarse block", dim, N, H.coarse.nu, "u dofs")
    ctx.set_linearization(dev(inp["u"]), dev(inp["phi"]), dev(inp["phi_old"]), dev(inp["active"]), dev(inp["phi_tilde"]))
    b = inp["rhs"]
    x = host(ctx.coarse_solve(dev(b)))
    # two correct inverses of a block with condition number up to ~5e5 agree to ~cond * 2^-53
    assert rel_err(x, H.coarse.solve(b)) <= 1e-9
    # the same context linearised again at phi = phi~ = 1 (g = 1, G_uu definite) is back on the
    # Cholesky path
    one = np.ones(cfg.n_nodes)
    ctx.set_linearization(dev(inp["u"]), dev(one), dev(one), dev(inp["active"]), dev(one))
    H2 = mg.Hierarchy(cfg, [(cfg.N, cfg.k)], inp["u"], one, one, inp["active"])
    assert H2.coarse.fu[0] == "chol"
    assert rel_err(host(ctx.coarse_solve(dev(b))), H2.coarse.solve(b)) <= 1e-10


def test_fully_broken_material_at_rest_rejected():
    # kappa = 0, phi = phi~ = 0, u = 0: g = 0 and tr e = 0 (tension branch), so every free
    # displacement row of G is zero: the coarse Cholesky fails and the LU meets a zero pivot
    # (the oracle rejects the same state, as a singular block)
    from paper_2005_00331_amd import MfpffError
    cfg = CONFIGS["C1"].with_(kappa=0.0)
    z = np.zeros(cfg.n_nodes)
    ctx = _ctx(cfg, level_list(cfg))
    with pytest.raises(MfpffError) as ei:
        ctx.set_linearization(dev(np.zeros((2, cfg.n_nodes))), dev(z), dev(z), dev(np.zeros(cfg.n_nodes, np.uint8)),
                              dev(z))
    assert ei.value.status == 6


def test_2d_level_past_the_offset_range_rejected():
    # the 2D Q1/Q2 kernel addresses nodes by 32-bit byte offsets: a level of 2^28 or more nodes
    # (16384^2 Q1 cells: 16385^2 nodes) is refused at set-up, before its storage is allocated
    from paper_2005_00331_amd import Context, MfpffError, problem_from
    cfg = CONFIGS["C1"].with_(N=16384, n_h_levels=1, p_coarse=())
    with pytest.raises(MfpffError) as ei:
        Context(problem_from(cfg, [(16384, 1)]))
    assert ei.value.status == 1


def test_oversized_coarse_level_rejected_without_allocation():
    from paper_2005_00331_amd import MfpffError
    cfg = CONFIGS["C5"]
    inp = make_inputs(cfg)
    ctx = _ctx(cfg, [(cfg.N, cfg.k)])
    with pytest.raises(MfpffError) as ei:
        ctx.set_linearization(dev(inp["u"]), dev(inp["phi"]), dev(inp["phi_old"]), dev(inp["active"]),
                              dev(inp["phi_tilde"]))
    assert ei.value.status == 1


@pytest.mark.parametrize("dim,levels", [(2, [(1, 1), (2, 1)]), (2, [(1, 1), (1, 2)]), (3, [(1, 1), (1, 2)])])
def test_smallest_meshes(dim, levels):
    from paper_2005_00331_amd import OP_G
    base = CONFIGS["C3"] if dim == 3 else CONFIGS["C2"]
    N, k = levels[-1]
    cfg = base.with_(dim=dim, N=N, k=k, n_h_levels=1, p_coarse=(), vcycle_prec="f64", active_p=0.2)
    inp = make_inputs(cfg, ("rhs",))
    H = mg.Hierarchy(cfg, levels, inp["u"], inp["phi"], inp["phi_tilde"], inp["active"])
    ctx = _ctx(cfg, levels)
    ctx.set_linearization(dev(inp["u"]), dev(inp["phi"]), dev(inp["phi_old"]), dev(inp["active"]), dev(inp["phi_tilde"]))
    x = np.random.default_rng(0).standard_normal(cfg.n_dofs)
    for l, lev in enumerate(H.levels):
        xl = x[: lev.mesh.n_dofs]
        assert rel_err(host(ctx.apply_jacobian(l, dev(xl), op=OP_G)), lev.A @ xl) <= 1e-12
    assert rel_err(host(ctx.vcycle(dev(x))), H.vcycle(x)) <= 1e-10


def test_sizes_match_the_level_descriptions():
    """mfpff_sizes (host only) against mfpff_level_info and the mesh formula (k N + 1)^d nodes,
    (d + 1) dofs per node, on an h- and p-coarsened hierarchy; out-of-range levels are rejected."""
    import ctypes
    from paper_2005_00331_amd import MfpffError
    cfg = CONFIGS["C4"].with_(N=4, n_h_levels=2)
    levels = level_list(cfg)
    ctx = _ctx(cfg, levels)
    say("sizes")
    for l, (N, k) in enumerate(levels):
        nn, nd = ctx.sizes(l)
        d = ctx.level_info(l)
        assert (nn, nd) == (d.n_nodes, d.n_dofs) == ((k * N + 1) ** 3, 4 * (k * N + 1) ** 3)
    a, b = ctypes.c_size_t(), ctypes.c_size_t()
    assert ctx.lib.mfpff_sizes(ctx.h, len(levels), ctypes.byref(a), ctypes.byref(b)) == 1
    assert ctx.lib.mfpff_sizes(ctx.h, -1, ctypes.byref(a), ctypes.byref(b)) == 1
    with pytest.raises(MfpffError):
        ctx._check(ctx.lib.mfpff_sizes(ctx.h, 0, None, ctypes.byref(b)))
