"""GPU parity on the slit geometry of the notched tests (Section 5.1): duplicated slit nodes,
one level whose exact coarse solve preconditions FGMRES.  Products, diagonal, residual,
parameter cotangents, active set, a linear solve, Newton steps and load steps against the
oracle's slit mesh."""
import numpy as np
import pytest

from helpers import dev, host, rel_err, say
from oracle import multigrid as mg, newton
from oracle import operator as op
from oracle.fe import Mesh
from synth import CONFIGS, make_inputs

pytestmark = pytest.mark.gpu

# (base workload, overrides): 2D Q1/Q2 and 3D Q1/Q2, all at most 16,384 dofs (one dense level)
SLIT_CASES = [
    ("C1", dict(N=16)),
    ("C2", dict(N=8)),
    ("C1", dict(dim=3, N=6)),
    ("C3", dict(N=4, vcycle_prec="f64")),
]


def _cfg(name, kw, **extra):
    return CONFIGS[name].with_(n_h_levels=1, p_coarse=(), slit=True, **kw, **extra)


def _ctx(cfg):
    from paper_2005_00331_amd import Context, problem_from
    return Context(problem_from(cfg, [(cfg.N, cfg.k)]))


@pytest.mark.parametrize("name,kw", SLIT_CASES)
def test_slit_products_diagonal_residual(name, kw):
    from paper_2005_00331_amd import OP_BLOCKDIAG, OP_G, OP_GT
    # a smooth seeded phi (phi = 1 would make the Gc cotangent vanish identically)
    cfg = _cfg(name, kw, phi_mode="smooth")
    inp = make_inputs(cfg, ("cotangent",))
    mesh = Mesh(cfg.dim, cfg.N, cfg.k, slit=True)
    assert mesh.n_nodes == cfg.n_nodes
    H = mg.Hierarchy(cfg, [(cfg.N, cfg.k)], inp["u"], inp["phi"], inp["phi_tilde"], inp["active"])
    lev = H.levels[0]
    say(name, kw, "slit", mesh.n_dofs, "dofs", mesh.n_dup, "duplicates")
    ctx = _ctx(cfg)
    assert ctx.n_nodes == mesh.n_nodes
    ctx.set_linearization(dev(inp["u"]), dev(inp["phi"]), dev(inp["phi_old"]), dev(inp["active"]), dev(inp["phi_tilde"]))
    x = np.random.default_rng(5).standard_normal(mesh.n_dofs)
    for opn, ref in ((OP_G, lev.A @ x), (OP_GT, lev.A.T @ x), (OP_BLOCKDIAG, lev.Ablk @ x)):
        say("op", opn)
        assert rel_err(host(ctx.apply_jacobian(-1, dev(x), op=opn)), ref) <= 1e-12
    assert rel_err(host(ctx.diagonal(-1)), lev.D) <= 1e-12
    R = host(ctx.residual(dev(inp["u"]), dev(inp["phi"]), dev(inp["phi_tilde"])))
    Rref = op.residual(mesh, op.material_of(cfg), inp["u"], inp["phi"], inp["phi_tilde"])
    assert rel_err(R, Rref) <= 1e-12
    dGc, deps = ctx.residual_param_vjp(dev(inp["u"]), dev(inp["phi"]), dev(inp["phi_tilde"]), dev(inp["cotangent"]))
    rGc, reps = op.param_vjp(mesh, op.material_of(cfg), inp["u"], inp["phi"], inp["phi_tilde"], inp["cotangent"])
    assert abs(dGc - rGc) <= 1e-12 * abs(rGc) and abs(deps - reps) <= 1e-12 * abs(reps)
    # the exact coarse solve of the one level: FGMRES converges at once
    b = lev.pvec * np.random.default_rng(6).standard_normal(mesh.n_dofs)
    xs, info = ctx.gmres_solve(dev(b))
    assert info["converged"] == 1 and info["iterations"] <= 2
    assert np.linalg.norm(b - lev.A @ host(xs)) <= 1.001 * cfg.rtol * np.linalg.norm(b)


@pytest.mark.parametrize("name,kw", [("C1", dict(N=16)), ("C2", dict(N=8))])
def test_slit_newton_step(name, kw):
    cfg = _cfg(name, kw)
    inp = make_inputs(cfg)
    out = newton.newton_step(cfg, [(cfg.N, cfg.k)], inp["u"], inp["phi"], inp["phi_old"], inp["phi_tilde"])
    ctx = _ctx(cfg)
    u, phi = dev(inp["u"]), dev(inp["phi"])
    say(name, kw, "slit newton step")
    act, info = ctx.newton_step(u, phi, dev(inp["phi_old"]), dev(inp["phi_tilde"]))
    ind = out["indicator"]
    tie = np.abs(ind) <= 1e-12 * np.abs(ind).max()
    assert np.array_equal(host(act)[~tie], out["active"][~tie])
    dU = np.concatenate([host(u) - inp["u"].ravel(), host(phi) - inp["phi"]])
    assert np.linalg.norm(dU - out["dU"]) <= 1e-8 * np.linalg.norm(out["dU"])


@pytest.mark.parametrize("name,kw,du", [("C1", dict(N=16), 2e-3), ("C1", dict(dim=3, N=6), 1e-3), ("C2", dict(N=8), 5e-4)])
def test_slit_load_steps(name, kw, du):
    """Three load steps of the tension test on the slit mesh (phi = 1 everywhere, no notch band:
    the slit is the notch) with the projected active-set update, against the oracle: the state,
    the reactions and the active set off indicator ties."""
    import torch
    from oracle import loading
    cfg = _cfg(name, kw, phi_mode="ones", pdas_project=True)
    mesh = Mesh(cfg.dim, cfg.N, cfg.k, slit=True)
    direction = np.zeros(cfg.dim)
    direction[-1] = 1.0
    phi0 = np.ones(mesh.n_nodes)
    ref = loading.load_steps(cfg, [(cfg.N, cfg.k)], np.zeros((cfg.dim, mesh.n_nodes)), phi0, direction, du, 3, tol=1e-10)
    ctx = _ctx(cfg)
    u = torch.zeros(cfg.dim * mesh.n_nodes, dtype=torch.float64, device="cuda")
    phi_prev, phi_prev2, ref_prev = dev(phi0), None, phi0
    for t, rec in enumerate(ref, start=1):
        say(name, kw, "slit load step", t)
        phi = phi_prev.clone()
        act, info = ctx.load_step(u, phi, phi_prev, phi_prev2, t * du * direction, tol=1e-10)
        _, ind = newton.active_set(mesh, rec["R"], rec["phi"], ref_prev, cfg.as_c)
        tie = np.abs(ind) <= 1e-8 * np.abs(ind).max()
        say("gpu steps", info["newton_steps"], "oracle steps", rec["steps"], "reaction", info["reaction_top"])
        assert info["converged"] == 1 and rec["converged"]
        assert np.array_equal(host(act)[~tie], rec["active"][~tie])
        assert rel_err(host(u), rec["u"].ravel()) <= 1e-6 and rel_err(host(phi), rec["phi"]) <= 1e-6
        Ft = np.array(info["reaction_top"])
        assert np.abs(Ft - rec["reaction_top"]).max() <= 1e-6 * np.abs(rec["reaction_top"]).max()
        phi_prev2, phi_prev, ref_prev = phi_prev, phi, rec["phi"]
    # the slit opens: above it the displacement along the last axis exceeds the one below it
    uu = host(u).reshape(cfg.dim, mesh.n_nodes)[cfg.dim - 1]
    from synth.fields import slit_duplicates
    grid = slit_duplicates(cfg.dim, cfg.N, cfg.k)
    assert np.all(uu[mesh.n_grid:] - uu[grid] > 0)


def test_slit_problem_errors():
    from paper_2005_00331_amd import Context, problem_from
    cfg = CONFIGS["C1"].with_(slit=True)
    say("slit argument errors")
    for levels in ([(3, 1), (6, 1)], [(15, 1)]):    # an odd N on some level
        with pytest.raises(Exception):
            Context(problem_from(cfg.with_(N=levels[-1][0]), levels))
