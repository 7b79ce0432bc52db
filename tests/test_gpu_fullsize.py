"""Parity at the workloads' full sizes, in the launch configuration the
benchmark times: sampled rows of the products, the transposed products, the
diagonal and the residual against the oracle (which evaluates only the cells
touching the sampled nodes), and the C2 Newton step through its own checks."""
import numpy as np
import pytest

from helpers import dev, host, rel_err, say
from oracle import newton
from oracle import operator as op
from oracle.fe import Mesh
from synth import CONFIGS, level_list, make_inputs
from synth.fields import notch_mask

pytestmark = pytest.mark.gpu


def sample_nodes(cfg, n_random, seed):
    mesh = Mesh(cfg.dim, cfg.N, cfg.k)
    rng = np.random.default_rng(seed)
    picks = list(rng.choice(mesh.n_nodes, n_random, replace=False))
    picks += [0, mesh.n_nodes - 1]                                   # corners (Dirichlet faces)
    picks += list(rng.choice(np.flatnonzero(notch_mask(cfg)), 2, replace=False))
    picks.append((mesh.n_nodes // 2) // cfg.k * cfg.k)               # somewhere in the middle
    return np.array(sorted(set(int(p) for p in picks)))


@pytest.mark.parametrize("name,n_random,split", [("C2", 40, "amor"), ("C3", 24, "amor"), ("C4", 8, "amor"),
                                                 ("C5", 24, "amor"), ("C2", 24, "miehe"), ("C3", 12, "miehe")])
def test_fullsize_sampled_rows(name, n_random, split):
    from paper_2005_00331_amd import OP_G, OP_GT, Context, problem_from
    cfg = CONFIGS[name].with_(split=split)
    levels = level_list(cfg)
    inp = make_inputs(cfg)
    mesh = Mesh(cfg.dim, cfg.N, cfg.k)
    m = op.material_of(cfg)
    nodes = sample_nodes(cfg, n_random, 31)
    rows = np.stack([c * mesh.n_nodes + nodes for c in range(cfg.dim + 1)])
    pvec = op.free_vector(mesh, inp["active"], cfg.dirichlet)
    say(name, split, "full size", mesh.n_dofs, "dofs, levels", levels)
    ctx = Context(problem_from(cfg, levels))
    args = (dev(inp["u"]), dev(inp["phi"]), dev(inp["phi_old"]), dev(inp["active"]), dev(inp["phi_tilde"]))
    full = len(levels) > 1
    if full:
        ctx.set_linearization(*args)
    else:
        ctx.set_point(*args)
    x = np.random.default_rng(32).standard_normal(mesh.n_dofs)
    xd = dev(x)
    for opn, tr in ((OP_G, False), (OP_GT, True)):
        say(name, "op", opn)
        y = host(ctx.apply_jacobian(-1, xd, op=opn))[rows]
        ref = op.apply_rows(mesh, m, inp["u"], inp["phi"], inp["phi_tilde"], pvec, x, nodes, transpose=tr)
        assert rel_err(y, ref) <= 1e-12, (name, opn, rel_err(y, ref))
    if full:
        say(name, "diagonal")
        dref = op.diag_rows(mesh, m, inp["u"], inp["phi"], inp["phi_tilde"], pvec, nodes)
        assert rel_err(host(ctx.diagonal(-1))[rows], dref) <= 1e-12
    say(name, "residual")
    R = host(ctx.residual(dev(inp["u"]), dev(inp["phi"]), dev(inp["phi_tilde"])))[rows]
    Rref = op.residual_rows(mesh, m, inp["u"], inp["phi"], inp["phi_tilde"], nodes)
    assert rel_err(R, Rref) <= 1e-12


def test_c5_parameter_cotangents_fullsize():
    from paper_2005_00331_amd import Context, problem_from
    cfg = CONFIGS["C5"]
    inp = make_inputs(cfg, ("cotangent",))
    mesh = Mesh(cfg.dim, cfg.N, cfg.k)
    ctx = Context(problem_from(cfg, [(cfg.N, cfg.k)]))
    say("C5 param vjp")
    dGc, deps = ctx.residual_param_vjp(dev(inp["u"]), dev(inp["phi"]), dev(inp["phi_tilde"]), dev(inp["cotangent"]))
    rGc, reps = op.param_vjp(mesh, op.material_of(cfg), inp["u"], inp["phi"], inp["phi_tilde"], inp["cotangent"])
    assert abs(dGc - rGc) <= 1e-12 * abs(rGc) and abs(deps - reps) <= 1e-12 * abs(reps)


def test_c2_newton_step_fullsize():
    """The benchmark's step: active set against the oracle's rule, solve to rtol."""
    from paper_2005_00331_amd import OP_G, Context, problem_from
    cfg = CONFIGS["C2"]
    levels = level_list(cfg)
    inp = make_inputs(cfg)
    mesh = Mesh(cfg.dim, cfg.N, cfg.k)
    R = op.residual(mesh, op.material_of(cfg), inp["u"], inp["phi"], inp["phi_tilde"])
    act_ref, ind = newton.active_set(mesh, R, inp["phi"], inp["phi_old"], cfg.as_c)
    ctx = Context(problem_from(cfg, levels))
    u, phi = dev(inp["u"]), dev(inp["phi"])
    say("C2 newton step full size")
    Rg = ctx.residual(u, phi, dev(inp["phi_tilde"]))
    assert rel_err(host(Rg), R) <= 1e-12
    act, info = ctx.newton_step(u, phi, dev(inp["phi_old"]), dev(inp["phi_tilde"]))
    act = host(act)
    tie = np.abs(ind) <= 1e-12 * np.abs(ind).max()
    assert np.array_equal(act[~tie], act_ref[~tie])
    assert info["converged"] == 1 and info["rel_residual"] <= cfg.rtol
    say("C2 iterations", info["iterations"], "setup ms", info["ms_setup"], "solve ms", info["ms_solve"])
    # the update solves the linearised system: check with the product at the old state
    dU = np.concatenate([host(u) - inp["u"].ravel(), host(phi) - inp["phi"]])
    pvec = op.free_vector(mesh, act, cfg.dirichlet)
    b = -pvec * host(Rg)
    r = b - host(ctx.apply_jacobian(-1, dev(dU), op=OP_G))
    assert np.linalg.norm(r) <= 1.01 * cfg.rtol * np.linalg.norm(b)
    assert np.all(dU[pvec == 0] == 0)
