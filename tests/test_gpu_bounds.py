"""The bounds-checking debug build of the kernels (libmfpff_bounds.so, sources compiled with
-DMFPFF_BOUNDS): every node, cell and transfer index the kernels compute is checked against its
range, and an index outside it is counted (and replaced by 0, so nothing faults).  A child process
loads that build and runs every parity case through every entry point (products on every level,
diagonals, smoothing, transfers, coarse solve, V-cycle, FGMRES, residual and its cotangents), the
slit meshes and slit hierarchies, a full-size 2D product (the many-tile launch) and a load step; no index may be out
of range, and the finest-level products still match the oracle."""
import os
import subprocess
import sys

import pytest

from helpers import say

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
BOUNDS_LIB = os.path.join(ROOT, "paper_2005_00331_amd", "libmfpff_bounds.so")

CHILD = r"""
import sys
import numpy as np
sys.path[:0] = [ROOT, HERE]
import torch
from helpers import CASES, case_config, dev, host, rel_err
from oracle import multigrid as mg
from synth import CONFIGS, make_inputs
from paper_2005_00331_amd import Context, F32, OP_BLOCKDIAG, OP_G, OP_GT, problem_from, binding

def hits():
    return int(binding.load_library().mfpff_debug_bounds_hits())

def run_case(name, cfg, levels, oracle):
    inp = make_inputs(cfg, ("rhs", "cotangent"))
    ctx = Context(problem_from(cfg, levels))
    args = (dev(inp["u"]), dev(inp["phi"]), dev(inp["phi_old"]), dev(inp["active"]), dev(inp["phi_tilde"]))
    ctx.set_linearization(*args)
    rng = np.random.default_rng(3)
    for l in range(len(levels)):
        n = ctx.levels[l].n_dofs
        x = dev(rng.standard_normal(n))
        for op in (OP_G, OP_GT, OP_BLOCKDIAG):
            ctx.apply_jacobian(l, x, op=op)
            if cfg.vcycle_prec == "f32":
                ctx.apply_jacobian(l, x.float(), prec=F32, op=op)
        ctx.diagonal(l)
        if l > 0:
            ctx.smooth(l, x)
            ctx.transfer(l, 0, dev(rng.standard_normal(ctx.levels[l - 1].n_dofs)))
            ctx.transfer(l, 1, x)
    ctx.coarse_solve(dev(rng.standard_normal(ctx.levels[0].n_dofs)))
    ctx.vcycle(dev(inp["rhs"]))
    ctx.gmres_solve(dev(inp["rhs"]), raise_on_noconv=False)
    ctx.residual(dev(inp["u"]), dev(inp["phi"]), dev(inp["phi_tilde"]))
    ctx.residual_param_vjp(dev(inp["u"]), dev(inp["phi"]), dev(inp["phi_tilde"]), dev(inp["cotangent"]))
    if oracle:
        lev = mg.Level(*oracle(cfg, inp))
        xf = rng.standard_normal(lev.A.shape[0])
        e = rel_err(host(ctx.apply_jacobian(-1, dev(xf), op=OP_G)), lev.A @ xf)
        assert e <= 1e-12, (name, e)
    ctx.close()
    h = hits()
    print("case", name, "hits", h, flush=True)
    return h

def level_args(cfg, inp):
    from oracle import operator as op
    from oracle.fe import Mesh
    mesh = Mesh(cfg.dim, cfg.N, cfg.k, getattr(cfg, "slit", False))
    return (mesh, op.material_of(cfg), inp["u"], inp["phi"], inp["phi_tilde"], inp["active"], cfg.dirichlet)

assert binding.LIB_PATH.endswith("libmfpff_bounds.so"), binding.LIB_PATH
assert hits() == 0
for name in sorted(CASES):
    cfg, levels = case_config(name)
    run_case(name, cfg, levels, level_args)
for base, kw in (("C1", dict(N=16)), ("C2", dict(N=8)), ("C1", dict(dim=3, N=6))):
    cfg = CONFIGS[base].with_(n_h_levels=1, p_coarse=(), slit=True, phi_mode="smooth", **kw)
    run_case("slit_" + base + str(kw), cfg, [(cfg.N, cfg.k)], level_args)
# slit hierarchies: side-aware transfers, injection of duplicates, smoothing on slit levels
for base, levels, kw in (("C2", [(4, 1), (4, 2), (8, 2)], {}), ("C1", [(2, 1), (4, 1)], dict(dim=3))):
    cfg = CONFIGS[base].with_(N=levels[-1][0], k=levels[-1][1], n_h_levels=1, p_coarse=(), slit=True,
                              phi_mode="smooth", **kw)
    run_case("slit_mg_" + base + str(levels), cfg, levels, None)
# the full-size 2D Q2 level (1369 tiles: the many-workgroup launch of the 2D kernel)
cfg = CONFIGS["C2"]
inp = make_inputs(cfg)
ctx = Context(problem_from(cfg, [(cfg.N, cfg.k)]))
ctx.set_point(dev(inp["u"]), dev(inp["phi"]), dev(inp["phi_old"]), dev(inp["active"]), dev(inp["phi_tilde"]))
x = dev(np.random.default_rng(4).standard_normal(ctx.n_dofs))
for op in (OP_G, OP_GT, OP_BLOCKDIAG):
    ctx.apply_jacobian(-1, x, op=op)
ctx.residual(dev(inp["u"]), dev(inp["phi"]), dev(inp["phi_tilde"]))
ctx.close()
print("case C2 full size hits", hits(), flush=True)
# a load step (face values, reactions, the active-set loop)
cfg = CONFIGS["C1"].with_(N=16, n_h_levels=2, p_coarse=(), phi_mode="ones", pdas_project=True)
from synth import level_list
ctx = Context(problem_from(cfg, level_list(cfg)))
u = torch.zeros(cfg.dim * cfg.n_nodes, dtype=torch.float64, device="cuda")
phi = torch.ones(cfg.n_nodes, dtype=torch.float64, device="cuda")
ctx.load_step(u, phi, phi.clone(), None, np.array([0.0, 1e-3]), tol=1e-8)
ctx.close()
print("total hits", hits(), flush=True)
"""


def test_debug_build_finds_no_out_of_range_index():
    if not os.path.exists(BOUNDS_LIB):
        pytest.fail("libmfpff_bounds.so is not built; run __graft_entry__.build()")
    code = CHILD.replace("ROOT", repr(ROOT)).replace("HERE", repr(HERE))
    say("child process on", BOUNDS_LIB)
    r = subprocess.run([sys.executable, "-u", "-c", code], env=dict(os.environ, MFPFF_LIB=BOUNDS_LIB),
                       capture_output=True, text=True, timeout=600)
    print(r.stdout[-3000:], flush=True)
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-4000:]
    lines = [l for l in r.stdout.splitlines() if "hits" in l]
    assert lines and lines[-1] == "total hits 0", lines
    assert all(l.endswith(" 0") for l in lines), [l for l in lines if not l.endswith(" 0")]
