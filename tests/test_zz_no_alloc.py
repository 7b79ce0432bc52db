"""The allocation-free variant of the parameter cotangents (mfpff_residual_param_vjp_noalloc)
against the allocating entry point, through the C ABI: two calls in a row on different contexts
(the second smaller) share the library's static device scratch, and a context whose finest
level needs more partial-sum blocks than that scratch holds is refused with a message."""
import pytest
import torch

from helpers import dev, say
from synth import CONFIGS, make_inputs

pytestmark = pytest.mark.gpu


def _case(cfg):
    from paper_2005_00331_amd import Context, problem_from
    inp = make_inputs(cfg, ("cotangent",))
    ctx = Context(problem_from(cfg, [(cfg.N, cfg.k)]))
    args = (dev(inp["u"]), dev(inp["phi"]), dev(inp["phi_tilde"]), dev(inp["cotangent"]))
    return ctx, args


def test_noalloc_param_vjp_matches_the_allocating_entry_point():
    # larger first (3D Q2, 12^3 cells: 192 partial-sum blocks), then smaller (2D Q2, 16^2: 10 blocks),
    # so stale partials of the first call would show in the second
    cases = [CONFIGS["C5"].with_(N=12), CONFIGS["C2"].with_(N=16, n_h_levels=1, active_p=0.0, dirichlet=False)]
    for cfg in cases:
        say("noalloc param vjp", cfg.name, f"{cfg.dim}D N={cfg.N} Q{cfg.k}")
        ctx, args = _case(cfg)
        ref = ctx.residual_param_vjp(*args)
        got = ctx.residual_param_vjp_noalloc(*args)
        again = ctx.residual_param_vjp_noalloc(*args)
        say("  allocating", ref, "no-alloc", got, again)
        assert ref[0] != 0.0 and ref[1] != 0.0
        # same kernels and the same fixed reduction order: bit-identical
        assert got == ref and again == ref
        ctx.close()


def test_noalloc_param_vjp_refuses_contexts_beyond_its_scratch():
    # 2D Q1 with 2897^2 cells needs 131,142 blocks of 64 cells, above the 131,072 the scratch holds
    from paper_2005_00331_amd import Context, MfpffError, problem_from
    cfg = CONFIGS["C1"].with_(N=2897, n_h_levels=1, active_p=0.0, dirichlet=False)
    say("noalloc refusal", f"2D N={cfg.N} Q{cfg.k}", cfg.n_dofs, "dofs")
    ctx = Context(problem_from(cfg, [(cfg.N, cfg.k)]))
    nn = ctx.n_nodes
    u = torch.zeros(2 * nn, dtype=torch.float64, device="cuda")
    phi = torch.ones(nn, dtype=torch.float64, device="cuda")
    v = torch.zeros(3 * nn, dtype=torch.float64, device="cuda")
    with pytest.raises(MfpffError) as ei:
        ctx.residual_param_vjp_noalloc(u, phi, phi, v)
    assert ei.value.status == 1 and "static scratch holds 131072" in str(ei.value)
    # the allocating entry point still serves it
    a, b = ctx.residual_param_vjp(u, phi, phi, v)
    assert a == 0.0 and b == 0.0
    ctx.close()
