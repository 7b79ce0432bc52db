"""GPU parity against the oracle on small multi-tile cases with ragged tails.

Every level of each hierarchy is checked: operator products (G^, G^T,
diag(G^_uu, G^_phiphi)), the diagonal, Lanczos estimates, the Chebyshev
smoother, the transfers, the coarse solve and a whole V-cycle.
Tolerances (relative to the max-norm of the oracle result):
  products, diagonal       1e-12  (sum-factorised vs explicit element matrices, FP64)
  transfers                1e-14  (same few-term interpolation sums)
  Lanczos lambda           1e-10  (15 CG steps, different reduction order)
  smoother, V-cycle        1e-10  (coarse solve by the inverse factor W = L^-1)
  FP32 level products      2e-5   (single precision, ~ (k+1)^d-term sums)
"""
import numpy as np
import pytest

from helpers import CASES, dev, gpu_context, host, oracle_case, rel_err, say
from oracle import multigrid as mg

pytestmark = pytest.mark.gpu

_ctx_cache = {}


def ctx_for(name):
    if name not in _ctx_cache:
        cfg, levels, inp, H = oracle_case(name)
        say(name, "levels", levels, "dofs", H.levels[-1].mesh.n_dofs)
        _ctx_cache.clear()
        _ctx_cache[name] = gpu_context(cfg, levels, inp)
    return _ctx_cache[name]


NAMES = [n for n in CASES if not n.endswith("f32")]


@pytest.mark.parametrize("name", ["2d_q2", "3d_q2"])
def test_accumulate_flag_is_masked_product_without_identity(name):
    # y += P G P x on free rows, y left alone elsewhere
    from paper_2005_00331_amd import OP_ACCUMULATE, OP_G
    cfg, levels, inp, H = oracle_case(name)
    ctx = ctx_for(name)
    lev = H.levels[-1]
    x = np.random.default_rng(12).standard_normal(lev.mesh.n_dofs)
    y0 = np.random.default_rng(13).standard_normal(lev.mesh.n_dofs)
    say(name, "accumulate")
    import torch
    y = dev(y0)
    ctx.apply_jacobian(-1, dev(x), y, op=OP_G | OP_ACCUMULATE)
    p = lev.pvec
    ref = y0 + p * (lev.G @ (p * x))
    assert rel_err(host(y), ref) <= 1e-12


@pytest.mark.parametrize("name", NAMES)
def test_operator_products_every_level(name):
    cfg, levels, inp, H = oracle_case(name)
    ctx = ctx_for(name)
    from paper_2005_00331_amd import OP_BLOCKDIAG, OP_G, OP_GT
    rng = np.random.default_rng(7)
    for l, lev in enumerate(H.levels):
        x = rng.standard_normal(lev.mesh.n_dofs)
        for op, ref in ((OP_G, lev.A @ x), (OP_GT, lev.A.T @ x), (OP_BLOCKDIAG, lev.Ablk @ x)):
            say(name, "level", l, "op", op)
            y = host(ctx.apply_jacobian(l, dev(x), op=op))
            e = rel_err(y, ref)
            assert e <= 1e-12, (name, l, op, e)


@pytest.mark.parametrize("name", NAMES)
def test_diagonal_every_level(name):
    cfg, levels, inp, H = oracle_case(name)
    ctx = ctx_for(name)
    for l, lev in enumerate(H.levels):
        say(name, "diag level", l)
        e = rel_err(host(ctx.diagonal(l)), lev.D)
        assert e <= 1e-12, (name, l, e)


@pytest.mark.parametrize("name", NAMES)
def test_lanczos_and_smoother(name):
    cfg, levels, inp, H = oracle_case(name)
    ctx = ctx_for(name)
    rng = np.random.default_rng(8)
    for l in range(1, len(H.levels)):
        info = ctx.levels[l]
        for got, ref in ((info.lambda_u, H.lam[l][0]), (info.lambda_phi, H.lam[l][1])):
            assert abs(got - ref) <= 1e-10 * abs(ref), (name, l, got, ref)
        r = rng.standard_normal(H.levels[l].mesh.n_dofs)
        say(name, "smooth level", l)
        z = host(ctx.smooth(l, dev(r)))
        ref = mg.chebyshev_block(H.levels[l], H.lam[l], r, cfg.cheb_degree, cfg.cheb_lo, cfg.cheb_hi)
        assert rel_err(z, ref) <= 1e-10, (name, l, rel_err(z, ref))


@pytest.mark.parametrize("name", NAMES)
def test_transfers(name):
    cfg, levels, inp, H = oracle_case(name)
    ctx = ctx_for(name)
    rng = np.random.default_rng(9)
    for l in range(1, len(H.levels)):
        xc = rng.standard_normal(H.levels[l - 1].mesh.n_dofs)
        xf = rng.standard_normal(H.levels[l].mesh.n_dofs)
        say(name, "transfer level", l)
        assert rel_err(host(ctx.transfer(l, 0, dev(xc))), H.P[l] @ xc) <= 1e-14
        assert rel_err(host(ctx.transfer(l, 1, dev(xf))), H.P[l].T @ xf) <= 1e-14


@pytest.mark.parametrize("name", NAMES)
def test_coarse_solve_and_vcycle(name):
    cfg, levels, inp, H = oracle_case(name)
    ctx = ctx_for(name)
    rng = np.random.default_rng(10)
    r0 = rng.standard_normal(H.levels[0].mesh.n_dofs)
    say(name, "coarse solve")
    e = rel_err(host(ctx.coarse_solve(dev(r0))), H.coarse.solve(r0))
    assert e <= 1e-10, (name, e)
    r = rng.standard_normal(H.levels[-1].mesh.n_dofs)
    say(name, "vcycle")
    e = rel_err(host(ctx.vcycle(dev(r))), H.vcycle(r))
    assert e <= 1e-10, (name, e)


@pytest.mark.parametrize("name", ["3d_q2_f32", "3d_q3_f32", "3d_q4_f32", "2d_q2_f32", "2d_q2_miehe_f32", "3d_q2_miehe_f32",
                                  "3d_q3_mfma_f32", "3d_q4_mfma_f32", "3d_q4_mfma_ragged_f32"])
def test_fp32_level_products(name):
    import torch
    from paper_2005_00331_amd import F32, OP_BLOCKDIAG, OP_G
    cfg, levels, inp, H = oracle_case(name)
    ctx = ctx_for(name)
    rng = np.random.default_rng(11)
    for l, lev in enumerate(H.levels):
        x = rng.standard_normal(lev.mesh.n_dofs)
        for op, A in ((OP_G, lev.A), (OP_BLOCKDIAG, lev.Ablk)):
            say(name, "fp32 level", l, "op", op)
            y = host(ctx.apply_jacobian(l, dev(x, torch.float32), prec=F32, op=op))
            assert rel_err(y, A @ x.astype(np.float32).astype(np.float64)) <= 2e-5
    # mixed V-cycle: FP32 levels, FP64 coarse solve
    r = rng.standard_normal(H.levels[-1].mesh.n_dofs)
    e = rel_err(host(ctx.vcycle(dev(r))), H.vcycle(r))
    say(name, "fp32 vcycle rel err", e)
    assert e <= 1e-4


@pytest.mark.parametrize("name", ["2d_q1", "2d_q2", "3d_q2"])
def test_products_and_vcycle_are_bitwise_reproducible(name):
    # fixed summation orders (colour phases in 2D, ordered node gather in 3D, block-ordered
    # reductions): repeated calls give identical bits
    from paper_2005_00331_amd import OP_BLOCKDIAG, OP_G, OP_GT
    cfg, levels, inp, H = oracle_case(name)
    ctx = ctx_for(name)
    x = dev(np.random.default_rng(21).standard_normal(H.levels[-1].mesh.n_dofs))
    say(name, "reproducibility")
    for opn in (OP_G, OP_GT, OP_BLOCKDIAG):
        a = host(ctx.apply_jacobian(-1, x, op=opn))
        b = host(ctx.apply_jacobian(-1, x, op=opn))
        assert np.array_equal(a, b), opn
    assert np.array_equal(host(ctx.vcycle(x)), host(ctx.vcycle(x)))


@pytest.mark.parametrize("dim,N,k,split", [(2, 4, 1, "amor"), (2, 3, 2, "amor"), (2, 2, 4, "amor"),
                                           (3, 2, 2, "amor"), (3, 2, 4, "amor"), (2, 3, 2, "miehe"),
                                           (3, 2, 2, "miehe")])
def test_element_matrices_and_sparse_product(dim, N, k, split):
    # the unconstrained element matrices against the oracle's assembled Jacobian, and the
    # assembled CSR product against the matrix-free product with nothing constrained
    import torch
    from oracle import fe
    from oracle import operator as op
    from paper_2005_00331_amd import Context, OP_G, problem_from
    from paper_2005_00331_amd.assembly import assemble_csr
    from synth import CONFIGS, make_inputs
    cfg = (CONFIGS["C3"] if dim == 3 else CONFIGS["C2"]).with_(dim=dim, N=N, k=k, n_h_levels=1, p_coarse=(),
                                                               split=split, dirichlet=False, vcycle_prec="f64")
    inp = make_inputs(cfg)
    mesh = fe.Mesh(dim, N, k)
    ctx = Context(problem_from(cfg, [(N, k)]))
    zeros = np.zeros(mesh.n_nodes, np.uint8)
    ctx.set_point(dev(inp["u"]), dev(inp["phi"]), dev(inp["phi_old"]), dev(zeros), dev(inp["phi_tilde"]))
    say(dim, N, k, split, "element matrices")
    A = assemble_csr(ctx.element_matrices(-1), dim, N, k)
    G = op.assemble_jacobian(mesh, op.material_of(cfg), inp["u"], inp["phi"], inp["phi_tilde"]).toarray()
    assert np.abs(A.to_dense().cpu().numpy() - G).max() <= 1e-12 * np.abs(G).max()
    x = dev(np.random.default_rng(3).standard_normal(mesh.n_dofs))
    y = host(torch.mv(A, x))
    assert rel_err(y, host(ctx.apply_jacobian(-1, x, op=OP_G))) <= 1e-12


@pytest.mark.parametrize("k,N", [(3, 5), (4, 3)])
def test_mfma_products_match_the_vector_unit(k, N):
    # the matrix-core and the vector-unit contractions give the same products up to rounding,
    # in FP64 and FP32, for every operator mode
    import torch
    from paper_2005_00331_amd import F32, F64, OP_BLOCKDIAG, OP_G, OP_GT, Context, problem_from
    from synth import CONFIGS, make_inputs
    cfg = CONFIGS["C4"].with_(N=N, k=k, n_h_levels=1, p_coarse=(), vcycle_prec="f32")
    inp = make_inputs(cfg)
    ctxs = [Context(problem_from(cfg, [(N, k)], contraction=c)) for c in ("valu", "mfma")]
    for ctx in ctxs:
        ctx.set_linearization(dev(inp["u"]), dev(inp["phi"]), dev(inp["phi_old"]), dev(inp["active"]),
                              dev(inp["phi_tilde"]))
    x = np.random.default_rng(14).standard_normal(ctxs[0].n_dofs)
    for prec, dt, tol in ((F64, torch.float64, 1e-13), (F32, torch.float32, 1e-5)):
        for opn in (OP_G, OP_GT, OP_BLOCKDIAG):
            say("mfma vs valu", k, N, prec, opn)
            ys = [host(c.apply_jacobian(-1, dev(x, dt), prec=prec, op=opn)) for c in ctxs]
            assert rel_err(ys[1], ys[0]) <= tol
