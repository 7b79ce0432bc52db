"""Shared helpers of the GPU tests: seeded inputs, oracle hierarchies, device copies."""
import functools
import sys

import numpy as np

from oracle import multigrid as mg
from oracle import operator as op
from oracle.fe import Mesh
from synth import CONFIGS, make_inputs


def say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


def rel_err(got, ref):
    got, ref = np.asarray(got, dtype=np.float64), np.asarray(ref, dtype=np.float64)
    den = np.abs(ref).max()
    return float(np.abs(got - ref).max() / (den if den > 0 else 1.0))


def dev(a, dtype=None):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(a).ravel())
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def host(t):
    return t.detach().cpu().numpy()


# parity cases: (name, base config, levels coarse->fine, overrides)
CASES = {
    "2d_q1": ("C1", [(6, 1), (12, 1)], {}),
    "2d_q2": ("C2", [(5, 1), (5, 2), (10, 2)], {}),
    "2d_q3": ("C2", [(3, 1), (3, 3), (6, 3)], {}),
    "2d_q4": ("C4", [(3, 2), (3, 4), (6, 4)], dict(dim=2)),
    "3d_q1": ("C3", [(3, 1), (6, 1)], dict(vcycle_prec="f64")),
    "3d_q2": ("C3", [(2, 1), (2, 2), (4, 2)], dict(vcycle_prec="f64")),
    "3d_q3": ("C4", [(3, 1), (3, 3)], {}),
    "3d_q4": ("C4", [(2, 2), (2, 4), (4, 4)], {}),
    "3d_q2_f32": ("C3", [(2, 2), (4, 2)], dict(vcycle_prec="f32")),
    # spectral (Miehe) split
    "2d_q1_miehe": ("C1", [(6, 1), (12, 1)], dict(split="miehe")),
    "2d_q2_miehe": ("C2", [(5, 1), (5, 2), (10, 2)], dict(split="miehe")),
    "2d_q3_miehe": ("C2", [(3, 1), (3, 3), (6, 3)], dict(split="miehe")),
    "3d_q2_miehe": ("C3", [(2, 1), (2, 2), (4, 2)], dict(vcycle_prec="f64", split="miehe")),
    "3d_q4_miehe": ("C4", [(2, 2), (2, 4), (4, 4)], dict(split="miehe")),
    "2d_q2_miehe_f32": ("C2", [(5, 2), (10, 2)], dict(vcycle_prec="f32", split="miehe")),
    "3d_q2_miehe_f32": ("C3", [(2, 2), (4, 2)], dict(vcycle_prec="f32", split="miehe")),
    # isotropic model (no split)
    "2d_q1_none": ("C1", [(6, 1), (12, 1)], dict(split="none")),
    "2d_q2_none": ("C2", [(5, 1), (5, 2), (10, 2)], dict(split="none")),
    "2d_q3_none": ("C2", [(3, 1), (3, 3), (6, 3)], dict(split="none")),
    "3d_q2_none": ("C3", [(2, 1), (2, 2), (4, 2)], dict(vcycle_prec="f64", split="none")),
    "3d_q3_f32": ("C4", [(3, 1), (3, 3)], dict(vcycle_prec="f32")),
    "3d_q4_f32": ("C4", [(2, 1), (2, 2), (2, 4), (4, 4)], dict(vcycle_prec="f32")),
    "2d_q2_f32": ("C2", [(5, 2), (10, 2)], dict(vcycle_prec="f32")),
    # 3D Q3/Q4 products with the 1D contractions on the matrix cores (MFMA); 27-cell levels leave
    # a ragged last workgroup (the ragged Q4 case p-coarsens straight to Q1: a 3^3 Q2 coarse level
    # with the notch band would have cond(G^_uu) = 1.3e11, too ill-conditioned for the coarse-solve bound)
    "3d_q3_mfma": ("C4", [(3, 1), (3, 3)], dict(contraction="mfma")),
    "3d_q4_mfma": ("C4", [(2, 2), (2, 4), (4, 4)], dict(contraction="mfma")),
    "3d_q4_mfma_ragged": ("C4", [(3, 1), (3, 4)], dict(contraction="mfma")),
    "3d_q3_mfma_f32": ("C4", [(3, 1), (3, 3)], dict(vcycle_prec="f32", contraction="mfma")),
    "3d_q4_mfma_f32": ("C4", [(2, 1), (2, 2), (2, 4), (4, 4)], dict(vcycle_prec="f32", contraction="mfma")),
    "3d_q4_mfma_ragged_f32": ("C4", [(3, 1), (3, 4)], dict(vcycle_prec="f32", contraction="mfma")),
}


def case_config(name):
    base, levels, ov = CASES[name]
    N, k = levels[-1]
    cfg = CONFIGS[base].with_(N=N, k=k, n_h_levels=1, p_coarse=(), **ov)
    return cfg, levels


@functools.lru_cache(maxsize=4)
def oracle_case(name):
    cfg, levels = case_config(name)
    inp = make_inputs(cfg, ("rhs",))
    H = mg.Hierarchy(cfg, levels, inp["u"], inp["phi"], inp["phi_tilde"], inp["active"])
    return cfg, levels, inp, H


def gpu_context(cfg, levels, inp, **kw):
    from paper_2005_00331_amd import Context, problem_from
    ctx = Context(problem_from(cfg, levels, **kw))
    ctx.set_linearization(dev(inp["u"]), dev(inp["phi"]), dev(inp["phi_old"]), dev(inp["active"]),
                          dev(inp["phi_tilde"]))
    return ctx


def oracle_material(cfg):
    return op.material_of(cfg)


def mesh_of(cfg):
    return Mesh(cfg.dim, cfg.N, cfg.k)
