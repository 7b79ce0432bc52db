"""Pins of the oracle's load stepping (Section 5 boundary loading, Section 3 extrapolation).

Independent of the oracle's formulas:
  * equilibrium: the basis functions sum to one, so the displacement residual rows sum to
    zero over all nodes; at the end of a step the free rows vanish, so the top and bottom
    reactions cancel;
  * Clapeyron's identity: the split stress is positively homogeneous of degree one in the
    strain, so u . R_u(u) = 2 E_el(u; phi~) for any u; at the end of a step the free rows
    vanish, bottom values are zero, and the sum reduces to u_top . reaction_top, with E_el
    the elastic part of the energy functional evaluated at phi~;
  * linear response: from an undamaged body at rest the reaction is linear in the
    prescribed displacement up to the phase field's second-order response;
  * the extrapolation reproduces a phase field that changes linearly in time.
"""
import numpy as np
import pytest

from oracle import loading, operator as op
from oracle.fe import Mesh
from synth.configs import CONFIGS, level_list
from synth.fields import make_phi

# (workload, overrides, split, displacement increment per step)
CASES = [
    ("C1", dict(N=8, n_h_levels=2), "amor", 2e-3),
    ("C1", dict(N=8, n_h_levels=2), "miehe", 2e-3),
    ("C2", dict(N=8, n_h_levels=2), "amor", 5e-4),
    ("C1", dict(dim=3, N=4, n_h_levels=2), "amor", 1e-3),
]


def _setup(name, kw, split):
    cfg = CONFIGS[name].with_(split=split, phi_mode="ones", **kw)
    mesh = Mesh(cfg.dim, cfg.N, cfg.k)
    direction = np.zeros(cfg.dim)
    direction[-1] = 1.0
    return cfg, mesh, direction


def _elastic_energy(mesh, m, u, phi_t):
    # the fracture part of the functional does not depend on u
    return op.energy(mesh, m, u, phi_t) - op.energy(mesh, m, np.zeros_like(u), phi_t)


@pytest.mark.parametrize("name,kw,split,du", CASES)
def test_load_steps_equilibrium_and_clapeyron(name, kw, split, du):
    cfg, mesh, direction = _setup(name, kw, split)
    levels = level_list(cfg)
    m = op.material_of(cfg)
    u0 = np.zeros((cfg.dim, cfg.n_nodes))
    hist = loading.load_steps(cfg, levels, u0, make_phi(cfg), direction, du, 3, tol=1e-10)
    for t, rec in enumerate(hist, start=1):
        assert rec["converged"]
        Ft, Fb = rec["reaction_top"], rec["reaction_bottom"]
        assert np.abs(Ft + Fb).max() <= 1e-7 * np.abs(Ft).max()
        u_top = t * du * direction
        assert np.allclose(rec["u"][:, loading.face_nodes(mesh, True)], u_top[:, None], rtol=0, atol=0)
        assert np.all(rec["u"][:, loading.face_nodes(mesh, False)] == 0.0)
        W = float(u_top @ Ft)
        E = _elastic_energy(mesh, m, rec["u"], rec["phi_tilde"])
        assert abs(W - 2.0 * E) <= 1e-7 * abs(W), (t, W, 2 * E)
    # the crack is driven: the phase field decreases under the growing load
    assert hist[-1]["phi"].min() < hist[0]["phi"].min() + 1e-12
    assert float((hist[0]["phi"] - hist[-1]["phi"]).max()) > 0


def test_reaction_is_linear_for_an_undamaged_body():
    cfg, mesh, direction = _setup("C1", dict(N=8, n_h_levels=2), "amor")
    levels = level_list(cfg)
    u0 = np.zeros((cfg.dim, cfg.n_nodes))
    ones = np.ones(cfg.n_nodes)
    r1 = loading.load_step(cfg, levels, u0, ones, ones, None, 1e-5 * direction, tol=1e-10)
    r2 = loading.load_step(cfg, levels, u0, ones, ones, None, 2e-5 * direction, tol=1e-10)
    F1, F2 = r1["reaction_top"], r2["reaction_top"]
    assert F1[-1] > 0  # pulling the top face up needs an upward force
    assert np.allclose(F2, 2.0 * F1, rtol=1e-6, atol=1e-9 * abs(F1[-1]))


def test_extrapolation_is_exact_for_a_linear_history():
    rng = np.random.default_rng(31)
    a, b = rng.uniform(0, 1, 50), rng.uniform(-0.1, 0.1, 50)
    assert np.allclose(loading.extrapolate(a + b, a), a + 2 * b, rtol=0, atol=1e-15)
    assert np.array_equal(loading.extrapolate(a, None), a)


def test_face_nodes_are_the_last_axis_faces():
    for dim, N, k in ((2, 3, 2), (3, 2, 1)):
        mesh = Mesh(dim, N, k)
        bn = mesh.boundary_nodes(dim - 1)
        top, bot = loading.face_nodes(mesh, True), loading.face_nodes(mesh, False)
        assert top.size == bot.size == mesh.M ** (dim - 1)
        assert np.array_equal(np.sort(np.concatenate([top, bot])), np.flatnonzero(bn))
        assert np.all(top > bot.max())
