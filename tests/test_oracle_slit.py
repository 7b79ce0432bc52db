"""The slit geometry of the single-edge-notched tests (Section 5.1) in the oracle: dof counts
against the table printed in Section 5.2, the assembly on the slit mesh against the unslit
mesh with the duplicates merged back, and the structure of the cut."""
import json
import os

import numpy as np
import pytest
import scipy.sparse as sp

from oracle import operator as op
from oracle.fe import Mesh
from synth import CONFIGS, make_inputs
from synth.fields import slit_duplicates

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "slit_dofs.json")


def test_dof_counts_match_the_printed_table():
    tab = json.load(open(GOLDEN))
    assert len(tab["rows"]) == 8
    for level, p, dofs, cells in tab["rows"]:
        mesh = Mesh(2, 2 ** level, p, slit=True)
        assert mesh.n_dofs == dofs, (level, p, mesh.n_dofs, dofs)
        assert mesh.n_cells == cells
        # without the slit every count would be short by (d+1) k N / 2
        assert Mesh(2, 2 ** level, p).n_dofs == dofs - 3 * p * 2 ** level // 2


def _merge(mesh_s, mesh_f):
    """S: full-mesh dofs -> slit-mesh dofs, each duplicate takes the value of its grid node."""
    dup = slit_duplicates(mesh_f.dim, mesh_f.N, mesh_f.k)
    nn_s, nn_f = mesh_s.n_nodes, mesh_f.n_nodes
    rows = np.concatenate([np.arange(nn_f), nn_f + np.arange(dup.size)])
    cols = np.concatenate([np.arange(nn_f), dup])
    S1 = sp.csr_matrix((np.ones(rows.size), (rows, cols)), shape=(nn_s, nn_f))
    return sp.block_diag([S1] * (mesh_f.dim + 1)).tocsr(), S1


@pytest.mark.parametrize("dim,N,k", [(2, 4, 1), (2, 4, 2), (3, 2, 1), (3, 2, 2)])
def test_slit_assembly_merges_back_to_the_unslit_mesh(dim, N, k):
    # element matrices do not depend on the numbering; adding the duplicate rows and columns to
    # their grid nodes must give the unslit operator and residual exactly (up to rounding)
    base = CONFIGS["C2" if dim == 2 else "C3"].with_(dim=dim, N=N, k=k, n_h_levels=1, p_coarse=())
    cf, cs = base, base.with_(slit=True)
    inp = make_inputs(cf)
    ms, mf = Mesh(dim, N, k, slit=True), Mesh(dim, N, k)
    S, S1 = _merge(ms, mf)
    m = op.material_of(cf)
    us = (S1 @ inp["u"].T).T
    phs, pts = S1 @ inp["phi"], S1 @ inp["phi_tilde"]
    Gs = op.assemble_jacobian(ms, m, us, phs, pts)
    Gf = op.assemble_jacobian(mf, m, inp["u"], inp["phi"], inp["phi_tilde"])
    D = (S.T @ Gs @ S - Gf).toarray()
    assert np.abs(D).max() <= 1e-13 * abs(Gf).max()
    Rs = op.residual(ms, m, us, phs, pts)
    Rf = op.residual(mf, m, inp["u"], inp["phi"], inp["phi_tilde"])
    assert np.abs(S.T @ Rs - Rf).max() <= 1e-13 * np.abs(Rf).max()
    # the slit mesh's own inputs (synth) give the duplicates their grid node's values
    ins = make_inputs(cs)
    assert np.array_equal(ins["u"][:, mf.n_nodes:], ins["u"][:, slit_duplicates(dim, N, k)]) or cs.u_mode == "iid"


@pytest.mark.parametrize("dim,N,k", [(2, 4, 2), (3, 2, 2)])
def test_the_slit_cuts_the_coupling(dim, N, k):
    # no row of a duplicate (above the slit) couples to a node strictly below the slit plane, and
    # no grid node on the slit couples to a node strictly above it
    cfg = CONFIGS["C2" if dim == 2 else "C3"].with_(dim=dim, N=N, k=k, n_h_levels=1, p_coarse=(), slit=True)
    inp = make_inputs(cfg)
    ms = Mesh(dim, N, k, slit=True)
    G = op.assemble_jacobian(ms, op.material_of(cfg), inp["u"], inp["phi"], inp["phi_tilde"]).tocoo()
    nn = ms.n_nodes
    last = ms.node_multi(np.arange(nn))[:, dim - 1]
    mid = ms.M // 2
    rn, cn = G.row % nn, G.col % nn
    nz = np.abs(G.data) > 0
    dup_rows = rn >= ms.n_grid
    assert not np.any(nz & dup_rows & (last[cn] < mid))
    slit_grid = np.zeros(nn, bool)
    slit_grid[slit_duplicates(dim, N, k)] = True
    assert not np.any(nz & slit_grid[rn] & (last[cn] > mid))
    # and the duplicates do couple upwards, the grid nodes downwards (the cut is not everything)
    assert np.any(nz & dup_rows & (last[cn] > mid)) and np.any(nz & slit_grid[rn] & (last[cn] < mid))


def test_lumped_mass_splits_between_the_two_sides():
    # a slit node's mass is its half on each side: grid node + duplicate = the unslit node's mass
    ms, mf = Mesh(2, 8, 2, slit=True), Mesh(2, 8, 2)
    Ms, Mf = op.lumped_phi_mass(ms), op.lumped_phi_mass(mf)
    dup = slit_duplicates(2, 8, 2)
    merged = Ms[: mf.n_nodes].copy()
    np.add.at(merged, dup, Ms[mf.n_nodes:])
    assert np.allclose(merged, Mf, rtol=1e-14, atol=0)
    assert np.all(Ms > 0)
    assert np.allclose(Ms[dup], Ms[mf.n_nodes:], rtol=1e-14)   # symmetric about the slit plane


# ------------------------------------------------------------- multigrid on slit meshes
def _coarse_value(coarse: Mesh, vc, x, above):
    """The coarse slit-mesh finite-element function with nodal values vc at the point x, taken
    in a coarse cell that contains x; a point on the slit plane is taken on the side `above`
    names (the cells above the slit for a duplicate).  Elsewhere the function is continuous, so
    any containing cell gives the same value."""
    from oracle.fe import lagrange_values
    d, N, k = coarse.dim, coarse.N, coarse.k
    cm = [min(int(np.floor(x[a] * N + 1e-12)), N - 1) for a in range(d)]
    if abs(x[d - 1] - 0.5) < 1e-12:
        cm[d - 1] = N // 2 if above else N // 2 - 1
    cell = sum(cm[a] * N ** a for a in range(d))
    nodes = coarse.cell_nodes([cell])[0]
    lm = coarse.local_multi()
    basis = np.ones(len(nodes))
    for a in range(d):
        basis *= lagrange_values(k, np.array([x[a] * N - cm[a]]))[0][lm[:, a]]
    return basis @ vc[nodes]


def _positions(mesh):
    from synth.fields import node_coords
    X = node_coords(mesh.dim, mesh.N, mesh.k)
    return np.concatenate([X, X[slit_duplicates(mesh.dim, mesh.N, mesh.k)]])


@pytest.mark.parametrize("dim,levels", [(2, [(4, 1), (8, 1)]), (2, [(4, 2), (8, 2)]), (2, [(4, 1), (4, 2)]),
                                        (2, [(4, 2), (4, 4)]), (3, [(2, 1), (4, 1)]), (3, [(2, 1), (2, 2)])])
def test_slit_prolongation_interpolates_each_side(dim, levels):
    # P applied to any coarse slit-mesh function gives that function at every fine node, on the
    # fine node's own side of the slit (brute-force evaluation in the containing coarse cell)
    from oracle import multigrid as mg
    (Nc, kc), (Nf, kf) = levels
    mc, mf = Mesh(dim, Nc, kc, slit=True), Mesh(dim, Nf, kf, slit=True)
    P1 = sp.csr_matrix(mg.prolongation_1d(mf, mc))
    Pn = P1
    for _ in range(dim - 1):
        Pn = sp.kron(P1, Pn)
    P = mg.slit_prolongation(mf, mc, Pn)
    assert P.shape == (mf.n_nodes, mc.n_nodes)
    vc = np.random.default_rng(21).standard_normal(mc.n_nodes)
    X = _positions(mf)
    above = np.arange(mf.n_nodes) >= mf.n_grid
    ref = np.array([_coarse_value(mc, vc, X[i], above[i]) for i in range(mf.n_nodes)])
    assert np.abs(P @ vc - ref).max() <= 1e-13 * np.abs(ref).max()
    # and the jump across the slit survives: fine duplicates differ from their grid nodes
    dup_grid = slit_duplicates(dim, Nf, kf)
    assert np.abs((P @ vc)[mf.n_grid:] - (P @ vc)[dup_grid]).max() > 1e-3


@pytest.mark.parametrize("dim,levels", [(2, [(4, 1), (8, 1)]), (2, [(4, 1), (4, 2)]), (3, [(2, 1), (4, 1)])])
def test_slit_injection_keeps_the_side(dim, levels):
    # every coarse node is injected from the fine node at its position and on its side: a coarse
    # duplicate from a fine duplicate, a coarse grid node from a fine grid node
    from oracle import multigrid as mg
    (Nc, kc), (Nf, kf) = levels
    mc, mf = Mesh(dim, Nc, kc, slit=True), Mesh(dim, Nf, kf, slit=True)
    idx = mg.injection_index(mf, mc)
    Xc, Xf = _positions(mc), _positions(mf)
    assert np.allclose(Xf[idx], Xc, atol=1e-14)
    assert np.array_equal(idx >= mf.n_grid, np.arange(mc.n_nodes) >= mc.n_grid)
