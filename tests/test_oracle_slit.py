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
