"""Load stepping of the single-edge-notched tests (oracle; test infrastructure only).

Section 5 drives the crack by a displacement prescribed on the top boundary that grows
with the pseudo-time, u = t du (a direction times the step count) on the top face,
with u = 0 on the bottom face; Section 3 replaces phi in the degradation g of the
residual by phi~, the linear extrapolation of the solutions of the two previous time
steps.  One load step is then Algorithm 1 run to its stopping test from the previous
step's state.  Readings:
  * top and bottom are the two faces normal to the last axis (y in 2D, z in 3D); every
    displacement component is prescribed on both;
  * with a constant step, the linear extrapolation at the new step is
    phi~ = 2 phi_{n-1} - phi_{n-2}, not clipped; at the first step, where there is no
    second previous solution, phi~ = phi_{n-1};
  * phi_{n-1} is also U^old of the active-set rule (the irreversibility reference);
  * the load on a face is the sum, over the face's nodes, of the residual's
    displacement rows at the end of the step: the nodal reaction force.
"""
import numpy as np

from . import operator as op
from .fe import Mesh
from .newton import pdas_solve


def face_nodes(mesh: Mesh, top: bool) -> np.ndarray:
    """Indices of the nodes on the bottom (last-axis coordinate 0) or top (1) face."""
    i = mesh.node_multi(np.arange(mesh.n_nodes))[:, mesh.dim - 1]
    return np.flatnonzero(i == (mesh.M - 1 if top else 0))


def impose_displacement(mesh: Mesh, u, u_top):
    """u with every component set to 0 on the bottom face and to u_top on the top face."""
    u = np.array(u, dtype=np.float64, copy=True).reshape(mesh.dim, mesh.n_nodes)
    u[:, face_nodes(mesh, False)] = 0.0
    u[:, face_nodes(mesh, True)] = np.asarray(u_top, dtype=np.float64)[:, None]
    return u


def extrapolate(phi_prev, phi_prev2):
    """Linear extrapolation to the new step from the two previous solutions (equal steps)."""
    if phi_prev2 is None:
        return np.array(phi_prev, dtype=np.float64, copy=True)
    return 2.0 * np.asarray(phi_prev) - np.asarray(phi_prev2)


def face_reaction(mesh: Mesh, R, top: bool):
    """Per component, the sum of the displacement residual rows over the face's nodes."""
    nodes = face_nodes(mesh, top)
    return np.array([R[c * mesh.n_nodes + nodes].sum() for c in range(mesh.dim)])


def load_step(cfg, levels_nk, u, phi, phi_prev, phi_prev2, u_top, max_newton=20, tol=1e-8):
    """One load step: prescribe the boundary displacement, extrapolate phi~, run Algorithm 1
    to its stopping test from (u, phi); returns the new state, the loop's record, phi~ and the
    reactions on the top and bottom faces."""
    mesh = Mesh(cfg.dim, cfg.N, cfg.k, getattr(cfg, "slit", False))
    u0 = impose_displacement(mesh, u, u_top)
    pt = extrapolate(phi_prev, phi_prev2)
    out = pdas_solve(cfg, levels_nk, u0, np.array(phi, dtype=np.float64), np.asarray(phi_prev), pt, max_newton, tol)
    R = op.residual(mesh, op.material_of(cfg), out["u"], out["phi"], pt)
    out.update(phi_tilde=pt, R=R, reaction_top=face_reaction(mesh, R, True),
               reaction_bottom=face_reaction(mesh, R, False))
    return out


def load_steps(cfg, levels_nk, u, phi, direction, du, n_steps, max_newton=20, tol=1e-8):
    """n_steps load steps from (u, phi) with u_top = t du direction at step t = 1..n_steps;
    returns the per-step records."""
    hist = []
    phi_prev, phi_prev2 = np.array(phi, dtype=np.float64), None
    for t in range(1, n_steps + 1):
        rec = load_step(cfg, levels_nk, u, phi_prev, phi_prev, phi_prev2, t * du * np.asarray(direction), max_newton,
                        tol)
        hist.append(rec)
        u, phi_prev2, phi_prev = rec["u"], phi_prev, rec["phi"]
    return hist
