"""Directional central differences of <v, R> with the quadrature points whose tension/compression
branch changes between U + h d and U - h d counted, and the cells holding them taken out of both
sides of the comparison.

R is piecewise smooth in U: in the volumetric/deviatoric split, the branch of a quadrature point
is the sign of tr e, which is linear in U, so a point changes branch exactly when tr e(U + h d) and
tr e(U - h d) lie on different sides of 0 (H(0) = 1).  Such a point makes the central difference
an average of two tangents.  Its cell's share of <v, R(U +- h d)> and of <v, G d> comes from the
oracle's element vectors and matrices, and is subtracted from the assembled sums (which come from
the implementation under test), so the remaining gap measures the product on every other cell.
"""
import numpy as np

from oracle import fe
from oracle import operator as op


def traces_at_points(mesh, u):
    """tr e at every Gauss point: (n_cells, Q), u of shape (dim, n_nodes)."""
    tb = fe.TensorBasis(mesh.dim, mesh.k)
    nodes = mesh.cell_nodes()
    t = np.zeros((nodes.shape[0], tb.grad.shape[0]))
    for a in range(mesh.dim):
        t += u[a][nodes] @ (tb.grad[:, :, a].T / mesh.h)
    return t


def crossing_cells(t0, td, h):
    """Cells with a point whose branch differs between t0 + h td and t0 - h td, and the point count."""
    cross = (t0 + h * td >= 0) != (t0 - h * td >= 0)
    return np.flatnonzero(cross.any(axis=1)), int(cross.sum())


def cells_share(mesh, m, U, pt, v, dvec, h, cells):
    """(FD share, tangent share) of the given cells: sum over them of
    <v_c, R_c(U + h d) - R_c(U - h d)> / 2h and <v_c, G_c(U) d_c>."""
    if len(cells) == 0:
        return 0.0, 0.0
    d, nn = mesh.dim, mesh.n_nodes
    fd = 0.0
    for sgn in (1.0, -1.0):
        W = U + sgn * h * dvec
        Re, nodes = op.cell_residuals(mesh, m, W[: d * nn].reshape(d, nn), W[d * nn:], pt, cells)
        fd += sgn * float((v[op.local_dofs(mesh, nodes)] * Re).sum())
    Ge, nodes = op.element_jacobians(mesh, m, U[: d * nn].reshape(d, nn), U[d * nn:], pt, cells)
    ld = op.local_dofs(mesh, nodes)
    ad = float(np.einsum("ni,nij,nj->", v[ld], Ge, dvec[ld]))
    return fd / (2 * h), ad


def excluded_gaps(mesh, m, U, pt, v, dirs, h, fd_full, ad_full):
    """Per direction: (crossing points, crossing cells, full relative gap, relative gap with the
    crossing cells excluded).  fd_full[j], ad_full[j]: the assembled sums under test."""
    d, nn = mesh.dim, mesh.n_nodes
    t0 = traces_at_points(mesh, U[: d * nn].reshape(d, nn))
    out = []
    for j, dvec in enumerate(dirs):
        td = traces_at_points(mesh, dvec[: d * nn].reshape(d, nn))
        cells, npts = crossing_cells(t0, td, h)
        fx, ax = cells_share(mesh, m, U, pt, v, dvec, h, cells)
        full = abs(fd_full[j] - ad_full[j]) / abs(ad_full[j])
        rest = abs((fd_full[j] - fx) - (ad_full[j] - ax)) / abs(ad_full[j] - ax)
        out.append((npts, len(cells), full, rest))
    return out
