"""Residual, Jacobian, constraints and derivatives (oracle; test infrastructure only).

Follows, term by term:
  * eq. (residual) of Section 3.2: the nonlinear residual R(u, phi)(w, psi)
    with the extrapolation phi~ in the degradation of the u-equation;
  * eq. (G) of Section 3.2: its derivative with phi~ frozen, which makes
    the coupling block G_{u phi} vanish (block structure of Section 3.3);
  * Section 3.4: G dU = sum_k C^T P_k^T G_k P_k C dU -- here every element
    matrix G_k is formed explicitly and the global sparse matrix is
    assembled from them (duplicates summed), the plain definition the
    matrix-free product must reproduce;
  * Algorithm 1: degrees of freedom of the active set are fixed
    (delta phi = 0), read as identity rows and columns:
    G^ = P G P + (I - P), P = diag(free dofs); homogeneous Dirichlet
    conditions on delta u are handled the same way.

Local dof order inside a cell is (component, local node), component d
being phi; global dof = component * n_nodes + node.
"""
from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp

from . import material as mat
from .fe import Mesh, TensorBasis


@dataclass(frozen=True)
class Material:
    lam: float
    mu: float
    Gc: float
    eps: float
    kappa: float
    split: str = "amor"   # "amor" (volumetric/deviatoric), "miehe" (spectral) or "none" (isotropic)


def material_of(cfg, N=None) -> Material:
    N = cfg.N if N is None else N
    return Material(cfg.lam, cfg.mu, cfg.Gc, cfg.eps_factor / N, cfg.kappa, getattr(cfg, "split", "amor"))


class CellData:
    """Quadrature-point quantities of a set of cells (the linearisation point)."""

    def __init__(self, mesh: Mesh, tb: TensorBasis, m: Material, u, phi, phi_t, cells):
        d, h = mesh.dim, mesh.h
        self.cells = cells
        self.nodes = mesh.cell_nodes(cells)                 # (nc, P)
        self.gradN = tb.grad / h                            # (Q, P, d)
        self.N = tb.val                                     # (Q, P)
        self.JxW = tb.w * h ** d                            # (Q,)
        ul = u[:, self.nodes]                               # (d, nc, P)
        self.grad_u = np.einsum("qpa,cnp->nqca", self.gradN, ul)   # (nc, Q, d, d): [c][a] = du_c/dx_a
        pl = phi[self.nodes]
        self.phi = pl @ self.N.T                            # (nc, Q)
        self.grad_phi = np.einsum("qpa,np->nqa", self.gradN, pl)
        self.phi_t = phi_t[self.nodes] @ self.N.T
        split = {"miehe": mat.miehe_split, "none": mat.isotropic_split}.get(m.split, mat.amor_split)
        self.split = split(self.grad_u, m.lam, m.mu)
        self.gt = mat.g(self.phi_t, m.kappa)
        self.dg = mat.dg(self.phi, m.kappa)
        self.ddg = mat.ddg(self.phi, m.kappa)
        # Eb[q, c, p, i, j]: strain of the vector basis function N_p e_c
        Q, P = self.N.shape
        Eb = np.zeros((Q, d, P, d, d))
        for c in range(d):
            Eb[:, c, :, c, :] += 0.5 * self.gradN
            Eb[:, c, :, :, c] += 0.5 * self.gradN
        self.Eb = Eb


def _chunks(n, size):
    for s in range(0, n, size):
        yield np.arange(s, min(n, s + size))


def _chunk_size(mesh):
    return max(1, 2_000_000 // (mesh.P ** 2 * (mesh.dim + 1) ** 2))


def element_jacobians(mesh, m: Material, u, phi, phi_t, cells):
    """(nc, (d+1)P, (d+1)P) element matrices of eq. (G) for the given cells."""
    tb = TensorBasis(mesh.dim, mesh.k)
    cd = CellData(mesh, tb, m, u, phi, phi_t, cells)
    d, P = mesh.dim, mesh.P
    s = cd.split
    nc = len(cells)
    # delta sigma for every trial basis function: (nc, Q, d, P, d, d)
    if m.split == "miehe":
        sb = dict(H=s["H"][:, :, None, None], ev=s["ev"][:, :, None, None], V=s["V"][:, :, None, None])
        dsig = mat.dsigma_miehe(cd.Eb[None], sb, cd.gt[:, :, None, None], m.lam, m.mu)
    else:
        dsig = mat.dsigma(cd.Eb[None], s["H"][:, :, None, None], cd.gt[:, :, None, None], s["K"], m.mu)
    Ge = np.zeros((nc, (d + 1) * P, (d + 1) * P))
    # G_uu: (delta sigma(trial), e(test))
    Guu = np.einsum("q,nqCPij,qcpij->ncpCP", cd.JxW, dsig, cd.Eb)
    Ge[:, : d * P, : d * P] = Guu.reshape(nc, d * P, d * P)
    # G_phi u: (g'(phi) dE^+/de (trial), psi) with dE^+/de = sigma^+
    sp_e = np.einsum("nqij,qCPij->nqCP", s["sig_p"], cd.Eb)
    Gpu = np.einsum("q,nq,nqCP,qp->npCP", cd.JxW, cd.dg, sp_e, cd.N)
    Ge[:, d * P:, : d * P] = Gpu.reshape(nc, P, d * P)
    # G_phi phi: (g'' E^+ + Gc/eps) (dphi, psi) + Gc eps (grad dphi, grad psi)
    coef = cd.ddg * s["E_p"] + m.Gc / m.eps
    Gpp = (np.einsum("q,nq,qP,qp->npP", cd.JxW, coef, cd.N, cd.N)
           + m.Gc * m.eps * np.einsum("q,qPa,qpa->pP", cd.JxW, cd.gradN, cd.gradN)[None])
    Ge[:, d * P:, d * P:] = Gpp
    return Ge, cd.nodes


def local_dofs(mesh, nodes):
    """(nc, (d+1)P) global dof ids in local (component, node) order."""
    return np.concatenate([c * mesh.n_nodes + nodes for c in range(mesh.dim + 1)], axis=1)


def assemble_jacobian(mesh, m: Material, u, phi, phi_t):
    """Unconstrained global Jacobian of eq. (G) as CSR (duplicates summed)."""
    n = mesh.n_dofs
    G = sp.csr_matrix((n, n))
    for cells in _chunks(mesh.n_cells, _chunk_size(mesh)):
        Ge, nodes = element_jacobians(mesh, m, u, phi, phi_t, cells)
        ld = local_dofs(mesh, nodes)
        nl = ld.shape[1]
        rows = np.repeat(ld, nl, axis=1).ravel()
        cols = np.tile(ld, (1, nl)).ravel()
        G = G + sp.coo_matrix((Ge.ravel(), (rows, cols)), shape=(n, n)).tocsr()
    G.sum_duplicates()
    return G


def free_vector(mesh, active, dirichlet: bool):
    """1 for free dofs, 0 for constrained ones: Dirichlet u-dofs on the two
    faces normal to the last axis, and phi-dofs in the active set."""
    d = mesh.dim
    p = np.ones(mesh.n_dofs)
    if dirichlet:
        bn = mesh.boundary_nodes(d - 1)
        for c in range(d):
            p[c * mesh.n_nodes + np.flatnonzero(bn)] = 0.0
    p[d * mesh.n_nodes + np.flatnonzero(np.asarray(active) != 0)] = 0.0
    return p


def constrain(G, pvec):
    """G^ = P G P + (I - P)."""
    Pm = sp.diags(pvec)
    return (Pm @ G @ Pm + sp.diags(1.0 - pvec)).tocsr()


def cell_residuals(mesh, m: Material, u, phi, phi_t, cells):
    """Element residual vectors of eq. (residual) for the given cells: (nc, (d+1)P) in local
    (component, node) order, and the (nc, P) node ids.  The assembled residual is their sum."""
    tb = TensorBasis(mesh.dim, mesh.k)
    d = mesh.dim
    cd = CellData(mesh, tb, m, u, phi, phi_t, cells)
    s = cd.split
    stress = cd.gt[..., None, None] * s["sig_p"] + s["sig_m"]               # (nc, Q, d, d)
    Ru = np.einsum("q,nqij,qcpij->ncp", cd.JxW, stress, cd.Eb)              # (nc, d, P)
    Rp = (np.einsum("q,nq,qp->np", cd.JxW, cd.dg * s["E_p"] - m.Gc * (1.0 - cd.phi) / m.eps, cd.N)
          + m.Gc * m.eps * np.einsum("q,nqa,qpa->np", cd.JxW, cd.grad_phi, cd.gradN))
    nc = len(cells)
    return np.concatenate([Ru.reshape(nc, d * mesh.P), Rp], axis=1), cd.nodes


def residual(mesh, m: Material, u, phi, phi_t):
    """Assembled residual vector of eq. (residual), unconstrained."""
    R = np.zeros(mesh.n_dofs)
    for cells in _chunks(mesh.n_cells, 4 * _chunk_size(mesh)):
        Re, nodes = cell_residuals(mesh, m, u, phi, phi_t, cells)
        R += np.bincount(local_dofs(mesh, nodes).ravel(), Re.ravel(), minlength=mesh.n_dofs)
    return R


def energy(mesh, m: Material, u, phi):
    """Discrete energy of the split functional of Section 2.1 (phi~ = phi):
    sum_q w [g(phi) E^+ + E^- + Gc/2 ((1-phi)^2/eps + eps |grad phi|^2)]."""
    tb = TensorBasis(mesh.dim, mesh.k)
    E = 0.0
    for cells in _chunks(mesh.n_cells, 4 * _chunk_size(mesh)):
        cd = CellData(mesh, tb, m, u, phi, phi, cells)
        s = cd.split
        dens = (mat.g(cd.phi, m.kappa) * s["E_p"] + s["E_m"]
                + 0.5 * m.Gc * ((1.0 - cd.phi) ** 2 / m.eps + m.eps * (cd.grad_phi ** 2).sum(-1)))
        E += float((dens * cd.JxW[None]).sum())
    return E


def param_vjp(mesh, m: Material, u, phi, phi_t, v):
    """(dGc, deps) = <v, dR/dGc>, <v, dR/deps>; only the phi rows depend on them."""
    tb = TensorBasis(mesh.dim, mesh.k)
    d, nn = mesh.dim, mesh.n_nodes
    vphi = v[d * nn:]
    dGc = deps = 0.0
    for cells in _chunks(mesh.n_cells, 4 * _chunk_size(mesh)):
        cd = CellData(mesh, tb, m, u, phi, phi_t, cells)
        vl = vphi[cd.nodes]
        vq = vl @ cd.N.T
        gv = np.einsum("qpa,np->nqa", cd.gradN, vl)
        a = ((1.0 - cd.phi) * vq * cd.JxW[None]).sum()          # (1 - phi, v)
        b = ((cd.grad_phi * gv).sum(-1) * cd.JxW[None]).sum()    # (grad phi, grad v)
        dGc += -a / m.eps + m.eps * b
        deps += m.Gc * (a / m.eps ** 2 + b)
    return dGc, deps


def lumped_phi_mass(mesh):
    """Row sums of the phi mass matrix: M_L[i] = integral of psi_i."""
    tb = TensorBasis(mesh.dim, mesh.k)
    nodes = mesh.cell_nodes()
    w = (tb.val * (tb.w * mesh.h ** mesh.dim)[:, None]).sum(0)   # (P,)
    return np.bincount(nodes.ravel(), np.tile(w, mesh.n_cells), minlength=mesh.n_nodes)


def apply_rows(mesh, m: Material, u, phi, phi_t, pvec, x, nodes, transpose=False):
    """Rows (all components) of G^ x (or G^T x) at the given nodes, from the
    element matrices of the cells that touch them only.  Returns (d+1, len(nodes))."""
    nodes = np.asarray(nodes)
    cells = mesh.cells_of_nodes(nodes)
    d, nn = mesh.dim, mesh.n_nodes
    y = np.zeros(mesh.n_dofs)
    xm = pvec * x
    for ch in _chunks(len(cells), _chunk_size(mesh)):
        Ge, cn = element_jacobians(mesh, m, u, phi, phi_t, cells[ch])
        ld = local_dofs(mesh, cn)
        xl = xm[ld]
        yl = np.einsum("nji,nj->ni" if transpose else "nij,nj->ni", Ge, xl)
        np.add.at(y, ld.ravel(), yl.ravel())
    rows = np.stack([c * nn + nodes for c in range(d + 1)])
    return pvec[rows] * y[rows] + (1.0 - pvec[rows]) * x[rows]


def diag_rows(mesh, m: Material, u, phi, phi_t, pvec, nodes):
    """Diagonal entries of G^ at the given nodes, (d+1, len(nodes))."""
    nodes = np.asarray(nodes)
    cells = mesh.cells_of_nodes(nodes)
    d, nn = mesh.dim, mesh.n_nodes
    y = np.zeros(mesh.n_dofs)
    for ch in _chunks(len(cells), _chunk_size(mesh)):
        Ge, cn = element_jacobians(mesh, m, u, phi, phi_t, cells[ch])
        ld = local_dofs(mesh, cn)
        np.add.at(y, ld.ravel(), np.diagonal(Ge, axis1=1, axis2=2).ravel())
    rows = np.stack([c * nn + nodes for c in range(d + 1)])
    return pvec[rows] * y[rows] + (1.0 - pvec[rows])


def residual_rows(mesh, m: Material, u, phi, phi_t, nodes):
    """Rows of the residual at the given nodes from the touching cells only."""
    nodes = np.asarray(nodes)
    cells = mesh.cells_of_nodes(nodes)
    d, nn = mesh.dim, mesh.n_nodes
    Re, cn = cell_residuals(mesh, m, u, phi, phi_t, cells)
    R = np.bincount(local_dofs(mesh, cn).ravel(), Re.ravel(), minlength=mesh.n_dofs)
    rows = np.stack([c * nn + nodes for c in range(d + 1)])
    return R[rows]
