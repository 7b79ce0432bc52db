"""Finite-element building blocks (oracle; test infrastructure only).

Section 3.1 of the paper: continuous Q_p elements on quadrilateral or
hexahedral meshes, p in every coordinate direction.  The paper leaves the
node placement and the quadrature to deal.II; the readings used here are
equispaced nodes on each cell (so coarse nodes are a subset of fine
nodes) and Gauss-Legendre quadrature with p+1 points per direction.

Mesh: the unit square/cube, N cells per direction, h = 1/N, affine cells
(Jacobian h*I).  Global nodes are numbered lexicographically,
node = i0 + M*i1 (+ M^2*i2), M = k*N + 1.  Cells are numbered the same
way with N, local nodes and quadrature points lexicographically with the
first axis fastest.
"""
import itertools

import numpy as np


def gauss_legendre_01(q: int):
    """Gauss-Legendre points and weights mapped to [0, 1]."""
    x, w = np.polynomial.legendre.leggauss(q)
    return 0.5 * (x + 1.0), 0.5 * w


def lagrange_nodes(k: int) -> np.ndarray:
    return np.arange(k + 1) / k


def lagrange_values(k: int, x: np.ndarray) -> np.ndarray:
    """V[j, i] = l_i(x_j) for the equispaced Lagrange basis of degree k."""
    xi = lagrange_nodes(k)
    x = np.asarray(x, dtype=float)
    V = np.ones((x.size, k + 1))
    for i in range(k + 1):
        for m in range(k + 1):
            if m != i:
                V[:, i] *= (x - xi[m]) / (xi[i] - xi[m])
    return V


def lagrange_derivs(k: int, x: np.ndarray) -> np.ndarray:
    """D[j, i] = l_i'(x_j), by the product rule on the Lagrange product."""
    xi = lagrange_nodes(k)
    x = np.asarray(x, dtype=float)
    D = np.zeros((x.size, k + 1))
    for i in range(k + 1):
        for m in range(k + 1):
            if m == i:
                continue
            term = np.full(x.size, 1.0 / (xi[i] - xi[m]))
            for j in range(k + 1):
                if j != i and j != m:
                    term *= (x - xi[j]) / (xi[i] - xi[j])
            D[:, i] += term
    return D


class Mesh:
    """Structured Q_k mesh of the unit square/cube.

    slit=True: the geometry of the single-edge-notched tests (Section 5.1), a slit on the
    mid-plane of the last axis from the face x = 0 to x = 1/2, across which the cells do not
    connect.  The nodes on the slit (last-axis coordinate 1/2, first coordinate below 1/2; the
    tip at x = 1/2 is shared) exist twice: the grid node belongs to the cells below the slit, a
    duplicate appended after the M^dim grid nodes to the cells above it.  Duplicates are numbered
    like their grid nodes with the first axis fastest (3D: then the second axis).  N must be even."""

    def __init__(self, dim: int, N: int, k: int, slit: bool = False):
        self.dim, self.N, self.k = dim, N, k
        self.h = 1.0 / N
        self.M = k * N + 1
        self.slit = bool(slit)
        self.n_grid = self.M ** dim
        if self.slit:
            assert N % 2 == 0, "the slit lies on a cell face only for even N"
            self.n_slit_x = k * N // 2          # slit nodes per line along the first axis
            self.n_dup = self.n_slit_x * (self.M ** (dim - 2))
        else:
            self.n_slit_x = 0
            self.n_dup = 0
        self.n_nodes = self.n_grid + self.n_dup
        self.n_cells = N ** dim
        self.P = (k + 1) ** dim   # nodes per cell == quadrature points per cell

    @property
    def n_dofs(self):
        return (self.dim + 1) * self.n_nodes

    def local_multi(self):
        """(P, dim) local multi-indices, first axis fastest."""
        r = range(self.k + 1)
        return np.array([t[::-1] for t in itertools.product(*([r] * self.dim))])

    def cell_multi(self, cells=None):
        if cells is None:
            cells = np.arange(self.n_cells)
        cells = np.asarray(cells)
        return np.stack([(cells // self.N ** a) % self.N for a in range(self.dim)], axis=1)

    def cell_nodes(self, cells=None) -> np.ndarray:
        """(n_cells, P) global node ids of each cell's local nodes."""
        cm = self.cell_multi(cells)                       # (nc, dim)
        lm = self.local_multi()                           # (P, dim)
        g = self.k * cm[:, None, :] + lm[None, :, :]      # (nc, P, dim)
        stride = self.M ** np.arange(self.dim)
        ids = (g * stride).sum(-1)
        if self.slit:
            # cells just above the slit plane take the duplicates of their slit-plane nodes
            d = self.dim
            above = (cm[:, d - 1] == self.N // 2)[:, None] & (lm[None, :, d - 1] == 0)
            on_slit = above & (g[:, :, 0] < self.n_slit_x)
            dup = g[:, :, 0] + (self.n_slit_x * g[:, :, 1] if d == 3 else 0)
            ids = np.where(on_slit, self.n_grid + dup, ids)
        return ids

    def node_multi(self, nodes) -> np.ndarray:
        """(n, dim) grid multi-indices of nodes (a duplicate has the one of its grid node)."""
        nodes = np.asarray(nodes)
        if self.slit:
            j = nodes - self.n_grid
            orig = (j % self.n_slit_x) + self.M ** (self.dim - 1) * (self.M // 2)
            if self.dim == 3:
                orig = orig + self.M * (j // self.n_slit_x)
            nodes = np.where(nodes >= self.n_grid, orig, nodes)
        return np.stack([(nodes // self.M ** a) % self.M for a in range(self.dim)], axis=1)

    def cells_of_nodes(self, nodes) -> np.ndarray:
        """Sorted unique ids of all cells that contain any of the given nodes."""
        nm = self.node_multi(nodes)
        out = set()
        for row in nm:
            ranges = []
            for a in range(self.dim):
                i = row[a]
                lo = max((i - 1) // self.k, 0) if i % self.k == 0 else i // self.k
                hi = min(i // self.k, self.N - 1)
                ranges.append(range(lo, hi + 1))
            for t in itertools.product(*ranges):
                out.add(int(sum(t[a] * self.N ** a for a in range(self.dim))))
        return np.array(sorted(out), dtype=np.int64)

    def boundary_nodes(self, axis: int) -> np.ndarray:
        """Boolean mask of nodes on the two faces normal to ``axis``."""
        i = self.node_multi(np.arange(self.n_nodes))[:, axis]
        return (i == 0) | (i == self.M - 1)


class TensorBasis:
    """Full tensor-product basis tables on the unit cell.

    val[q, p]       = N_p(x_q)
    grad[q, p, a]   = dN_p/dx_a (x_q) on the unit cell (divide by h for the physical cell)
    w[q]            = quadrature weight on the unit cell
    """

    def __init__(self, dim: int, k: int, q1d: int = None):
        q1d = k + 1 if q1d is None else q1d
        x, w1 = gauss_legendre_01(q1d)
        B = lagrange_values(k, x)      # (q, k+1)
        D = lagrange_derivs(k, x)
        qm = np.array([t[::-1] for t in itertools.product(*([range(q1d)] * dim))])
        pm = np.array([t[::-1] for t in itertools.product(*([range(k + 1)] * dim))])
        nq, P = len(qm), len(pm)
        val = np.ones((nq, P))
        grad = np.ones((nq, P, dim))
        wq = np.ones(nq)
        for a in range(dim):
            val *= B[np.ix_(qm[:, a], pm[:, a])]
            wq *= w1[qm[:, a]]
            for b in range(dim):
                grad[:, :, b] *= (D if a == b else B)[np.ix_(qm[:, a], pm[:, a])]
        self.val, self.grad, self.w = val, grad, wq
        self.dim, self.k, self.nq, self.P = dim, k, nq, P
