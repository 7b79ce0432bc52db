"""Monolithic geometric multigrid (oracle; test infrastructure only).

Section 3.3: P^-1 = GMG(G) with the block-diagonal smoother
diag(S(G_uu), S(G_phiphi)), S a Chebyshev-Jacobi smoother on the interval
[c lambda_max, C lambda_max], c = 0.24, C = 1.2, lambda_max estimated by
CG.  Readings where the paper is silent:
  * levels: h-steps (N -> N/2) at the fine degree, optionally one p-step
    to a lower degree on the coarsest mesh;
  * level operators are rediscretised (eq. (G)) at injected fields
    u, phi, phi~ and injected active sets (coarse nodes are fine nodes);
  * transfers: P = Kronecker product of 1D interpolation matrices per
    component, masked on both sides, restriction = P^T;
  * smoothing step x <- x + diag(C_u, C_phi)(b - G^ x): the residual uses
    the full level operator, each block a Chebyshev polynomial of degree s
    (s - 1 block products) built by the textbook three-term recurrence
    with Jacobi scaling (Saad, Iterative Methods, Alg. 12.1);
  * lambda_max: k_L steps of Jacobi-preconditioned CG from a SplitMix64
    start vector, Ritz value of the CG-Lanczos tridiagonal
    (Saad, Section 6.7.3);
  * coarsest level: exact FP64 solve using the block lower-triangular
    structure (Cholesky of G_uu and G_phiphi; LU with partial pivoting for
    a block that is not positive definite, which takes kappa < 0; a
    singular block is an error), in place of the Chebyshev coarse solver
    the paper uses.
"""
import warnings

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

from . import operator as op
from .fe import Mesh, lagrange_values
from .splitmix import uniform_pm1


def injection_index(fine: Mesh, coarse: Mesh) -> np.ndarray:
    """For each coarse node, the fine node at the same position (on slit meshes a coarse
    duplicate maps to the fine duplicate there: the same side of the slit)."""
    num = fine.k * fine.N
    den = coarse.k * coarse.N
    assert num % den == 0
    r = num // den
    cm = coarse.node_multi(np.arange(coarse.n_nodes))
    stride = fine.M ** np.arange(fine.dim)
    idx = ((cm * r) * stride).sum(1)
    if coarse.slit:
        assert fine.slit
        dup = np.arange(coarse.n_grid, coarse.n_nodes)
        fm = cm[dup] * r
        idx[dup] = fine.n_grid + fm[:, 0] + (fine.n_slit_x * fm[:, 1] if fine.dim == 3 else 0)
    return idx


def slit_prolongation(fine: Mesh, coarse: Mesh, Pn) -> sp.csr_matrix:
    """Per-component prolongation between two slit meshes: the tensor-product interpolation Pn
    between the grid nodes, with every fine node taking the coarse values of its own side of the
    slit.  Where a fine node strictly above the slit plane, or a fine duplicate, reads a coarse
    slit node (a grid node with a duplicate), it reads that node's duplicate instead; below the
    slit, on the plane's grid nodes and at the shared tip nothing changes.  A fine duplicate
    interpolates like its grid node, along the plane."""
    d = fine.dim
    Pg = sp.csr_matrix(Pn)
    cm = coarse.node_multi(np.arange(coarse.n_grid))
    c_slit = (cm[:, d - 1] == coarse.M // 2) & (cm[:, 0] < coarse.n_slit_x)
    c_dup = coarse.n_grid + cm[:, 0] + (coarse.n_slit_x * cm[:, 1] if d == 3 else 0)
    fm = fine.node_multi(np.arange(fine.n_grid))
    f_above = fm[:, d - 1] > fine.M // 2

    def remap(block, above_rows):
        b = block.tocoo()
        m = above_rows[b.row] & c_slit[b.col]
        return b.row, np.where(m, c_dup[b.col], b.col), b.data

    r1, c1, v1 = remap(Pg, f_above)
    dup_grid = fine.node_multi(np.arange(fine.n_grid, fine.n_nodes))
    dup_grid = (dup_grid * (fine.M ** np.arange(d))).sum(1)
    r2, c2, v2 = remap(Pg[dup_grid], np.ones(dup_grid.size, bool))
    rows = np.concatenate([r1, fine.n_grid + r2])
    cols = np.concatenate([c1, c2])
    vals = np.concatenate([v1, v2])
    return sp.csr_matrix((vals, (rows, cols)), shape=(fine.n_nodes, coarse.n_nodes))


def prolongation_1d(fine: Mesh, coarse: Mesh) -> np.ndarray:
    """P1[i, j] = value of the coarse global basis function j at fine node i."""
    P1 = np.zeros((fine.M, coarse.M))
    den = fine.k * fine.N
    for i in range(fine.M):
        cell = min(i * coarse.N // den, coarse.N - 1)
        xi = (i * coarse.N - cell * den) / den
        vals = lagrange_values(coarse.k, np.array([xi]))[0]
        P1[i, coarse.k * cell: coarse.k * cell + coarse.k + 1] = vals
    return P1


class Level:
    def __init__(self, mesh: Mesh, m: op.Material, u, phi, phi_t, active, dirichlet):
        self.mesh, self.m = mesh, m
        self.u, self.phi, self.phi_t, self.active = u, phi, phi_t, active
        self.G = op.assemble_jacobian(mesh, m, u, phi, phi_t)
        self.pvec = op.free_vector(mesh, active, dirichlet)
        self.A = op.constrain(self.G, self.pvec)
        d, nn = mesh.dim, mesh.n_nodes
        nu = d * nn
        # block-diagonal part diag(G^_uu, G^_phiphi)
        A = self.A.tocoo()
        keep = (A.row < nu) == (A.col < nu)
        self.Ablk = sp.csr_matrix((A.data[keep], (A.row[keep], A.col[keep])), shape=A.shape)
        self.D = self.A.diagonal()
        self.nu = nu


class Hierarchy:
    """Levels 0 (coarsest) .. L (finest) with transfers and smoother data."""

    def __init__(self, cfg, levels_nk, u, phi, phi_t, active, dirichlet=None, m=None):
        dirichlet = cfg.dirichlet if dirichlet is None else dirichlet
        self.cfg = cfg
        self.m = op.material_of(cfg) if m is None else m
        slit = getattr(cfg, "slit", False)
        meshes = [Mesh(cfg.dim, N, k, slit) for (N, k) in levels_nk]
        L = len(meshes) - 1
        fields = [None] * (L + 1)
        fields[L] = (u, phi, phi_t, np.asarray(active).astype(np.uint8))
        for l in range(L - 1, -1, -1):
            idx = injection_index(meshes[l + 1], meshes[l])
            uf, pf, ptf, af = fields[l + 1]
            fields[l] = (uf[:, idx], pf[idx], ptf[idx], af[idx])
        self.levels = [Level(meshes[l], self.m, *fields[l], dirichlet) for l in range(L + 1)]
        self.L = L
        # transfers between l-1 (coarse) and l (fine)
        self.P = [None] * (L + 1)
        for l in range(1, L + 1):
            f, c = self.levels[l], self.levels[l - 1]
            P1 = sp.csr_matrix(prolongation_1d(f.mesh, c.mesh))
            Pn = P1
            for _ in range(cfg.dim - 1):
                Pn = sp.kron(P1, Pn)
            if slit:
                Pn = slit_prolongation(f.mesh, c.mesh, Pn)
            Pfull = sp.block_diag([Pn] * (cfg.dim + 1))
            self.P[l] = (sp.diags(f.pvec) @ Pfull @ sp.diags(c.pvec)).tocsr()
        # smoother intervals on levels >= 1
        self.lam = [None] * (L + 1)
        for l in range(1, L + 1):
            self.lam[l] = lanczos_block_estimates(self.levels[l], l, cfg.lanczos_steps, cfg.lanczos_seed)
        # coarse solver
        self.coarse = CoarseSolver(self.levels[0])

    def vcycle(self, b, l=None):
        """V_l(b) of the monolithic multigrid."""
        l = self.L if l is None else l
        lev = self.levels[l]
        if l == 0:
            return self.coarse.solve(b)
        s = self.cfg.cheb_degree
        lo, hi = self.cfg.cheb_lo, self.cfg.cheb_hi
        x = chebyshev_block(lev, self.lam[l], b, s, lo, hi)
        r = b - lev.A @ x
        xc = self.vcycle(self.P[l].T @ r, l - 1)
        x = x + self.P[l] @ xc
        r = b - lev.A @ x
        x = x + chebyshev_block(lev, self.lam[l], r, s, lo, hi)
        return x


def lanczos_ritz_max(alphas, betas):
    """Largest eigenvalue of the CG-Lanczos tridiagonal:
    T_jj = 1/a_j + b_{j-1}/a_{j-1},  T_{j,j+1} = sqrt(b_j)/a_j."""
    n = len(alphas)
    if n == 0:
        return 1.0
    diag = np.array([1.0 / alphas[j] + (betas[j - 1] / alphas[j - 1] if j > 0 else 0.0) for j in range(n)])
    off = np.array([np.sqrt(betas[j]) / alphas[j] for j in range(n - 1)])
    if n == 1:
        return float(diag[0])
    return float(sla.eigh_tridiagonal(diag, off, eigvals_only=True)[-1])


def cg_lanczos(A, Dvec, v, steps):
    """Jacobi-preconditioned CG on A from r0 = v; returns (alphas, betas).
    Stops early on r^T z == 0 or p^T A p <= 0."""
    r = v.copy()
    z = r / Dvec
    p = z.copy()
    rz = float(r @ z)
    alphas, betas = [], []
    for _ in range(steps):
        if rz == 0.0:
            break
        Ap = A @ p
        pAp = float(p @ Ap)
        if not pAp > 0.0:
            break
        a = rz / pAp
        alphas.append(a)
        r = r - a * Ap
        z = r / Dvec
        rz_new = float(r @ z)
        b = rz_new / rz
        betas.append(b)
        rz = rz_new
        p = z + b * p
    return alphas, betas


def start_vector(lev: Level, level_index: int, block: int, seed: int):
    nu, n = lev.nu, lev.mesh.n_dofs
    if block == 0:
        v = uniform_pm1(seed, 2 * level_index, nu) * lev.pvec[:nu]
    else:
        v = uniform_pm1(seed, 2 * level_index + 1, n - nu) * lev.pvec[nu:]
    return v


def lanczos_block_estimates(lev: Level, level_index: int, steps: int, seed: int):
    """(lambda_u, lambda_phi): Ritz estimates of lambda_max(D^-1 A_bb) per block."""
    nu = lev.nu
    out = []
    for b, sl in ((0, slice(0, nu)), (1, slice(nu, None))):
        Ab = lev.A[sl, sl]
        v = start_vector(lev, level_index, b, seed)
        al, be = cg_lanczos(Ab, lev.D[sl], v, steps)
        out.append(lanczos_ritz_max(al, be))
    return tuple(out)


def chebyshev_block(lev: Level, lam, r, s, lo_f, hi_f):
    """x = diag(C_u, C_phi) r: degree-s Chebyshev-Jacobi polynomial per block, x0 = 0."""
    nu = lev.nu
    theta = np.empty_like(r)
    delta = np.empty_like(r)
    for sl, lm in ((slice(0, nu), lam[0]), (slice(nu, None), lam[1])):
        lo, hi = lo_f * lm, hi_f * lm
        theta[sl] = 0.5 * (hi + lo)
        delta[sl] = 0.5 * (hi - lo)
    sigma = theta / delta
    rho = 1.0 / sigma
    d = r / lev.D / theta
    x = d.copy()
    for _ in range(1, s):
        res = r - lev.Ablk @ x
        rho_new = 1.0 / (2.0 * sigma - rho)
        d = rho_new * rho * d + (2.0 * rho_new / delta) * (res / lev.D)
        x = x + d
        rho = rho_new
    return x


class CoarseSolver:
    """Exact solve of the block lower-triangular coarse system (Section 3.3):
    x_u = G_uu^-1 r_u, x_phi = G_phiphi^-1 (r_phi - G_phiu x_u)."""

    def __init__(self, lev: Level):
        A = lev.A.toarray()
        nu = lev.nu
        self.nu = nu
        self.Auu = A[:nu, :nu]
        self.App = A[nu:, nu:]
        self.Apu = A[nu:, :nu]
        self.fu = self._factor(self.Auu)
        self.fp = self._factor(self.App)

    @staticmethod
    def _factor(B):
        """Cholesky where the block is positive definite (always, for kappa >= 0 and a regular
        state); otherwise LU with partial pivoting.  A zero pivot in the LU means a singular
        block, which has no solve: it is reported, not returned as inf/NaN."""
        try:
            return ("chol", sla.cho_factor(B, lower=True))
        except np.linalg.LinAlgError:
            pass
        with np.errstate(all="ignore"), warnings.catch_warnings():
            warnings.simplefilter("ignore")
            lu, piv = sla.lu_factor(B)
        if np.any(np.diag(lu) == 0.0):
            raise np.linalg.LinAlgError("coarse block is singular: zero pivot in the LU factorisation")
        return ("lu", (lu, piv))

    @staticmethod
    def _solve(f, r):
        kind, fac = f
        return sla.cho_solve(fac, r) if kind == "chol" else sla.lu_solve(fac, r)

    def solve(self, r):
        nu = self.nu
        xu = self._solve(self.fu, r[:nu])
        xp = self._solve(self.fp, r[nu:] - self.Apu @ xu)
        return np.concatenate([xu, xp])
