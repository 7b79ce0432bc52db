"""Workload descriptions (data only).

Material values are the table of Section 5.1 ("Material parameters and
configuration"), restated in N/mm units (lambda, mu and G_c scaled by
1e3; ratios unchanged).  kappa is the same table's regularisation.  The
Chebyshev interval factors 0.24 and 1.2 are the ones Section 3.3 states.
The coarse grid and sweep count follow Section 6.2; the level counts per
workload are the readings listed beside each entry.
"""
from dataclasses import dataclass, field, replace


@dataclass(frozen=True)
class Config:
    name: str
    dim: int
    N: int                 # cells per direction on the finest level
    k: int                 # polynomial degree Q_k on the finest level
    n_h_levels: int        # number of levels at degree k (N, N/2, ...)
    p_coarse: tuple = ()   # degrees of extra p-levels on the coarsest mesh, finest first, e.g. (2, 1)
    lam: float = 121.15e3
    mu: float = 80.77e3
    Gc: float = 2.7
    kappa: float = 1e-10
    eps_factor: float = 2.0   # eps = eps_factor * h with h = 1/N (edge length)
    as_c: float = 1.0         # constant c of the active-set rule
    cheb_degree: int = 5
    cheb_lo: float = 0.24
    cheb_hi: float = 1.2
    lanczos_steps: int = 15
    restart: int = 30
    max_iter: int = 300
    rtol: float = 1e-8
    vcycle_prec: str = "f64"
    active_p: float = 0.05
    phi_mode: str = "smooth"  # "ones" (1 off the notch) or "smooth"
    u_mode: str = "smooth"    # "iid" (U[0,1e-3] per node) or "smooth"
    dirichlet: bool = True    # delta u = 0 on the two faces normal to the last axis
    split: str = "amor"       # tension/compression split: "amor" (workloads), "miehe" (spectral), "none" (isotropic)
    pdas_project: bool = False  # Algorithm 1 as written (delta phi = 0 on A) or phi := phi_old on A first
    slit: bool = False          # geometry of Section 5.1: a slit from x = 0 to 1/2 on the mid-plane of the
                                # last axis, its nodes duplicated (on every level); no phi = 0 notch band then
    contraction: str = "valu"   # 3D products at degree 3/4: 1D contractions on the vector unit or the matrix cores ("mfma")
    seed_index: int = 0
    lanczos_seed: int = 20050331

    @property
    def h(self) -> float:
        return 1.0 / self.N

    @property
    def eps(self) -> float:
        return self.eps_factor / self.N

    @property
    def M(self) -> int:
        return self.k * self.N + 1

    @property
    def n_nodes(self) -> int:
        # the slit's duplicated nodes: k N / 2 per line along the first axis, M lines in 3D
        dup = (self.k * self.N // 2) * self.M ** (self.dim - 2) if self.slit else 0
        return self.M ** self.dim + dup

    @property
    def n_dofs(self) -> int:
        return (self.dim + 1) * self.n_nodes

    def with_(self, **kw) -> "Config":
        return replace(self, **kw)


def level_list(cfg: Config):
    """Levels from coarsest (index 0) to finest as (N, k) pairs."""
    lv = []
    N = cfg.N
    for _ in range(cfg.n_h_levels):
        lv.append((N, cfg.k))
        N //= 2
    lv.reverse()
    for deg in cfg.p_coarse:
        lv.insert(0, (lv[0][0], deg))
    return lv


CONFIGS = {
    # 2D 32x32 Q1, two-level GMG, phi = 1 off the notch, ~10% active
    "C1": Config("C1", 2, 32, 1, 2, active_p=0.10, phi_mode="ones", u_mode="iid", seed_index=1),
    # 2D 256x256 Q2, five-level GMG, full Newton step
    "C2": Config("C2", 2, 256, 2, 5, active_p=0.05, seed_index=2),
    # 3D 64^3 Q2, FP32 V-cycle with Chebyshev degree 4 inside FP64 GMRES; the workload names only
    # the notch plane, so phi = 1 off the notch (as in C1)
    "C3": Config("C3", 3, 64, 2, 5, cheb_degree=4, vcycle_prec="f32", active_p=0.05, phi_mode="ones", seed_index=3),
    # 3D 32^3 Q4, four h-levels plus p-coarsening to Q1 on 4^3 (taken as Q4 -> Q2 -> Q1)
    "C4": Config("C4", 3, 32, 4, 4, p_coarse=(2, 1), active_p=0.05, seed_index=4),
    # 3D 48^3 Q2, residual and its hand-written backward (no constraints)
    "C5": Config("C5", 3, 48, 2, 1, active_p=0.0, dirichlet=False, seed_index=5),
}


def config_by_name(name: str) -> Config:
    return CONFIGS[name]
