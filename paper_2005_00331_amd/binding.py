"""ctypes binding of libmfpff (include/mfpff.h), argument marshalling only.

Every function here has the name of the C entry point it calls and checks
dtype, device, contiguity and length of its tensor arguments before the
call.  All arithmetic runs in the library's HIP kernels; when the library
or a GPU is missing the binding raises, it never falls back to anything.
"""
import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
# MFPFF_LIB selects another build of the library (the bounds-checking debug build in its test)
LIB_PATH = os.environ.get("MFPFF_LIB", os.path.join(_HERE, "libmfpff.so"))
MAX_LEVELS = 16

F64, F32 = 0, 1
OP_G, OP_GT, OP_BLOCKDIAG = 0, 1, 2
SPLITS = {"amor": 0, "miehe": 1, "none": 2}   # mfpff_split
CONTRACTIONS = {"valu": 0, "mfma": 1}          # mfpff_contraction
OP_ACCUMULATE = 16

STATUS = {0: "OK", 1: "ERR_ARG", 2: "ERR_STATE", 3: "ERR_OOM", 4: "ERR_HIP", 5: "ERR_NOCONV", 6: "ERR_NUMERIC"}


class MfpffError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"mfpff {STATUS.get(status, status)}: {msg}")
        self.status = status


class Problem(ctypes.Structure):
    _fields_ = [
        ("dim", ctypes.c_int),
        ("n_levels", ctypes.c_int),
        ("level_N", ctypes.c_int * MAX_LEVELS),
        ("level_k", ctypes.c_int * MAX_LEVELS),
        ("dirichlet", ctypes.c_int),
        ("lambda_", ctypes.c_double),
        ("mu", ctypes.c_double),
        ("Gc", ctypes.c_double),
        ("eps", ctypes.c_double),
        ("kappa", ctypes.c_double),
        ("as_c", ctypes.c_double),
        ("cheb_degree", ctypes.c_int),
        ("cheb_lo", ctypes.c_double),
        ("cheb_hi", ctypes.c_double),
        ("lanczos_steps", ctypes.c_int),
        ("lanczos_seed", ctypes.c_ulonglong),
        ("vcycle_prec", ctypes.c_int),
        ("restart", ctypes.c_int),
        ("max_iter", ctypes.c_int),
        ("rtol", ctypes.c_double),
        ("split", ctypes.c_int),
        ("pdas_project", ctypes.c_int),
        ("contraction", ctypes.c_int),
        ("slit", ctypes.c_int),
    ]


class SolveInfo(ctypes.Structure):
    _fields_ = [
        ("iterations", ctypes.c_int),
        ("converged", ctypes.c_int),
        ("rel_residual", ctypes.c_double),
        ("ms_setup", ctypes.c_double),
        ("ms_solve", ctypes.c_double),
        ("n_active", ctypes.c_int),
    ]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class PdasInfo(ctypes.Structure):
    _fields_ = [
        ("newton_steps", ctypes.c_int),
        ("converged", ctypes.c_int),
        ("gmres_iterations", ctypes.c_int),
        ("n_active", ctypes.c_int),
        ("rel_residual", ctypes.c_double),
        ("ms_total", ctypes.c_double),
    ]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class LoadInfo(ctypes.Structure):
    _fields_ = [
        ("pdas", PdasInfo),
        ("reaction_top", ctypes.c_double * 3),
        ("reaction_bottom", ctypes.c_double * 3),
    ]

    def as_dict(self, dim):
        out = self.pdas.as_dict()
        out["reaction_top"] = [self.reaction_top[a] for a in range(dim)]
        out["reaction_bottom"] = [self.reaction_bottom[a] for a in range(dim)]
        return out


class LevelDesc(ctypes.Structure):
    _fields_ = [
        ("N", ctypes.c_int),
        ("k", ctypes.c_int),
        ("n_nodes", ctypes.c_longlong),
        ("n_dofs", ctypes.c_longlong),
        ("lambda_u", ctypes.c_double),
        ("lambda_phi", ctypes.c_double),
        ("lanczos_steps_u", ctypes.c_int),
        ("lanczos_steps_phi", ctypes.c_int),
    ]


EXPORTS = [
    "mfpff_setup_mesh_levels", "mfpff_destroy", "mfpff_last_error", "mfpff_level_info", "mfpff_set_linearization",
    "mfpff_set_point",
    "mfpff_apply_jacobian", "mfpff_diagonal", "mfpff_smooth", "mfpff_transfer", "mfpff_coarse_solve",
    "mfpff_vcycle", "mfpff_gmres_solve", "mfpff_residual", "mfpff_residual_param_vjp", "mfpff_active_set",
    "mfpff_residual_param_vjp_noalloc",
    "mfpff_newton_step", "mfpff_pdas_solve", "mfpff_element_matrices", "mfpff_load_step", "mfpff_sizes",
    "mfpff_debug_bounds_hits",
]

_lib = None


def load_library(path=LIB_PATH):
    """Load libmfpff.so (after torch, so that both share one HIP runtime)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"libmfpff.so is not built ({path}); run paper_2005_00331_amd/build.py")
    lib = ctypes.CDLL(path)
    P, I, D, VP = ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_void_p
    sig = {
        "mfpff_setup_mesh_levels": ([ctypes.POINTER(Problem), VP, ctypes.POINTER(VP)], I),
        "mfpff_destroy": ([VP], None),
        "mfpff_last_error": ([VP], ctypes.c_char_p),
        "mfpff_level_info": ([VP, I, ctypes.POINTER(LevelDesc)], I),
        "mfpff_set_linearization": ([VP, P, P, P, P, P], I),
        "mfpff_set_point": ([VP, P, P, P, P, P], I),
        "mfpff_apply_jacobian": ([VP, I, P, P, I, I], I),
        "mfpff_diagonal": ([VP, I, P], I),
        "mfpff_smooth": ([VP, I, P, P], I),
        "mfpff_transfer": ([VP, I, I, P, P], I),
        "mfpff_coarse_solve": ([VP, P, P], I),
        "mfpff_vcycle": ([VP, P, P], I),
        "mfpff_gmres_solve": ([VP, P, P, ctypes.POINTER(SolveInfo)], I),
        "mfpff_residual": ([VP, P, P, P, P], I),
        "mfpff_residual_param_vjp": ([VP, P, P, P, P, ctypes.POINTER(D), ctypes.POINTER(D)], I),
        "mfpff_residual_param_vjp_noalloc": ([VP, P, P, P, P, ctypes.POINTER(D), ctypes.POINTER(D)], I),
        "mfpff_active_set": ([VP, P, P, P, P], I),
        "mfpff_newton_step": ([VP, P, P, P, P, P, ctypes.POINTER(SolveInfo)], I),
        "mfpff_pdas_solve": ([VP, P, P, P, P, P, I, D, ctypes.POINTER(PdasInfo)], I),
        "mfpff_element_matrices": ([VP, I, P], I),
        "mfpff_load_step": ([VP, P, P, P, P, ctypes.POINTER(D), P, I, D, ctypes.POINTER(LoadInfo)], I),
        "mfpff_sizes": ([VP, I, ctypes.POINTER(ctypes.c_size_t), ctypes.POINTER(ctypes.c_size_t)], I),
        "mfpff_debug_bounds_hits": ([], ctypes.c_longlong),
    }
    for name, (args, res) in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = res
    _lib = lib
    return lib


def make_problem(dim, levels, *, dirichlet=True, lam=121.15e3, mu=80.77e3, Gc=2.7, eps, kappa=1e-10, as_c=1.0,
                 cheb_degree=5, cheb_lo=0.24, cheb_hi=1.2, lanczos_steps=15, lanczos_seed=20050331,
                 vcycle_prec=F64, restart=30, max_iter=300, rtol=1e-8, split="amor", pdas_project=False,
                 contraction="valu", slit=False):
    """levels: list of (N, k) from the coarsest to the finest."""
    p = Problem()
    p.dim = dim
    p.n_levels = len(levels)
    for i, (N, k) in enumerate(levels):
        p.level_N[i] = N
        p.level_k[i] = k
    p.dirichlet = int(bool(dirichlet))
    p.lambda_, p.mu, p.Gc, p.eps, p.kappa, p.as_c = lam, mu, Gc, eps, kappa, as_c
    p.cheb_degree, p.cheb_lo, p.cheb_hi = cheb_degree, cheb_lo, cheb_hi
    p.lanczos_steps, p.lanczos_seed = lanczos_steps, lanczos_seed
    p.vcycle_prec = vcycle_prec
    p.restart, p.max_iter, p.rtol = restart, max_iter, rtol
    if split not in SPLITS:
        raise ValueError(f"split must be one of {sorted(SPLITS)}")
    p.split = SPLITS[split]
    p.pdas_project = 1 if pdas_project else 0
    if contraction not in CONTRACTIONS:
        raise ValueError(f"contraction must be one of {sorted(CONTRACTIONS)}")
    p.contraction = CONTRACTIONS[contraction]
    p.slit = 1 if slit else 0
    return p


def _ptr(t, dtype, n, name, allow_none=False):
    if t is None:
        if allow_none:
            return None
        raise ValueError(f"{name} is required")
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch.Tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name}: dtype {t.dtype}, expected {dtype}")
    if t.device.type != "cuda":
        raise ValueError(f"{name} must be on a HIP device")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if t.numel() != n:
        raise ValueError(f"{name}: {t.numel()} entries, expected {n}")
    return ctypes.c_void_p(t.data_ptr())


class Context:
    """Owns one mfpff_ctx; methods carry the C names without the prefix."""

    def __init__(self, problem: Problem, stream=None):
        if not torch.cuda.is_available():
            raise RuntimeError("mfpff needs a HIP device; none is visible")
        self.lib = load_library()
        s = torch.cuda.current_stream() if stream is None else stream
        self.stream = s
        self.problem = problem
        h = ctypes.c_void_p()
        st = self.lib.mfpff_setup_mesh_levels(ctypes.byref(problem), ctypes.c_void_p(s.cuda_stream), ctypes.byref(h))
        if st != 0:
            raise MfpffError(st, "mfpff_setup_mesh_levels failed")
        self.h = h
        self.dim = problem.dim
        self.levels = [self.level_info(l) for l in range(problem.n_levels)]
        fine = self.levels[-1]
        self.n_nodes, self.n_dofs = fine.n_nodes, fine.n_dofs

    def close(self):
        if getattr(self, "h", None):
            self.lib.mfpff_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, st):
        if st != 0:
            raise MfpffError(st, self.lib.mfpff_last_error(self.h).decode())

    def _lvl(self, level):
        return self.levels[level if level >= 0 else len(self.levels) + level]

    # ---- entry points
    def sizes(self, level):
        """(n_nodes, n_dofs) of a level (0 = coarsest), from the host."""
        nn, nd = ctypes.c_size_t(), ctypes.c_size_t()
        level = level % len(self.levels)
        self._check(self.lib.mfpff_sizes(self.h, level, ctypes.byref(nn), ctypes.byref(nd)))
        return nn.value, nd.value

    def level_info(self, level):
        d = LevelDesc()
        self._check(self.lib.mfpff_level_info(self.h, level, ctypes.byref(d)))
        return d

    def set_linearization(self, u, phi, phi_old, active, phi_tilde=None):
        nn = self.n_nodes
        self._check(self.lib.mfpff_set_linearization(
            self.h, _ptr(u, torch.float64, self.dim * nn, "u"), _ptr(phi, torch.float64, nn, "phi"),
            _ptr(phi_old, torch.float64, nn, "phi_old"), _ptr(active, torch.uint8, nn, "active"),
            _ptr(phi_tilde, torch.float64, nn, "phi_tilde", allow_none=True)))
        self.levels = [self.level_info(l) for l in range(len(self.levels))]

    def set_point(self, u, phi, phi_old, active, phi_tilde=None):
        nn = self.n_nodes
        self._check(self.lib.mfpff_set_point(
            self.h, _ptr(u, torch.float64, self.dim * nn, "u"), _ptr(phi, torch.float64, nn, "phi"),
            _ptr(phi_old, torch.float64, nn, "phi_old"), _ptr(active, torch.uint8, nn, "active"),
            _ptr(phi_tilde, torch.float64, nn, "phi_tilde", allow_none=True)))

    def apply_jacobian(self, level, x, y=None, prec=F64, op=OP_G):
        lv = self._lvl(level)
        dt = torch.float64 if prec == F64 else torch.float32
        if y is None:
            y = torch.empty(lv.n_dofs, dtype=dt, device=x.device)
        self._check(self.lib.mfpff_apply_jacobian(self.h, level % len(self.levels), _ptr(x, dt, lv.n_dofs, "x"),
                                                  _ptr(y, dt, lv.n_dofs, "y"), prec, op))
        return y

    def diagonal(self, level):
        lv = self._lvl(level)
        out = torch.empty(lv.n_dofs, dtype=torch.float64, device="cuda")
        self._check(self.lib.mfpff_diagonal(self.h, level % len(self.levels), _ptr(out, torch.float64, lv.n_dofs, "diag")))
        return out

    def smooth(self, level, r):
        lv = self._lvl(level)
        z = torch.empty_like(r)
        self._check(self.lib.mfpff_smooth(self.h, level % len(self.levels), _ptr(r, torch.float64, lv.n_dofs, "r"),
                                          _ptr(z, torch.float64, lv.n_dofs, "z")))
        return z

    def transfer(self, level, direction, x):
        level = level % len(self.levels)
        fine, coarse = self.levels[level], self.levels[level - 1]
        nin, nout = (coarse.n_dofs, fine.n_dofs) if direction == 0 else (fine.n_dofs, coarse.n_dofs)
        out = torch.empty(nout, dtype=torch.float64, device=x.device)
        self._check(self.lib.mfpff_transfer(self.h, level, direction, _ptr(x, torch.float64, nin, "in"),
                                            _ptr(out, torch.float64, nout, "out")))
        return out

    def coarse_solve(self, r):
        n = self.levels[0].n_dofs
        x = torch.empty(n, dtype=torch.float64, device=r.device)
        self._check(self.lib.mfpff_coarse_solve(self.h, _ptr(r, torch.float64, n, "r"), _ptr(x, torch.float64, n, "x")))
        return x

    def vcycle(self, r):
        z = torch.empty_like(r)
        self._check(self.lib.mfpff_vcycle(self.h, _ptr(r, torch.float64, self.n_dofs, "r"),
                                          _ptr(z, torch.float64, self.n_dofs, "z")))
        return z

    def gmres_solve(self, b, x=None, raise_on_noconv=True):
        if x is None:
            x = torch.empty_like(b)
        info = SolveInfo()
        st = self.lib.mfpff_gmres_solve(self.h, _ptr(b, torch.float64, self.n_dofs, "b"),
                                        _ptr(x, torch.float64, self.n_dofs, "x"), ctypes.byref(info))
        if st != 5 or raise_on_noconv:
            self._check(st)
        return x, info.as_dict()

    def residual(self, u, phi, phi_tilde):
        nn = self.n_nodes
        R = torch.empty(self.n_dofs, dtype=torch.float64, device=u.device)
        self._check(self.lib.mfpff_residual(self.h, _ptr(u, torch.float64, self.dim * nn, "u"),
                                            _ptr(phi, torch.float64, nn, "phi"),
                                            _ptr(phi_tilde, torch.float64, nn, "phi_tilde"),
                                            _ptr(R, torch.float64, self.n_dofs, "R")))
        return R

    def residual_param_vjp(self, u, phi, phi_tilde, v):
        nn = self.n_nodes
        a, b = ctypes.c_double(), ctypes.c_double()
        self._check(self.lib.mfpff_residual_param_vjp(
            self.h, _ptr(u, torch.float64, self.dim * nn, "u"), _ptr(phi, torch.float64, nn, "phi"),
            _ptr(phi_tilde, torch.float64, nn, "phi_tilde"), _ptr(v, torch.float64, self.n_dofs, "v"),
            ctypes.byref(a), ctypes.byref(b)))
        return a.value, b.value

    def residual_param_vjp_noalloc(self, u, phi, phi_tilde, v):
        nn = self.n_nodes
        a, b = ctypes.c_double(), ctypes.c_double()
        self._check(self.lib.mfpff_residual_param_vjp_noalloc(
            self.h, _ptr(u, torch.float64, self.dim * nn, "u"), _ptr(phi, torch.float64, nn, "phi"),
            _ptr(phi_tilde, torch.float64, nn, "phi_tilde"), _ptr(v, torch.float64, self.n_dofs, "v"),
            ctypes.byref(a), ctypes.byref(b)))
        return a.value, b.value

    def active_set(self, R, phi, phi_old):
        nn = self.n_nodes
        act = torch.empty(nn, dtype=torch.uint8, device=R.device)
        self._check(self.lib.mfpff_active_set(self.h, _ptr(R, torch.float64, self.n_dofs, "R"),
                                              _ptr(phi, torch.float64, nn, "phi"),
                                              _ptr(phi_old, torch.float64, nn, "phi_old"),
                                              _ptr(act, torch.uint8, nn, "active")))
        return act

    def newton_step(self, u, phi, phi_old, phi_tilde=None, active=None, raise_on_noconv=True):
        nn = self.n_nodes
        if active is None:
            active = torch.empty(nn, dtype=torch.uint8, device=u.device)
        info = SolveInfo()
        st = self.lib.mfpff_newton_step(self.h, _ptr(u, torch.float64, self.dim * nn, "u"),
                                        _ptr(phi, torch.float64, nn, "phi"), _ptr(phi_old, torch.float64, nn, "phi_old"),
                                        _ptr(phi_tilde, torch.float64, nn, "phi_tilde", allow_none=True),
                                        _ptr(active, torch.uint8, nn, "active"), ctypes.byref(info))
        if st != 5 or raise_on_noconv:
            self._check(st)
        self.levels = [self.level_info(l) for l in range(len(self.levels))]
        return active, info.as_dict()

    def element_matrices(self, level=-1):
        """Unconstrained element matrices of a level, (n_cells, nl, nl) FP64 on the device."""
        lv = self._lvl(level)
        nl = (self.dim + 1) * (lv.k + 1) ** self.dim
        nc = lv.N ** self.dim
        em = torch.empty((nc, nl, nl), dtype=torch.float64, device="cuda")
        self._check(self.lib.mfpff_element_matrices(self.h, level % len(self.levels),
                                                    _ptr(em.view(-1), torch.float64, nc * nl * nl, "em")))
        return em

    def pdas_solve(self, u, phi, phi_old, phi_tilde=None, active=None, max_newton=20, tol=1e-8,
                   raise_on_noconv=True):
        """Algorithm 1 to its stopping test (u, phi updated in place); returns the final active
        set and the loop's counts."""
        nn = self.n_nodes
        if active is None:
            active = torch.empty(nn, dtype=torch.uint8, device=u.device)
        info = PdasInfo()
        st = self.lib.mfpff_pdas_solve(self.h, _ptr(u, torch.float64, self.dim * nn, "u"),
                                       _ptr(phi, torch.float64, nn, "phi"), _ptr(phi_old, torch.float64, nn, "phi_old"),
                                       _ptr(phi_tilde, torch.float64, nn, "phi_tilde", allow_none=True),
                                       _ptr(active, torch.uint8, nn, "active"), int(max_newton), float(tol),
                                       ctypes.byref(info))
        if st != 5 or raise_on_noconv:
            self._check(st)
        self.levels = [self.level_info(l) for l in range(len(self.levels))]
        return active, info.as_dict()

    def load_step(self, u, phi, phi_prev, phi_prev2, u_top, active=None, max_newton=20, tol=1e-8,
                  raise_on_noconv=True):
        """One load step: u := 0 on the bottom face and u_top on the top face, phi~ from the two
        previous phase fields (phi_prev2 None: phi~ = phi_prev), Algorithm 1 from (u, phi) with
        phi_old = phi_prev (u, phi updated in place); returns the final active set and the
        loop's counts with the face reactions."""
        nn = self.n_nodes
        if active is None:
            active = torch.empty(nn, dtype=torch.uint8, device=u.device)
        top = [float(v) for v in u_top]
        if len(top) != self.dim:
            raise ValueError(f"u_top needs {self.dim} values")
        top_c = (ctypes.c_double * 3)(*(top + [0.0] * (3 - self.dim)))
        info = LoadInfo()
        st = self.lib.mfpff_load_step(self.h, _ptr(u, torch.float64, self.dim * nn, "u"),
                                      _ptr(phi, torch.float64, nn, "phi"),
                                      _ptr(phi_prev, torch.float64, nn, "phi_prev"),
                                      _ptr(phi_prev2, torch.float64, nn, "phi_prev2", allow_none=True),
                                      top_c, _ptr(active, torch.uint8, nn, "active"), int(max_newton), float(tol),
                                      ctypes.byref(info))
        if st != 5 or raise_on_noconv:
            self._check(st)
        self.levels = [self.level_info(l) for l in range(len(self.levels))]
        return active, info.as_dict(self.dim)


def problem_from(cfg, levels, vcycle_prec=None, dirichlet=None, **overrides):
    """Problem from any object with the workload attributes (dim, lam, mu, Gc, eps,
    kappa, as_c, cheb_*, lanczos_*, restart, max_iter, rtol, vcycle_prec, dirichlet)."""
    vp = cfg.vcycle_prec if vcycle_prec is None else vcycle_prec
    if isinstance(vp, str):
        vp = F32 if vp == "f32" else F64
    kw = dict(dirichlet=cfg.dirichlet if dirichlet is None else dirichlet, lam=cfg.lam, mu=cfg.mu, Gc=cfg.Gc,
              eps=cfg.eps, kappa=cfg.kappa, as_c=cfg.as_c, cheb_degree=cfg.cheb_degree, cheb_lo=cfg.cheb_lo,
              cheb_hi=cfg.cheb_hi, lanczos_steps=cfg.lanczos_steps, lanczos_seed=cfg.lanczos_seed,
              vcycle_prec=vp, restart=cfg.restart, max_iter=cfg.max_iter, rtol=cfg.rtol,
              split=getattr(cfg, "split", "amor"), pdas_project=getattr(cfg, "pdas_project", False),
              contraction=getattr(cfg, "contraction", "valu"), slit=getattr(cfg, "slit", False))
    kw.update(overrides)
    return make_problem(cfg.dim, levels, **kw)
