"""Seeded synthetic fields (data only, no method arithmetic).

They stand in for the states of the single-edge-notched tests of
Section 5, which are not available: a random displacement, a phase field
with a one-cell notch band (phi = 0) and a smooth random field elsewhere,
a random active set, a random right-hand side, a random cotangent and
random directions.  Node numbering is lexicographic,
node = i0 + M*i1 (+ M*M*i2), with M = k*N + 1 and node coordinate
i/(k*N) along each axis.  Vectors are component-blocked:
[u_0 | ... | u_{d-1} | phi], each block of M**d entries.
"""
import numpy as np

_STREAMS = ("u", "phi", "active", "rhs", "cotangent", "directions")


def _rng(cfg, stream: str):
    ss = np.random.SeedSequence(200500331 + cfg.seed_index).spawn(len(_STREAMS))
    return np.random.default_rng(ss[_STREAMS.index(stream)])


def node_coords(dim: int, N: int, k: int) -> np.ndarray:
    """(n_nodes, dim) coordinates of the lexicographically numbered nodes."""
    M = k * N + 1
    idx = np.arange(M ** dim)
    out = np.empty((M ** dim, dim))
    for a in range(dim):
        out[:, a] = (idx // (M ** a)) % M / (k * N)
    return out


def slit_duplicates(dim: int, N: int, k: int) -> np.ndarray:
    """Grid node of each duplicated slit node, in the order the duplicates are numbered after the
    M**dim grid nodes: the slit-plane nodes (last-axis index k*N/2) with first index below k*N/2,
    first axis fastest (3D: then the second axis)."""
    M = k * N + 1
    i0 = np.arange(k * N // 2)
    if dim == 2:
        return i0 + M * (k * N // 2)
    i1 = np.arange(M)
    return (i0[None, :] + M * i1[:, None] + M * M * (k * N // 2)).ravel()


def _coords(cfg):
    X = node_coords(cfg.dim, cfg.N, cfg.k)
    if getattr(cfg, "slit", False):
        X = np.concatenate([X, X[slit_duplicates(cfg.dim, cfg.N, cfg.k)]])
    return X


def notch_mask(cfg) -> np.ndarray:
    """Nodes of the one-cell band on the mid-plane of the last axis, first half of axis 0 (none
    on a slit mesh, where the slit itself is the notch)."""
    X = _coords(cfg)
    if getattr(cfg, "slit", False):
        return np.zeros(X.shape[0], dtype=bool)
    h = cfg.h
    y = X[:, cfg.dim - 1]
    return (np.abs(y - 0.5) <= h / 2 + 1e-12) & (X[:, 0] < 0.5 - 1e-12)


def make_u(cfg) -> np.ndarray:
    """Displacement state.  "iid": U[0, 1e-3] per node and component;
    "smooth": per component 1e-3 * (1/2 + 1/2 sum_m a_m cos(2 pi k_m.x + t_m) / sum|a_m|),
    eight modes with k_m in {0..3}^d, so tension and compression occupy regions."""
    g = _rng(cfg, "u")
    if cfg.u_mode == "iid":
        return g.uniform(0.0, 1e-3, size=(cfg.dim, cfg.n_nodes))
    X = _coords(cfg)
    u = np.empty((cfg.dim, cfg.n_nodes))
    for c in range(cfg.dim):
        nm = 8
        a = g.uniform(-1.0, 1.0, size=nm)
        kv = g.integers(0, 4, size=(nm, cfg.dim))
        th = g.uniform(0.0, 2 * np.pi, size=nm)
        s = np.zeros(cfg.n_nodes)
        for m in range(nm):
            s += a[m] * np.cos(2 * np.pi * (X @ kv[m]) + th[m])
        u[c] = 1e-3 * (0.5 + 0.5 * s / np.abs(a).sum())
    return u


def make_phi(cfg) -> np.ndarray:
    if cfg.phi_mode == "ones":
        phi = np.ones(cfg.n_nodes)
    else:
        g = _rng(cfg, "phi")
        nm = 8
        a = g.uniform(-1.0, 1.0, size=nm)
        kv = g.integers(0, 4, size=(nm, cfg.dim))
        th = g.uniform(0.0, 2 * np.pi, size=nm)
        X = _coords(cfg)
        s = np.zeros(cfg.n_nodes)
        for m in range(nm):
            s += a[m] * np.cos(2 * np.pi * (X @ kv[m]) + th[m])
        phi = 0.5 + 0.5 * s / np.abs(a).sum()
        phi = np.clip(phi, 0.0, 1.0)
    phi[notch_mask(cfg)] = 0.0
    return phi


def make_active(cfg) -> np.ndarray:
    xi = _rng(cfg, "active").random(cfg.n_nodes)
    return (xi < cfg.active_p).astype(np.uint8)


def make_rhs(cfg) -> np.ndarray:
    return _rng(cfg, "rhs").uniform(-1.0, 1.0, size=cfg.n_dofs)


def make_cotangent(cfg) -> np.ndarray:
    return _rng(cfg, "cotangent").standard_normal(cfg.n_dofs)


def make_directions(cfg, n: int = 32) -> np.ndarray:
    g = _rng(cfg, "directions")
    d = g.standard_normal((n, cfg.n_dofs))
    d[:, : cfg.dim * cfg.n_nodes] *= 1e-3
    return d


def make_inputs(cfg, extra=()) -> dict:
    """Core inputs of a workload; ``extra`` may name 'rhs', 'cotangent', 'directions'."""
    phi = make_phi(cfg)
    out = {
        "u": make_u(cfg),
        "phi": phi,
        "phi_old": phi.copy(),
        "phi_tilde": phi.copy(),
        "active": make_active(cfg),
    }
    if "rhs" in extra:
        out["rhs"] = make_rhs(cfg)
    if "cotangent" in extra:
        out["cotangent"] = make_cotangent(cfg)
    if "directions" in extra:
        out["directions"] = make_directions(cfg)
    return out
