"""Active-set rule and one semi-smooth Newton step (oracle; test infrastructure only).

Algorithm 1 (primal-dual active set).  Readings:
  * the update U_{k+1} = U_k + G^-1 R_k and the active-set test
    (M^-1 R)_i + c (U - U_old)_i > 0 are consistent when R_k is minus
    the residual of eq. (residual); with R the residual as written there,
    the Newton step solves G^ dU = -P R and the active set is
        A = { phi-dofs i : -(M_L^-1 R)_i + c (phi - phi_old)_i > 0 },
    i.e. the multiplier -R_i wants phi to grow above phi_old;
  * M is the row-sum-lumped phi mass matrix, c = 1;
  * the Newton step keeps phi on A_k (delta phi = 0 there, as the algorithm is written) unless
    cfg.pdas_project is set: then phi := phi_old on A_k first, the residual is evaluated again at
    that point and the step is taken from there (the primal-dual active-set update of
    Hintermueller, Ito and Kunisch, which puts the iterate on the obstacle on the active set).
"""
import numpy as np

from . import operator as op
from .fe import Mesh
from .krylov import fgmres
from .multigrid import Hierarchy


def active_set(mesh: Mesh, R, phi, phi_old, c=1.0):
    ML = op.lumped_phi_mass(mesh)
    Rp = R[mesh.dim * mesh.n_nodes:]
    ind = -Rp / ML + c * (phi - phi_old)
    return (ind > 0.0).astype(np.uint8), ind


def newton_step(cfg, levels_nk, u, phi, phi_old, phi_t):
    """One step: residual, active set, linearisation, FGMRES + GMG, update."""
    mesh = Mesh(cfg.dim, cfg.N, cfg.k, getattr(cfg, "slit", False))
    m = op.material_of(cfg)
    R = op.residual(mesh, m, u, phi, phi_t)
    act, ind = active_set(mesh, R, phi, phi_old, cfg.as_c)
    R_at_start = R
    if getattr(cfg, "pdas_project", False):
        phi = np.where(act != 0, phi_old, phi)
        R = op.residual(mesh, m, u, phi, phi_t)
    hier = Hierarchy(cfg, levels_nk, u, phi, phi_t, act)
    fine = hier.levels[-1]
    b = -fine.pvec * R
    dU, info = fgmres(lambda v: fine.A @ v, hier.vcycle, b, cfg.restart, cfg.rtol, cfg.max_iter)
    d, nn = cfg.dim, mesh.n_nodes
    u_new = u + dU[: d * nn].reshape(d, nn)
    phi_new = phi + dU[d * nn:]
    return dict(R=R_at_start, active=act, indicator=ind, b=b, dU=dU, u=u_new, phi=phi_new, info=info, hier=hier)


def pdas_solve(cfg, levels_nk, u, phi, phi_old, phi_t, max_newton=20, tol=1e-8):
    """Algorithm 1 to its stopping test: repeat (active set from the residual at U_k, Newton step
    on the inactive set) until the active set equals the previous one and the residual on the
    free dofs, ||P_k R_k||, is at most tol ||P_0 R_0|| (reading: the paper's eps_as taken relative
    to the first iterate).  Returns the final state, the number of Newton steps taken, the norms
    and the FGMRES iteration counts."""
    mesh = Mesh(cfg.dim, cfg.N, cfg.k, getattr(cfg, "slit", False))
    m = op.material_of(cfg)
    prev = None
    norms, iters = [], []
    converged = False
    r0 = None
    for k in range(max_newton + 1):
        R = op.residual(mesh, m, u, phi, phi_t)
        act, _ = active_set(mesh, R, phi, phi_old, cfg.as_c)
        pvec = op.free_vector(mesh, act, cfg.dirichlet)
        rn = float(np.linalg.norm(pvec * R))
        r0 = rn if r0 is None else r0
        norms.append(rn)
        if prev is not None and np.array_equal(act, prev) and rn <= tol * r0:
            converged = True
            break
        if k == max_newton:
            break
        out = newton_step(cfg, levels_nk, u, phi, phi_old, phi_t)
        u, phi = out["u"], out["phi"]
        iters.append(out["info"]["iterations"])
        prev = act
    return dict(u=u, phi=phi, active=act, steps=len(iters), converged=converged, norms=norms, gmres_iterations=iters)
