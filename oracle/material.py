"""Degradation function and tension/compression split (oracle; test infrastructure only).

Section 2.1: g(phi) = (1 - kappa) phi^2 + kappa; solid energy
E_s(e) = lambda/2 tr(e)^2 + mu e:e with e = sym(grad u); the split
E_s = E_s^+ + E_s^- with sigma^+ = dE_s^+/de.

The paper defines the spectral (Miehe) split; the workloads use the
volumetric/deviatoric (Amor) split, which the paper cites but does not
write out.  Reading used here, with K = lambda + 2 mu / d the bulk
modulus in d dimensions and dev e = e - tr(e)/d I:
    E^+ = K/2 <tr e>_+^2 + mu dev e : dev e,   E^- = K/2 <tr e>_-^2
    sigma^+ = K <tr e>_+ I + 2 mu dev e,       sigma^- = K <tr e>_- I
so that E^+ + E^- = E_s.  The tangent uses the one-sided Heaviside
H = [tr e >= 0] (H(0) = 1).
"""
import numpy as np


def g(phi, kappa):
    return (1.0 - kappa) * phi ** 2 + kappa


def dg(phi, kappa):
    return 2.0 * (1.0 - kappa) * phi


def ddg(phi, kappa):
    return 2.0 * (1.0 - kappa) * np.ones_like(phi)


def sym(A):
    return 0.5 * (A + np.swapaxes(A, -1, -2))


def trace(A):
    return np.trace(A, axis1=-2, axis2=-1)


def eye_like(A):
    d = A.shape[-1]
    return np.broadcast_to(np.eye(d), A.shape)


def amor_split(grad_u, lam, mu):
    """Return dict with e, t, H, sig_p, sig_m, E_p, E_m for strains at quadrature points."""
    d = grad_u.shape[-1]
    e = sym(grad_u)
    t = trace(e)
    K = lam + 2.0 * mu / d
    I = eye_like(e)
    dev = e - (t / d)[..., None, None] * I
    tp = np.maximum(t, 0.0)
    tm = np.minimum(t, 0.0)
    sig_p = K * tp[..., None, None] * I + 2.0 * mu * dev
    sig_m = K * tm[..., None, None] * I
    E_p = 0.5 * K * tp ** 2 + mu * np.einsum("...ij,...ij->...", dev, dev)
    E_m = 0.5 * K * tm ** 2
    H = (t >= 0.0).astype(float)
    return dict(e=e, t=t, H=H, K=K, sig_p=sig_p, sig_m=sig_m, E_p=E_p, E_m=E_m)


def dsigma(de, H, gt, K, mu):
    """Directional derivative of g(phi~) sigma^+ + sigma^- in strain direction de.

    de: (..., d, d) strain directions; H, gt: broadcastable per-point
    Heaviside and g(phi~).  Follows the definitions above term by term:
    g(phi~) [K H tr(de) I + 2 mu dev(de)] + K (1 - H) tr(de) I.
    """
    d = de.shape[-1]
    tde = trace(de)
    I = eye_like(de)
    dev = de - (tde / d)[..., None, None] * I
    return (gt[..., None, None] * (K * (H * tde)[..., None, None] * I + 2.0 * mu * dev)
            + K * ((1.0 - H) * tde)[..., None, None] * I)
