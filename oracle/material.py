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

The spectral (Miehe) split of Section 2.1, with (lambda_i, v_i) the
eigensystem of e, e^+ = sum_i <lambda_i>_+ v_i v_i^T and e^- = e - e^+:
    E^+ = lambda/2 <tr e>_+^2 + mu tr(e^+ e^+),  E^- = lambda/2 <tr e>_-^2 + mu tr(e^- e^-)
    sigma^+ = lambda <tr e>_+ I + 2 mu e^+,      sigma^- = lambda <tr e>_- I + 2 mu e^-
and, Section 3.5, d sigma^+(de) = lambda H tr(de) I + 2 mu d e^+(de).  The
derivative of the positive part is taken in the eigenbasis with divided
differences (Daleckii-Krein): [V^T de^+ V]_ij = F_ij [V^T de V]_ij with
F_ij = (<lambda_i>_+ - <lambda_j>_+) / (lambda_i - lambda_j), and
F_ij = [lambda_i >= 0] where lambda_i = lambda_j.  On distinct eigenvalues
this is the result of Algorithm 2; on repeated ones it does not depend on
the eigenvectors chosen, which Algorithm 2 with D^dagger = 0 does.
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


def isotropic_split(grad_u, lam, mu):
    """The model without a split (the isotropic case of Section 5): the whole solid energy and Hooke's
    stress are degraded, E^+ = E_s = lambda/2 tr(e)^2 + mu e:e, sigma^+ = lambda tr(e) I + 2 mu e,
    E^- = 0, sigma^- = 0.  Same keys as amor_split, with H = 1 everywhere, so that dsigma gives
    g(phi~) (lambda tr(de) I + 2 mu de)."""
    d = grad_u.shape[-1]
    e = sym(grad_u)
    t = trace(e)
    I = eye_like(e)
    sig_p = lam * t[..., None, None] * I + 2.0 * mu * e
    E_p = 0.5 * lam * t ** 2 + mu * np.einsum("...ij,...ij->...", e, e)
    return dict(e=e, t=t, H=np.ones_like(t), K=lam + 2.0 * mu / d, sig_p=sig_p, sig_m=np.zeros_like(sig_p),
                E_p=E_p, E_m=np.zeros_like(E_p))


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


def miehe_split(grad_u, lam, mu):
    """Spectral split: dict with e, t, H, sig_p, sig_m, E_p, E_m and the
    eigensystem (ev: eigenvalues, V: eigenvectors as columns)."""
    e = sym(grad_u)
    t = trace(e)
    ev, V = np.linalg.eigh(e)
    evp = np.maximum(ev, 0.0)
    ep = np.einsum("...ik,...k,...jk->...ij", V, evp, V)
    em = e - ep
    tp = np.maximum(t, 0.0)
    tm = np.minimum(t, 0.0)
    I = eye_like(e)
    sig_p = lam * tp[..., None, None] * I + 2.0 * mu * ep
    sig_m = lam * tm[..., None, None] * I + 2.0 * mu * em
    E_p = 0.5 * lam * tp ** 2 + mu * np.einsum("...ij,...ij->...", ep, ep)
    E_m = 0.5 * lam * tm ** 2 + mu * np.einsum("...ij,...ij->...", em, em)
    H = (t >= 0.0).astype(float)
    return dict(e=e, t=t, H=H, sig_p=sig_p, sig_m=sig_m, E_p=E_p, E_m=E_m, ev=ev, V=V)


def divided_differences(ev):
    """F_ij of the positive part (..., d, d) for eigenvalues ev (..., d)."""
    li = ev[..., :, None]
    lj = ev[..., None, :]
    num = np.maximum(li, 0.0) - np.maximum(lj, 0.0)
    den = li - lj
    same = den == 0.0
    return np.where(same, (li >= 0.0).astype(float) * np.ones_like(den), num / np.where(same, 1.0, den))


def dpositive_part(ev, V, de):
    """d e^+ (de) at e = V diag(ev) V^T.  ev, V broadcast against de (..., d, d)."""
    F = divided_differences(ev)
    Vt_de_V = np.einsum("...ki,...kl,...lj->...ij", V, de, V)
    return np.einsum("...ik,...kl,...jl->...ij", V, F * Vt_de_V, V)


def dsigma_miehe(de, s, gt, lam, mu):
    """Directional derivative of g(phi~) sigma^+ + sigma^- (spectral split) in
    strain direction de; s from miehe_split with its point axes broadcast
    against de, gt the per-point g(phi~)."""
    tde = trace(de)
    I = eye_like(de)
    H = s["H"]
    dep = dpositive_part(s["ev"], s["V"], de)
    dsp = lam * (H * tde)[..., None, None] * I + 2.0 * mu * dep
    dsm = lam * ((1.0 - H) * tde)[..., None, None] * I + 2.0 * mu * (de - dep)
    return gt[..., None, None] * dsp + dsm
