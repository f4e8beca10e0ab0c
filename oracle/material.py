"""Hyperelastic closures (paper Appendix A) in plain FP64 on the unshifted F.

Test infrastructure only (see the package docstring).

Conventions: ``F`` has shape (2, 2, ...) with ``F[i, A]`` = F_iA (spatial row i, material
column A); extra trailing axes are grid axes and broadcast against ``mu`` and ``lam``.
The kinematic quantities follow eq:constitutive-kinematic-quantities:
C = F^T F, E = (C - I)/2, J = det F, H = F^{-T}.

The tangent C_iAkB = dP_iA/dF_kB is required by eq:stress-and-tangent but not printed in
the paper; the closed forms below are derived by differentiating each P and are pinned in
the tests by central differences of P (and P itself by central differences of W).
"""
import numpy as np

LAWS = ("lognh", "nh", "svk")


def det(F):
    return F[0, 0] * F[1, 1] - F[0, 1] * F[1, 0]


def inv_transpose(F):
    """H = F^{-T}."""
    J = det(F)
    return np.array([[F[1, 1], -F[1, 0]], [-F[0, 1], F[0, 0]]]) / J


def _eye_like(F):
    I = np.zeros_like(F)
    I[0, 0] = 1.0
    I[1, 1] = 1.0
    return I


def green_lagrange(F):
    C = np.einsum("mA...,mB...->AB...", F, F)
    return 0.5 * (C - _eye_like(F))


def energy(law, F, mu, lam):
    """Strain energy density W(F) per reference area (Appendix A)."""
    J = det(F)
    trC = np.einsum("mA...,mA...->...", F, F)
    if law == "lognh":                       # eq:lognh-model
        L = np.log(J)
        return 0.5 * mu * (trC - 2.0 - 2.0 * L) + 0.5 * lam * L * L
    if law == "nh":                          # eq:nh-model
        L = np.log(J)
        return 0.5 * mu * (trC - 2.0 - 2.0 * L) + 0.25 * lam * (J * J - 1.0 - 2.0 * L)
    if law == "svk":                         # eq:svk-model
        E = green_lagrange(F)
        trE = E[0, 0] + E[1, 1]
        EE = np.einsum("AB...,AB...->...", E, E)
        return 0.5 * lam * trE * trE + mu * EE
    raise ValueError(law)


def stress(law, F, mu, lam):
    """First Piola-Kirchhoff stress P(F) (Appendix A)."""
    if law in ("lognh", "nh"):
        J = det(F)
        H = inv_transpose(F)
        if law == "lognh":                   # P = mu (F - H) + lam ln J H
            vol = lam * np.log(J)
        else:                                # P = mu (F - H) + lam/2 (J^2 - 1) H
            vol = 0.5 * lam * (J * J - 1.0)
        return mu * (F - H) + vol * H
    if law == "svk":                         # P = F [lam tr(E) I + 2 mu E]
        E = green_lagrange(F)
        trE = E[0, 0] + E[1, 1]
        S = 2.0 * mu * E + lam * trE * _eye_like(F)
        return np.einsum("iC...,CA...->iA...", F, S)
    raise ValueError(law)


def tangent(law, F, mu, lam):
    """C_iAkB = dP_iA / dF_kB, shape (2, 2, 2, 2, ...)."""
    d = np.eye(2)
    shape = F.shape[2:]
    dd = np.einsum("ik,AB->iAkB", d, d).reshape((2, 2, 2, 2) + (1,) * len(shape))
    if law in ("lognh", "nh"):
        J = det(F)
        H = inv_transpose(F)
        HiB_HkA = np.einsum("iB...,kA...->iAkB...", H, H)
        HiA_HkB = np.einsum("iA...,kB...->iAkB...", H, H)
        if law == "lognh":
            a = mu - lam * np.log(J)
            b = lam * np.ones_like(J)
        else:
            a = mu - 0.5 * lam * (J * J - 1.0)
            b = lam * J * J
        return mu * dd + a * HiB_HkA + b * HiA_HkB
    if law == "svk":
        E = green_lagrange(F)
        trE = E[0, 0] + E[1, 1]
        S = 2.0 * mu * E + lam * trE * _eye_like(F)
        FFt = np.einsum("iC...,kC...->ik...", F, F)
        t1 = np.einsum("ik,AB...->iAkB...", d, S)
        t2 = lam * np.einsum("iA...,kB...->iAkB...", F, F)
        t3 = mu * (np.einsum("iB...,kA...->iAkB...", F, F)
                   + np.einsum("ik...,AB->iAkB...", FFt, d))
        return t1 + t2 + t3
    raise ValueError(law)


def stress_parameter_partials(law, F):
    """(dP/dmu, dP/dlam).  Every law here is linear in (mu, lam), so these are P at unit
    parameters."""
    return stress(law, F, 1.0, 0.0), stress(law, F, 0.0, 1.0)


def tangent_parameter_partials(law, F):
    return tangent(law, F, 1.0, 0.0), tangent(law, F, 0.0, 1.0)


def acoustic_tensor(law, F, mu, lam, n):
    """Q_ik(n; F) = n_A C_iAkB n_B (eq:acoustic-tensor-section2)."""
    Cc = tangent(law, F, mu, lam)
    n = np.asarray(n, dtype=np.float64)
    return np.einsum("A,iAkB...,B->ik...", n, Cc, n)


def max_tangent_speed(law, F, mu, lam, dtheta_deg=0.25):
    """Largest tangent wave speed max_n sqrt(lambda_max(Q(n; F))) over a scan of
    theta in [0, pi) (the audit of Sec. 4 scans with a 0.25 degree step)."""
    best = None
    for th in np.arange(0.0, 180.0, dtheta_deg):
        t = np.deg2rad(th)
        Q = acoustic_tensor(law, F, mu, lam, (np.cos(t), np.sin(t)))
        tr = Q[0, 0] + Q[1, 1]
        dt = Q[0, 0] * Q[1, 1] - Q[0, 1] * Q[1, 0]
        lmax = 0.5 * tr + np.sqrt(np.maximum(0.25 * tr * tr - dt, 0.0))
        best = lmax if best is None else np.maximum(best, lmax)
    return np.sqrt(best)


def cauchy(law, F, mu, lam):
    """sigma = J^{-1} P F^T (Sec. 3.5)."""
    P = stress(law, F, mu, lam)
    return np.einsum("iA...,kA...->ik...", P, F) / det(F)
