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
INVARIANT_LAWS = ("mr", "yeoh", "gent")
ALL_LAWS = LAWS + INVARIANT_LAWS

# Law constants of the invariant-based closures.  The coefficients are given as multiples
# of mu, so that P stays linear in (mu, lam) over a heterogeneous mu field:
#   mr:   (k10, k01)      c10 = k10 mu, c01 = k01 mu
#   yeoh: (k1, k2, k3)    c1 = k1 mu, c2 = k2 mu, c3 = k3 mu
#   gent: (J_m,)
# Appendix A fixes c10 + c01 = mu/2 and c1 = mu/2 when no constants are supplied; the
# split of the Mooney-Rivlin pair, the higher Yeoh coefficients and the Gent limit are not
# printed, the defaults below are readings.
DEFAULT_PARAMS = {"mr": (0.3, 0.2), "yeoh": (0.5, 0.05, 0.01), "gent": (20.0,)}


def law_name(law):
    """A law is a name from ALL_LAWS or a pair (name, constants) for the invariant laws."""
    return law[0] if isinstance(law, tuple) else law


def _law(law, params):
    if isinstance(law, tuple):
        return law[0], tuple(law[1])
    return law, (DEFAULT_PARAMS.get(law) if params is None else tuple(params))


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


def _invariants(F):
    """eq:modified-invariants with the plane-strain embedding (out-of-plane stretch 1):
    I1 = tr C + 1, I2 = J^2 + tr C, barI1 = J^(-2/3) I1, barI2 = J^(-4/3) I2."""
    J = det(F)
    trC = np.einsum("mA...,mA...->...", F, F)
    I1 = trC + 1.0
    I2 = J * J + trC
    return J, I1, I2, J ** (-2.0 / 3.0) * I1, J ** (-4.0 / 3.0) * I2


def _G1_G2(F):
    """eq:modified-invariant-gradients: G1 = d barI1/dF, G2 = d barI2/dF."""
    J, I1, I2, _, _ = _invariants(F)
    H = inv_transpose(F)
    G1 = J ** (-2.0 / 3.0) * (2.0 * F - (2.0 / 3.0) * I1 * H)
    G2 = J ** (-4.0 / 3.0) * (2.0 * F + (2.0 * J * J - (4.0 / 3.0) * I2) * H)
    return G1, G2


def energy(law, F, mu, lam, params=None):
    """Strain energy density W(F) per reference area (Appendix A)."""
    law, prm = _law(law, params)
    if law in INVARIANT_LAWS:
        J, I1, I2, bI1, bI2 = _invariants(F)
        vol = 0.5 * lam * np.log(J) ** 2
        A = bI1 - 3.0
        if law == "mr":                      # eq:mr-model
            return prm[0] * mu * A + prm[1] * mu * (bI2 - 3.0) + vol
        if law == "yeoh":                    # eq:yeoh-model
            return prm[0] * mu * A + prm[1] * mu * A ** 2 + prm[2] * mu * A ** 3 + vol
        Jm = prm[0]                          # eq:gent-model
        return -0.5 * mu * Jm * np.log(1.0 - A / Jm) + vol
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


def stress(law, F, mu, lam, params=None):
    """First Piola-Kirchhoff stress P(F) (Appendix A)."""
    law, prm = _law(law, params)
    if law in INVARIANT_LAWS:
        J, I1, I2, bI1, bI2 = _invariants(F)
        G1, G2 = _G1_G2(F)
        H = inv_transpose(F)
        vol = lam * np.log(J) * H
        A = bI1 - 3.0
        if law == "mr":                      # P = c10 G1 + c01 G2 + lam ln J H
            return prm[0] * mu * G1 + prm[1] * mu * G2 + vol
        if law == "yeoh":                    # P = (c1 + 2 c2 A + 3 c3 A^2) G1 + lam ln J H
            return (prm[0] + 2.0 * prm[1] * A + 3.0 * prm[2] * A ** 2) * mu * G1 + vol
        Jm = prm[0]                          # P = mu / (2 (1 - A/J_m)) G1 + lam ln J H
        return mu / (2.0 * (1.0 - A / Jm)) * G1 + vol
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


def tangent(law, F, mu, lam, params=None):
    """C_iAkB = dP_iA / dF_kB, shape (2, 2, 2, 2, ...)."""
    law, params = _law(law, params)
    if law in INVARIANT_LAWS:
        # complex-step differentiation of P: dP/dF_kB = Im P(F + i h e_kB) / h, exact to
        # rounding for real-analytic P (no subtraction of nearly equal numbers)
        h = 1e-30
        out = np.empty((2, 2, 2, 2) + F.shape[2:])
        mu_c = np.asarray(mu) + 0j
        lam_c = np.asarray(lam) + 0j
        for k in range(2):
            for B in range(2):
                Fc = F.astype(np.complex128)
                Fc[k, B] += 1j * h
                out[:, :, k, B] = stress(law, Fc, mu_c, lam_c, params).imag / h
        return out
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


def stress_parameter_partials(law, F, params=None):
    """(dP/dmu, dP/dlam).  Every law here is linear in (mu, lam) (the invariant laws'
    constants are multiples of mu), so these are P at unit parameters."""
    return stress(law, F, 1.0, 0.0, params), stress(law, F, 0.0, 1.0, params)


def tangent_parameter_partials(law, F, params=None):
    return tangent(law, F, 1.0, 0.0, params), tangent(law, F, 0.0, 1.0, params)


def acoustic_tensor(law, F, mu, lam, n, params=None):
    """Q_ik(n; F) = n_A C_iAkB n_B (eq:acoustic-tensor-section2)."""
    Cc = tangent(law, F, mu, lam, params)
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


def cauchy(law, F, mu, lam, params=None):
    """sigma = J^{-1} P F^T (Sec. 3.5)."""
    P = stress(law, F, mu, lam, params)
    return np.einsum("iA...,kA...->ik...", P, F) / det(F)
