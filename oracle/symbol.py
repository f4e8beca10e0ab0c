"""Fourier symbol of the D2Q4 x 6 step linearised about a uniform state, FP64.

Test infrastructure only (see the package docstring).

About a uniform state U0 = (0, 0, F0) with b = 0, a perturbation f = f(U0) + df evolves
as df^{n+1}_q(X) = [(1 - omega) df^n_q + omega (f^eq_q)'(U0) dU](X - c_q dt) with
dU = sum_q df_q (eq:moment-U, eq:collision, eq:streaming) and (f^eq_q)' from
eq:feq-derivative with the Jacobian actions of eq:jacobian-actions.  For a Fourier mode
exp(i k.X) the step is the 24 x 24 matrix G(k) = S(k) [(1 - omega) I + omega E R], with
S(k) = diag(exp(-i k.c_q dt)) (x I6), E the stacked equilibrium derivatives and R the
moment sum.  Its eigenvalues give the linear stability (|z| <= 1) and, for the six modes
near z = 1, the lattice dispersion of the elastic waves whose continuum speeds are the
square roots of the acoustic-tensor eigenvalues (eq:predeformed-acoustic-eigenproblem).
"""
import numpy as np

from . import material as mat

DIRS = ((1, 0), (0, 1), (-1, 0), (0, -1))


def jacobians(Cc):
    """Dense 6 x 6 A_X, A_Y of eq:jacobian-actions for a tangent C (2, 2, 2, 2)."""
    AX = np.zeros((6, 6))
    AY = np.zeros((6, 6))
    for k in range(2):
        for B in range(2):
            col = 2 + 2 * k + B
            AX[0, col] = -Cc[0, 0, k, B]
            AX[1, col] = -Cc[1, 0, k, B]
            AY[0, col] = -Cc[0, 1, k, B]
            AY[1, col] = -Cc[1, 1, k, B]
    AX[2, 0] = AX[4, 1] = -1.0
    AY[3, 0] = AY[5, 1] = -1.0
    return AX, AY


def step_matrix(kvec, c, omega, law, mu, lam, dx=1.0, F0=None):
    F0 = np.eye(2) if F0 is None else np.asarray(F0, dtype=np.float64)
    Cc = mat.tangent(law, F0, mu, lam)
    AX, AY = jacobians(Cc)
    E = np.vstack([0.25 * (np.eye(6) + (2.0 / c) * (i * AX + j * AY)) for (i, j) in DIRS])
    R = np.hstack([np.eye(6)] * 4)
    coll = (1.0 - omega) * np.eye(24) + omega * E @ R
    ph = np.repeat([np.exp(-1j * (kvec[0] * i + kvec[1] * j) * dx) for (i, j) in DIRS], 6)
    return ph[:, None] * coll


def spectral_radius(c, omega, law, mu, lam, n=64, dx=1.0, F0=None):
    """max |z| over the eigenvalues of G(k) for every wavevector of an n x n periodic grid."""
    rho = 0.0
    for a in range(n):
        for b in range(n):
            kv = (2.0 * np.pi * a / (n * dx), 2.0 * np.pi * b / (n * dx))
            z = np.linalg.eigvals(step_matrix(kv, c, omega, law, mu, lam, dx, F0))
            rho = max(rho, float(np.abs(z).max()))
    return rho


def elastic_modes(kvec, c, omega, law, mu, lam, dx=1.0, F0=None):
    """The six eigenpairs nearest z = 1 (the macroscopic modes), as a list of
    (phase speed, z, moment vector sum_q f_q of the eigenvector), sorted by speed.
    The phase speed is |arg z| / (dt |k|) with dt = dx / c."""
    G = step_matrix(kvec, c, omega, law, mu, lam, dx, F0)
    z, V = np.linalg.eig(G)
    order = np.argsort(np.abs(z - 1.0))[:6]
    dt = dx / c
    kn = float(np.hypot(*kvec))
    out = []
    for idx in order:
        mom = V[:, idx].reshape(4, 6).sum(0)
        out.append((abs(np.angle(z[idx])) / (dt * kn), z[idx], mom))
    out.sort(key=lambda t: t[0])
    return out
