"""Wave speeds about predeformed states, Sec. 5.2 (eq:predeformed-acoustic-eigenproblem,
eq:predeformed-acoustic-reference, eq:predeformed-acoustic-F), FP64.

Test infrastructure only (see the package docstring).

A small plane wave u' = eps q sin(k X), v' = -eps k c_ac q cos(k X) travels along the
material direction n = (1, 0) on top of a uniform predeformation F0, where (c_ac^2, q) is
an eigenpair of the acoustic tensor Q(n; F0).  The lattice phase speed is measured from
the fundamental Fourier mode of v_q = q . v: phi(t) = atan2(a_s, a_c) with
a_c = 2 <v_q cos kX>, a_s = 2 <v_q sin kX>, unwrapped, c_num = (phi(t) - phi(0)) / (k t).

Setup of the paper: periodic n = 80, c = 5, omega = 2, k = 2 pi, eps = 1e-4, two
predeformations (area-preserving stretch 1.2 and simple shear 0.3).  Readings (not
printed): mu = 0.5, lam = 0.5; measurement over t = 1 (400 steps); the wave is uniform
in Y, so the oracle may run it on a grid of few rows (the lattice update of a Y-uniform
field is Y-uniform node by node).
"""
import numpy as np

from . import lbm
from . import material as mat

MU, LAM = 0.5, 0.5
EPS = 1e-4
K = 2.0 * np.pi
PREDEFORMATIONS = {"aps": np.array([[1.2, 0.0], [0.0, 1.0 / 1.2]]),
                   "shear": np.array([[1.0, 0.3], [0.0, 1.0]])}


def modes(law, F0):
    """Acoustic speeds and polarisations for n = (1, 0), slow branch first."""
    Q = mat.acoustic_tensor(law, F0, MU, LAM, (1.0, 0.0))
    w, V = np.linalg.eigh(Q)
    return np.sqrt(w), V


def initial_fields(nx, ny, law, F0, branch):
    """(v0, F-field, c_ac, q) of the travelling perturbation (eq:predeformed-acoustic-reference,
    eq:predeformed-acoustic-F at t = 0)."""
    cs, V = modes(law, F0)
    c_ac, q = cs[branch], V[:, branch]
    x = (np.arange(nx) + 0.5) / nx
    X = np.broadcast_to(x[None, :], (ny, nx))
    v0 = -EPS * K * c_ac * q[:, None, None] * np.cos(K * X)[None]
    F = np.empty((2, 2, ny, nx))
    for i in range(2):
        for A in range(2):
            F[i, A] = F0[i, A] + (EPS * K * q[i] * np.cos(K * X) if A == 0 else 0.0)
    return v0, F, c_ac, q


def problem(nx, ny, law, c=5.0, omega=2.0):
    return lbm.Problem(nx=nx, ny=ny, c=c, omega=omega, law=law, mu=MU, lam=LAM, dx=1.0 / nx)


def phase(v, q, nx):
    """phi = atan2(a_s, a_c) of v_q averaged over rows."""
    x = (np.arange(nx) + 0.5) / nx
    vq = (q[0] * v[0] + q[1] * v[1]).mean(axis=0)
    ac = 2.0 * (vq * np.cos(K * x)).mean()
    a_s = 2.0 * (vq * np.sin(K * x)).mean()
    return np.arctan2(a_s, ac)


def phase_speed(phases, dt):
    """c_num = (phi(t_end) - phi(0)) / (k t_end) after unwrapping."""
    ph = np.unwrap(np.asarray(phases))
    return (ph[-1] - ph[0]) / (K * dt * (len(ph) - 1))


def measure(law, F0, branch, nx=80, ny=4, t_end=1.0, c=5.0):
    pb = problem(nx, ny, law, c)
    v0, F, c_ac, q = initial_fields(nx, ny, law, F0, branch)
    st = lbm.initial_state(pb, v0, F0=F)
    nsteps = int(round(t_end / pb.dt))
    phases = [phase(v0, q, nx)]
    for _ in range(nsteps):
        lbm.step(pb, st)
        U, _ = lbm.observe(pb, st)
        phases.append(phase(U[0:2], q, nx))
    c_num = phase_speed(phases, pb.dt)
    return dict(c_ac=float(c_ac), c_num=float(c_num), rel=float(abs(c_num - c_ac) / c_ac))
