"""Affine finite-strain patch of Sec. 5.1 (eq:affine-patch-motion, eq:affine-exact-fields,
eq:affine-deformation-paths), FP64.

Test infrastructure only (see the package docstring).

On the unit square with velocity walls on all four sides, the affine motion
u = (F(t) - I) X, v = (F* - I)/T X, F(t) = I + (t/T)(F* - I) solves eq:displacement-form
exactly without body force for every law (P is uniform, so Div P = 0).  The lattice run
starts from F = I, v = (F* - I)/T X with the second-order initialisation, prescribes the
exact wall velocity at the half-way wall points, and is compared with F*, P(F*) and
sigma(F*) at t = T.

Readings (the paper does not print them): T = 1, mu = 0.5, lam = 0.5 (nu = 0.25), so the
largest tangent speed on every path stays below 0.42 c at c = 5; omega = 2 - 1.6 dx as in
eq:benchmark-omega; the terminal states use the largest parameter of each family
(lambda_s = 1.45 and 1.40, gamma = kappa = 0.80).
"""
import numpy as np

from . import lbm
from . import material as mat

MU, LAM = 0.5, 0.5
T_LOAD = 1.0


def terminal_state(path, s=None):
    """F* of eq:affine-deformation-paths for parameter s (default: the largest used)."""
    if path == "uni":
        s = 1.45 if s is None else s
        return np.array([[s, 0.0], [0.0, 1.0]])
    if path == "aps":
        s = 1.40 if s is None else s
        return np.array([[s, 0.0], [0.0, 1.0 / s]])
    if path == "sh":
        s = 0.80 if s is None else s
        return np.array([[1.0, s], [0.0, 1.0]])
    if path == "ss":
        s = 0.80 if s is None else s
        return np.array([[1.15, s], [0.0, 1.0 / 1.15]])
    raise ValueError(path)


PATHS = ("uni", "aps", "sh", "ss")


def grid(n):
    x = (np.arange(n) + 0.5) / n
    return np.meshgrid(x, x, indexing="xy")


def problem(n, law, Fs, c=5.0, omega=None):
    """Velocity walls carrying v = (F* - I)/T X at the half-way wall points."""
    from .lbm import Edge, XMIN, XMAX, YMIN, YMAX
    G = (np.asarray(Fs) - np.eye(2)) / T_LOAD
    s = (np.arange(n) + 0.5) / n
    pts = {XMIN: (np.zeros(n), s), XMAX: (np.ones(n), s), YMIN: (s, np.zeros(n)), YMAX: (s, np.ones(n))}

    def data(e):
        Xw, Yw = pts[e]
        vw = np.array([G[0, 0] * Xw + G[0, 1] * Yw, G[1, 0] * Xw + G[1, 1] * Yw])
        return lambda t: vw
    edges = [Edge("velocity", data(e)) for e in range(4)]
    om = 2.0 - 1.6 / n if omega is None else omega
    return lbm.Problem(nx=n, ny=n, c=c, omega=om, law=law, mu=MU, lam=LAM, dx=1.0 / n, edges=edges)


def initial_velocity(n, Fs):
    X, Y = grid(n)
    G = (np.asarray(Fs) - np.eye(2)) / T_LOAD
    return np.array([G[0, 0] * X + G[0, 1] * Y, G[1, 0] * X + G[1, 1] * Y])


def steps(n, c=5.0):
    return int(round(T_LOAD / (1.0 / (n * c))))


def run(n, law, path, c=5.0):
    """Relative L2 errors of F, P, sigma and u at t = T (norms over all nodes and
    components, as in Sec. 4)."""
    Fs = terminal_state(path)
    pb = problem(n, law, Fs, c)
    st = lbm.initial_state(pb, initial_velocity(n, Fs))
    N = steps(n, c)
    U, u = lbm.run(pb, st, N)
    X, Y = grid(n)
    Fh = lbm.F_of(U)
    Fe = np.broadcast_to(Fs[:, :, None, None], Fh.shape)
    Ph, Pe = mat.stress(law, Fh, MU, LAM), mat.stress(law, Fe, MU, LAM)
    Sh, Se = mat.cauchy(law, Fh, MU, LAM), mat.cauchy(law, Fe, MU, LAM)
    ue = np.array([(Fs[0, 0] - 1.0) * X + Fs[0, 1] * Y, Fs[1, 0] * X + (Fs[1, 1] - 1.0) * Y])

    def rel(a, b):
        return float(np.sqrt(((a - b) ** 2).sum() / (b ** 2).sum()))
    return dict(F=rel(Fh, Fe), P=rel(Ph, Pe), sigma=rel(Sh, Se), u=rel(u, ue), steps=N, U=U, u_h=u)
