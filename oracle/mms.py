"""Periodic manufactured solution of Sec. 4.1, FP64.

Test infrastructure only (see the package docstring).

Exact displacement (eq:periodic-mms-displacement), A = 0.08, k = 2 pi on (0, 1)^2:
  u_x = A sin(k(X - 0.23 t)) cos(k(Y - 0.17 t)) sin(k(t - 0.11)),
  u_y = A cos(k(X + 0.19 t)) sin(k(Y - 0.29 t)) cos(k(t + 0.07)),
with the body acceleration of eq:mms-body-force, b = d_t^2 u - Div P(I + grad u), so the
field solves eq:displacement-form exactly.  The divergence is evaluated as
d_A P_iA = C_iAkB d_A F_kB with analytic second derivatives of u.  Derivatives of u are
produced symbolically (sympy) once and evaluated in numpy.
"""
import functools

import numpy as np

from . import lbm
from . import material as mat

AMP = 0.08
K = 2.0 * np.pi


@functools.lru_cache(maxsize=1)
def _derivative_functions():
    import sympy as sp
    X, Y, t = sp.symbols("X Y t", real=True)
    A, k = sp.Float(AMP, 30), 2 * sp.pi
    ux = A * sp.sin(k * (X - sp.Rational(23, 100) * t)) * sp.cos(k * (Y - sp.Rational(17, 100) * t)) \
        * sp.sin(k * (t - sp.Rational(11, 100)))
    uy = A * sp.cos(k * (X + sp.Rational(19, 100) * t)) * sp.sin(k * (Y - sp.Rational(29, 100) * t)) \
        * sp.cos(k * (t + sp.Rational(7, 100)))
    names = {}
    for nm, u in (("x", ux), ("y", uy)):
        names[nm] = {
            "u": u, "t": sp.diff(u, t), "tt": sp.diff(u, t, 2),
            "X": sp.diff(u, X), "Y": sp.diff(u, Y),
            "XX": sp.diff(u, X, 2), "XY": sp.diff(u, X, Y), "YY": sp.diff(u, Y, 2),
            "tX": sp.diff(u, t, X), "tY": sp.diff(u, t, Y),
        }
    return {nm: {key: sp.lambdify((X, Y, t), expr, "numpy") for key, expr in d.items()}
            for nm, d in names.items()}


def fields(X, Y, t):
    """Exact u, v, F, and the material derivatives of v and F at (X, Y, t)."""
    fn = _derivative_functions()
    ev = {key: np.array([np.broadcast_to(fn[c][key](X, Y, t), np.broadcast(X, Y).shape)
                         for c in ("x", "y")]) for key in fn["x"]}
    u, v, a = ev["u"], ev["t"], ev["tt"]
    F = np.array([[1.0 + ev["X"][0], ev["Y"][0]], [ev["X"][1], 1.0 + ev["Y"][1]]])
    dF_dX = np.array([[ev["XX"][0], ev["XY"][0]], [ev["XX"][1], ev["XY"][1]]])
    dF_dY = np.array([[ev["XY"][0], ev["YY"][0]], [ev["XY"][1], ev["YY"][1]]])
    dv_dX, dv_dY = ev["tX"], ev["tY"]
    return dict(u=u, v=v, a=a, F=F, dF_dX=dF_dX, dF_dY=dF_dY, dv_dX=dv_dX, dv_dY=dv_dY)


def body_force(law, mu, lam, X, Y, t):
    f = fields(X, Y, t)
    Cc = mat.tangent(law, f["F"], mu, lam)
    divP = (np.einsum("iAkB...,kB...->iA...", Cc, f["dF_dX"])[:, 0]
            + np.einsum("iAkB...,kB...->iA...", Cc, f["dF_dY"])[:, 1])
    return f["a"] - divP


def grid(n):
    x = (np.arange(n) + 0.5) / n
    return np.meshgrid(x, x, indexing="xy")          # X[b, a], Y[b, a]


def setup(n, c=5.0, omega=2.0, law="lognh", mu=1.0, lam=2.0 / 3.0, second_order=True):
    """Periodic MMS problem on an n x n grid of (0, 1)^2 (Sec. 4.1: log-NH, lam = 2/3,
    mu = 1, c = 5, omega = 2) and its initial state with analytic derivatives."""
    X, Y = grid(n)
    dx = 1.0 / n
    dt = dx / c
    pb = lbm.Problem(nx=n, ny=n, c=c, omega=omega, law=law, mu=mu, lam=lam, dx=dx,
                     body=lambda m: body_force(law, mu, lam, X, Y, m * dt))
    f0 = fields(X, Y, 0.0)
    F0 = f0["F"]
    U0 = np.array([f0["v"][0], f0["v"][1], F0[0, 0], F0[0, 1], F0[1, 0], F0[1, 1]])
    dUdX = np.array([f0["dv_dX"][0], f0["dv_dX"][1], f0["dF_dX"][0, 0], f0["dF_dX"][0, 1],
                     f0["dF_dX"][1, 0], f0["dF_dX"][1, 1]])
    dUdY = np.array([f0["dv_dY"][0], f0["dv_dY"][1], f0["dF_dY"][0, 0], f0["dF_dY"][0, 1],
                     f0["dF_dY"][1, 0], f0["dF_dY"][1, 1]])
    if second_order:
        f = lbm.second_order_populations(pb, U0, dUdX, dUdY, pb.B(0))
    else:
        f, _ = lbm.equilibrium_of_state(pb, U0)
    st = lbm.State(f=f, ustar=f0["u"] - 0.5 * dt * f0["v"], n=0)
    return pb, st, (X, Y)


def relative_errors(n, t_end=0.1, second_order=True, **kw):
    """E_L2 of u, P and sigma (Sec. 4, norms over all nodes and components) at t_end."""
    pb, st, (X, Y) = setup(n, second_order=second_order, **kw)
    nsteps = int(round(t_end / pb.dt))
    U, u = lbm.run(pb, st, nsteps)
    ex = fields(X, Y, nsteps * pb.dt)
    Fh = lbm.F_of(U)
    Ph = mat.stress(pb.law, Fh, pb.mu, pb.lam)
    Pe = mat.stress(pb.law, ex["F"], pb.mu, pb.lam)
    Sh = mat.cauchy(pb.law, Fh, pb.mu, pb.lam)
    Se = mat.cauchy(pb.law, ex["F"], pb.mu, pb.lam)

    def rel(a, b):
        return float(np.sqrt(((a - b) ** 2).sum()) / np.sqrt((b ** 2).sum()))
    return dict(u=rel(u, ex["u"]), P=rel(Ph, Pe), sigma=rel(Sh, Se), steps=nsteps)


# ----------------------------------------------------------------------------- boundary MMS

def boundary_setup(n, mode="dirichlet", c=5.0, omega=2.0, law="lognh", mu=1.0, lam=2.0 / 3.0):
    """Manufactured solution of Sec. 4.2 on the bounded square (0, 1)^2 with half-way walls.

    mode 'dirichlet': exact material velocity v = d_t u on every side
    (eq:boundary-mms-dirichlet); mode 'mixed': exact velocity on X = 0 and Y = 0, exact
    nominal traction P(I + grad u) N on X = 1 and Y = 1 (eq:boundary-mms-mixed).  The wall
    data are evaluated at the half-way wall points and at t^{n+1/2} (eq:boundary-general)."""
    from .lbm import Edge, XMIN, XMAX, YMIN, YMAX
    X, Y = grid(n)
    dx = 1.0 / n
    dt = dx / c
    s = (np.arange(n) + 0.5) / n

    def wall_points(e):
        if e == XMIN:
            return np.zeros(n), s
        if e == XMAX:
            return np.ones(n), s
        if e == YMIN:
            return s, np.zeros(n)
        return s, np.ones(n)

    normals = {XMIN: (-1.0, 0.0), XMAX: (1.0, 0.0), YMIN: (0.0, -1.0), YMAX: (0.0, 1.0)}

    def velocity_data(e):
        Xw, Yw = wall_points(e)
        return lambda t: fields(Xw, Yw, t)["v"]

    def traction_data(e):
        Xw, Yw = wall_points(e)
        N = np.array(normals[e])

        def T(t):
            P = mat.stress(law, fields(Xw, Yw, t)["F"], mu, lam)
            return np.einsum("iA...,A->i...", P, N)
        return T

    kinds = {XMIN: "velocity", YMIN: "velocity",
             XMAX: "velocity" if mode == "dirichlet" else "traction",
             YMAX: "velocity" if mode == "dirichlet" else "traction"}
    edges = []
    for e in range(4):
        data = velocity_data(e) if kinds[e] == "velocity" else traction_data(e)
        edges.append(Edge(kinds[e], data))
    pb = lbm.Problem(nx=n, ny=n, c=c, omega=omega, law=law, mu=mu, lam=lam, dx=dx,
                     body=lambda m: body_force(law, mu, lam, X, Y, m * dt), edges=edges)
    f0 = fields(X, Y, 0.0)
    F0 = f0["F"]
    U0 = np.array([f0["v"][0], f0["v"][1], F0[0, 0], F0[0, 1], F0[1, 0], F0[1, 1]])
    dUdX = np.array([f0["dv_dX"][0], f0["dv_dX"][1], f0["dF_dX"][0, 0], f0["dF_dX"][0, 1],
                     f0["dF_dX"][1, 0], f0["dF_dX"][1, 1]])
    dUdY = np.array([f0["dv_dY"][0], f0["dv_dY"][1], f0["dF_dY"][0, 0], f0["dF_dY"][0, 1],
                     f0["dF_dY"][1, 0], f0["dF_dY"][1, 1]])
    f = lbm.second_order_populations(pb, U0, dUdX, dUdY, pb.B(0))
    st = lbm.State(f=f, ustar=f0["u"] - 0.5 * dt * f0["v"], n=0)
    return pb, st, (X, Y)


def boundary_errors(n, mode="dirichlet", t_end=0.1, layers=2, **kw):
    """E_L2 of u, P and sigma over the full domain and after removing `layers` grid layers
    next to the boundary (Sec. 4.2, Table tab:mms-error-summary)."""
    pb, st, (X, Y) = boundary_setup(n, mode, **kw)
    nsteps = int(round(t_end / pb.dt))
    U, u = lbm.run(pb, st, nsteps)
    ex = fields(X, Y, nsteps * pb.dt)
    Fh = lbm.F_of(U)
    Ph, Pe = mat.stress(pb.law, Fh, pb.mu, pb.lam), mat.stress(pb.law, ex["F"], pb.mu, pb.lam)
    Sh, Se = mat.cauchy(pb.law, Fh, pb.mu, pb.lam), mat.cauchy(pb.law, ex["F"], pb.mu, pb.lam)

    def rel(a, b, sl=(slice(None), slice(None))):
        a = a[(Ellipsis,) + sl]
        b = b[(Ellipsis,) + sl]
        return float(np.sqrt(((a - b) ** 2).sum()) / np.sqrt((b ** 2).sum()))
    inner = (slice(layers, n - layers), slice(layers, n - layers))
    return dict(u=rel(u, ex["u"]), P=rel(Ph, Pe), sigma=rel(Sh, Se),
                u_in=rel(u, ex["u"], inner), P_in=rel(Ph, Pe, inner), sigma_in=rel(Sh, Se, inner),
                steps=nsteps)
