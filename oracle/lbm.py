"""One time step of the D2Q4 x 6 vectorial LBM (paper Sec. 3), plain FP64 numpy.

Test infrastructure only (see the package docstring).

Layout: populations ``f[q, k, b, a]`` with q the D2Q4 direction in the paper's order
(1,0), (0,1), (-1,0), (0,-1) (Sec. 3.1), k the state component in the order of
eq:state-vector, U = (v1, v2, F11, F12, F21, F22), b the row (Y) index and a the column
(X) index.  Node (a, b) sits at X = ((a + 1/2) dx, (b + 1/2) dx), so half-way walls lie at
X = 0, X = nx dx, Y = 0, Y = ny dx (Sec. 3.6).  The oracle stores the unshifted F.

The state advanced by ``step`` is the pre-collision population f^n and the auxiliary
displacement u*^n of eq:trapezoid-u.  Readings of points the paper leaves open are marked
"Reading" and are the same ones the library implements.
"""
from dataclasses import dataclass, field
from typing import Callable, Optional, Sequence

import numpy as np

from . import material as mat

DIRS = ((1, 0), (0, 1), (-1, 0), (0, -1))
OPP = (2, 3, 0, 1)
XMIN, XMAX, YMIN, YMAX = 0, 1, 2, 3

# Per grid-aligned edge: outward normal N, the material axis A that N is aligned with,
# and the missing incoming direction d = -N (Sec. 3.6).
EDGE_NORMAL = {XMIN: (-1, 0), XMAX: (1, 0), YMIN: (0, -1), YMAX: (0, 1)}
EDGE_AXIS = {XMIN: 0, XMAX: 0, YMIN: 1, YMAX: 1}
EDGE_MISSING = {XMIN: 0, XMAX: 2, YMIN: 1, YMAX: 3}

# eq:dirichlet-boundary-rule and eq:neumann-boundary-rule
D_DIRICHLET = np.array([-1.0, -1.0, 1.0, 1.0, 1.0, 1.0])
D_NEUMANN = np.array([1.0, 1.0, -1.0, -1.0, -1.0, -1.0])


@dataclass
class Edge:
    kind: str = "periodic"                      # 'periodic' | 'velocity' | 'traction'
    data: Optional[Callable] = None             # t -> (2,) or (2, L): v_D or nominal T


@dataclass
class Problem:
    nx: int
    ny: int
    c: float                                    # lattice speed dx/dt (Sec. 2.1)
    omega: float                                # BGK relaxation rate (eq:collision)
    law: object = "lognh"                       # name, or (name, constants) for MR / Yeoh / Gent
    mu: object = 0.1                            # scalar or (ny, nx)
    lam: object = 0.2
    dx: float = 1.0
    body: object = None                         # None, (2, ny, nx) array, or n -> (2, ny, nx)
    ramp: Optional[Callable] = None             # n -> r(n) multiplying a fixed body field
    edges: Sequence[Edge] = field(default_factory=lambda: [Edge(), Edge(), Edge(), Edge()])
    newton_max_iter: int = 50
    newton_tol: float = 1e-14

    def __post_init__(self):
        self.mu = np.broadcast_to(np.asarray(self.mu, dtype=np.float64), (self.ny, self.nx))
        self.lam = np.broadcast_to(np.asarray(self.lam, dtype=np.float64), (self.ny, self.nx))
        kinds = [e.kind for e in self.edges]
        if (kinds[XMIN] == "periodic") != (kinds[XMAX] == "periodic"):
            raise ValueError("x edges must both be periodic or both be walls")
        if (kinds[YMIN] == "periodic") != (kinds[YMAX] == "periodic"):
            raise ValueError("y edges must both be periodic or both be walls")

    @property
    def dt(self):
        return self.dx / self.c

    @property
    def periodic_x(self):
        return self.edges[XMIN].kind == "periodic"

    @property
    def periodic_y(self):
        return self.edges[YMIN].kind == "periodic"

    def B(self, n):
        """Body acceleration field b at time level n, shape (2, ny, nx)."""
        if self.body is None:
            return np.zeros((2, self.ny, self.nx))
        if callable(self.body):
            return np.asarray(self.body(n), dtype=np.float64)
        r = 1.0 if self.ramp is None else float(self.ramp(n))
        return r * np.broadcast_to(np.asarray(self.body, dtype=np.float64), (2, self.ny, self.nx))


# ----------------------------------------------------------------------------- moments

def F_of(U):
    """Deformation gradient (2, 2, ...) from the state vector (eq:state-vector)."""
    return np.array([[U[2], U[3]], [U[4], U[5]]])


def moments(f, B, dt):
    """eq:moment-U: U = sum_q f_q + (dt/2) B, with B = (b1, b2, 0, 0, 0, 0)."""
    U = f[0] + f[1] + f[2] + f[3]
    U = U.copy()
    U[0] += 0.5 * dt * B[0]
    U[1] += 0.5 * dt * B[1]
    return U


def fluxes(U, P):
    """eq:flux-vectors: Phi_X = (-P11, -P21, -v1, 0, -v2, 0), Phi_Y = (-P12, -P22, 0, -v1, 0, -v2)."""
    z = np.zeros_like(U[0])
    PhiX = np.array([-P[0, 0], -P[1, 0], -U[0], z, -U[1], z])
    PhiY = np.array([-P[0, 1], -P[1, 1], z, -U[0], z, -U[1]])
    return PhiX, PhiY


def equilibrium(U, PhiX, PhiY, c):
    """eq:feq: f^eq_ij = 1/4 [U + (2/c)(i Phi_X + j Phi_Y)]."""
    return np.array([0.25 * (U + (2.0 / c) * (i * PhiX + j * PhiY)) for (i, j) in DIRS])


def equilibrium_of_state(pb, U):
    P = mat.stress(pb.law, F_of(U), pb.mu, pb.lam)
    PhiX, PhiY = fluxes(U, P)
    return equilibrium(U, PhiX, PhiY, pb.c), P


def collide(f, feq, B, omega, dt):
    """eq:collision: f* = f + omega (f^eq - f) + dt (2 - omega) w B, w = 1/8."""
    fs = f + omega * (feq - f)
    src = dt * (2.0 - omega) * 0.125
    fs[:, 0] += src * B[0]
    fs[:, 1] += src * B[1]
    return fs


# ----------------------------------------------------------------------------- streaming

def stream(pb, fstar):
    """eq:streaming: f_q(X + c_q dt) = f*_q(X).  Entries whose source lies outside a wall are
    left as NaN; the boundary rules must fill every one of them."""
    out = np.full_like(fstar, np.nan)
    for q, (i, j) in enumerate(DIRS):
        src = fstar[q]
        if i != 0:
            if pb.periodic_x:
                out[q] = np.roll(src, i, axis=-1)
            elif i == 1:
                out[q][..., 1:] = src[..., :-1]
            else:
                out[q][..., :-1] = src[..., 1:]
        else:
            if pb.periodic_y:
                out[q] = np.roll(src, j, axis=-2)
            elif j == 1:
                out[q][..., 1:, :] = src[..., :-1, :]
            else:
                out[q][..., :-1, :] = src[..., 1:, :]
    return out


# ----------------------------------------------------------------------------- walls

def wall_row(arr, e, row, nx, ny):
    """Values on the wall row (row=0) or the first interior row (row=1) of edge e, as an
    array whose last axis runs along the edge."""
    if e == XMIN:
        return arr[..., :, row]
    if e == XMAX:
        return arr[..., :, nx - 1 - row]
    if e == YMIN:
        return arr[..., row, :]
    return arr[..., ny - 1 - row, :]


def set_wall_row(arr, e, vals, nx, ny):
    if e == XMIN:
        arr[..., :, 0] = vals
    elif e == XMAX:
        arr[..., :, nx - 1] = vals
    elif e == YMIN:
        arr[..., 0, :] = vals
    else:
        arr[..., ny - 1, :] = vals


def fd_along(g, periodic, h):
    """Second-order first derivative along the last axis: central differences, and at the
    ends of a non-periodic axis the one-sided three-point formula (Sec. 3.4 uses
    one-sided stencils next to nonperiodic boundaries)."""
    d = np.empty_like(g)
    if periodic:
        return (np.roll(g, -1, axis=-1) - np.roll(g, 1, axis=-1)) / (2.0 * h)
    d[..., 1:-1] = (g[..., 2:] - g[..., :-2]) / (2.0 * h)
    d[..., 0] = (-3.0 * g[..., 0] + 4.0 * g[..., 1] - g[..., 2]) / (2.0 * h)
    d[..., -1] = (3.0 * g[..., -1] - 4.0 * g[..., -2] + g[..., -3]) / (2.0 * h)
    return d


def edge_values(edge, t, L):
    vals = np.asarray(edge.data(t) if edge.data is not None else np.zeros(2), dtype=np.float64)
    if vals.ndim == 1:
        vals = np.repeat(vals[:, None], L, axis=1)
    return vals


def neumann_guess_and_tangent(pb, e, U):
    """Reading of Sec. 3.6, which says only that the tangential column of F^b comes from
    the interior nodes: it is the tangential column of the wall node's own F at level n,
    and the Newton initial guess for the normal column is that node's normal column.  Run
    to t = 0.05, the boundary manufactured solution of Sec. 4.2 with this reading gives
    every printed digit of the two boundary blocks of Table tab:mms-error-summary, and the
    cantilever of Sec. 5.4 gives the printed J range at t = 12."""
    A = EDGE_AXIS[e]
    F0 = wall_row(F_of(U), e, 0, pb.nx, pb.ny)
    return F0[:, 1 - A].copy(), F0[:, A].copy()


def _assemble(A, a, tang):
    L = a.shape[-1]
    F = np.empty((2, 2, L))
    F[:, A] = a
    F[:, 1 - A] = tang
    return F


def _solve2(M, r):
    det = M[0, 0] * M[1, 1] - M[0, 1] * M[1, 0]
    x0 = (M[1, 1] * r[0] - M[0, 1] * r[1]) / det
    x1 = (-M[1, 0] * r[0] + M[0, 0] * r[1]) / det
    return np.array([x0, x1])


def newton_normal_column(law, A, NA, tang, T, mu, lam, guess, max_iter, tol):
    """Solve P_iA(F^b) N_A = T_i (i = 1, 2) for the normal column a_i = F^b_iA of the
    boundary deformation gradient (Sec. 3.6), vectorised over the nodes of one edge.

    Reading of "Newton iteration with line search, rejecting det F^b <= 0": full step
    delta = -J^{-1} r with J_ik = N_A C_iAkA(F^b); step lengths 1, 1/2, ..., 2^-10 are tried
    and the first one with det F^b > 0 and a strictly smaller |r| is taken; a node stops
    when |r| <= tol (|T| + mu |F^b - I|), when no step length is accepted, or after
    max_iter updates.  Returns (a, failed) where failed flags |r| above 1e-4 of that scale
    (plus the rounding floor of the unshifted evaluation) or det F^b <= 0."""
    Bax = 1 - A

    def residual(a):
        P = mat.stress(law, _assemble(A, a, tang), mu, lam)
        return NA * P[:, A] - T

    def scale_of(a):
        F = _assemble(A, a, tang)
        Ft = F.copy()
        Ft[0, 0] -= 1.0
        Ft[1, 1] -= 1.0
        return np.sqrt((T * T).sum(0)) + mu * np.sqrt((Ft * Ft).sum((0, 1)))

    a = guess.copy()
    r = residual(a)
    active = np.ones(a.shape[-1], dtype=bool)
    for _ in range(max_iter):
        rn = np.sqrt((r * r).sum(0))
        active &= ~(rn <= tol * scale_of(a))
        if not active.any():
            break
        F = _assemble(A, a, tang)
        Cc = mat.tangent(law, F, mu, lam)
        Jm = NA * Cc[:, A, :, A]
        delta = -_solve2(Jm, r)
        accepted = np.zeros_like(active)
        a_new, r_new = a.copy(), r.copy()
        alpha = 1.0
        for _ls in range(11):
            cand = active & ~accepted
            if not cand.any():
                break
            a_try = a + alpha * delta
            Jt = mat.det(_assemble(A, a_try, tang))
            ok = cand & (Jt > 0)
            if ok.any():
                r_try = np.full_like(r, np.inf)
                sub = _assemble(A, a_try[:, ok], tang[:, ok])
                P = mat.stress(law, sub, mu[ok], lam[ok])
                r_try[:, ok] = NA * P[:, A] - T[:, ok]
                ok &= np.sqrt((r_try * r_try).sum(0)) < rn
                a_new[:, ok] = a_try[:, ok]
                r_new[:, ok] = r_try[:, ok]
                accepted |= ok
            alpha *= 0.5
        active &= accepted
        a, r = a_new, r_new
    rn = np.sqrt((r * r).sum(0))
    # the unshifted F leaves a rounding floor of order eps (|T| + 2 mu) in the residual
    floor = 1e3 * np.finfo(np.float64).eps * (np.sqrt((T * T).sum(0)) + 2.0 * mu)
    failed = (rn > 1e-4 * scale_of(a) + floor) | (mat.det(_assemble(A, a, tang)) <= 0)
    del Bax
    return a, failed


def neumann_boundary_F(pb, e, U, T):
    """Boundary deformation gradient F^b (2, 2, L) for the traction rule of edge e."""
    A = EDGE_AXIS[e]
    NA = float(EDGE_NORMAL[e][A])
    tang, guess = neumann_guess_and_tangent(pb, e, U)
    mu_b = wall_row(pb.mu, e, 0, pb.nx, pb.ny)
    lam_b = wall_row(pb.lam, e, 0, pb.nx, pb.ny)
    a, failed = newton_normal_column(pb.law, A, NA, tang, T, mu_b, lam_b, guess,
                                     pb.newton_max_iter, pb.newton_tol)
    return _assemble(A, a, tang), failed


def apply_walls(pb, fnew, fstar, U, t_half):
    """eq:boundary-general: f_d(t + dt) = D f*_{-d}(t) + S_d(t + dt/2) for every missing
    incoming direction d = -N at the wall nodes of each non-periodic edge.  Each missing
    link is rebuilt by its own edge's rule (reading for corner nodes, which the paper
    leaves to future work).  Returns a dict of per-edge F^b (traction edges)."""
    out = {}
    for e in range(4):
        edge = pb.edges[e]
        if edge.kind == "periodic":
            continue
        d = EDGE_MISSING[e]
        N = EDGE_NORMAL[e]
        L = pb.ny if EDGE_AXIS[e] == 0 else pb.nx
        outgoing = wall_row(fstar[OPP[d]], e, 0, pb.nx, pb.ny)          # (6, L)
        data = edge_values(edge, t_half, L)                              # (2, L)
        if edge.kind == "velocity":
            vD = data
            S = np.array([0.5 * vD[0], 0.5 * vD[1],
                          N[0] * vD[0] / pb.c, N[1] * vD[0] / pb.c,
                          N[0] * vD[1] / pb.c, N[1] * vD[1] / pb.c])
            val = D_DIRICHLET[:, None] * outgoing + S
        elif edge.kind == "traction":
            T = data
            Fb, failed = neumann_boundary_F(pb, e, U, T)
            S = np.array([T[0] / pb.c, T[1] / pb.c,
                          0.5 * Fb[0, 0], 0.5 * Fb[0, 1], 0.5 * Fb[1, 0], 0.5 * Fb[1, 1]])
            val = D_NEUMANN[:, None] * outgoing + S
            out[e] = (Fb, failed)
        else:
            raise ValueError(edge.kind)
        set_wall_row(fnew[d], e, val, pb.nx, pb.ny)
    return out


# ----------------------------------------------------------------------------- init

def fd_gradient(pb, g):
    """(d/dX g, d/dY g) by second-order differences; one-sided at non-periodic walls."""
    gx = fd_along(g, pb.periodic_x, pb.dx)
    gy = np.swapaxes(fd_along(np.swapaxes(g, -1, -2), pb.periodic_y, pb.dx), -1, -2)
    return gx, gy


def second_order_populations(pb, U0, dUdX, dUdY, B0):
    """eq:init-compact with eq:init-Zq-components, eq:init-deltaPq, eq:init-expanded:
    f_q(0) = f^eq(U0) - (dt/2) D_q f^eq(U0), D_q = d_t + c i d_X + c j d_Y, where the time
    derivative comes from the continuum system and d_alpha P = C(F0) : d_alpha F."""
    c, dt = pb.c, pb.dt
    F0 = F_of(U0)
    Cc = mat.tangent(pb.law, F0, pb.mu, pb.lam)
    feq, _ = equilibrium_of_state(pb, U0)
    dFX, dFY = F_of(dUdX), F_of(dUdY)
    dPX = np.einsum("iAkB...,kB...->iA...", Cc, dFX)
    dPY = np.einsum("iAkB...,kB...->iA...", Cc, dFY)
    f = np.empty((4, 6) + U0.shape[1:])
    for q, (i, j) in enumerate(DIRS):
        Z1 = B0[0] + dPX[0, 0] + dPY[0, 1] + c * (i * dUdX[0] + j * dUdY[0])
        Z2 = B0[1] + dPX[1, 0] + dPY[1, 1] + c * (i * dUdX[1] + j * dUdY[1])
        Z3 = dUdX[0] + c * (i * dFX[0, 0] + j * dFY[0, 0])
        Z4 = dUdY[0] + c * (i * dFX[0, 1] + j * dFY[0, 1])
        Z5 = dUdX[1] + c * (i * dFX[1, 0] + j * dFY[1, 0])
        Z6 = dUdY[1] + c * (i * dFX[1, 1] + j * dFY[1, 1])
        ZF = np.array([[Z3, Z4], [Z5, Z6]])
        dP = np.einsum("iAkB...,kB...->iA...", Cc, ZF)
        Dfeq = 0.25 * np.array([
            Z1 - (2.0 / c) * (i * dP[0, 0] + j * dP[0, 1]),
            Z2 - (2.0 / c) * (i * dP[1, 0] + j * dP[1, 1]),
            Z3 - (2.0 * i / c) * Z1,
            Z4 - (2.0 * j / c) * Z1,
            Z5 - (2.0 * i / c) * Z2,
            Z6 - (2.0 * j / c) * Z2,
        ])
        f[q] = feq[q] - 0.5 * dt * Dfeq
    return f


@dataclass
class State:
    f: np.ndarray          # pre-collision populations f^n, (4, 6, ny, nx)
    ustar: np.ndarray      # u*^n, (2, ny, nx)
    n: int = 0


def initial_state(pb, v0, u0=None, second_order=True, dU=None, F0=None):
    """Populations at t = 0 from v0 (2, ny, nx) and u0 (2, ny, nx) (Sec. 3.4): F0 = I + grad u0
    by finite differences unless F0 is given; derivatives by finite differences unless
    ``dU = (dU/dX, dU/dY)`` is given (manufactured solutions use analytic ones).
    u*^0 = u0 - (dt/2) v0 (eq:trapezoid-u)."""
    ny, nx = pb.ny, pb.nx
    v0 = np.asarray(v0, dtype=np.float64)
    u0 = np.zeros((2, ny, nx)) if u0 is None else np.asarray(u0, dtype=np.float64)
    if F0 is None:
        ux, uy = fd_gradient(pb, u0)
        F0 = np.array([[1.0 + ux[0], uy[0]], [ux[1], 1.0 + uy[1]]])
    U0 = np.array([v0[0], v0[1], F0[0, 0], F0[0, 1], F0[1, 0], F0[1, 1]])
    B0 = pb.B(0)
    if second_order:
        if dU is None:
            dUdX, dUdY = fd_gradient(pb, U0)
        else:
            dUdX, dUdY = dU
        f = second_order_populations(pb, U0, dUdX, dUdY, B0)
    else:
        f, _ = equilibrium_of_state(pb, U0)
    return State(f=f, ustar=u0 - 0.5 * pb.dt * v0, n=0)


# ----------------------------------------------------------------------------- step

def step(pb, st, record=None):
    """Sec. 3.7, steps 1-6, advancing level n to n + 1 in place.  Returns U^n and u^n."""
    n, dt = st.n, pb.dt
    B = pb.B(n)
    U = moments(st.f, B, dt)                                   # 1
    feq, P = equilibrium_of_state(pb, U)                       # 2, 3
    fstar = collide(st.f, feq, B, pb.omega, dt)                # 3
    v = U[0:2]
    u_n = st.ustar + 0.5 * dt * v                              # 6
    ustar_next = u_n + 0.5 * dt * v
    fnew = stream(pb, fstar)                                   # 4
    walls = apply_walls(pb, fnew, fstar, U, (n + 0.5) * dt)    # 5
    if record is not None:
        record.append(dict(n=n, U=U, fstar=fstar, walls=walls))
    if np.isnan(fnew).any():
        raise FloatingPointError("a missing link was not reconstructed")
    st.f, st.ustar, st.n = fnew, ustar_next, n + 1
    return U, u_n


def observe(pb, st):
    """U^n and u^n of the current level without stepping."""
    U = moments(st.f, pb.B(st.n), pb.dt)
    return U, st.ustar + 0.5 * pb.dt * U[0:2]


def post_collision(pb, st):
    """f*^n of the current level (what the library stores)."""
    B = pb.B(st.n)
    U = moments(st.f, B, pb.dt)
    feq, _ = equilibrium_of_state(pb, U)
    return collide(st.f, feq, B, pb.omega, pb.dt)


def run(pb, st, nsteps, record=None):
    for _ in range(nsteps):
        step(pb, st, record)
    return observe(pb, st)


def diagnostics(pb, U):
    """Total momentum, sum of F - I, elastic + kinetic energy, min J, max |F - I|_F."""
    F = F_of(U)
    W = mat.energy(pb.law, F, pb.mu, pb.lam)
    Ft = F.copy()
    Ft[0, 0] -= 1.0
    Ft[1, 1] -= 1.0
    kin = 0.5 * (U[0] ** 2 + U[1] ** 2)
    return dict(
        momentum=np.array([U[0].sum(), U[1].sum()]),
        sumFt=Ft.reshape(4, -1).sum(1),
        energy=float((kin + W).sum() * pb.dx * pb.dx),
        minJ=float(mat.det(F).min()),
        maxFt=float(np.sqrt((Ft * Ft).sum((0, 1))).max()),
    )
