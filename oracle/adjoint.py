"""Hand-written reverse sweep of the oracle's forward map, FP64.

Test infrastructure only (see the package docstring).

Forward map (notation of Sec. 3): f(0) = f^eq(U0) - (dt/2) D_q f^eq(U0) (eq:init-compact);
for levels m = 0, 1, ...: U^m = sum_q f^m_q + (dt/2) B^m (eq:moment-U),
f*^m = (1 - omega) f^m + omega f^eq(U^m) + dt (2 - omega) B^m / 8 (eq:collision),
f^{m+1}_q(X) = f*^m_q(X - c_q) or, on a missing link, D f*^m_{-q}(X) + S_q
(eq:streaming, eq:boundary-general).  Displacement by eq:trapezoid-u:
u^N = u0 - (dt/2) v0 + dt sum_{m<N} v^m + (dt/2) v^N.

Loss: L = sum_p |u^N(X_p) - u_target,p|^2 over probe cells.  The sweep returns dL/dmu,
dL/dlam (per cell), dL/db (per cell, for a fixed body field times a ramp) and dL/dv0.

Adjoint variables: lam^m = dL/df^m (pre-collision) and lam*^m = dL/df*^m.  With
g^m = dL/dU^m:
  g^m = omega sum_q (f^eq_q)'(U^m)^T lam*^m_q + (probe source) + (traction-wall source),
  lam^m_q = (1 - omega) lam*^m_q + g^m,
  lam*^m_q(X) = lam^{m+1}_q(X + c_q), or D lam^{m+1}_d(X) for the outgoing slot -d = N of
  a wall node (transposes of streaming and of eq:boundary-general).
(f^eq_q)'^T follows from eq:feq-derivative and the Jacobian actions of
eq:jacobian-actions, using the tangent of eq:stress-and-tangent.
"""
import numpy as np

from . import lbm
from . import material as mat


# ------------------------------------------------------------------ linear pieces

def AX_T(lam, Cc):
    """A_X^T lam: A_X dU = (-dP11, -dP21, -dv1, 0, -dv2, 0) with dP = C : dF."""
    M = -(lam[0] * Cc[0, 0] + lam[1] * Cc[1, 0])              # (2, 2, ...) over (k, B)
    return np.array([-lam[2], -lam[4], M[0, 0], M[0, 1], M[1, 0], M[1, 1]])


def AY_T(lam, Cc):
    """A_Y^T lam: A_Y dU = (-dP12, -dP22, 0, -dv1, 0, -dv2)."""
    M = -(lam[0] * Cc[0, 1] + lam[1] * Cc[1, 1])
    return np.array([-lam[3], -lam[5], M[0, 0], M[0, 1], M[1, 0], M[1, 1]])


def feq_prime_T_sum(lstar, Cc, c):
    """sum_q (f^eq_q)'(U)^T lstar_q = 1/4 [sum_q l_q + (2/c)(A_X^T (l_0 - l_2) + A_Y^T (l_1 - l_3))]."""
    s = lstar[0] + lstar[1] + lstar[2] + lstar[3]
    dxl = lstar[0] - lstar[2]
    dyl = lstar[1] - lstar[3]
    return 0.25 * (s + (2.0 / c) * (AX_T(dxl, Cc) + AY_T(dyl, Cc)))


def feq_param_T(lstar, Pp, c):
    """sum_q lstar_q . d f^eq_q / dp for a parameter p with dP/dp = Pp."""
    dxl = lstar[0] - lstar[2]
    dyl = lstar[1] - lstar[3]
    return (0.5 / c) * -(dxl[0] * Pp[0, 0] + dxl[1] * Pp[1, 0] + dyl[0] * Pp[0, 1] + dyl[1] * Pp[1, 1])


def fd_along_T(gbar, periodic, h):
    """Transpose of lbm.fd_along (along the last axis)."""
    if periodic:
        return (np.roll(gbar, 1, axis=-1) - np.roll(gbar, -1, axis=-1)) / (2.0 * h)
    out = np.zeros_like(gbar)
    s = gbar / (2.0 * h)
    out[..., 2:] += s[..., 1:-1]
    out[..., :-2] -= s[..., 1:-1]
    out[..., 0] += -3.0 * s[..., 0]
    out[..., 1] += 4.0 * s[..., 0]
    out[..., 2] += -1.0 * s[..., 0]
    out[..., -1] += 3.0 * s[..., -1]
    out[..., -2] += -4.0 * s[..., -1]
    out[..., -3] += 1.0 * s[..., -1]
    return out


def fd_gradient_T(pb, gx_bar, gy_bar):
    out = fd_along_T(gx_bar, pb.periodic_x, pb.dx)
    out += np.swapaxes(fd_along_T(np.swapaxes(gy_bar, -1, -2), pb.periodic_y, pb.dx), -1, -2)
    return out


def stream_T(pb, lam_next):
    """lam*_q(X) = lam_q(X + c_q); slots whose partner lies beyond a wall are NaN here and
    are filled by the wall transposes."""
    out = np.full_like(lam_next, np.nan)
    for q, (i, j) in enumerate(lbm.DIRS):
        src = lam_next[q]
        if i != 0:
            if pb.periodic_x:
                out[q] = np.roll(src, -i, axis=-1)
            elif i == 1:
                out[q][..., :-1] = src[..., 1:]
            else:
                out[q][..., 1:] = src[..., :-1]
        else:
            if pb.periodic_y:
                out[q] = np.roll(src, -j, axis=-2)
            elif j == 1:
                out[q][..., :-1, :] = src[..., 1:, :]
            else:
                out[q][..., 1:, :] = src[..., :-1, :]
    return out


def _add_wall_row(arr, e, row, vals, nx, ny):
    if e == lbm.XMIN:
        arr[..., :, row] += vals
    elif e == lbm.XMAX:
        arr[..., :, nx - 1 - row] += vals
    elif e == lbm.YMIN:
        arr[..., row, :] += vals
    else:
        arr[..., ny - 1 - row, :] += vals


def walls_T(pb, lstar, lam_next, U, g_mu, g_lam, t_half):
    """Wall transposes for the step m -> m + 1.  Fills the outgoing slots of lstar and
    returns the traction-wall source E = dL/dU^m through F^b (Sec. 3.6: its tangential
    column is the wall node's F, its normal column solves P(F^b) N = T and is
    differentiated by the implicit function theorem)."""
    nx, ny = pb.nx, pb.ny
    E = np.zeros((6, ny, nx))
    for e in range(4):
        edge = pb.edges[e]
        if edge.kind == "periodic":
            continue
        d = lbm.EDGE_MISSING[e]
        ell = lbm.wall_row(lam_next[d], e, 0, nx, ny)                       # (6, L)
        D = lbm.D_DIRICHLET if edge.kind == "velocity" else lbm.D_NEUMANN
        od = lbm.OPP[d]
        cur = lbm.wall_row(lstar[od], e, 0, nx, ny)
        if not np.isnan(cur).all():
            raise AssertionError("outgoing wall slot already filled")
        lbm.set_wall_row(lstar[od], e, D[:, None] * ell, nx, ny)
        if edge.kind != "traction":
            continue
        A = lbm.EDGE_AXIS[e]
        Bax = 1 - A
        NA = float(lbm.EDGE_NORMAL[e][A])
        L = ell.shape[-1]
        T = lbm.edge_values(edge, t_half, L)
        Fb, _ = lbm.neumann_boundary_F(pb, e, U, T)
        mu_b = lbm.wall_row(pb.mu, e, 0, nx, ny)
        lam_b = lbm.wall_row(pb.lam, e, 0, nx, ny)
        Fbar = 0.5 * np.array([[ell[2], ell[3]], [ell[4], ell[5]]])       # dL/dF^b
        abar = Fbar[:, A]
        Cc = mat.tangent(pb.law, Fb, mu_b, lam_b)
        Jm = NA * Cc[:, A, :, A]                                            # J_ik
        JT = np.array([[Jm[0, 0], Jm[1, 0]], [Jm[0, 1], Jm[1, 1]]])
        y = lbm._solve2(JT, abar)                                           # J^{-T} abar
        tbar = Fbar[:, Bax] - NA * np.einsum("i...,ij...->j...", y, Cc[:, A, :, Bax])
        Pm, Pl = mat.stress_parameter_partials(pb.law, Fb)
        _add_wall_row(g_mu, e, 0, -NA * (y[0] * Pm[0, A] + y[1] * Pm[1, A]), nx, ny)
        _add_wall_row(g_lam, e, 0, -NA * (y[0] * Pl[0, A] + y[1] * Pl[1, A]), nx, ny)
        # F^b's tangential column is the wall node's own (reading of Sec. 3.6); the normal
        # column is the Newton root, which depends on it only through the traction equations
        for k in range(2):
            _add_wall_row(E[2 + 2 * k + Bax], e, 0, tbar[k], nx, ny)
    return E


# ------------------------------------------------------------------ init transpose

def init_T(pb, U0, dUdX, dUdY, lam0, g_mu, g_lam):
    """Transpose of lbm.second_order_populations with respect to v0 (through U0 and its
    finite-difference gradient), mu, lam and the body force B0.  F0 is held fixed.
    Returns (dL/dv0, dL/dB0)."""
    c, dt = pb.c, pb.dt
    F0 = lbm.F_of(U0)
    Cc = mat.tangent(pb.law, F0, pb.mu, pb.lam)
    Cm, Cl = mat.tangent_parameter_partials(pb.law, F0)
    Pm, Pl = mat.stress_parameter_partials(pb.law, F0)
    dFX, dFY = lbm.F_of(dUdX), lbm.F_of(dUdY)
    shape = U0.shape[1:]
    v_bar = np.zeros((2,) + shape)
    vX_bar = np.zeros((2,) + shape)
    vY_bar = np.zeros((2,) + shape)
    B_bar = np.zeros((2,) + shape)
    dPX_bar = np.zeros((2, 2) + shape)
    dPY_bar = np.zeros((2, 2) + shape)
    for q, (i, j) in enumerate(lbm.DIRS):
        ell = lam0[q]
        # equilibrium part f^eq_q(U0)
        v_bar[0] += 0.25 * (ell[0] - (2.0 / c) * (i * ell[2] + j * ell[3]))
        v_bar[1] += 0.25 * (ell[1] - (2.0 / c) * (i * ell[4] + j * ell[5]))
        feq_p = (0.5 / c) * -(i * (ell[0] * Pm[0, 0] + ell[1] * Pm[1, 0])
                              + j * (ell[0] * Pm[0, 1] + ell[1] * Pm[1, 1]))
        feq_l = (0.5 / c) * -(i * (ell[0] * Pl[0, 0] + ell[1] * Pl[1, 0])
                              + j * (ell[0] * Pl[0, 1] + ell[1] * Pl[1, 1]))
        g_mu += feq_p
        g_lam += feq_l
        # correction part -(dt/2) D_q f^eq
        w = -0.5 * dt * ell
        Z1b = 0.25 * (w[0] - (2.0 * i / c) * w[2] - (2.0 * j / c) * w[3])
        Z2b = 0.25 * (w[1] - (2.0 * i / c) * w[4] - (2.0 * j / c) * w[5])
        dPb = np.array([[-(0.5 / c) * i * w[0], -(0.5 / c) * j * w[0]],
                        [-(0.5 / c) * i * w[1], -(0.5 / c) * j * w[1]]])
        ZFb = 0.25 * np.array([[w[2], w[3]], [w[4], w[5]]]) + np.einsum("iAkB...,iA...->kB...", Cc, dPb)
        # recompute Z_F for the parameter terms of dP = C : Z_F
        Z3 = dUdX[0] + c * (i * dFX[0, 0] + j * dFY[0, 0])
        Z4 = dUdY[0] + c * (i * dFX[0, 1] + j * dFY[0, 1])
        Z5 = dUdX[1] + c * (i * dFX[1, 0] + j * dFY[1, 0])
        Z6 = dUdY[1] + c * (i * dFX[1, 1] + j * dFY[1, 1])
        ZF = np.array([[Z3, Z4], [Z5, Z6]])
        g_mu += np.einsum("iA...,iA...->...", dPb, np.einsum("iAkB...,kB...->iA...", Cm, ZF))
        g_lam += np.einsum("iA...,iA...->...", dPb, np.einsum("iAkB...,kB...->iA...", Cl, ZF))
        # Z1 = B0_1 + dPX_11 + dPY_12 + c (i vX_1 + j vY_1), Z2 likewise
        B_bar[0] += Z1b
        B_bar[1] += Z2b
        dPX_bar[0, 0] += Z1b
        dPY_bar[0, 1] += Z1b
        dPX_bar[1, 0] += Z2b
        dPY_bar[1, 1] += Z2b
        vX_bar[0] += c * i * Z1b + ZFb[0, 0]
        vY_bar[0] += c * j * Z1b + ZFb[0, 1]
        vX_bar[1] += c * i * Z2b + ZFb[1, 0]
        vY_bar[1] += c * j * Z2b + ZFb[1, 1]
    # d_alpha P = C : d_alpha F0 with F0 fixed: only the parameter dependence of C
    g_mu += np.einsum("iA...,iA...->...", dPX_bar, np.einsum("iAkB...,kB...->iA...", Cm, dFX))
    g_mu += np.einsum("iA...,iA...->...", dPY_bar, np.einsum("iAkB...,kB...->iA...", Cm, dFY))
    g_lam += np.einsum("iA...,iA...->...", dPX_bar, np.einsum("iAkB...,kB...->iA...", Cl, dFX))
    g_lam += np.einsum("iA...,iA...->...", dPY_bar, np.einsum("iAkB...,kB...->iA...", Cl, dFY))
    v_bar += fd_gradient_T(pb, vX_bar, vY_bar)
    return v_bar, B_bar


# ------------------------------------------------------------------ driver

def initial_U(pb, v0, u0=None):
    """U0 = (v0, I + grad u0) exactly as lbm.initial_state builds it."""
    u0 = np.zeros((2, pb.ny, pb.nx)) if u0 is None else np.asarray(u0, dtype=np.float64)
    ux, uy = lbm.fd_gradient(pb, u0)
    return np.array([v0[0], v0[1], 1.0 + ux[0], uy[0], ux[1], 1.0 + uy[1]])


def forward(pb, v0, nsteps, u0=None):
    """Run the forward map and keep U^m for m = 0..N.  Returns (Us, u^N, state)."""
    st = lbm.initial_state(pb, v0, u0)
    Us = []
    for _ in range(nsteps):
        U, _u = lbm.step(pb, st)
        Us.append(U)
    UN, uN = lbm.observe(pb, st)
    Us.append(UN)
    return Us, uN, st


def probe_loss(uN, probes, target):
    ys, xs = probes
    diff = uN[:, ys, xs] - target
    return float((diff * diff).sum()), 2.0 * diff


def gradients(pb, v0, nsteps, probes, target, u0=None):
    """Loss and its gradients (dict with 'mu', 'lam', 'body', 'v0') for a problem whose
    body force is a fixed field times pb.ramp (or None)."""
    if callable(pb.body):
        raise ValueError("gradients need a fixed body field times a ramp")
    Us, uN, _ = forward(pb, v0, nsteps, u0)
    L, ubar = probe_loss(uN, probes, target)
    N = nsteps
    nx, ny, c, dt, om = pb.nx, pb.ny, pb.c, pb.dt, pb.omega
    ys, xs = probes
    g_mu = np.zeros((ny, nx))
    g_lam = np.zeros((ny, nx))
    g_b = np.zeros((2, ny, nx))
    lam_next = None
    for m in range(N, -1, -1):
        U = Us[m]
        F = lbm.F_of(U)
        Cc = mat.tangent(pb.law, F, pb.mu, pb.lam)
        if m == N:
            lstar = np.zeros((4, 6, ny, nx))
            E = 0.0
        else:
            lstar = stream_T(pb, lam_next)
            E = walls_T(pb, lstar, lam_next, U, g_mu, g_lam, (m + 0.5) * dt)
            if np.isnan(lstar).any():
                raise AssertionError("unfilled adjoint slot")
        src = np.zeros((6, ny, nx))
        wgt = 0.5 if m == N else 1.0
        np.add.at(src[0], (ys, xs), dt * wgt * ubar[0])
        np.add.at(src[1], (ys, xs), dt * wgt * ubar[1])
        gU = om * feq_prime_T_sum(lstar, Cc, c) + src + E
        Pm, Pl = mat.stress_parameter_partials(pb.law, F)
        g_mu += om * feq_param_T(lstar, Pm, c)
        g_lam += om * feq_param_T(lstar, Pl, c)
        r = 1.0 if pb.ramp is None else float(pb.ramp(m))
        lsum_v = lstar[:, 0:2].sum(0)
        g_b += r * (0.5 * dt * gU[0:2] + dt * (2.0 - om) * 0.125 * lsum_v)
        lam_next = (1.0 - om) * lstar + gU[None]
    # init: lam_next is dL/df(0)
    U0 = initial_U(pb, v0, u0)
    dUdX, dUdY = lbm.fd_gradient(pb, U0)
    g_v0, B_bar = init_T(pb, U0, dUdX, dUdY, lam_next, g_mu, g_lam)
    r0 = 1.0 if pb.ramp is None else float(pb.ramp(0))
    g_b += r0 * B_bar
    np.add.at(g_v0[0], (ys, xs), -0.5 * dt * ubar[0])
    np.add.at(g_v0[1], (ys, xs), -0.5 * dt * ubar[1])
    return L, dict(mu=g_mu, lam=g_lam, body=g_b, v0=g_v0)


def loss_only(pb, v0, nsteps, probes, target, u0=None):
    _, uN, _ = forward(pb, v0, nsteps, u0)
    return probe_loss(uN, probes, target)[0]
