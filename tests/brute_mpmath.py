"""Brute-force, per-link, arbitrary-precision implementation of the vectorial LBM for tiny
grids (Sec. 3 of the paper), used only to pin the numpy oracle.

It is written independently of ``oracle/`` in the most literal form: explicit loops over
nodes, directions and components, mpmath numbers at 40 significant digits, the tangent
C = dP/dF obtained by numerical differentiation of P at that precision (not from the
oracle's closed forms), a hand 2 x 2 solve for the boundary Newton iteration.  The readings
of the points the paper leaves open are the same as the oracle's (they are readings of
the paper, not of the oracle's code): tangential column of F^b = that of the wall node's
own F; Newton guess = the wall node's normal column; backtracking 1, 1/2, ..., 2^-10 with
det > 0 and decreasing |r|.
"""
import mpmath as mp

mp.mp.dps = 40
DIRS = [(1, 0), (0, 1), (-1, 0), (0, -1)]


def _det(F):
    return F[0][0] * F[1][1] - F[0][1] * F[1][0]


def piola(law, F, mu, lam):
    J = _det(F)
    if law in ("lognh", "nh"):
        H = [[F[1][1] / J, -F[1][0] / J], [-F[0][1] / J, F[0][0] / J]]
        vol = lam * mp.log(J) if law == "lognh" else lam / 2 * (J * J - 1)
        return [[mu * (F[i][A] - H[i][A]) + vol * H[i][A] for A in range(2)] for i in range(2)]
    # St. Venant-Kirchhoff
    C = [[sum(F[m][A] * F[m][B] for m in range(2)) for B in range(2)] for A in range(2)]
    E = [[(C[A][B] - (1 if A == B else 0)) / 2 for B in range(2)] for A in range(2)]
    trE = E[0][0] + E[1][1]
    S = [[2 * mu * E[A][B] + (lam * trE if A == B else 0) for B in range(2)] for A in range(2)]
    return [[sum(F[i][C_] * S[C_][A] for C_ in range(2)) for A in range(2)] for i in range(2)]


def tangent(law, F, mu, lam):
    """C[i][A][k][B] by central differences of P at 40 digits (step 1e-18)."""
    h = mp.mpf("1e-18")
    out = [[[[None] * 2 for _ in range(2)] for _ in range(2)] for _ in range(2)]
    for k in range(2):
        for B in range(2):
            Fp = [row[:] for row in F]
            Fm = [row[:] for row in F]
            Fp[k][B] += h
            Fm[k][B] -= h
            Pp, Pm = piola(law, Fp, mu, lam), piola(law, Fm, mu, lam)
            for i in range(2):
                for A in range(2):
                    out[i][A][k][B] = (Pp[i][A] - Pm[i][A]) / (2 * h)
    return out


def Fmat(U):
    return [[U[2], U[3]], [U[4], U[5]]]


def feq(U, P, c, i, j):
    PhiX = [-P[0][0], -P[1][0], -U[0], 0, -U[1], 0]
    PhiY = [-P[0][1], -P[1][1], 0, -U[0], 0, -U[1]]
    return [(U[k] + 2 / c * (i * PhiX[k] + j * PhiY[k])) / 4 for k in range(6)]


class Brute:
    def __init__(self, nx, ny, c, omega, law, mu, lam, dx, body, ramp, kinds, data):
        """mu, lam: [b][a] lists; body: [2][b][a]; kinds: 4 strings (xmin, xmax, ymin,
        ymax); data: 4 pairs (v_D or traction, constant in time and along the edge)."""
        self.nx, self.ny = nx, ny
        self.c, self.omega, self.law = mp.mpf(c), mp.mpf(omega), law
        self.dx = mp.mpf(dx)
        self.dt = self.dx / self.c
        self.mu = [[mp.mpf(x) for x in row] for row in mu]
        self.lam = [[mp.mpf(x) for x in row] for row in lam]
        self.body = [[[mp.mpf(x) for x in row] for row in comp] for comp in body]
        self.ramp = ramp
        self.kinds = kinds
        self.data = [[mp.mpf(x) for x in d] for d in data]
        self.px = kinds[0] == "periodic"
        self.py = kinds[2] == "periodic"

    def B(self, n, b, a):
        r = mp.mpf(self.ramp(n))
        return [r * self.body[0][b][a], r * self.body[1][b][a]]

    # --- finite differences along x or y with wrap or one-sided ends
    def d_dx(self, g, b, a):
        nx, h = self.nx, self.dx
        if self.px:
            return (g[b][(a + 1) % nx] - g[b][(a - 1) % nx]) / (2 * h)
        if a == 0:
            return (-3 * g[b][0] + 4 * g[b][1] - g[b][2]) / (2 * h)
        if a == nx - 1:
            return (3 * g[b][nx - 1] - 4 * g[b][nx - 2] + g[b][nx - 3]) / (2 * h)
        return (g[b][a + 1] - g[b][a - 1]) / (2 * h)

    def d_dy(self, g, b, a):
        ny, h = self.ny, self.dx
        if self.py:
            return (g[(b + 1) % ny][a] - g[(b - 1) % ny][a]) / (2 * h)
        if b == 0:
            return (-3 * g[0][a] + 4 * g[1][a] - g[2][a]) / (2 * h)
        if b == ny - 1:
            return (3 * g[ny - 1][a] - 4 * g[ny - 2][a] + g[ny - 3][a]) / (2 * h)
        return (g[b + 1][a] - g[b - 1][a]) / (2 * h)

    def initialise(self, v0, u0):
        nx, ny, c, dt = self.nx, self.ny, self.c, self.dt
        u0m = [[[mp.mpf(u0[k][b][a]) for a in range(nx)] for b in range(ny)] for k in range(2)]
        v0m = [[[mp.mpf(v0[k][b][a]) for a in range(nx)] for b in range(ny)] for k in range(2)]
        # U0 = (v0, I + grad u0)
        U0 = [[[None] * nx for _ in range(ny)] for _ in range(6)]
        for b in range(ny):
            for a in range(nx):
                U0[0][b][a] = v0m[0][b][a]
                U0[1][b][a] = v0m[1][b][a]
                U0[2][b][a] = 1 + self.d_dx(u0m[0], b, a)
                U0[3][b][a] = self.d_dy(u0m[0], b, a)
                U0[4][b][a] = self.d_dx(u0m[1], b, a)
                U0[5][b][a] = 1 + self.d_dy(u0m[1], b, a)
        self.f = [[[[None] * nx for _ in range(ny)] for _ in range(6)] for _ in range(4)]
        for b in range(ny):
            for a in range(nx):
                U = [U0[k][b][a] for k in range(6)]
                dX = [self.d_dx(U0[k], b, a) for k in range(6)]
                dY = [self.d_dy(U0[k], b, a) for k in range(6)]
                mu, lam = self.mu[b][a], self.lam[b][a]
                F = Fmat(U)
                P = piola(self.law, F, mu, lam)
                Cc = tangent(self.law, F, mu, lam)
                dFX, dFY = Fmat(dX), Fmat(dY)
                dPX = [[sum(Cc[i][A][k][B_] * dFX[k][B_] for k in range(2) for B_ in range(2))
                        for A in range(2)] for i in range(2)]
                dPY = [[sum(Cc[i][A][k][B_] * dFY[k][B_] for k in range(2) for B_ in range(2))
                        for A in range(2)] for i in range(2)]
                B0 = self.B(0, b, a)
                for q, (i, j) in enumerate(DIRS):
                    Z = [B0[0] + dPX[0][0] + dPY[0][1] + c * (i * dX[0] + j * dY[0]),
                         B0[1] + dPX[1][0] + dPY[1][1] + c * (i * dX[1] + j * dY[1])]
                    for k in range(2):
                        for B_ in range(2):
                            dv = dX[k] if B_ == 0 else dY[k]
                            Z.append(dv + c * (i * dFX[k][B_] + j * dFY[k][B_]))
                    ZF = [[Z[2], Z[3]], [Z[4], Z[5]]]
                    dP = [[sum(Cc[ii][A][k][B_] * ZF[k][B_] for k in range(2) for B_ in range(2))
                           for A in range(2)] for ii in range(2)]
                    D = [Z[0] - 2 / c * (i * dP[0][0] + j * dP[0][1]),
                         Z[1] - 2 / c * (i * dP[1][0] + j * dP[1][1]),
                         Z[2] - 2 * i / c * Z[0], Z[3] - 2 * j / c * Z[0],
                         Z[4] - 2 * i / c * Z[1], Z[5] - 2 * j / c * Z[1]]
                    fe = feq(U, P, c, i, j)
                    for k in range(6):
                        self.f[q][k][b][a] = fe[k] - dt / 2 * D[k] / 4
        self.ustar = [[[u0m[k][b][a] - dt / 2 * v0m[k][b][a] for a in range(nx)]
                       for b in range(ny)] for k in range(2)]
        self.n = 0

    def moments(self, b, a):
        Bv = self.B(self.n, b, a)
        U = [sum(self.f[q][k][b][a] for q in range(4)) for k in range(6)]
        U[0] += self.dt / 2 * Bv[0]
        U[1] += self.dt / 2 * Bv[1]
        return U

    def step(self):
        nx, ny, c, om, dt = self.nx, self.ny, self.c, self.omega, self.dt
        Us = [[self.moments(b, a) for a in range(nx)] for b in range(ny)]
        fs = [[[[None] * nx for _ in range(ny)] for _ in range(6)] for _ in range(4)]
        for b in range(ny):
            for a in range(nx):
                U = Us[b][a]
                P = piola(self.law, Fmat(U), self.mu[b][a], self.lam[b][a])
                Bv = self.B(self.n, b, a)
                for q, (i, j) in enumerate(DIRS):
                    fe = feq(U, P, c, i, j)
                    for k in range(6):
                        src = dt * (2 - om) / 8 * Bv[k] if k < 2 else 0
                        fs[q][k][b][a] = self.f[q][k][b][a] + om * (fe[k] - self.f[q][k][b][a]) + src
                for k in range(2):
                    un = self.ustar[k][b][a] + dt / 2 * U[k]
                    self.ustar[k][b][a] = un + dt / 2 * U[k]
        t_half = (self.n + mp.mpf(1) / 2) * dt
        del t_half   # edge data are constant in time here
        fn = [[[[None] * nx for _ in range(ny)] for _ in range(6)] for _ in range(4)]
        for b in range(ny):
            for a in range(nx):
                for q, (i, j) in enumerate(DIRS):
                    sa, sb = a - i, b - j
                    if self.px:
                        sa %= nx
                    if self.py:
                        sb %= ny
                    if 0 <= sa < nx and 0 <= sb < ny:
                        for k in range(6):
                            fn[q][k][b][a] = fs[q][k][sb][sa]
                    else:
                        vals = self.wall_link(q, b, a, fs, Us)
                        for k in range(6):
                            fn[q][k][b][a] = vals[k]
        self.f = fn
        self.n += 1

    def wall_link(self, q, b, a, fs, Us):
        i, j = DIRS[q]
        N = (-i, -j)                          # missing incoming d = -N
        e = {(-1, 0): 0, (1, 0): 1, (0, -1): 2, (0, 1): 3}[N]
        kind = self.kinds[e]
        opp = DIRS.index(N)
        out = [fs[opp][k][b][a] for k in range(6)]
        c = self.c
        w = self.data[e]
        if kind == "velocity":
            S = [w[0] / 2, w[1] / 2, N[0] * w[0] / c, N[1] * w[0] / c, N[0] * w[1] / c, N[1] * w[1] / c]
            Dg = [-1, -1, 1, 1, 1, 1]
            return [Dg[k] * out[k] + S[k] for k in range(6)]
        assert kind == "traction"
        Fb = self.boundary_F(e, b, a, Us, w)
        S = [w[0] / c, w[1] / c, Fb[0][0] / 2, Fb[0][1] / 2, Fb[1][0] / 2, Fb[1][1] / 2]
        Dg = [1, 1, -1, -1, -1, -1]
        return [Dg[k] * out[k] + S[k] for k in range(6)]

    def boundary_F(self, e, b, a, Us, T):
        A = 0 if e in (0, 1) else 1
        Bx = 1 - A
        NA = -1 if e in (0, 2) else 1
        # the wall node's own F: tangential column kept, normal column the Newton guess
        F0 = Fmat(Us[b][a])
        tang = [F0[k][Bx] for k in range(2)]
        acol = [F0[k][A] for k in range(2)]
        mu, lam = self.mu[b][a], self.lam[b][a]

        def build(ac):
            F = [[None, None], [None, None]]
            for k in range(2):
                F[k][A] = ac[k]
                F[k][Bx] = tang[k]
            return F

        def resid(ac):
            P = piola(self.law, build(ac), mu, lam)
            return [NA * P[k][A] - T[k] for k in range(2)]

        r = resid(acol)
        for _ in range(60):
            rn = mp.sqrt(r[0] ** 2 + r[1] ** 2)
            if rn <= mp.mpf("1e-32"):
                break
            Cc = tangent(self.law, build(acol), mu, lam)
            Jm = [[NA * Cc[ii][A][k][A] for k in range(2)] for ii in range(2)]
            dt_ = Jm[0][0] * Jm[1][1] - Jm[0][1] * Jm[1][0]
            d0 = -(Jm[1][1] * r[0] - Jm[0][1] * r[1]) / dt_
            d1 = -(-Jm[1][0] * r[0] + Jm[0][0] * r[1]) / dt_
            alpha, accepted = mp.mpf(1), False
            for _ls in range(11):
                trial = [acol[0] + alpha * d0, acol[1] + alpha * d1]
                if _det(build(trial)) > 0:
                    rt = resid(trial)
                    if mp.sqrt(rt[0] ** 2 + rt[1] ** 2) < rn:
                        acol, r, accepted = trial, rt, True
                        break
                alpha /= 2
            if not accepted:
                break
        return build(acol)

    def state(self):
        """U (6, ny, nx), u (2, ny, nx) and f (4, 6, ny, nx) of the current level, as floats."""
        nx, ny = self.nx, self.ny
        U = [[[0.0] * nx for _ in range(ny)] for _ in range(6)]
        u = [[[0.0] * nx for _ in range(ny)] for _ in range(2)]
        for b in range(ny):
            for a in range(nx):
                m = self.moments(b, a)
                for k in range(6):
                    U[k][b][a] = float(m[k])
                for k in range(2):
                    u[k][b][a] = float(self.ustar[k][b][a] + self.dt / 2 * m[k])
        f = [[[[float(self.f[q][k][b][a]) for a in range(nx)] for b in range(ny)]
              for k in range(6)] for q in range(4)]
        return U, u, f
