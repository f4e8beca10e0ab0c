"""Pins of the oracle's lattice algebra and step: exact identities and invariants."""
import numpy as np
import pytest

import lbm_inputs as li
from oracle import lbm
from oracle import material as mat


def random_state(rng, shape, strain=0.05):
    U = np.empty((6,) + shape)
    U[0:2] = 1e-2 * rng.standard_normal((2,) + shape)
    U[2:6] = strain * rng.standard_normal((4,) + shape)
    U[2] += 1.0
    U[5] += 1.0
    return U


@pytest.mark.parametrize("law", mat.LAWS)
def test_equilibrium_moments_and_pair_identities(law):
    """eq:equilibrium-moments (four vector constraints) and the pair identities
    f_d + f_-d = U/2, f_d - f_-d = d_A Phi_A / c (eq:appendix-pair-identities)."""
    rng = np.random.default_rng(5)
    U = random_state(rng, (7,))
    c = 2.3
    pb = lbm.Problem(nx=7, ny=1, c=c, omega=2.0, law=law, mu=0.3, lam=0.6)
    P = mat.stress(law, lbm.F_of(U), 0.3, 0.6)
    PhiX, PhiY = lbm.fluxes(U, P)
    f = lbm.equilibrium(U, PhiX, PhiY, c)
    del pb
    dirs = np.array(lbm.DIRS, dtype=float)
    assert np.allclose(f.sum(0), U, atol=1e-15)
    assert np.allclose(np.einsum("q,qk...->k...", c * dirs[:, 0], f), PhiX, atol=1e-15)
    assert np.allclose(np.einsum("q,qk...->k...", c * dirs[:, 1], f), PhiY, atol=1e-15)
    ghost = np.einsum("q,qk...->k...", c * c * (dirs[:, 0] ** 2 - dirs[:, 1] ** 2), f)
    assert np.allclose(ghost, 0.0, atol=1e-14)
    for d in range(4):
        od = lbm.OPP[d]
        i, j = lbm.DIRS[d]
        assert np.allclose(f[d] + f[od], 0.5 * U, atol=1e-15)
        assert np.allclose(f[d] - f[od], (i * PhiX + j * PhiY) / c, atol=1e-15)


@pytest.mark.parametrize("omega", [2.0, 1.9, 1.3])
def test_post_collision_moment_identity(omega):
    """Sum of eq:collision over q with sum_q w = 1/2: sum_q f* = U + (dt/2) B for any omega,
    so the state is recoverable from stored post-collision populations."""
    rng = np.random.default_rng(6)
    f = 0.25 * random_state(rng, (4, 5))[None] + 1e-3 * rng.standard_normal((4, 6, 4, 5))
    B = 1e-2 * rng.standard_normal((2, 4, 5))
    dt = 0.4
    pb = lbm.Problem(nx=5, ny=4, c=2.5, omega=omega, mu=0.2, lam=0.3)
    U = lbm.moments(f, B, dt)
    feq, _ = lbm.equilibrium_of_state(pb, U)
    fs = lbm.collide(f, feq, B, omega, dt)
    expect = U.copy()
    expect[0:2] += 0.5 * dt * B
    assert np.allclose(fs.sum(0), expect, atol=1e-15)


def _bounded(nx, ny, kinds, data=None, **kw):
    data = data or [np.zeros(2)] * 4
    edges = [lbm.Edge(k, (lambda t, d=d: np.asarray(d))) for k, d in zip(kinds, data)]
    return lbm.Problem(nx=nx, ny=ny, edges=edges, **kw)


@pytest.mark.parametrize("kinds", [
    ("periodic",) * 4,
    ("velocity", "traction", "traction", "traction"),
    ("traction",) * 4,
    ("velocity",) * 4,
])
def test_second_order_init_recovers_state(kinds):
    """Sum_q f_q(0) + (dt/2) B^0 = U0 exactly when the same finite differences feed the
    time derivative and the spatial terms of eq:init-Zq-components (sum of
    eq:init-expanded over q reproduces d_t U + d_X Phi_X + d_Y Phi_Y = B)."""
    rng = np.random.default_rng(7)
    nx, ny = 12, 9
    pb = _bounded(nx, ny, kinds, c=2.5, omega=1.95, mu=li.lognormal_field(nx, ny, 1, 0.1, 0.3, 4.0),
                  lam=0.3, body=li.uniform_body(nx, ny, (2e-3, -1e-3)), ramp=lambda n: 0.7)
    v0 = 1e-3 * rng.standard_normal((2, ny, nx))
    u0 = 1e-2 * rng.standard_normal((2, ny, nx))
    st = lbm.initial_state(pb, v0, u0)
    U, _ = lbm.observe(pb, st)
    ux, uy = lbm.fd_gradient(pb, u0)
    assert np.allclose(U[0:2], v0, atol=2e-17)
    assert np.allclose(U[2], 1 + ux[0], atol=4e-16)
    assert np.allclose(U[3], uy[0], atol=4e-16)
    assert np.allclose(U[4], ux[1], atol=4e-16)
    assert np.allclose(U[5], 1 + uy[1], atol=4e-16)


@pytest.mark.parametrize("kinds", [
    ("periodic",) * 4,
    ("velocity", "traction", "traction", "traction"),
    ("traction",) * 4,
    ("periodic", "periodic", "velocity", "traction"),
])
@pytest.mark.parametrize("law", mat.LAWS)
def test_rest_state_is_bitwise_invariant(kinds, law):
    """F0 = I, v0 = 0, b = 0 and zero boundary data: P(I) = 0 keeps every population
    exactly at its equilibrium value."""
    pb = _bounded(10, 8, kinds, c=2.0, omega=1.9, law=law, mu=0.1, lam=0.2)
    st = lbm.initial_state(pb, np.zeros((2, 8, 10)))
    f0 = st.f.copy()
    lbm.run(pb, st, 30)
    assert np.array_equal(st.f, f0)
    assert np.array_equal(st.ustar, np.zeros((2, 8, 10)))


def test_uniform_translation():
    """Constant v with F = I on a periodic grid is an exact solution: U stays constant and
    u^n = u0 + n dt v (eq:trapezoid-u)."""
    nx, ny = 9, 7
    pb = lbm.Problem(nx=nx, ny=ny, c=2.0, omega=2.0, mu=0.1, lam=0.2)
    v = np.array([3e-3, -2e-3])
    v0 = np.broadcast_to(v[:, None, None], (2, ny, nx)).copy()
    st = lbm.initial_state(pb, v0)
    U, u = lbm.run(pb, st, 50)
    assert np.allclose(U[0:2], v0, rtol=1e-14, atol=0)
    assert np.allclose(U[2:], np.array([1, 0, 0, 1.0])[:, None, None], atol=1e-15)
    assert np.allclose(u, 50 * pb.dt * v0, rtol=1e-13)


def test_periodic_momentum_and_mean_F_conserved():
    """Periodic streaming permutes populations and the source vanishes for b = 0, so
    sum_X v and sum_X F are conserved (shear-wave workload, 64 x 64, 200 steps)."""
    pb = lbm.Problem(nx=64, ny=64, c=2.0, omega=2.0, law="lognh", mu=0.1, lam=0.2)
    rng = np.random.default_rng(8)
    v0 = li.shear_wave_v0(64, 64) + 1e-4 * rng.standard_normal((2, 64, 64))
    st = lbm.initial_state(pb, v0)
    U0, _ = lbm.observe(pb, st)
    d0 = lbm.diagnostics(pb, U0)
    U, _ = lbm.run(pb, st, 200)
    d1 = lbm.diagnostics(pb, U)
    vrms = np.sqrt((v0 ** 2).mean())
    assert np.all(np.abs(d1["momentum"] - d0["momentum"]) <= 1e-13 * 64 * 64 * vrms)
    assert np.all(np.abs(d1["sumFt"] - d0["sumFt"]) <= 1e-10)


def test_energy_is_nearly_conserved_at_omega_two():
    """omega = 2 is the nondissipative setting (Sec. 3.3): the discrete elastic + kinetic
    energy of a small-amplitude wave drifts by far less than under omega = 1.5."""
    def drift(omega):
        pb = lbm.Problem(nx=32, ny=32, c=2.0, omega=omega, law="lognh", mu=0.1, lam=0.2)
        st = lbm.initial_state(pb, li.shear_wave_v0(32, 32))
        e0 = lbm.diagnostics(pb, lbm.observe(pb, st)[0])["energy"]
        U, _ = lbm.run(pb, st, 200)
        return abs(lbm.diagnostics(pb, U)["energy"] - e0) / e0
    assert drift(2.0) < 1e-3
    assert drift(1.5) > 10 * drift(2.0)


def test_prestressed_patch_is_steady():
    """A uniform predeformation F* with v = 0 held by matching nominal tractions
    T = P(F*) N on traction edges (and v_D = 0 on velocity edges) is an exact steady state:
    at a traction link f*_N,v = -P N / (2c) and the rule returns P N / (2c) = f^eq_{-N},
    the F rows return F* / 4 when F^b = F* (linear extrapolation of a constant is exact
    and the Newton solve recovers F*'s normal column)."""
    Fs = np.array([[1.08, 0.05], [-0.03, 0.94]])
    for law in mat.LAWS:
        mu, lam = 0.1, 0.3
        P = mat.stress(law, Fs, mu, lam)
        data = []
        kinds = ("velocity", "traction", "traction", "traction")
        for e, kind in enumerate(kinds):
            N = np.array(lbm.EDGE_NORMAL[e], dtype=float)
            data.append(np.zeros(2) if kind == "velocity" else P @ N)
        pb = _bounded(9, 7, kinds, data, c=2.5, omega=1.9, law=law, mu=mu, lam=lam)
        st = lbm.initial_state(pb, np.zeros((2, 7, 9)), F0=np.broadcast_to(Fs[:, :, None, None], (2, 2, 7, 9)))
        f0 = st.f.copy()
        lbm.run(pb, st, 40)
        assert np.abs(st.f - f0).max() <= 1e-14


def test_newton_solves_traction_equation():
    """The boundary Newton solve returns P(F^b) N = T with det F^b > 0 (Sec. 3.6), and on a
    case with a unique admissible root it agrees with a brute-force grid search."""
    law, mu, lam = "lognh", np.array([0.1, 0.1, 0.2]), np.array([0.3, 0.3, 0.1])
    A, NA = 0, 1.0
    tang = np.array([[0.02, 0.1, -0.05], [1.01, 0.95, 1.1]])
    T = np.array([[1e-3, 0.02, -0.01], [-2e-3, 0.01, 0.0]])
    guess = np.array([[1.0, 1.0, 1.0], [0.0, 0.0, 0.0]])
    a, failed = lbm.newton_normal_column(law, A, NA, tang, T, mu, lam, guess, 50, 1e-14)
    assert not failed.any()
    F = lbm._assemble(A, a, tang)
    P = mat.stress(law, F, mu, lam)
    assert np.abs(NA * P[:, A] - T).max() <= 1e-14
    assert (mat.det(F) > 0).all()
    # grid search for node 0
    g0 = np.linspace(0.8, 1.2, 401)
    g1 = np.linspace(-0.2, 0.2, 401)
    G0, G1 = np.meshgrid(g0, g1)
    Fg = np.empty((2, 2) + G0.shape)
    Fg[0, 0], Fg[1, 0] = G0, G1
    Fg[0, 1], Fg[1, 1] = tang[0, 0], tang[1, 0]
    ok = mat.det(Fg) > 0
    Pg = mat.stress(law, np.where(ok, Fg, np.eye(2)[:, :, None, None]), mu[0], lam[0])
    res = np.hypot(Pg[0, 0] - T[0, 0], Pg[1, 0] - T[1, 0])
    idx = np.unravel_index(np.argmin(np.where(ok, res, np.inf)), res.shape)
    assert abs(G0[idx] - a[0, 0]) <= 1e-3 and abs(G1[idx] - a[1, 0]) <= 1e-3


def test_walls_fill_every_missing_link():
    """After streaming, every entry whose source lies beyond a wall is rebuilt (the
    oracle's streaming leaves those entries NaN and raises if any survives)."""
    pb = _bounded(6, 5, ("velocity", "traction", "traction", "velocity"),
                  [np.array([1e-3, 0.0]), np.zeros(2), np.array([0.0, 1e-4]), np.zeros(2)],
                  c=2.5, omega=1.9, mu=0.1, lam=0.3)
    st = lbm.initial_state(pb, np.zeros((2, 5, 6)))
    lbm.run(pb, st, 5)
    assert np.isfinite(st.f).all()
