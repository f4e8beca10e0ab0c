"""Second workloads of the paper on the GPU, checked against the oracle on the same
inputs: the finite-amplitude periodic shear wave (Sec. 5.3, an exact travelling wave of
both neo-Hookean laws) and the cantilever bending wave (Sec. 5.4: clamped left edge,
traction-free top and bottom, Ricker-pulse traction on the right edge with a corner
taper; run-only, the finite-element reference is not available).

Bars: F64 1e-10 and F32 1e-5 relative L2 against the oracle (F - I normalised by
max(|F - I|, |v| / c_p) as in test_gpu_forward).
"""
import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu


def _rel(a, b):
    return float(np.sqrt(((a - b) ** 2).sum() / (b ** 2).sum()))


def _errors(Ug, ug, Uo, uo, cp):
    Uo = Uo.copy()
    Uo[2] -= 1.0
    Uo[5] -= 1.0
    ft_norm = max(np.sqrt((Uo[2:] ** 2).sum()), np.sqrt((Uo[:2] ** 2).sum()) / cp)
    return (_rel(Ug[:2], Uo[:2]), float(np.sqrt(((Ug[2:] - Uo[2:]) ** 2).sum()) / ft_norm), _rel(ug, uo))


def _shear_wave_inputs(n, Ak, mu):
    k = 4 * np.pi
    A = Ak / k
    cs = np.sqrt(mu)
    X = np.broadcast_to(((np.arange(n) + 0.5) / n)[None, :], (n, n))
    u0 = np.zeros((2, n, n))
    u0[1] = A * np.sin(k * X)
    v0 = np.zeros((2, n, n))
    v0[1] = -A * cs * k * np.cos(k * X)
    return u0, v0, X, k, A, cs


@pytest.mark.parametrize("law", ["nh", "lognh"])
@pytest.mark.parametrize("storage,bar", [("f64", 1e-10), ("f32", 1e-5)])
def test_finite_shear_wave(law, storage, bar):
    """Sec. 5.3 with mu = 2, k = 4 pi, n = 80, c = 5, omega = 2, Ak = 0.5, one period; the
    library against the oracle (finite-difference initialisation on both sides), and the
    library's error against the exact wave is independent of the amplitude (the lattice
    dynamics on the J = 1 path is linear)."""
    from oracle import lbm
    from paper_2605_26677_amd.solver import Solver
    n, mu, lam, c = 80, 2.0, 1.0, 5.0
    steps = int(round((0.5 / np.sqrt(mu)) / (1.0 / n / c)))
    exact_err = {}
    for Ak in (0.2, 0.5):
        u0, v0, X, k, A, cs = _shear_wave_inputs(n, Ak, mu)
        sv = Solver(n, n, c=c, omega=2.0, dx=1.0 / n, material=law, storage=storage, mu=mu, lam=lam)
        sv.init(v0, u0)
        for m in range(steps):
            sv.step(m)
        U = sv.moments().cpu().numpy()
        u = sv.displacement().cpu().numpy()
        torch.cuda.synchronize()
        assert sv.faults() == 0
        t = steps / n / c
        v2 = -A * cs * k * np.cos(k * X - cs * k * t)
        exact_err[Ak] = _rel(U[1], v2)
        if Ak == 0.5:
            pb = lbm.Problem(nx=n, ny=n, c=c, omega=2.0, law=law, mu=mu, lam=lam, dx=1.0 / n)
            st = lbm.initial_state(pb, v0, u0)
            Uo, uo = lbm.run(pb, st, steps)
            ev, eF, eu = _errors(U, u, Uo, uo, np.sqrt(lam + 2 * mu))
            print(f"\n[shear wave {law} {storage}] v={ev:.2e} F-I={eF:.2e} u={eu:.2e} "
                  f"exact-wave error {exact_err}")
            assert ev <= bar and eF <= bar and eu <= bar
    if storage == "f64":
        assert abs(exact_err[0.2] - exact_err[0.5]) <= 1e-6 * exact_err[0.5]


@pytest.mark.parametrize("storage,bar", [("f64", 1e-10), ("f32", 1e-5)])
def test_cantilever_pulse(storage, bar):
    """Sec. 5.4 cantilever over the loading pulse (t = 3, 1200 steps)."""
    from oracle import cantilever as cv
    from oracle import lbm
    from paper_2605_26677_amd.solver import Solver
    pb = cv.problem()
    steps = 1200
    st = lbm.initial_state(pb, np.zeros((2, cv.NY, cv.NX)))
    Uo, uo = lbm.run(pb, st, steps)
    sv = Solver(cv.NX, cv.NY, c=cv.C, omega=cv.OMEGA, dx=pb.dx, material="nh", storage=storage, mu=cv.MU,
                lam=cv.LAM, bc=("velocity", "traction", "traction", "traction"))
    sv.init(np.zeros((2, cv.NY, cv.NX)))
    w = cv.taper()
    dev = sv.device
    for m in range(steps):
        T = torch.tensor(np.array([np.zeros(cv.NY), cv.ricker((m + 0.5) * pb.dt) * w]), dtype=torch.float64,
                         device=dev)
        sv.step(m, edges=[(0, 0), T, (0, 0), (0, 0)])
    U = sv.moments().cpu().numpy()
    u = sv.displacement().cpu().numpy()
    torch.cuda.synchronize()
    assert sv.faults() == 0
    ev, eF, eu = _errors(U, u, Uo, uo, np.sqrt(cv.LAM + 2 * cv.MU))
    print(f"\n[cantilever {storage}] v={ev:.2e} F-I={eF:.2e} u={eu:.2e} max|u|={np.abs(uo).max():.3e}")
    assert ev <= bar and eF <= bar and eu <= bar
    from gpu_cases import WALL_BAR, shifted_state, wall_line_errors
    we = wall_line_errors(U, u, shifted_state(Uo), uo, ("velocity",) * 4)
    print(f"[cantilever {storage}] wall lines: " + " ".join(f"{k}={v:.2e}" for k, v in we.items()))
    assert max(we.values()) <= WALL_BAR[storage], we


@pytest.mark.parametrize("storage", ["f64", "f32"])
def test_cantilever_printed_values(storage):
    """The library's own run of the Sec. 5.4 cantilever to t = 12 (4800 steps) reproduces
    the printed J range, largest |u_y| on the loaded end and largest |u| over the beam, each
    at the printed number of decimals (tests/golden/cantilever_t12.txt)."""
    import os
    from oracle import cantilever as cv
    from paper_2605_26677_amd.solver import Solver
    want = {}
    with open(os.path.join(os.path.dirname(__file__), "golden", "cantilever_t12.txt")) as fh:
        for line in fh:
            if line.strip() and not line.startswith("#"):
                key, val, dec = line.split()
                want[key] = (float(val), int(dec))
    pb = cv.problem()
    sv = Solver(cv.NX, cv.NY, c=cv.C, omega=cv.OMEGA, dx=pb.dx, material="nh", storage=storage, mu=cv.MU,
                lam=cv.LAM, bc=("velocity", "traction", "traction", "traction"))
    sv.init(np.zeros((2, cv.NY, cv.NX)))
    w = cv.taper()
    dev = sv.device
    steps = int(round(12.0 / pb.dt))
    zero = torch.zeros((2, cv.NY), dtype=torch.float64, device=dev)
    for m in range(steps):
        p = cv.ricker((m + 0.5) * pb.dt)
        T = torch.tensor(np.array([np.zeros(cv.NY), p * w]), dtype=torch.float64, device=dev) if p != 0.0 else zero
        sv.step(m, edges=[(0, 0), T, (0, 0), (0, 0)])
    U = sv.moments().cpu().numpy()
    u = sv.displacement().cpu().numpy()
    torch.cuda.synchronize()
    assert sv.faults() == 0
    J = (1 + U[2]) * (1 + U[5]) - U[3] * U[4]
    got = dict(J_min=J.min(), J_max=J.max(), tip=np.abs(u[1, :, -1]).max(), umag=np.sqrt((u ** 2).sum(0)).max())
    print(f"\n[cantilever t=12 {storage}] " + " ".join(f"{k}={v:.5e}" for k, v in got.items()))
    for key, (val, dec) in want.items():
        assert round(float(got[key]), dec) == pytest.approx(val, abs=1e-12), (key, got[key], val)
