"""The six hyperelastic closures of Appendix A on the GPU: stress recovery at finite
strain, FP32 dynamics at tiny strain (the shifted evaluation must not cancel), the
affine-patch suite of Sec. 5.1 against its closed form and the predeformed acoustic
suite of Sec. 5.2 against the oracle and the acoustic-tensor speeds.

Bars: F64 1e-10 (stress 1e-12), F32 1e-5 relative L2 against the FP64 oracle; affine
patch 1e-12 (F64) and 1e-5 (F32) against the exact affine motion; acoustic phase speed
1e-9 (F64) and 2e-5 (F32) against the oracle's measured speed on the same inputs, and
5e-4 against the continuum acoustic-tensor speed (the paper's maximum is 2.18e-4).
"""
import numpy as np
import pytest
import torch

import lbm_inputs as li
from gpu_cases import ALL_LAWS, LAW_K, Case, oracle_law, rel_l2, run_library, run_oracle, shifted_state

pytestmark = pytest.mark.gpu


def _solver(law, storage, nx, ny, **kw):
    from paper_2605_26677_amd.solver import Solver
    return Solver(nx, ny, material=law, storage=storage, law_k=LAW_K.get(law), **kw)


@pytest.mark.parametrize("law", ALL_LAWS)
@pytest.mark.parametrize("storage,bar", [("f64", 1e-12), ("f32", 2e-6)])
def test_stress_recovery_finite_strain(law, storage, bar):
    """lbm_stress after lbm_init on F = I + grad u0 with |grad u0| ~ 0.2, against the
    oracle's P and sigma of its own initial state."""
    from oracle import lbm
    from oracle import material as mat
    nx, ny = 72, 40
    u0 = np.stack([li.gaussian_random_field(nx, ny, 21, 0.12), li.gaussian_random_field(nx, ny, 22, 0.12)])
    mu, lam = 0.5, 0.7
    sv = _solver(law, storage, nx, ny, c=8.0, omega=2.0, mu=mu, lam=lam)
    sv.init(np.zeros((2, ny, nx)), u0)
    P, sig = sv.stress()
    P, sig = P.cpu().numpy(), sig.cpu().numpy()
    torch.cuda.synchronize()
    assert sv.faults() == 0
    pb = lbm.Problem(nx=nx, ny=ny, c=8.0, omega=2.0, law=oracle_law(law), mu=mu, lam=lam)
    st = lbm.initial_state(pb, np.zeros((2, ny, nx)), u0)
    U, _ = lbm.observe(pb, st)
    F = lbm.F_of(U)
    Po = mat.stress(oracle_law(law), F, mu, lam)
    So = mat.cauchy(oracle_law(law), F, mu, lam)
    eP, eS = rel_l2(P, Po), rel_l2(sig, So)
    print(f"\n[stress {law} {storage}] |F-I| max {np.abs(U[2:] - [[[1]], [[0]], [[0]], [[1]]]).max():.2f} "
          f"P={eP:.2e} sigma={eS:.2e}")
    assert eP <= bar and eS <= bar


@pytest.mark.parametrize("law", ALL_LAWS)
def test_fp32_tiny_strain_dynamics(law):
    """Waves with strains ~1e-7: F - I is carried as the shift, and every closure is
    evaluated without subtracting O(1) quantities, so FP32 keeps ~1e-6 relative accuracy
    (an evaluation on the plain F would lose all digits at this amplitude)."""
    nx, ny = 96, 40
    v0 = np.stack([li.gaussian_random_field(nx, ny, 31, 3e-8), li.gaussian_random_field(nx, ny, 32, 3e-8)])
    case = Case(f"tiny_{law}", nx, ny, 2.0, 2.0, 100, law=law, v0=v0)
    Uo, uo, _ = run_oracle(case)
    sv, Ug, ug = run_library(case, "f32")
    Uo_s = shifted_state(Uo)
    ev, eF, eu = rel_l2(Ug[:2], Uo_s[:2]), rel_l2(Ug[2:], Uo_s[2:]), rel_l2(ug, uo)
    print(f"\n[tiny strain {law} f32] max|F-I|={np.abs(Uo_s[2:]).max():.1e} v={ev:.2e} F-I={eF:.2e} u={eu:.2e}")
    assert sv.faults() == 0
    assert ev <= 1e-5 and eF <= 1e-5 and eu <= 1e-5


@pytest.mark.parametrize("law", ALL_LAWS)
@pytest.mark.parametrize("storage,bar", [("f64", 1e-12), ("f32", 1e-5)])
def test_affine_patch(law, storage, bar):
    """Sec. 5.1: velocity walls carrying v = (F* - I) X / T, start from F = I with that
    velocity; at t = T the lattice holds F*, P(F*), sigma(F*) and u = (F* - I) X."""
    from oracle import affine
    from oracle import material as mat
    n = 20
    lawo = oracle_law(law)
    for path in affine.PATHS:
        Fs = affine.terminal_state(path)
        pb = affine.problem(n, lawo, Fs)
        sv = _solver(law, storage, n, n, c=pb.c, omega=pb.omega, dx=pb.dx, bc=("velocity",) * 4,
                     mu=affine.MU, lam=affine.LAM)
        sv.init(affine.initial_velocity(n, Fs))
        N = affine.steps(n)
        edges = [torch.tensor(e.data(0.0), dtype=torch.float64, device=sv.device) for e in pb.edges]
        for m in range(N):
            sv.step(m, 1.0, 1.0, edges=edges)
        U = sv.moments().cpu().numpy()
        u = sv.displacement().cpu().numpy()
        P, sig = sv.stress()
        P, sig = P.cpu().numpy(), sig.cpu().numpy()
        torch.cuda.synchronize()
        assert sv.faults() == 0
        X, Y = affine.grid(n)
        Fe = np.broadcast_to((Fs - np.eye(2)).reshape(4, 1, 1), (4, n, n))
        Pe = np.broadcast_to(mat.stress(lawo, Fs, affine.MU, affine.LAM)[:, :, None, None], (2, 2, n, n))
        Se = np.broadcast_to(mat.cauchy(lawo, Fs, affine.MU, affine.LAM)[:, :, None, None], (2, 2, n, n))
        ue = np.array([(Fs[0, 0] - 1.0) * X + Fs[0, 1] * Y, Fs[1, 0] * X + (Fs[1, 1] - 1.0) * Y])
        eF = float(np.sqrt(((U[2:] - Fe) ** 2).sum() / ((Fe + np.eye(2).reshape(4, 1, 1)) ** 2).sum()))
        errs = dict(F=eF, P=rel_l2(P, Pe), sigma=rel_l2(sig, Se), u=rel_l2(u, ue))
        print(f"\n[affine {law} {path} {storage}] " + " ".join(f"{k}={v:.2e}" for k, v in errs.items()))
        assert max(errs.values()) <= bar, (path, errs)


def _oracle_phase_speed(law, F0, branch, u0, nx, ny):
    """The oracle's phase speed on the library's inputs: F = F0 + grad u0 by the same
    second-order differences the library uses."""
    from oracle import acoustic, lbm
    pb = acoustic.problem(nx, ny, oracle_law(law))
    cs, V = acoustic.modes(oracle_law(law), F0)
    q = V[:, branch]
    v0, _, c_ac, _ = acoustic.initial_fields(nx, ny, oracle_law(law), F0, branch)
    gx, gy = lbm.fd_gradient(pb, u0)
    F = np.array([[F0[0, 0] + gx[0], F0[0, 1] + gy[0]], [F0[1, 0] + gx[1], F0[1, 1] + gy[1]]])
    st = lbm.initial_state(pb, v0, u0, F0=F)
    nsteps = int(round(1.0 / pb.dt))
    ph = [acoustic.phase(v0, q, nx)]
    for _ in range(nsteps):
        lbm.step(pb, st)
        U, _ = lbm.observe(pb, st)
        ph.append(acoustic.phase(U[:2], q, nx))
    return acoustic.phase_speed(ph, pb.dt), c_ac, q, v0


@pytest.mark.parametrize("law", ALL_LAWS)
@pytest.mark.parametrize("storage,bar", [("f64", 1e-9), ("f32", 2e-5)])
def test_predeformed_acoustic_speeds(law, storage, bar):
    """Sec. 5.2 on the GPU (80 x 80, c = 5, omega = 2, k = 2 pi, eps = 1e-4, n = (1, 0)),
    both predeformations and both branches."""
    from oracle import acoustic
    nx = ny = 80
    x = (np.arange(nx) + 0.5) / nx
    for name, F0 in acoustic.PREDEFORMATIONS.items():
        for branch in (0, 1):
            cs, V = acoustic.modes(oracle_law(law), F0)
            q = V[:, branch]
            u0 = acoustic.EPS * q[:, None, None] * np.broadcast_to(np.sin(acoustic.K * x)[None, :], (ny, nx))[None]
            c_or, c_ac, _, v0 = _oracle_phase_speed(law, F0, branch, u0[:, :4], nx, 4)
            v0f = np.broadcast_to(v0[:, :1], (2, ny, nx))
            sv = _solver(law, storage, nx, ny, c=5.0, omega=2.0, dx=1.0 / nx, mu=acoustic.MU, lam=acoustic.LAM)
            sv.init(v0f, u0, Fbar=F0)
            nsteps = int(round(1.0 / sv.dt))
            ph = [acoustic.phase(v0f, q, nx)]
            for m in range(nsteps):
                sv.step(m)
                ph.append(acoustic.phase(sv.moments()[:2].cpu().numpy(), q, nx))
            torch.cuda.synchronize()
            assert sv.faults() == 0
            c_gpu = acoustic.phase_speed(ph, sv.dt)
            d_or, d_ac = abs(c_gpu - c_or) / c_or, abs(c_gpu - c_ac) / c_ac
            print(f"\n[acoustic {law} {name} branch {branch} {storage}] c_ac={c_ac:.6f} c_gpu={c_gpu:.9f} "
                  f"vs oracle {d_or:.2e} vs acoustic tensor {d_ac:.2e}")
            assert d_or <= bar and d_ac <= 5e-4


def test_gent_locking_limit_is_reported():
    """A shear wave with max F21 = 0.3 has barI1 - 3 = 0.09 (J = 1): beyond a Gent limit
    J_m = 0.05 the state is inadmissible and fault bit 1 is raised (init and step); with
    J_m = 1 the same run is clean."""
    from paper_2605_26677_amd.solver import Solver
    n = 64
    k = 2 * np.pi / n
    x = np.arange(n) + 0.5
    u0 = np.zeros((2, n, n))
    u0[1] = np.broadcast_to((0.3 / k) * np.sin(k * x)[None, :], (n, n))
    for jm, expect in ((0.05, True), (1.0, False)):
        sv = Solver(n, n, c=4.0, omega=2.0, material="gent", storage="f32", mu=0.1, lam=0.2,
                    law_k=(jm, 0.0, 0.0))
        sv.init(np.zeros((2, n, n)), u0)
        sv.step(0)
        torch.cuda.synchronize()
        assert bool(sv.faults() & 1) == expect, (jm, sv.faults())


@pytest.mark.parametrize("law", ALL_LAWS)
@pytest.mark.parametrize("storage,bar", [("f64", 1e-11), ("f32", 1e-5)])
def test_diagnostics_at_finite_strain(law, storage, bar):
    """lbm_diagnostics on F = I + grad u0 with |F - I| ~ 0.2: sum of F - I, energy
    sum(|v|^2/2 + W(F)) dx^2, min J, max |F - I| and the tangent-speed audit
    max_X max_n sqrt(lam_max(Q(n; F))) / c over the same 180 one-degree directions,
    against the oracle."""
    from oracle import lbm
    from oracle import material as mat
    nx, ny = 72, 40
    mu, lam, c, dx = 0.5, 0.7, 8.0, 0.05
    # displacement in units of dx, so that |F - I| ~ 0.2 whatever the spacing
    u0 = dx * np.stack([li.gaussian_random_field(nx, ny, 21, 0.12), li.gaussian_random_field(nx, ny, 22, 0.12)])
    v0 = np.stack([li.gaussian_random_field(nx, ny, 23, 1e-2), li.gaussian_random_field(nx, ny, 24, 1e-2)])
    sv = _solver(law, storage, nx, ny, c=c, omega=2.0, dx=dx, mu=mu, lam=lam)
    sv.init(v0, u0)
    d = sv.diagnostics().cpu().numpy()
    torch.cuda.synchronize()
    pb = lbm.Problem(nx=nx, ny=ny, c=c, omega=2.0, law=oracle_law(law), mu=mu, lam=lam, dx=dx)
    st = lbm.initial_state(pb, v0, u0)
    U, _ = lbm.observe(pb, st)
    do = lbm.diagnostics(pb, U)
    F = lbm.F_of(U)
    audit = float(mat.max_tangent_speed(oracle_law(law), F, mu, lam, dtheta_deg=1.0).max()) / c
    rel = lambda a, b: abs(a - b) / abs(b)
    # sum of F - I of a periodic displacement vanishes up to rounding: compare it on the
    # scale of its terms (node count times max |F - I|)
    errs = dict(sumFt=float(np.abs(d[2:6] - do["sumFt"]).max() / (nx * ny * do["maxFt"])),
                energy=rel(d[6], do["energy"]), minJ=abs(d[7] - do["minJ"]), maxFt=rel(d[8], do["maxFt"]),
                audit=rel(d[9], audit))
    print(f"\n[diagnostics {law} {storage}] audit {d[9]:.6f} " + " ".join(f"{k}={v:.1e}" for k, v in errs.items()))
    assert max(errs.values()) <= bar, errs
