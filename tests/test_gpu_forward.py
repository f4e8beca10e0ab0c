"""Parity of the HIP forward path (lbm_init, lbm_step, lbm_moments, lbm_displacement,
lbm_diagnostics) with the FP64 oracle on the same seeded inputs.

On grids with walls every case also checks the wall line and the first interior line of
each wall edge element by element: max |GPU - oracle| over those lines, divided by the
largest oracle value of that quantity, at most 1e-10 (F64), 3e-5 (F32), 5e-2 (F16).

Bars (relative L2 over all nodes and components):
  F64 plain storage: 1e-10 on v, F - I, u and the populations (both sides carry the
      unshifted F in FP64; the bound allows ~1e-16 rounding per operation on O(1) values
      relative to |F - I| ~ 1e-4..1e-2 and its growth over the steps);
  F32 shifted storage: 1e-5 on v, F, F - I and u;
  F16 shifted storage: 2e-2 (measured and stated, see the test).
The F - I error is normalised by max(|F - I|, |v| / c_p), c_p = sqrt(lam + 2 mu): in an
elastic wave |F - I| ~ |v| / c_wave, and a standing wave passes through instants where
F - I is near zero while v carries the amplitude (the 64 x 64 shear wave is at half
period after 200 steps), where the plain relative error of F - I says nothing.
"""
import numpy as np
import pytest

import lbm_inputs as li
from gpu_cases import (ALL_LAWS, WALL_BAR, Case, block_case, mixed_case, random_field_case, rel_l2, run_library,
                       run_oracle, shear_wave_case, shifted_state, make_solver, wall_line_errors)

pytestmark = pytest.mark.gpu

BAR = {"f64": 1e-10, "f32": 1e-5, "f16": 2e-2}


def _compare(case, storage, report=None):
    Uo, uo, fo = run_oracle(case)
    sv, Ug, ug = run_library(case, storage)
    Uo_s = shifted_state(Uo)
    cp = np.sqrt(np.max(case.lam) + 2 * np.max(case.mu))
    ft_norm = max(np.sqrt((Uo_s[2:6] ** 2).sum()), np.sqrt((Uo_s[0:2] ** 2).sum()) / cp)
    Fg = Ug[2:6].copy()
    Fg[0] += 1.0
    Fg[3] += 1.0
    errs = dict(v=rel_l2(Ug[0:2], Uo_s[0:2]), F=rel_l2(Fg, Uo[2:6]),
                Ft=float(np.sqrt(((Ug[2:6] - Uo_s[2:6]) ** 2).sum()) / ft_norm), u=rel_l2(ug, uo))
    pops = sv.populations().double().cpu().numpy()
    ref = fo.copy()
    if storage != "f64":
        ref[:, 2] -= 0.25
        ref[:, 5] -= 0.25
    errs["pop"] = rel_l2(pops, ref)
    print(f"\n[{case.name} {storage}] rel L2: " + " ".join(f"{k}={v:.3e}" for k, v in errs.items()))
    assert sv.faults() == 0
    if any(k != "periodic" for k in case.kinds):
        we = wall_line_errors(Ug, ug, Uo_s, uo, case.kinds)
        print(f"[{case.name} {storage}] wall lines, max |err| / max |oracle|: "
              + " ".join(f"{k}={v:.3e}" for k, v in we.items()))
        assert max(we.values()) <= WALL_BAR[storage], we
    return errs


@pytest.mark.parametrize("storage", ["f64", "f32", "f16"])
def test_shear_wave_parity(storage):
    errs = _compare(shear_wave_case(), storage)
    bar = BAR[storage]
    assert errs["v"] <= bar and errs["Ft"] <= bar and errs["u"] <= bar and errs["F"] <= bar
    if storage == "f64":
        assert errs["pop"] <= bar


@pytest.mark.parametrize("law", ALL_LAWS)
@pytest.mark.parametrize("storage", ["f64", "f32"])
def test_random_field_parity(law, storage):
    """Periodic grid spanning several 256-wide tiles with a ragged tail (300 x 40)."""
    case = random_field_case(300, 40, 150, law=law)
    errs = _compare(case, storage)
    bar = BAR[storage]
    assert errs["v"] <= bar and errs["Ft"] <= bar and errs["u"] <= bar


@pytest.mark.parametrize("fields", [False, True])
@pytest.mark.parametrize("storage", ["f64", "f32"])
def test_block_with_walls_parity(fields, storage):
    """Velocity wall + traction-free walls + ramped body force, uniform and per-node
    parameters (the per-node path reads mu, lam and b from fields)."""
    errs = _compare(block_case(fields=fields), storage)
    bar = BAR[storage]
    assert errs["v"] <= bar and errs["Ft"] <= bar and errs["u"] <= bar


@pytest.mark.parametrize("law", ALL_LAWS)
@pytest.mark.parametrize("storage", ["f64", "f32"])
def test_mixed_edges_parity(law, storage):
    """Moving velocity walls and loaded traction walls, F0 = I + grad u0, corners."""
    errs = _compare(mixed_case(law=law), storage)
    bar = BAR[storage]
    assert errs["v"] <= bar and errs["Ft"] <= bar and errs["u"] <= bar


def test_ragged_wall_grid_parity():
    case = mixed_case(nx=259, ny=21, steps=60)
    errs = _compare(case, "f32")
    assert max(errs["v"], errs["Ft"], errs["u"]) <= BAR["f32"]


@pytest.mark.parametrize("storage", ["f64", "f32", "f16"])
@pytest.mark.parametrize("kinds", [("periodic",) * 4, ("velocity", "traction", "traction", "traction"),
                                   ("traction",) * 4, ("periodic", "periodic", "velocity", "traction")])
@pytest.mark.parametrize("law", ALL_LAWS)
def test_rest_state_bitwise(storage, kinds, law):
    """F0 = I, v0 = 0, b = 0, zero wall data: P(I) = 0 keeps every stored population exactly
    at its reference value (0 in shifted storage, U_ref/4 in plain)."""
    import torch
    case = Case("rest", 40, 24, 2.0, 1.9, 50, law=law, kinds=kinds, v0=np.zeros((2, 24, 40)))
    sv, U, u = run_library(case, storage)
    pops = sv.populations().double().cpu().numpy()
    ref = np.zeros((4, 6, 24, 40))
    if storage == "f64":
        ref[:, 2] = ref[:, 5] = 0.25
    assert np.array_equal(pops, ref)
    assert np.array_equal(U, np.zeros_like(U)) and np.array_equal(u, np.zeros_like(u))
    del torch


@pytest.mark.parametrize("storage", ["f64", "f32"])
def test_init_recovers_initial_state(storage):
    """After lbm_init the stored f*^0 gives back U0 = (v0, grad u0) (second-order init
    preserves the state exactly, then the collision preserves the moments)."""
    case = mixed_case()
    sv, U, u = run_library(case, storage, steps=0)
    from oracle import lbm
    from gpu_cases import oracle_problem
    pb = oracle_problem(case)
    ux, uy = lbm.fd_gradient(pb, case.u0)
    want = np.array([case.v0[0], case.v0[1], ux[0], uy[0], ux[1], uy[1]])
    tol = 1e-14 if storage == "f64" else 1e-6
    assert np.abs(U - want).max() <= tol * max(1.0, np.abs(want).max())
    assert np.abs(u - case.u0).max() <= tol * np.abs(case.u0).max() + 1e-15


@pytest.mark.parametrize("storage", ["f64", "f32"])
def test_momentum_conserved_fp64_reduction(storage):
    """Periodic, b = 0: sum_X v is conserved; the FP64 reduction of lbm_diagnostics sees it
    to 1e-6 of N v_rms in FP32 storage (1e-12 in FP64)."""
    import torch
    case = random_field_case(256, 256, 200)
    case.v0 = case.v0 + np.array([2e-3, -1e-3])[:, None, None]
    sv = make_solver(case, storage)
    sv.init(case.v0)
    d0 = sv.diagnostics().cpu().numpy()
    for n in range(case.steps):
        sv.step(n)
    d1 = sv.diagnostics().cpu().numpy()
    torch.cuda.synchronize()
    N = case.nx * case.ny
    vrms = np.sqrt((case.v0 ** 2).mean())
    tol = 1e-12 if storage == "f64" else 1e-6
    assert np.all(np.abs(d1[0:2] - d0[0:2]) <= tol * N * vrms)
    # oracle energy and extrema at level 200
    from oracle import lbm
    from gpu_cases import oracle_problem
    Uo, _, _ = run_oracle(case)
    do = lbm.diagnostics(oracle_problem(case), Uo)
    assert abs(d1[6] - do["energy"]) <= 1e-5 * do["energy"]
    assert abs(d1[7] - do["minJ"]) <= 1e-6
    assert abs(d1[8] - do["maxFt"]) <= 1e-5 * do["maxFt"]
    assert abs(d1[9] - np.sqrt(0.2 + 0.2) / 2.0) <= 2e-2


def test_cfl_refusal():
    from paper_2605_26677_amd import _lib as L
    case = shear_wave_case()
    case.c = 1.0
    sv = make_solver(case, "f32")
    with pytest.raises(L.LBMError) as ei:
        sv.init(case.v0)
    assert ei.value.status == L.LBM_ERR_CFL


def test_fault_bits_forced_from_host():
    import torch
    # non-finite initial velocity at one node
    case = shear_wave_case(steps=2)
    v0 = case.v0.copy()
    v0[0, 5, 7] = np.nan
    case.v0 = v0
    sv, _, _ = run_library(case, "f32")
    assert sv.faults() & 2
    # an inverted element: u0 with grad u = -2 gives det F0 < 0
    case = shear_wave_case(steps=1)
    u0 = np.zeros((2, 64, 64))
    u0[0, :, 10:13] = np.array([0.0, -2.0, -4.0])
    case.u0 = u0
    sv, _, _ = run_library(case, "f32")
    assert sv.faults() & 1
    # a traction solve cut to one Newton update against a large load
    from paper_2605_26677_amd.solver import Solver
    sv = Solver(16, 16, c=2.5, omega=1.9, storage="f32", bc=("velocity", "traction", "traction", "traction"),
                mu=0.1, lam=0.3, newton_max_iter=1)
    sv.init(np.zeros((2, 16, 16)))
    sv.step(0, edges=[(0, 0), (0.05, 0.02), (0, 0), (0, 0)])
    torch.cuda.synchronize()
    assert sv.faults() & 4


@pytest.mark.parametrize("storage,bar", [("f64", 1e-10), ("f32", 1e-5)])
@pytest.mark.parametrize("law", ["lognh", "nh", "svk"])
def test_stress_recovery(storage, bar, law):
    """lbm_stress: P(F) and sigma = J^-1 P F^T (Sec. 3.5) of the recovered state."""
    from oracle import material as mat
    case = mixed_case(law=law)
    Uo, _, _ = run_oracle(case)
    sv, _, _ = run_library(case, storage)
    P, S = (t.cpu().numpy() for t in sv.stress(case.ramp(case.steps)))
    F = np.array([[Uo[2], Uo[3]], [Uo[4], Uo[5]]])
    Pe = mat.stress(law, F, case.mu, case.lam)
    Se = mat.cauchy(law, F, case.mu, case.lam)
    eP = rel_l2(P, Pe)
    eS = rel_l2(S, Se)
    print(f"\n[stress {law} {storage}] P={eP:.2e} sigma={eS:.2e}")
    assert eP <= bar and eS <= bar


@pytest.mark.parametrize("kinds,storage", [(("periodic",) * 4, "f32"),
                                           (("velocity", "traction", "traction", "traction"), "f32"),
                                           (("velocity", "traction", "traction", "traction"), "f64")])
def test_step_graph_replays_match_eager(kinds, storage):
    """A captured block of steps replayed four times, with eager work (moments, a host
    synchronisation) between the replays, gives bitwise the eager result after every
    replay; ``advance`` (captured blocks plus an eager tail) matches too."""
    import torch
    from gpu_cases import block_case
    case = block_case(nx=96, ny=80, steps=0)
    case.kinds = kinds
    case.ramp_steps = 0
    data = [(0.0, 0.0), (1e-4, 0.0), (0.0, 0.0), (0.0, -1e-4)]
    eager = make_solver(case, storage)
    graph = make_solver(case, storage)
    for sv in (eager, graph):
        sv.init(case.v0, r0=1.0)
        for m in range(16):                    # also loads the kernels before any capture
            sv.step(m, edges=data)
    # a block of 16 levels: replays keep the phase of the 16-level displacement fold
    g = graph.capture([dict(n=m, edges=data) for m in range(16, 32)])
    for rep in range(4):
        for m in range(16 + 16 * rep, 32 + 16 * rep):
            eager.step(m, edges=data)
        g.replay()
        Ue, Ug = eager.moments(), graph.moments()
        torch.cuda.synchronize()
        assert torch.equal(Ue, Ug), rep
        assert torch.equal(eager.displacement(), graph.displacement())
    eager2 = make_solver(case, storage)
    adv = make_solver(case, storage)
    for sv in (eager2, adv):
        sv.init(case.v0, r0=1.0)
    for m in range(150):
        eager2.step(m, edges=data)
    adv.advance(0, 150, edges=lambda n: data, block=32, graph=True)
    assert torch.equal(eager2.moments(), adv.moments())
    assert eager2.faults() == 0 and adv.faults() == 0


# (F11, F12, F21, F22) of uniform states: J from 0.3 to 4 on both sides of the boundaries
# -1/4 and 1/2 of J - 1 where the FP32 ln(1 + (J - 1)) changes method, strains down to
# 1e-7, and a shear at J = 1
PIOLA_STATES = [(1 + 1e-7, 0.0, 0.0, 1.0), (1.0, 3e-6, 0.0, 1 - 2e-6), (1 + 1e-4, 2e-4, -1e-4, 1 - 3e-4),
                (1.05, 0.01, 0.02, 0.97), (1.2, 0.1, -0.05, 1.1), (0.9, 0.0, 0.0, 0.8334),
                (0.866, 0.0, 0.0, 0.866), (0.8661, 0.0, 0.0, 0.8661), (1.2247, 0.0, 0.0, 1.2247),
                (1.2248, 0.0, 0.0, 1.2248), (0.5, 0.1, 0.0, 0.6), (1.0, 0.5, 0.0, 1.0),
                (2.0, 0.3, 0.2, 2.0), (0.3, 0.0, 0.0, 1.0), (4.0, 0.0, 0.0, 1.0)]


@pytest.mark.parametrize("Fbar", PIOLA_STATES)
def test_piola_fp32_accuracy(Fbar):
    """The FP32 collision's first Piola stress (log-NH: mu (F - F^-T) + lam ln J F^-T, ln J by
    the kernels' own ln(1 + (J - 1))) within 8 units in the last place of its terms.  A
    uniform state, one step at omega = 1: the post-collision population of direction (1, 0)
    in the v1 row is U_v1 / 4 - P11 / (2c), and that of (0, 1) is U_v1 / 4 - P12 / (2c); the
    reference forms the step's moments from the stored level-0 populations in the kernel's
    FP32 order and P in FP64."""
    import torch
    c, mu, lam = 2.0, 0.1, 0.2
    n = 4
    case = Case("piola", n, n, c, 1.0, 1, mu=mu, lam=lam, v0=np.zeros((2, n, n)), force_unstable=True)
    sv = make_solver(case, "f32")
    sv.init(case.v0, Fbar=np.array(Fbar, dtype=np.float64).reshape(2, 2))
    f0 = sv.populations()[:, :, 0, 0].cpu().numpy()            # (4, 6) float32, uniform
    sv.step(0)
    f1 = sv.populations()[:, :, 0, 0].cpu().numpy().astype(np.float64)
    torch.cuda.synchronize()
    U = ((f0[0] + f0[1]) + f0[2]) + f0[3]                      # float32, q0 .. q3 in order
    t = U[2:6].astype(np.float64)
    F = np.array([[1 + t[0], t[1]], [t[2], 1 + t[3]]])
    J = np.linalg.det(F)
    H = np.linalg.inv(F).T
    P = mu * (F - H) + lam * np.log(J) * H
    cq = float(np.float32(1.0 / (2 * c)))                      # omega / (2c) as the kernel rounds it
    scale = cq * (mu * np.abs(F - H) + lam * abs(np.log(J)) * np.abs(H)).max() + 1e-30
    ulp = 2.0 ** -24
    exp = {(0, 0): U[0] / 4 - cq * P[0, 0], (1, 0): U[0] / 4 - cq * P[0, 1],
           (0, 1): U[1] / 4 - cq * P[1, 0], (1, 1): U[1] / 4 - cq * P[1, 1]}
    for (q, k), e in exp.items():
        err = abs(f1[q, k] - e) / scale
        assert err <= 8 * ulp, (Fbar, q, k, f1[q, k], e, err / ulp)
