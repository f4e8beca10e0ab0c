"""Parity at the benchmark sizes.

8192 x 8192 periodic random-field workload, in the launch configuration bench.py times:
after k steps a node depends only on the nodes within k of it (one cell per step), so
sampled windows are checked against the oracle run on a small periodic window holding
the sample plus a margin of k + 2 nodes (the margin absorbs the wrong values that enter
from the window's artificial wrap).  Plus the FP64 momentum reduction at full size.

1024 x 1024 block (velocity wall left, traction-free elsewhere, ramped body force
(0, -1e-5) over 500 steps, log-NH mu = 0.1, lam = 0.3, c = 10, omega = 2 - 1.6/1024):
FP32 shifted and FP64 plain against the FP64 oracle after 1000 steps, on the oracle's
stored samples (tests/golden/block1024_samples.txt, written by make_block1024.py, which
calls only the oracle); FP32 against FP64 on the GPU after 20000 steps, where the block
has reached |F - I| of about 0.3.
"""
import os
import numpy as np
import pytest
import torch

import lbm_inputs as li

pytestmark = pytest.mark.gpu

N = 8192
STEPS = 16
WIN = 32
MARGIN = STEPS + 2


@pytest.fixture(scope="module")
def v0_full():
    return np.stack([li.gaussian_random_field(N, N, 301, 5e-3), li.gaussian_random_field(N, N, 302, 5e-3)])


def _oracle_window(v0, y0, x0, steps, law="lognh"):
    from oracle import lbm
    size = WIN + 2 * MARGIN
    ys = (np.arange(size) + y0 - MARGIN) % N
    xs = (np.arange(size) + x0 - MARGIN) % N
    vw = v0[:, ys][:, :, xs]
    pb = lbm.Problem(nx=size, ny=size, c=2.0, omega=2.0, law=law, mu=0.1, lam=0.2)
    st = lbm.initial_state(pb, vw)
    U, u = lbm.run(pb, st, steps)
    sl = slice(MARGIN, MARGIN + WIN)
    U = U[:, sl, sl].copy()
    U[2] -= 1.0
    U[5] -= 1.0
    return U, u[:, sl, sl]


@pytest.mark.parametrize("storage,bar,law", [("f32", 1e-5, "lognh"), ("f64", 1e-10, "lognh"),
                                            ("f32", 1e-5, "svk"), ("f16", 2e-2, "lognh")])
def test_fullsize_windows_match_oracle(v0_full, storage, bar, law):
    from paper_2605_26677_amd.solver import Solver
    sv = Solver(N, N, c=2.0, omega=2.0, material=law, storage=storage, mu=0.1, lam=0.2)
    sv.init(v0_full)
    d0 = sv.diagnostics().cpu().numpy()
    for k in range(STEPS):
        sv.step(k)
    U = sv.moments()
    u = sv.displacement()
    d1 = sv.diagnostics().cpu().numpy()
    torch.cuda.synchronize()
    assert sv.faults() == 0
    rng = np.random.default_rng(7)
    corners = [(0, 0), (N - WIN, N - WIN)] + [tuple(rng.integers(0, N - WIN, 2)) for _ in range(3)]
    cp = np.sqrt(0.2 + 2 * 0.1)
    for (y0, x0) in corners:
        Ug = U[:, y0:y0 + WIN, x0:x0 + WIN].cpu().numpy()
        ug = u[:, y0:y0 + WIN, x0:x0 + WIN].cpu().numpy()
        Uo, uo = _oracle_window(v0_full, y0, x0, STEPS, law)
        ev = np.sqrt(((Ug[:2] - Uo[:2]) ** 2).sum() / (Uo[:2] ** 2).sum())
        ft_norm = max(np.sqrt((Uo[2:] ** 2).sum()), np.sqrt((Uo[:2] ** 2).sum()) / cp)
        eF = np.sqrt(((Ug[2:] - Uo[2:]) ** 2).sum()) / ft_norm
        eu = np.sqrt(((ug - uo) ** 2).sum() / (uo ** 2).sum())
        print(f"\n[8192 window {law} {storage} at {y0},{x0}] v={ev:.2e} F-I={eF:.2e} u={eu:.2e}")
        assert ev <= bar and eF <= bar and eu <= bar
    # periodic, b = 0: total momentum is conserved (FP64 reduction over 67M nodes)
    vrms = np.sqrt((v0_full ** 2).mean())
    assert np.all(np.abs(d1[0:2] - d0[0:2]) <= (1e-12 if storage == "f64" else 1e-6) * N * N * vrms)


GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "block1024_samples.txt")


def _block_run(storage, steps):
    from paper_2605_26677_amd.solver import Solver
    n = 1024
    omega = 2.0 - 1.6 / n
    sv = Solver(n, n, c=10.0, omega=omega, material="lognh", storage=storage, mu=0.1, lam=0.3,
                body=(0.0, -1e-5), bc=("velocity", "traction", "traction", "traction"))
    ramp = lambda k: min(1.0, k / 500)
    sv.init(np.zeros((2, n, n)), r0=ramp(0))
    edges = [(0.0, 0.0)] * 4
    for k in range(steps):
        sv.step(k, ramp(k), ramp(k + 1), edges=edges)
    U = sv.moments(ramp(steps)).cpu().numpy()
    u = sv.displacement(ramp(steps)).cpu().numpy()
    torch.cuda.synchronize()
    assert sv.faults() == 0
    return U, u


def _rel(a, b):
    return float(np.sqrt(((a - b) ** 2).sum() / (b ** 2).sum()))


@pytest.mark.skipif(not os.path.exists(GOLDEN), reason="oracle samples not generated")
@pytest.mark.parametrize("storage,bar", [("f64", 1e-10), ("f32", 1e-5)])
def test_block_1024_against_oracle_samples(storage, bar):
    ref = np.loadtxt(GOLDEN)
    ys, xs = ref[:, 0].astype(int), ref[:, 1].astype(int)
    U, u = _block_run(storage, 1000)
    Ug = U[:, ys, xs].T
    ug = u[:, ys, xs].T
    ev, eF, eu = _rel(Ug[:, :2], ref[:, 2:4]), _rel(Ug[:, 2:6], ref[:, 4:8]), _rel(ug, ref[:, 8:10])
    print(f"\n[block 1024 {storage} vs oracle samples, 1000 steps] v={ev:.2e} F-I={eF:.2e} u={eu:.2e}")
    assert ev <= bar and eF <= bar and eu <= bar
    # element by element on the sampled wall lines and first interior lines (rows and
    # columns 0, 1, N-2, N-1), each scaled by the largest sampled oracle value
    N = 1024
    on_wall = (ys <= 1) | (ys >= N - 2) | (xs <= 1) | (xs >= N - 2)
    got = np.concatenate([Ug, ug], axis=1)[on_wall]
    want = ref[on_wall, 2:10]
    werr = {}
    for key, cols in (("v", slice(0, 2)), ("Ft", slice(2, 6)), ("u", slice(6, 8))):
        werr[key] = float(np.abs(got[:, cols] - want[:, cols]).max() / np.abs(ref[:, 2:10][:, cols]).max())
    print(f"[block 1024 {storage}] wall lines: " + " ".join(f"{k}={v:.2e}" for k, v in werr.items()))
    from gpu_cases import WALL_BAR
    assert max(werr.values()) <= WALL_BAR[storage], werr


def test_block_1024_fp32_against_fp64_20000_steps():
    """FP32 shifted storage against FP64 after 20000 steps, when the block has sagged to
    |F - I| of about 0.35.  The FP64 problem is well conditioned (a one-ulp relative change
    of b moves the FP64 result by the same 6e-8), but FP32 rounding of this slowly varying,
    quasi-static field repeats almost identically from step to step and acts as a
    persistent forcing, so the FP32 difference grows about linearly in time (5e-6 at 1000
    steps, 5e-5 at 5000, 1e-4 at 10000, 3e-4 at 20000), spread evenly over the interior,
    and is unchanged by a tighter Newton tolerance or an FP32-exact omega.  Bar: 1e-3."""
    U32, u32 = _block_run("f32", 20000)
    U64, u64 = _block_run("f64", 20000)
    ev, eF, eu = _rel(U32[:2], U64[:2]), _rel(U32[2:], U64[2:]), _rel(u32, u64)
    Ft = np.sqrt((U64[2:] ** 2).sum(0))
    print(f"\n[block 1024 f32 vs f64, 20000 steps] v={ev:.2e} F-I={eF:.2e} u={eu:.2e} max|F-I|={Ft.max():.3f}")
    assert ev <= 1e-3 and eF <= 1e-3 and eu <= 1e-3
    assert 0.2 <= Ft.max() <= 0.5


def test_periodic_1024_fp32_against_fp64_20000_steps():
    """Periodic random field (the throughput workload's recipe at 1024^2, c = 2, omega = 2):
    with no quasi-static drift the FP32 rounding behaves as noise and the difference to FP64
    grows like the square root of the step count (2.4e-6 at 1000 steps, 1.2e-5 at 20000).
    Bar: 3e-5 on v and F - I, 1e-5 on u."""
    from paper_2605_26677_amd.solver import Solver
    m = 1024
    v0 = np.stack([li.gaussian_random_field(m, m, 301, 5e-3), li.gaussian_random_field(m, m, 302, 5e-3)])
    res = {}
    for storage in ("f32", "f64"):
        sv = Solver(m, m, c=2.0, omega=2.0, material="lognh", storage=storage, mu=0.1, lam=0.2)
        sv.init(v0)
        for k in range(20000):
            sv.step(k)
        res[storage] = (sv.moments().cpu().numpy(), sv.displacement().cpu().numpy())
        assert sv.faults() == 0
    (U32, u32), (U64, u64) = res["f32"], res["f64"]
    ev, eF, eu = _rel(U32[:2], U64[:2]), _rel(U32[2:], U64[2:]), _rel(u32, u64)
    print(f"\n[periodic 1024 f32 vs f64, 20000 steps] v={ev:.2e} F-I={eF:.2e} u={eu:.2e}")
    assert ev <= 3e-5 and eF <= 3e-5 and eu <= 1e-5


def test_largest_fp32_grid_windows():
    """The largest FP32 grid one MI355X holds, ragged in x: 32700 x 32768 nodes
    (1.07e9; two population buffers of 103 GB, u* 17 GB), periodic, 16 steps.  Buffer
    offsets pass 2^32 elements, so every index of the step kernel must be 64-bit.  The
    stored populations of sampled windows (the corners, the ragged x wrap and random
    places) are read straight from the tiled buffers and compared with the oracle's
    post-collision populations on a periodic window with a k + 2 margin.  The initial
    velocity is a sum of three periodic plane waves (amplitude 5e-3), built on the
    device; the oracle takes the same values read back.  Bar: 1e-5 relative L2."""
    from oracle import lbm
    from paper_2605_26677_amd.solver import Solver
    nx, ny, steps, win = 32700, 32768, 16, 24
    margin = steps + 2
    dev = "cuda"
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    sv = Solver(nx, ny, c=2.0, omega=2.0, material="lognh", storage="f32", mu=0.1, lam=0.2)
    rng = np.random.default_rng(11)
    modes = [(int(rng.integers(1, 40)), int(rng.integers(1, 40)), float(rng.uniform(0, 2 * np.pi))) for _ in range(3)]

    def v0_block(ys, xs):
        Y, X = np.meshgrid(ys.astype(np.float64), xs.astype(np.float64), indexing="ij")
        out = np.zeros((2,) + Y.shape)
        for i, (kx, ky, ph) in enumerate(modes):
            w = 2 * np.pi * (kx * (X + 0.5) / nx + ky * (Y + 0.5) / ny) + ph
            out[i % 2] += 5e-3 * np.sin(w)
        return out

    v0 = torch.zeros((2, ny, nx), dtype=torch.float64, device=dev)
    X = torch.arange(nx, dtype=torch.float64, device=dev)[None, :]
    rows = 2048
    for y0 in range(0, ny, rows):
        Y = torch.arange(y0, min(ny, y0 + rows), dtype=torch.float64, device=dev)[:, None]
        for i, (kx, ky, ph) in enumerate(modes):
            w = 2 * np.pi * (kx * (X + 0.5) / nx + ky * (Y + 0.5) / ny) + ph
            v0[i % 2, y0:y0 + rows] += 5e-3 * torch.sin(w)
    sv.init(v0)
    del v0
    torch.cuda.empty_cache()
    for k in range(steps):
        sv.step(k)
    torch.cuda.synchronize()
    assert sv.faults() == 0
    T = (nx + 63) // 64
    pop = sv.pop[sv.s.cur].view(torch.float32)
    starts = [(0, 0), (ny - win, nx - win), (100, nx - 10), (ny - 7, 5)] + \
             [(int(rng.integers(0, ny - win)), int(rng.integers(0, nx - win))) for _ in range(2)]
    for (y0, x0) in starts:
        ys = (np.arange(win) + y0) % ny
        xs = (np.arange(win) + x0) % nx
        p = np.arange(24)
        idx = ((ys[None, :, None] * T + xs[None, None, :] // 64) * 24 + p[:, None, None]) * 64 + xs[None, None, :] % 64
        g = pop[torch.from_numpy(idx.reshape(-1)).to(dev)].double().cpu().numpy().reshape(4, 6, win, win)
        size = win + 2 * margin
        wy = (np.arange(size) + y0 - margin) % ny
        wx = (np.arange(size) + x0 - margin) % nx
        pb = lbm.Problem(nx=size, ny=size, c=2.0, omega=2.0, law="lognh", mu=0.1, lam=0.2)
        st = lbm.initial_state(pb, v0_block(wy, wx))
        lbm.run(pb, st, steps)
        fo = lbm.post_collision(pb, st)[:, :, margin:margin + win, margin:margin + win].copy()
        fo[:, 2] -= 0.25
        fo[:, 5] -= 0.25
        err = float(np.sqrt(((g - fo) ** 2).sum() / (fo ** 2).sum()))
        print(f"\n[largest grid {nx}x{ny} f32 window at {y0},{x0}] populations rel L2 {err:.2e}")
        assert err <= 1e-5
    del sv, pop
    torch.cuda.empty_cache()
