"""The traction-wall modes and the audit that bounds them (lbm_wall_mode_growth,
lbm_check_cfl).

Traction walls carry modes confined to the wall line and its corners (mostly the F rows of
the tangential column) whose growth per step at omega = 2 depends on c_p / c and not on the
grid size, so 2 - omega = 1.6 / n stops damping them once n is large.  These runs start
from noise of 1e-9 on a 512^2 FP64 grid with traction walls on all four sides (mu = 0.1,
lam = 0.3, c_p = 0.707) and measure the growth of max |U| over steps 2000 - 4000 (the
amplitude stays below 1e-3, in the linear range): the audit refuses exactly the growing
cases."""
import ctypes

import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu

N = 512


def _growth(c, omega, steps=4000):
    from paper_2605_26677_amd.solver import Solver
    rng = np.random.default_rng(5)
    v0 = 1e-9 * rng.standard_normal((2, N, N))
    sv = Solver(N, N, c=c, omega=omega, storage="f64", bc=("traction",) * 4, mu=0.1, lam=0.3,
                force_unstable=True)
    sv.init(v0)
    sv.advance(0, steps // 2, block=64)
    m1 = float(sv.moments().abs().max())
    sv.advance(steps // 2, steps // 2, block=64)
    m2 = float(sv.moments().abs().max())
    assert sv.faults() == 0 and m2 < 1e-3
    est = sv.lib.lbm_wall_mode_growth(ctypes.byref(sv.p), 0.1, 0.3)
    ok = sv.lib.lbm_check_cfl(ctypes.byref(sv.p), 0.1, 0.3)
    del sv
    torch.cuda.empty_cache()
    return np.log(m2 / m1) / (steps // 2), est, ok


@pytest.mark.parametrize("c,omega,grows", [(2.5, 2.0 - 1.6 / N, True), (2.5, 1.99, False), (3.5, 1.998, True),
                                           (3.5, 1.995, False), (10.0, 1.9995, False)])
def test_wall_modes_and_audit(c, omega, grows):
    from paper_2605_26677_amd import _lib as L
    g, est, ok = _growth(c, omega)
    print(f"\n[wall modes c={c} omega={omega:.6f}] measured {g:+.2e} per step, estimate {est:+.2e}")
    assert (g > 0) == grows
    # the audit refuses an estimated growth above 2e-4 per step (e-folding within 5000 steps)
    assert (est > 2e-4) == grows
    assert (ok == L.LBM_ERR_CFL) == grows
