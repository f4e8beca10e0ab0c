"""lbm_diagnostics_noalloc (the variant of lbm_diagnostics that keeps its reduction
partials in the library's own device array instead of caller scratch) against
lbm_diagnostics, through the C ABI: bit for bit on two calls in a row, the second on a
smaller grid, so the shared array holds the first call's partials when the second runs."""
import ctypes

import numpy as np
import pytest

from gpu_cases import block_case, make_solver, random_field_case

pytestmark = pytest.mark.gpu


def _both(sv, r_n):
    import torch
    from paper_2605_26677_amd import _lib as L
    from paper_2605_26677_amd.solver import _ptr, _stream
    ref = sv.diagnostics(r_n)
    out = torch.full((L.LBM_DIAG_COUNT,), float("nan"), dtype=torch.float64, device=sv.device)
    L.check(sv.lib.lbm_diagnostics_noalloc(ctypes.byref(sv.p), ctypes.byref(sv.s), float(r_n), _ptr(out),
                                           _stream()), "lbm_diagnostics_noalloc")
    torch.cuda.synchronize()
    return ref.cpu().numpy(), out.cpu().numpy()


@pytest.mark.parametrize("storage", ["f32", "f64"])
def test_noalloc_diagnostics_match(storage):
    runs = [(random_field_case(300, 260, 20), 1.0), (block_case(96, 80, 30), 0.5)]
    for case, r_n in runs:
        print(f"\n[noalloc diagnostics {case.name} {storage}]", flush=True)
        sv = make_solver(case, storage)
        sv.init(case.v0, case.u0, r0=case.ramp(0))
        for n in range(case.steps):
            sv.step(n, case.ramp(n), case.ramp(n + 1), edges=list(case.data))
        ref, got = _both(sv, r_n)
        assert np.all(np.isfinite(got))
        np.testing.assert_array_equal(got, ref)
