"""Host-side checks of the C ABI: the library loads, exports every entry point that
include/lbm.h declares, and its size and validation functions behave as documented.
No call here touches the GPU."""
import ctypes
import os
import re

import pytest

from paper_2605_26677_amd import _lib as L

HEADER = os.path.join(os.path.dirname(os.path.dirname(__file__)), "include", "lbm.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(lbm_[a-z_0-9]+)\s*\(", text)))


def test_every_declared_symbol_is_exported():
    lib = L.lib()
    names = declared_functions()
    assert len(names) >= 15
    for name in names:
        assert hasattr(lib, name), name
        assert name in L.SIGNATURES, name


def _params(nx=64, ny=64, storage=L.LBM_F32_SHIFTED, bc=(0, 0, 0, 0), c=2.0, omega=2.0):
    p = L.lbm_params()
    p.nx, p.ny, p.storage, p.material = nx, ny, storage, L.LBM_LOGNH
    for e in range(4):
        p.bc[e] = bc[e]
    p.dx, p.c, p.omega = 1.0, c, omega
    return p


def test_sizes():
    lib = L.lib()
    assert lib.lbm_tile_width() == 64
    p = _params(8192, 8192)
    assert lib.lbm_padded_nodes(ctypes.byref(p)) == 8192 * 8192
    assert lib.lbm_pop_bytes(ctypes.byref(p)) == 24 * 8192 * 8192 * 4
    assert lib.lbm_ustar_bytes(ctypes.byref(p)) == (2 * 4 + 2 * 8) * 8192 * 8192   # S float + U double
    assert lib.lbm_record_bytes(ctypes.byref(p)) == 6 * 8192 * 8192 * 4
    p64 = _params(100, 37, storage=L.LBM_F64_PLAIN)
    assert lib.lbm_padded_nodes(ctypes.byref(p64)) == 128 * 37        # rows padded to whole tiles
    assert lib.lbm_pop_bytes(ctypes.byref(p64)) == 24 * 128 * 37 * 8
    p16 = _params(100, 37, storage=L.LBM_F16_SHIFTED)
    assert lib.lbm_pop_bytes(ctypes.byref(p16)) == 24 * 128 * 37 * 2
    assert lib.lbm_adj_bytes(ctypes.byref(p16)) == 24 * 128 * 37 * 4


@pytest.mark.parametrize("mutate,code", [
    (lambda p: setattr(p, "nx", 2), L.LBM_ERR_ARG),
    (lambda p: setattr(p, "storage", 7), L.LBM_ERR_ARG),
    (lambda p: setattr(p, "material", -1), L.LBM_ERR_ARG),
    (lambda p: p.bc.__setitem__(0, L.LBM_VELOCITY), L.LBM_ERR_ARG),      # unpaired periodic
    (lambda p: setattr(p, "omega", 2.5), L.LBM_ERR_ARG),
    (lambda p: setattr(p, "c", 0.0), L.LBM_ERR_ARG),
    (lambda p: setattr(p, "nx", 70000), L.LBM_ERR_ARG),                    # nx * ny >= 2^31
])
def test_parameter_validation(mutate, code):
    lib = L.lib()
    p = _params(ny=40000)
    p.ny = 64
    mutate(p)
    if p.nx == 70000:
        p.ny = 40000
    assert lib.lbm_check_params(ctypes.byref(p)) == code


@pytest.mark.parametrize("material,law_k,code", [
    (L.LBM_MR, (0.3, 0.2, 0.0), L.LBM_OK),
    (L.LBM_MR, (0.5, 0.0, 0.0), L.LBM_OK),
    (L.LBM_MR, (0.0, 0.0, 0.0), L.LBM_ERR_ARG),       # no shear stiffness
    (L.LBM_MR, (0.6, -0.1, 0.0), L.LBM_ERR_ARG),
    (L.LBM_YEOH, (0.5, 0.05, 0.01), L.LBM_OK),
    (L.LBM_YEOH, (0.0, 0.05, 0.01), L.LBM_ERR_ARG),
    (L.LBM_GENT, (20.0, 0.0, 0.0), L.LBM_OK),
    (L.LBM_GENT, (0.0, 0.0, 0.0), L.LBM_ERR_ARG),
    (L.LBM_SVK, (0.0, 0.0, 0.0), L.LBM_OK),           # ignored by the Lame-parametrised laws
    (6, (0.0, 0.0, 0.0), L.LBM_ERR_ARG),
])
def test_law_constant_validation(material, law_k, code):
    lib = L.lib()
    p = _params()
    p.material = material
    for i in range(3):
        p.law_k[i] = law_k[i]
    assert lib.lbm_check_params(ctypes.byref(p)) == code


def test_cfl_audit_invariant_laws():
    """The invariant laws' small-strain P-wave speed is sqrt(lam + 4 G / 3) with G the
    small-strain shear modulus: MR 2 (c10 + c01), Yeoh 2 c1, Gent mu."""
    lib = L.lib()
    p = _params(c=2.0)
    mu, lam = 1.0, 0.5
    for material, k, G in ((L.LBM_MR, (0.3, 0.2, 0), 1.0), (L.LBM_YEOH, (0.75, 0, 0), 1.5),
                           (L.LBM_GENT, (20.0, 0, 0), 1.0)):
        p.material = material
        for i in range(3):
            p.law_k[i] = k[i]
        cp = (lam + 4.0 * G / 3.0) ** 0.5
        p.c = 2.0 * cp * 1.001
        assert lib.lbm_check_cfl(ctypes.byref(p), mu, lam) == L.LBM_OK
        p.c = 2.0 * cp * 0.999
        assert lib.lbm_check_cfl(ctypes.byref(p), mu, lam) == L.LBM_ERR_CFL


def test_walls_need_four_nodes():
    lib = L.lib()
    p = _params(3, 16, bc=(1, 2, 0, 0))
    assert lib.lbm_check_params(ctypes.byref(p)) == L.LBM_ERR_ARG
    p.nx = 4
    assert lib.lbm_check_params(ctypes.byref(p)) == L.LBM_OK


def test_cfl_audit():
    """sqrt(lam + 2 mu) / c <= 1/2: c = 2 passes and c = 1 is refused for mu = 0.1,
    lam = 0.2 (the oracle's linear symbol shows the c = 1 step is unstable)."""
    lib = L.lib()
    p = _params(c=2.0)
    assert lib.lbm_check_cfl(ctypes.byref(p), 0.1, 0.2) == L.LBM_OK
    p.c = 1.0
    assert lib.lbm_check_cfl(ctypes.byref(p), 0.1, 0.2) == L.LBM_ERR_CFL


def test_calls_reject_missing_buffers():
    lib = L.lib()
    p = _params()
    s = L.lbm_state()
    assert lib.lbm_step(ctypes.byref(p), ctypes.byref(s), 0, 1.0, 1.0, None, None, None) == L.LBM_ERR_ARG
    assert lib.lbm_init(ctypes.byref(p), ctypes.byref(s), None, None, None, 0.0, None) == L.LBM_ERR_ARG
    a = L.lbm_adj_state()
    assert lib.lbm_adjoint_step(ctypes.byref(p), ctypes.byref(s), ctypes.byref(a), 0, 1.0, None, None,
                                None) == L.LBM_ERR_ARG
    for st in range(5):
        assert lib.lbm_status_string(st)


def test_adjoint_step_requires_block_sums_for_shifted_storage():
    """Gradients of a F32/F16 adjoint step are summed through lbm_adj_state.gsum: a call
    with a gradient pointer and no gsum is refused before any launch; FP64 storage adds to
    the gradients directly and needs none."""
    lib = L.lib()
    fake = 256                       # never dereferenced: argument checks come first
    s = L.lbm_state()
    s.pop[0], s.pop[1], s.fault = fake, fake, fake
    a = L.lbm_adj_state()
    a.adj[0], a.adj[1] = fake, fake
    a.g_mu = fake
    a.nsteps = 10
    p = _params()
    assert lib.lbm_adj_sum_bytes(ctypes.byref(p)) == 4 * 64 * 64 * 4
    assert lib.lbm_adjoint_step(ctypes.byref(p), ctypes.byref(s), ctypes.byref(a), 3, 1.0, None,
                                ctypes.c_void_p(fake), None) == L.LBM_ERR_ARG


def test_walls_need_boundary_data():
    """lbm_step on a grid with walls refuses a NULL at_half before any launch."""
    lib = L.lib()
    fake = 256
    p = _params(bc=(L.LBM_VELOCITY, L.LBM_VELOCITY, 0, 0))
    s = L.lbm_state()
    s.pop[0], s.pop[1], s.fault = fake, fake, fake
    assert lib.lbm_step(ctypes.byref(p), ctypes.byref(s), 0, 1.0, 1.0, None, None, None) == L.LBM_ERR_ARG


def test_step2_argument_checks():
    """lbm_step2 (two fused levels) refuses missing buffers, and on a grid with walls missing
    boundary data of either half step or a missing staging buffer, before any launch."""
    lib = L.lib()
    fake = 256
    s = L.lbm_state()
    p = _params()
    assert lib.lbm_step2(ctypes.byref(p), ctypes.byref(s), 0, 1.0, 1.0, 1.0, None, None, None, None,
                         None) == L.LBM_ERR_ARG
    s.pop[0], s.pop[1], s.fault = fake, fake, fake
    p = _params(bc=(L.LBM_VELOCITY, L.LBM_VELOCITY, 0, 0))
    ed = L.lbm_edge_data()
    s.aux = fake
    assert lib.lbm_step2(ctypes.byref(p), ctypes.byref(s), 0, 1.0, 1.0, 1.0, ctypes.byref(ed), None, None, None,
                         None) == L.LBM_ERR_ARG
    assert lib.lbm_step2(ctypes.byref(p), ctypes.byref(s), 0, 1.0, 1.0, 1.0, None, ctypes.byref(ed), None, None,
                         None) == L.LBM_ERR_ARG
    s.aux = None
    assert lib.lbm_step2(ctypes.byref(p), ctypes.byref(s), 0, 1.0, 1.0, 1.0, ctypes.byref(ed), ctypes.byref(ed),
                         None, None, None) == L.LBM_ERR_ARG


@pytest.mark.parametrize("bc", [(2, 2, 2, 2), (1, 2, 2, 2), (0, 0, 2, 2)])
def test_traction_wall_stability_region(bc):
    """Traction walls carry modes that grow at omega = 2 at a rate set by c_p / c; the audit
    refuses what the measured map (FP64, 512^2) shows growing, and passes what it shows
    decaying.  mu = 0.1, lam = 0.3 (c_p = 0.707):
      c = 2.5, omega = 1.996875 (2 - 1.6/512): grows (+3e-3 per step) -> refused;
      c = 2.5, omega = 1.99: decays -> passes;
      c = 3.5, omega = 1.998: grows (+7e-4) -> refused;  omega = 1.995: decays -> passes;
      c = 10, omega = 1.9995: decays -> passes;
      periodic grids and velocity walls only: no wall term."""
    lib = L.lib()
    mu, lam = 0.1, 0.3
    p = _params(64, 64, bc=bc)
    for c, om, ok in ((2.5, 2.0 - 1.6 / 512, False), (2.5, 1.99, True), (3.5, 1.998, False),
                      (3.5, 1.995, True), (10.0, 1.9995, True), (10.0, 2.0, False)):
        p.c, p.omega = c, om
        want = L.LBM_OK if ok else L.LBM_ERR_CFL
        assert lib.lbm_check_cfl(ctypes.byref(p), mu, lam) == want, (c, om)
        g = lib.lbm_wall_mode_growth(ctypes.byref(p), mu, lam)
        assert (g <= 2e-4) == ok, (c, om, g)
    p = _params(64, 64, bc=(1, 1, 1, 1))
    p.c, p.omega = 2.5, 2.0
    assert lib.lbm_wall_mode_growth(ctypes.byref(p), mu, lam) == 0.0
    assert lib.lbm_check_cfl(ctypes.byref(p), mu, lam) == L.LBM_OK
