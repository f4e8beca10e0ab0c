"""Pin of the vectorised oracle against a literal per-link mpmath implementation on tiny
grids, for every law and every kind of edge (periodic, velocity, traction, corners)."""
import numpy as np
import pytest

import lbm_inputs as li
from brute_mpmath import Brute
from oracle import lbm

COMBOS = [
    ("periodic", "periodic", "periodic", "periodic"),
    ("velocity", "velocity", "periodic", "periodic"),
    ("periodic", "periodic", "traction", "velocity"),
    ("velocity", "traction", "traction", "traction"),
    ("traction", "traction", "traction", "traction"),
    ("velocity", "velocity", "velocity", "velocity"),
]
DATA = [(1e-3, -5e-4), (2e-4, 1e-3), (-1e-3, 3e-4), (5e-4, 5e-4)]


@pytest.mark.parametrize("law", ["lognh", "nh", "svk"])
@pytest.mark.parametrize("kinds", COMBOS)
def test_oracle_matches_brute_force(law, kinds):
    nx, ny = 4, 4
    mu = li.lognormal_field(nx, ny, 1, 0.1, 0.3, 2.0)
    lam = li.lognormal_field(nx, ny, 2, 0.2, 0.3, 2.0)
    body = li.uniform_body(nx, ny, (1e-3, -2e-3))
    v0 = np.stack([li.gaussian_random_field(nx, ny, 3, 2e-3), li.gaussian_random_field(nx, ny, 4, 2e-3)])
    u0 = np.stack([li.gaussian_random_field(nx, ny, 5, 1e-2), li.gaussian_random_field(nx, ny, 6, 1e-2)])
    ramp = lambda n: min(1.0, n / 4)
    pb = lbm.Problem(nx=nx, ny=ny, c=2.5, omega=1.9, law=law, mu=mu, lam=lam, body=body, ramp=ramp,
                     edges=[lbm.Edge(k, (lambda t, d=d: np.array(d))) for k, d in zip(kinds, DATA)])
    st = lbm.initial_state(pb, v0, u0)
    br = Brute(nx, ny, 2.5, 1.9, law, mu, lam, 1.0, body, ramp, kinds, DATA)
    br.initialise(v0, u0)
    for _ in range(6):
        lbm.step(pb, st)
        br.step()
    U, u = lbm.observe(pb, st)
    Ub, ub, fb = (np.array(x) for x in br.state())
    assert np.abs(U - Ub).max() <= 1e-14
    assert np.abs(u - ub).max() <= 1e-14
    assert np.abs(st.f - fb).max() <= 1e-14
