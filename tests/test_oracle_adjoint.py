"""Pins of the oracle's hand-written adjoint: central finite differences of the forward
map for every parameter group, every kind of edge and omega = 2 and omega < 2."""
import numpy as np
import pytest

import lbm_inputs as li
from oracle import adjoint as adj
from oracle import lbm

NX, NY = 10, 8
SCALE = dict(mu=0.1, lam=0.2, body=1e-3, v0=1e-3)


def _problem(mu, lam, body, kinds, omega, law):
    edges = [lbm.Edge(k, (lambda t: np.array([1e-3, -2e-3])) if k == "traction" else None) for k in kinds]
    return lbm.Problem(nx=NX, ny=NY, c=2.5, omega=omega, law=law, mu=mu, lam=lam, body=body,
                       ramp=lambda n: min(1.0, n / 5), edges=edges)


@pytest.mark.parametrize("kinds", [
    ("periodic",) * 4,
    ("velocity",) * 4,
    ("velocity", "traction", "traction", "traction"),
    ("traction",) * 4,
])
@pytest.mark.parametrize("omega,law", [(2.0, "lognh"), (1.9, "lognh"), (1.95, "svk"), (1.95, "nh"),
                                       (1.95, ("mr", (0.3, 0.2))), (2.0, ("yeoh", (0.5, 0.2, 0.1))),
                                       (1.95, ("gent", (3.0,)))])
def test_adjoint_matches_central_differences(kinds, omega, law):
    mu = li.lognormal_field(NX, NY, 1, 0.1, 0.3, 3.0)
    lam = li.lognormal_field(NX, NY, 2, 0.2, 0.3, 3.0)
    body = li.uniform_body(NX, NY, (0.0, -2e-3))
    v0 = np.stack([li.gaussian_random_field(NX, NY, 3, 2e-3), li.gaussian_random_field(NX, NY, 4, 2e-3)])
    probes = li.random_probes(NX, NY, 5, 7, margin=1)
    target = np.full((2, 5), 1e-3)
    N = 12
    pb = _problem(mu, lam, body, kinds, omega, law)
    _, g = adj.gradients(pb, v0, N, probes, target)
    base = dict(mu=mu, lam=lam, body=body, v0=v0)
    for d in li.fd_directions({k: base[k].shape for k in base}, 2, 406):
        eps = 1e-4

        def L(s):
            kw = {k: base[k] + s * eps * SCALE[k] * d[k] for k in base}
            return adj.loss_only(_problem(kw["mu"], kw["lam"], kw["body"], kinds, omega, law),
                                 kw["v0"], N, probes, target)
        fd = (L(1) - L(-1)) / (2 * eps)
        an = sum((g[k] * SCALE[k] * d[k]).sum() for k in base)
        assert abs(fd - an) <= 1e-6 * abs(fd), (fd, an)
