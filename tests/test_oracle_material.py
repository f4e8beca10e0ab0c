"""Pins of the oracle's constitutive closures (paper Appendix A, eq:stress-and-tangent)."""
import numpy as np
import pytest

from oracle import material as mat

LAWS = mat.LAWS


def random_F(rng, n, strain=0.3):
    F = np.eye(2)[:, :, None] + strain * rng.standard_normal((2, 2, n))
    J = mat.det(F)
    keep = J > 0.3
    return F[:, :, keep]


@pytest.mark.parametrize("law", LAWS)
def test_stress_is_energy_gradient(law):
    """P = dW/dF (Appendix A defines P as the derivative of W): central differences."""
    rng = np.random.default_rng(1)
    F = random_F(rng, 40)
    mu, lam = 0.7, 1.3
    P = mat.stress(law, F, mu, lam)
    h = 1e-6
    for k in range(2):
        for B in range(2):
            Fp, Fm = F.copy(), F.copy()
            Fp[k, B] += h
            Fm[k, B] -= h
            fd = (mat.energy(law, Fp, mu, lam) - mat.energy(law, Fm, mu, lam)) / (2 * h)
            assert np.allclose(fd, P[k, B], rtol=1e-7, atol=1e-8)


@pytest.mark.parametrize("law", LAWS)
def test_tangent_is_stress_gradient(law):
    """C_iAkB = dP_iA/dF_kB (eq:stress-and-tangent): central differences."""
    rng = np.random.default_rng(2)
    F = random_F(rng, 40)
    mu, lam = 0.4, 0.9
    Cc = mat.tangent(law, F, mu, lam)
    h = 1e-6
    for k in range(2):
        for B in range(2):
            Fp, Fm = F.copy(), F.copy()
            Fp[k, B] += h
            Fm[k, B] -= h
            fd = (mat.stress(law, Fp, mu, lam) - mat.stress(law, Fm, mu, lam)) / (2 * h)
            assert np.allclose(fd, Cc[:, :, k, B], rtol=1e-7, atol=1e-8)


@pytest.mark.parametrize("law", LAWS)
def test_reference_state_is_stress_free_exactly(law):
    """P(I) = 0 for every law of Appendix A, bit for bit (the rest state is invariant)."""
    F = np.repeat(np.eye(2)[:, :, None], 5, axis=2)
    for mu, lam in ((0.1, 0.2), (1.0, 2.0 / 3.0), (0.137, 0.411)):
        assert np.array_equal(mat.stress(law, F, mu, lam), np.zeros((2, 2, 5)))


@pytest.mark.parametrize("law", LAWS)
def test_small_strain_limit_is_lame(law):
    """C(I) = mu (d_ik d_AB + d_iB d_kA) + lam d_iA d_kB (linear elasticity)."""
    mu, lam = 0.3, 0.8
    Cc = mat.tangent(law, np.eye(2), mu, lam)
    d = np.eye(2)
    lame = (mu * (np.einsum("ik,AB->iAkB", d, d) + np.einsum("iB,kA->iAkB", d, d))
            + lam * np.einsum("iA,kB->iAkB", d, d))
    assert np.allclose(Cc, lame, atol=1e-15)


@pytest.mark.parametrize("law", LAWS)
def test_acoustic_speeds_at_rest(law):
    """Eigenvalues of Q(n; I) are mu and lam + 2 mu for every direction n
    (eq:acoustic-tensor-section2 at F = I: S- and P-wave speeds)."""
    mu, lam = 0.1, 0.2
    for th in np.linspace(0, np.pi, 7):
        Q = mat.acoustic_tensor(law, np.eye(2), mu, lam, (np.cos(th), np.sin(th)))
        ev = np.sort(np.linalg.eigvalsh(Q))
        assert np.allclose(ev, [mu, lam + 2 * mu], atol=1e-15)
    assert np.isclose(mat.max_tangent_speed(law, np.eye(2), mu, lam), np.sqrt(lam + 2 * mu))


@pytest.mark.parametrize("law", LAWS)
def test_frame_indifference_and_symmetric_cauchy(law):
    rng = np.random.default_rng(3)
    F = random_F(rng, 20)
    mu, lam = 0.5, 0.5
    th = 0.7
    R = np.array([[np.cos(th), -np.sin(th)], [np.sin(th), np.cos(th)]])
    RF = np.einsum("ij,jA...->iA...", R, F)
    assert np.allclose(mat.energy(law, RF, mu, lam), mat.energy(law, F, mu, lam), rtol=1e-12, atol=1e-14)
    s = mat.cauchy(law, F, mu, lam)
    assert np.allclose(s[0, 1], s[1, 0], rtol=1e-12, atol=1e-14)


@pytest.mark.parametrize("law", ["nh", "lognh"])
def test_isochoric_shear_path(law):
    """On F = [[1, 0], [g, 1]] (J = 1), P21 = mu F21 for both neo-Hookean laws
    (eq:finite-amplitude-shear-stress)."""
    g = np.linspace(-0.5, 0.5, 11)
    F = np.zeros((2, 2, g.size))
    F[0, 0] = F[1, 1] = 1.0
    F[1, 0] = g
    P = mat.stress(law, F, 2.0, 7.0)
    assert np.allclose(P[1, 0], 2.0 * g, atol=1e-15)


def test_parameter_partials_are_linear():
    rng = np.random.default_rng(4)
    F = random_F(rng, 10)
    for law in LAWS:
        Pm, Pl = mat.stress_parameter_partials(law, F)
        assert np.allclose(mat.stress(law, F, 0.3, 0.7), 0.3 * Pm + 0.7 * Pl, atol=1e-14)
