"""Pins of the oracle's constitutive closures (paper Appendix A, eq:stress-and-tangent)."""
import numpy as np
import pytest

from oracle import material as mat

LAWS = mat.ALL_LAWS


def lame_tangent(mu, lam):
    d = np.eye(2)
    return (mu * (np.einsum("ik,AB->iAkB", d, d) + np.einsum("iB,kA->iAkB", d, d))
            + lam * np.einsum("iA,kB->iAkB", d, d))


def small_strain_lambda(law, mu, lam):
    """In-plane Lame constant of the linearised law.  The invariant laws split W into an
    isochoric part in the 3D modified invariants (out-of-plane stretch 1) and the bulk
    term lam/2 (ln J)^2, so their small-strain energy is mu |dev3 eps|^2 + lam/2 (tr eps)^2
    = mu eps:eps + (lam - 2 mu / 3)/2 (tr eps)^2: the plane Lame constant is lam - 2 mu/3."""
    return lam - 2.0 * mu / 3.0 if law in mat.INVARIANT_LAWS else lam


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
    """C(I) = mu (d_ik d_AB + d_iB d_kA) + lam' d_iA d_kB (linear elasticity), with
    lam' = lam for the Lame-parametrised laws and lam - 2 mu/3 for the invariant laws,
    whose shear modulus is 2 (c10 + c01) = 2 c1 = mu (Appendix A)."""
    mu, lam = 0.3, 0.8
    Cc = mat.tangent(law, np.eye(2), mu, lam)
    assert np.allclose(Cc, lame_tangent(mu, small_strain_lambda(law, mu, lam)), atol=1e-14)


@pytest.mark.parametrize("law", LAWS)
def test_acoustic_speeds_at_rest(law):
    """Eigenvalues of Q(n; I) are mu and lam' + 2 mu for every direction n
    (eq:acoustic-tensor-section2 at F = I: S- and P-wave speeds)."""
    mu, lam = 0.1, 0.2
    lp = small_strain_lambda(law, mu, lam)
    for th in np.linspace(0, np.pi, 7):
        Q = mat.acoustic_tensor(law, np.eye(2), mu, lam, (np.cos(th), np.sin(th)))
        ev = np.sort(np.linalg.eigvalsh(Q))
        assert np.allclose(ev, [mu, lp + 2 * mu], atol=1e-14)
    assert np.isclose(mat.max_tangent_speed(law, np.eye(2), mu, lam), np.sqrt(lp + 2 * mu))


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


@pytest.mark.parametrize("law", mat.INVARIANT_LAWS)
def test_invariant_laws_on_isochoric_shear(law):
    """On F = [[1, 0], [g, 1]]: J = 1, barI1 - 3 = barI2 - 3 = g^2, so W reduces to a
    polynomial (or log) in g and P21 = dW/dg in closed form: MR 2 (c10 + c01) g, Yeoh
    2 c1 g + 4 c2 g^3 + 6 c3 g^5, Gent mu g / (1 - g^2 / J_m)."""
    g = np.linspace(-0.6, 0.6, 13)
    F = np.zeros((2, 2, g.size))
    F[0, 0] = F[1, 1] = 1.0
    F[1, 0] = g
    mu = 1.7
    prm = {"mr": (0.2, 0.45), "yeoh": (0.5, 0.11, 0.03), "gent": (2.5,)}[law]
    P = mat.stress(law, F, mu, 9.0, prm)
    if law == "mr":
        want = 2 * (prm[0] + prm[1]) * mu * g
    elif law == "yeoh":
        want = 2 * prm[0] * mu * g + 4 * prm[1] * mu * g ** 3 + 6 * prm[2] * mu * g ** 5
    else:
        want = mu * g / (1.0 - g * g / prm[0])
    assert np.allclose(P[1, 0], want, rtol=1e-13, atol=1e-15)
    W = mat.energy(law, F, mu, 9.0, prm)
    if law == "mr":
        Wwant = (prm[0] + prm[1]) * mu * g ** 2
    elif law == "yeoh":
        Wwant = prm[0] * mu * g ** 2 + prm[1] * mu * g ** 4 + prm[2] * mu * g ** 6
    else:
        Wwant = -mu * prm[0] / 2 * np.log(1 - g ** 2 / prm[0])
    assert np.allclose(W, Wwant, rtol=1e-13, atol=1e-15)


def test_invariant_law_special_cases_coincide():
    """Yeoh with c2 = c3 = 0, Mooney-Rivlin with c01 = 0 and Gent as J_m -> infinity all
    reduce to the same isochoric neo-Hookean law mu/2 (barI1 - 3) + lam/2 (ln J)^2."""
    rng = np.random.default_rng(7)
    F = random_F(rng, 30)
    mu, lam = 0.9, 1.4
    P_y = mat.stress("yeoh", F, mu, lam, (0.5, 0.0, 0.0))
    P_m = mat.stress(("mr", (0.5, 0.0)), F, mu, lam)
    P_g = mat.stress("gent", F, mu, lam, (1e12,))
    assert np.allclose(P_y, P_m, rtol=1e-14, atol=1e-15)
    assert np.allclose(P_g, P_m, rtol=1e-10, atol=1e-12)
    C_y = mat.tangent("yeoh", F, mu, lam, (0.5, 0.0, 0.0))
    C_m = mat.tangent(("mr", (0.5, 0.0)), F, mu, lam)
    assert np.allclose(C_y, C_m, rtol=1e-13, atol=1e-14)


def test_parameter_partials_are_linear():
    rng = np.random.default_rng(4)
    F = random_F(rng, 10)
    for law in LAWS:
        Pm, Pl = mat.stress_parameter_partials(law, F)
        assert np.allclose(mat.stress(law, F, 0.3, 0.7), 0.3 * Pm + 0.7 * Pl, atol=1e-14)
