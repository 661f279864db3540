"""Pins of the oracle's stout and over-improved stout smearing (Sec. II.B)."""
import numpy as np
import pytest

from helpers import center_links, gauge_transform, unitarity_error

L4 = (4, 4, 4, 4)


@pytest.fixture(scope="module")
def U(S):
    return S.heatbath_field(L4, S.sub_seed(101), 5.7, 10)


def test_rho_zero_and_n_zero_are_identity_bitwise(O, U):
    assert np.array_equal(O.smear(U, 0.0, 1.0, 3), U)
    assert np.array_equal(O.smear(U, 0.0, -0.25, 2), U)
    assert np.array_equal(O.smear(U, 0.1, 1.0, 0), U)


@pytest.mark.parametrize("eps", [1.0, -0.25, 0.0])
def test_gauge_covariance(O, S, U, eps):
    """S(U^g) = S(U)^g for a Haar-random gauge transform g."""
    g = S.haar_gauge(L4, S.sub_seed(102))
    a = O.smear(gauge_transform(U, g), 0.1, eps, 3)
    b = gauge_transform(O.smear(U, 0.1, eps, 3), g)
    assert np.abs(a - b).max() < 1e-13


@pytest.mark.parametrize("eps", [1.0, -0.25])
def test_center_field_is_fixed_point(O, S, eps):
    """Every staple of a gauge-transformed Z3 field is c g(x) g(x+mu)^dag, so
    Omega is a multiple of 1, TA(Omega) = 0 and smearing changes nothing."""
    m = S.z3_links(L4, S.sub_seed(103))
    g = S.haar_gauge(L4, S.sub_seed(104))
    U = gauge_transform(center_links(m), g)
    # five steps, each exact up to ~1e-15 rounding
    assert np.abs(O.smear(U, 0.1, eps, 5) - U).max() < 5e-14


def test_oi_eps_one_is_plain_stout(O, U):
    """eps = 1 gives plaquette weight 1 and rectangle weight 0; compare with
    the plain stout staples written out as explicit products."""
    for site in (0, 37, 255):
        for mu in range(4):
            a = O.staple_sum(U, site, mu, 0.1, 1.0)
            b = O.stout_staple_plain(U, site, mu, 0.1)
            assert np.abs(a - b).max() < 1e-15


def test_smeared_links_stay_in_su3(O, U):
    for eps in (1.0, -0.25):
        Sm = O.smear(U, 0.1, eps, 5).reshape(-1, 3, 3)
        assert unitarity_error(Sm) < 1e-13
        assert np.abs(np.linalg.det(Sm) - 1).max() < 1e-13


def _abelian_step(theta, rho, eps):
    """Closed form of one smearing step for a diagonal field.

    theta[a, t, z, y, x, mu] are the phases of the three diagonal entries.
    For commuting links the phase of a closed loop is the signed sum of the
    plaquette fluxes F_{mu nu}(x) it encloses (Stokes), so
    Omega_mu(x) = C U^dag = rho sum_nu [ wp (e^{-i F(x)} + e^{i F(x-nu)})
      + wr (e^{-i(F(x)+F(x+mu))} + e^{-i(F(x-mu)+F(x))} + e^{-i(F(x)+F(x+nu))}
            + e^{i(F(x-nu)+F(x-nu+mu))} + e^{i(F(x-mu-nu)+F(x-nu))} + e^{i(F(x-nu)+F(x-2nu))}) ]
    with F = F_{mu nu}, and U' = exp(TA(Omega)) U is diagonal with phases
    theta + Im(omega) - mean(Im(omega))."""
    wp, wr = (5 - 2 * eps) / 3, -(1 - eps) / 12

    def sh(a, d, s):
        return np.roll(a, -s, axis=4 - d)  # axes: a, t, z, y, x

    out = theta.copy()
    for mu in range(4):
        om = np.zeros(theta.shape[:5], complex)
        for nu in range(4):
            if nu == mu:
                continue
            th_mu, th_nu = theta[..., mu], theta[..., nu]
            F = th_mu + sh(th_nu, mu, 1) - sh(th_mu, nu, 1) - th_nu
            Fm = lambda dm, dn: sh(sh(F, mu, dm), nu, dn)  # noqa: E731
            om += wp * (np.exp(-1j * F) + np.exp(1j * Fm(0, -1)))
            om += wr * (np.exp(-1j * (F + Fm(1, 0))) + np.exp(-1j * (Fm(-1, 0) + F))
                        + np.exp(-1j * (F + Fm(0, 1)))
                        + np.exp(1j * (Fm(0, -1) + Fm(1, -1))) + np.exp(1j * (Fm(-1, -1) + Fm(0, -1)))
                        + np.exp(1j * (Fm(0, -1) + Fm(0, -2))))
        im = np.imag(rho * om)
        out[..., mu] = theta[..., mu] + im - im.mean(axis=0, keepdims=True)
    return out


@pytest.mark.parametrize("eps", [1.0, -0.25, 0.0])
def test_abelian_closed_form(O, eps):
    L = (4, 4, 4, 6)
    rng = np.random.default_rng(7)
    th = rng.uniform(-np.pi, np.pi, size=(2, L[3], L[2], L[1], L[0], 4))
    theta = np.concatenate([th, -th.sum(axis=0, keepdims=True)], axis=0)
    U = np.zeros((L[3], L[2], L[1], L[0], 4, 3, 3), complex)
    for a in range(3):
        U[..., a, a] = np.exp(1j * theta[a])
    got = O.smear_step(U, 0.1, eps)
    want_theta = _abelian_step(theta, 0.1, eps)
    want = np.zeros_like(U)
    for a in range(3):
        want[..., a, a] = np.exp(1j * want_theta[a])
    assert np.abs(got - want).max() < 1e-13


def test_smear_link_matches_full_step(O, U):
    full = O.smear_step(U, 0.1, -0.25)
    for site, mu in ((0, 0), (100, 3), (255, 1)):
        t, r = divmod(site, 64)
        z, r = divmod(r, 16)
        y, x = divmod(r, 4)
        assert np.array_equal(O.smear_link(U, site, mu, 0.1, -0.25), full[t, z, y, x, mu])
