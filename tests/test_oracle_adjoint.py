"""Pins of the oracle's FP64 adjoint of the smeared-field MCG loss
L = R(S_n(U; rho, eps)^{G*}) at fixed G*."""
import numpy as np
import pytest

from helpers import dag, inner, random_su3

L4 = (4, 4, 4, 4)


@pytest.fixture(scope="module")
def setup(S, O):
    U = S.heatbath_field(L4, S.sub_seed(501), 5.7, 10)
    Sm = O.smear(U, 0.06, -0.25, 3)
    G, info, _ = O.mcg_fix(Sm, tol=1e-12, max_sweeps=3000)
    return U, G


def _tangent(S, L, seed):
    return S.su3_tangent(L, S.sub_seed(seed))


def _fd(f, h):
    """Fourth-order central difference of f at 0 with step h: the rho
    direction has a large third derivative, so the second-order stencil
    carries a truncation error of ~1e-6 relative at h = 1e-4."""
    return (-f(2 * h) + 8 * f(h) - 8 * f(-h) + f(-2 * h)) / (12 * h)


@pytest.mark.parametrize("eps", [1.0, -0.25])
def test_grad_matches_central_differences(O, S, setup, eps):
    U, G = setup
    rho, n, h = 0.06, 3, 1e-4
    g, drho, deps, loss = O.smear_loss_grad(U, rho, eps, n, G)
    assert abs(loss - O.smear_loss(U, rho, eps, n, G)) < 1e-15
    fd_rho = _fd(lambda s: O.smear_loss(U, rho + s, eps, n, G), h)
    assert abs(fd_rho - drho) <= 1e-6 * max(abs(drho), 1e-3)
    fd_eps = _fd(lambda s: O.smear_loss(U, rho, eps + s, n, G), h)
    assert abs(fd_eps - deps) <= 1e-6 * max(abs(deps), 1e-3)
    # random su(3) tangent: U_l -> exp(h X_l) U_l, dL/dh = sum <grad_l, X_l U_l>
    X = _tangent(S, L4, 502)
    Xf = X.reshape(-1, 3, 3)

    def moved(s):
        E = np.array([O.exp_taylor(s * x) for x in Xf]).reshape(U.shape)
        return E @ U

    fd = _fd(lambda s: O.smear_loss(moved(s), rho, eps, n, G), h)
    an = inner(g, X @ U)
    assert abs(fd - an) <= 1e-6 * max(abs(an), 1e-3)


@pytest.mark.parametrize("eps", [1.0, -0.25])
def test_dot_product_jvp_vjp(O, S, eps):
    """<J v, w> = <v, J^T w> for one smearing step: the forward-mode and
    reverse-mode codes are independent."""
    U = S.heatbath_field(L4, S.sub_seed(503), 5.7, 5)
    rng = np.random.default_rng(1)
    v = rng.normal(size=U.shape) + 1j * rng.normal(size=U.shape)
    w = rng.normal(size=U.shape) + 1j * rng.normal(size=U.shape)
    Jv = O.step_jvp(U, v, 0.1, eps)
    JTw, _, _ = O.step_vjp(U, w, 0.1, eps)
    a, b = inner(Jv, w), inner(v, JTw)
    assert abs(a - b) <= 1e-13 * max(abs(a), 1.0)


def test_jvp_matches_finite_difference(O, S):
    U = S.heatbath_field(L4, S.sub_seed(504), 5.7, 5)
    X = _tangent(S, L4, 505)
    dU = X @ U
    h = 1e-5
    Xf = X.reshape(-1, 3, 3)
    Ep = np.array([O.exp_taylor(h * x) for x in Xf]).reshape(U.shape)
    Em = np.array([O.exp_taylor(-h * x) for x in Xf]).reshape(U.shape)
    fd = (O.smear_step(Ep @ U, 0.1, -0.25) - O.smear_step(Em @ U, 0.1, -0.25)) / (2 * h)
    assert np.abs(fd - O.step_jvp(U, dU, 0.1, -0.25)).max() < 1e-8


def test_rho_zero_gives_zero_eps_derivative(O, setup):
    U, G = setup
    _, drho, deps, _, scale = O.smear_loss_grad(U, 0.0, -0.25, 2, G, want_eps_scale=True)
    assert deps == 0.0 and scale == 0.0


def test_eps_term_scale_bounds_the_derivative(O, setup):
    """The summed magnitude of the terms of dL/deps bounds |dL/deps| (triangle inequality) and
    does not depend on checkpointing; the gradient itself is unchanged by asking for it."""
    U, G = setup
    a = O.smear_loss_grad(U, 0.06, -0.25, 4, G, ckpt_every=2, want_eps_scale=True)
    b = O.smear_loss_grad(U, 0.06, -0.25, 4, G, ckpt_every=0, want_eps_scale=True)
    c = O.smear_loss_grad(U, 0.06, -0.25, 4, G, ckpt_every=2)
    assert a[4] >= abs(a[2]) > 0 and a[4] == b[4]
    assert np.array_equal(a[0], c[0]) and a[1:4] == c[1:4]


def test_checkpointing_is_bitwise(O, setup):
    U, G = setup
    a = O.smear_loss_grad(U, 0.06, -0.25, 6, G, ckpt_every=1)
    b = O.smear_loss_grad(U, 0.06, -0.25, 6, G, ckpt_every=5)
    c = O.smear_loss_grad(U, 0.06, -0.25, 6, G, ckpt_every=0)
    for other in (b, c):
        assert np.array_equal(a[0], other[0]) and a[1:] == other[1:]


def test_gradient_orthogonal_to_gauge_directions_at_stationary_g(O, S):
    """L(U^Lambda) at G* Lambda^dag equals L(U) at G*; at a stationary G* the
    derivative along G* vanishes, so the gradient is orthogonal to every
    infinitesimal gauge direction U_mu(x) -> U_mu(x) + lam(x) U_mu(x) - U_mu(x) lam(x+mu)."""
    U = S.heatbath_field(L4, S.sub_seed(506), 5.7, 10)
    Sm = O.smear(U, 0.1, 1.0, 2)
    G, info, _ = O.mcg_fix(Sm, tol=1e-14, max_sweeps=5000)
    assert info["theta"] < 1e-10
    g, _, _, _ = O.smear_loss_grad(U, 0.1, 1.0, 2, G)
    rng = np.random.default_rng(8)
    lam = random_su3(rng, 256, 1.0).reshape(G.shape)
    dU = np.empty_like(U)
    for mu in range(4):
        dU[..., mu, :, :] = lam @ U[..., mu, :, :] - U[..., mu, :, :] @ np.roll(lam, -1, axis=3 - mu)
    gauge_part = inner(g, dU)
    scale = np.sqrt(inner(g, g) * inner(dU, dU))
    assert abs(gauge_part) < 1e-6 * scale
    # generic directions of the same size are far from orthogonal
    ctrl = []
    for s in range(5):
        X = S.su3_tangent(L4, S.sub_seed(507 + s)) @ U
        X *= np.sqrt(inner(dU, dU) / inner(X, X))
        ctrl.append(abs(inner(g, X)))
    assert max(ctrl) > 1e-3 * scale
