"""Checks of the seeded input generator (inputs only, no method arithmetic)."""
import ctypes as C

import numpy as np
import pytest

from helpers import dag, unitarity_error


def test_elementary_functions(S):
    xs = np.random.default_rng(0).uniform(1e-300, 1, 2000)
    lib = S.cpu()
    assert max(abs(lib.sy_cpu_log(float(x)) - np.log(x)) for x in xs) < 2e-15 * 700
    assert max(abs(lib.sy_cpu_log(float(x)) - np.log(x)) / abs(np.log(x)) for x in xs) < 1e-15
    assert max(abs(lib.sy_cpu_sqrt(float(x)) - np.sqrt(x)) / np.sqrt(x) for x in xs) < 1e-15
    assert max(abs(lib.sy_cpu_recip(float(x)) * x - 1) for x in xs) < 1e-15
    s, c = C.c_double(), C.c_double()
    for r in np.linspace(0, 1, 1001):
        lib.sy_cpu_sincos_turn(float(r), C.byref(s), C.byref(c))
        assert abs(s.value - np.sin(2 * np.pi * r)) < 1e-15
        assert abs(c.value - np.cos(2 * np.pi * r)) < 1e-15


def test_determinism_and_seeds(S):
    L = (4, 4, 4, 4)
    a = S.haar_links(L, 7)
    assert np.array_equal(a, S.haar_links(L, 7))
    assert not np.array_equal(a, S.haar_links(L, 8))
    h = S.heatbath_field(L, 3, 5.7, 2)
    assert np.array_equal(h, S.heatbath_field(L, 3, 5.7, 2))
    assert not np.array_equal(S.haar_gauge(L, 3, 0), S.haar_gauge(L, 3, 1))


def test_haar_moments(S):
    """Haar SU(3): E tr U = 0, E |tr U|^2 = 1, E |tr U|^4 = 2."""
    U = S.haar_links((8, 8, 8, 8), 11).reshape(-1, 3, 3)
    assert unitarity_error(U) < 1e-14
    assert np.abs(np.linalg.det(U) - 1).max() < 1e-14
    t = np.trace(U, axis1=1, axis2=2)
    n = len(t)
    assert abs(t.mean()) < 5 / np.sqrt(n)
    assert abs(np.mean(np.abs(t) ** 2) - 1) < 5 / np.sqrt(n)
    assert abs(np.mean(np.abs(t) ** 4) - 2) < 5 * np.sqrt(24 / n)


def test_gaussian_moments(S):
    z = S.gaussians(200000, 5)
    assert abs(z.mean()) < 5 / np.sqrt(len(z))
    assert abs(z.var() - 1) < 5 * np.sqrt(2 / len(z))


def test_z3_uniform(S):
    m = S.z3_links((8, 8, 8, 8), 9)
    assert set(np.unique(m)) == {-1, 0, 1}
    f = np.array([(m == k).mean() for k in (-1, 0, 1)])
    assert np.abs(f - 1 / 3).max() < 0.01


def test_heatbath_plaquette_beta_5p7(S, O):
    """50 sweeps from a Haar start at beta = 5.7: the plaquette approaches its
    equilibrium value (about 0.549 for the Wilson action)."""
    U = S.heatbath_field((8, 8, 8, 8), S.sub_seed(601), 5.7, 50)
    assert unitarity_error(U) < 1e-14
    P = O.plaquette(U)
    assert 0.53 < P < 0.56


# ---- Luscher-Weisz heatbath ----------------------------------------------------------
def _shift(A, mu, k):
    """field value at x + k mu (array axes [t, z, y, x, ...])"""
    return np.roll(A, -k, axis=3 - mu)


def _lw_action(U, beta, c0, c1):
    """beta sum over plaquettes of c0 (1 - Re tr P / 3) plus c1 times the same
    over all 2x1 rectangles (both orientations in each plane), every loop
    multiplied out explicitly."""
    def link(mu, shift=None):
        A = U[..., mu, :, :]
        for nu, k in (shift or {}).items():
            A = _shift(A, nu, k)
        return A

    def dag(A):
        return np.conj(np.swapaxes(A, -1, -2))

    def rtr(A):
        return np.trace(A, axis1=-2, axis2=-1).real / 3

    S = 0.0
    V = U.shape[0] * U.shape[1] * U.shape[2] * U.shape[3]
    for mu in range(4):
        for nu in range(mu + 1, 4):
            P = link(mu) @ link(nu, {mu: 1}) @ dag(link(mu, {nu: 1})) @ dag(link(nu))
            S += c0 * (V - rtr(P).sum())
            # 2x1 long in mu, 2x1 long in nu
            R1 = (link(mu) @ link(mu, {mu: 1}) @ link(nu, {mu: 2}) @ dag(link(mu, {mu: 1, nu: 1}))
                  @ dag(link(mu, {nu: 1})) @ dag(link(nu)))
            R2 = (link(mu) @ link(nu, {mu: 1}) @ link(nu, {mu: 1, nu: 1}) @ dag(link(mu, {nu: 2}))
                  @ dag(link(nu, {nu: 1})) @ dag(link(nu)))
            S += c1 * (2 * V - rtr(R1).sum() - rtr(R2).sum())
    return beta * S


def test_lw_staple_gives_the_action_change_of_one_link(S):
    """The action is linear in each link (no loop holds a link twice), so
    replacing U_mu(x) by V changes it by -(beta/3) Re tr((V - U_mu(x)) A)."""
    import ctypes as C
    L = (4, 4, 4, 4)
    U = S.heatbath_lw_field(L, S.sub_seed(710), 4.52, 2, 0.9)
    beta, u0 = 4.52, 0.9
    c0, c1 = 5 / 3, -1 / (12 * u0 * u0)
    S0 = _lw_action(U, beta, c0, c1)
    rng = np.random.default_rng(3)
    for x, mu in ((0, 0), (37, 2), (255, 3), (100, 1)):
        A = np.empty((3, 3), np.complex128)
        S.cpu().sy_cpu_lw_staple(S._I4(L), U.ctypes.data_as(C.c_void_p), x, mu, c0, c1,
                                 A.ctypes.data_as(C.c_void_p))
        t, r = divmod(x, 64)
        z, r = divmod(r, 16)
        y, xx = divmod(r, 4)
        Vn = S.haar_links((2, 2, 2, 2), 720 + x)[0, 0, 0, 0, int(rng.integers(4))]
        U2 = U.copy()
        old = U2[t, z, y, xx, mu].copy()
        U2[t, z, y, xx, mu] = Vn
        dS = _lw_action(U2, beta, c0, c1) - S0
        want = -(beta / 3) * np.trace((Vn - old) @ A).real
        assert abs(dS - want) < 1e-10 * max(1.0, abs(want)), (x, mu)


def test_lw_colours_separate_links_of_a_common_loop(S):
    """No two links of one direction and one colour lie in a common plaquette
    or rectangle (exhaustive on 4^4 and 8x4x4x4)."""
    for L in ((4, 4, 4, 4), (8, 4, 4, 4)):
        V = L[0] * L[1] * L[2] * L[3]

        def idx(c):
            return (c[0] % L[0]) + L[0] * ((c[1] % L[1]) + L[1] * ((c[2] % L[2]) + L[2] * (c[3] % L[3])))

        col = {(x, mu): S.cpu().sy_cpu_lw_colour(S._I4(L), x, mu) for x in range(V) for mu in range(4)}
        for x in range(V):
            c = [x % L[0], (x // L[0]) % L[1], (x // (L[0] * L[1])) % L[2], x // (L[0] * L[1] * L[2])]
            for mu in range(4):
                for nu in range(4):
                    if nu == mu:
                        continue
                    for d in ({nu: 1}, {nu: 2}, {mu: 1}, {mu: 1, nu: 1}, {mu: 1, nu: -1}):
                        y = list(c)
                        for a, k in d.items():
                            y[a] += k
                        assert col[(x, mu)] != col[(idx(y), mu)], (L, x, mu, d)
        assert sorted(set(col.values())) == list(range(8))


def test_lw_heatbath_thermalises(S, O):
    U = S.heatbath_lw_field((8, 8, 8, 8), S.sub_seed(700), 4.52, 30, 0.884)
    assert unitarity_error(U) < 1e-14
    P = O.plaquette(U)
    # tadpole self-consistency: u0 = P^(1/4) for the chosen u0 = 0.884
    assert 0.59 < P < 0.63 and abs(P ** 0.25 - 0.884) < 0.01
    W21 = O.wilson_loop(U, 2, 1)
    assert 0 < W21 < O.wilson_loop(U, 1, 1)
    with pytest.raises(ValueError, match="divisible by 4"):
        S.heatbath_lw_field((6, 4, 4, 4), 1, 4.52, 1)
