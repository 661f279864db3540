"""Pins of the oracle's update-rule variants: re-linearisation hits of the
local MCG update and the block-wise stop test (Sec. II.A, Table I's blocks of
50 iterations).

- one hit is the plain update, bit for bit;
- every further hit is again a minorise-maximise step: the local functional
  F(g) = sum_k |tr(g M_k)|^2 never decreases from hit to hit (random,
  non-unitary M, omega in [0, 2]);
- for a single link M = U in SU(3) the maximum of |tr(g U)|^2 is 9, at g = z U^dagger
  with z a centre element; repeated hits reach it;
- at convergence of the hits the local problem is stationary: the traceless
  anti-Hermitian part of g X_g vanishes;
- a block-wise stop test changes only where the iteration stops, on a sweep
  number that is a multiple of the block, with the same trajectory.
"""
import numpy as np
import pytest


def rand_m(rng, n=8, unitary=False, S=None):
    if unitary:
        return np.stack([S.haar_links((2, 2, 2, 2), 900 + i)[0, 0, 0, 0, 0] for i in range(n)])
    return rng.normal(size=(n, 3, 3)) + 1j * rng.normal(size=(n, 3, 3))


def F(g, M):
    return sum(abs(np.trace(g @ m)) ** 2 for m in M)


def test_one_hit_is_the_plain_update(O):
    rng = np.random.default_rng(1)
    for _ in range(5):
        M = rand_m(rng)
        assert np.array_equal(O.site_g_hits(M, 1.7, 1), O.site_g(M, 1.7))


@pytest.mark.parametrize("omega", [0.5, 1.0, 1.7, 2.0])
def test_each_hit_never_lowers_the_local_functional(O, omega):
    rng = np.random.default_rng(2)
    for _ in range(20):
        M = rand_m(rng)
        prev = F(np.eye(3), M)
        for h in range(1, 7):
            g = O.site_g_hits(M, omega, h)
            f = F(g, M)
            assert f >= prev - 1e-10 * max(prev, 1.0), (omega, h)
            assert np.abs(g @ g.conj().T - np.eye(3)).max() < 1e-13 and abs(np.linalg.det(g) - 1) < 1e-13
            prev = f


def test_single_link_reaches_the_centre_maximum(O, S):
    U = rand_m(None, 1, True, S)[0]
    M = np.zeros((8, 3, 3), np.complex128)
    M[0] = U
    g = O.site_g_hits(M, 1.0, 400)
    assert abs(F(g, M) - 9.0) < 1e-9
    # g U is a centre element
    z = np.trace(g @ U) / 3
    assert abs(abs(z) - 1) < 1e-9 and abs(z ** 3 - 1) < 1e-8
    assert np.abs(g @ U - z * np.eye(3)).max() < 1e-6


def test_converged_hits_are_stationary(O, S):
    M = rand_m(None, 8, True, S)
    g = O.site_g_hits(M, 1.0, 2000)
    X = sum(np.conj(np.trace(g @ m)) * m for m in M)
    Y = g @ X
    A = (Y - Y.conj().T) / 2
    A -= np.trace(A) / 3 * np.eye(3)
    assert np.abs(A).max() < 1e-9 * np.abs(Y).max()
    # while after one hit it is not
    g1 = O.site_g_hits(M, 1.0, 1)
    Y1 = g1 @ sum(np.conj(np.trace(g1 @ m)) * m for m in M)
    A1 = (Y1 - Y1.conj().T) / 2
    assert np.abs(A1 - np.trace(A1) / 3 * np.eye(3)).max() > 1e-3 * np.abs(Y1).max()


def test_fix_with_hits_raises_r_per_halfsweep(O, S):
    L = (4, 4, 4, 4)
    U = S.heatbath_field(L, S.sub_seed(6000), 5.7, 3)
    G = S.haar_gauge(L, S.sub_seed(6001))
    W = O.apply_gauge(U, G)
    r = O.functional(W)
    for par in (0, 1, 0, 1):
        W, G = O.halfsweep(W, G, par, 1.7, hits=3)
        r2 = O.functional(W)
        assert r2 >= r - 1e-14
        r = r2
    # W stays the transform of U by the accumulated G
    assert np.abs(O.apply_gauge(U, G) - W).max() < 1e-12


def test_block_stop_only_moves_the_stop(O, S):
    L = (4, 4, 4, 4)
    U = S.heatbath_field(L, S.sub_seed(6002), 5.7, 5)
    Ga, ia, ta = O.mcg_fix(U, tol=1e-9, max_sweeps=2000, want_traj=True)
    Gb, ib, tb = O.mcg_fix(U, tol=1e-9, max_sweeps=2000, want_traj=True, stop_every=50)
    assert ia["status"] == ib["status"] == 0
    assert ib["sweeps"] % 50 == 0 and ib["sweeps"] >= ia["sweeps"]
    Gc, ic, tc = O.mcg_fix(U, tol=-1.0, max_sweeps=ib["sweeps"], want_traj=True)
    assert np.array_equal(tb, tc) and np.array_equal(Gb, Gc)
    assert np.array_equal(ta, tc[: ia["sweeps"] + 1])
