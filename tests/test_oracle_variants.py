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
  number that is a multiple of the block, with the same trajectory;
- exact maximisation over a subgroup: the maximiser of a^T Q a + 2 h.a on the
  unit sphere beats 200000 sampled points and meets the Lagrange conditions
  (also when h = 0 and when h has no component along the top eigenvector, a
  closed form); exact updates never lower the local functional (omega = 1),
  reach the single-link maximum 9 and a stationary point, and on average end
  above the linearised update.
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


# ---- exact maximisation over each SU(2) subgroup ---------------------------------------
def _f(Q, h, a):
    return a @ Q @ a + 2 * h @ a


def _sphere_samples(rng, n):
    a = rng.normal(size=(n, 4))
    return a / np.linalg.norm(a, axis=1)[:, None]


def test_sphere_max_beats_dense_sampling_and_is_stationary(O):
    rng = np.random.default_rng(5)
    A = _sphere_samples(rng, 200000)
    for _ in range(10):
        B = rng.normal(size=(4, 4))
        Q = B + B.T
        h = rng.normal(size=4)
        a = O.sphere_max(Q, h)
        assert abs(np.linalg.norm(a) - 1) < 1e-13
        best = (np.einsum("ni,ij,nj->n", A, Q, A) + 2 * A @ h).max()
        assert _f(Q, h, a) >= best - 1e-12
        # Lagrange: Q a + h = lambda a with lambda >= the top eigenvalue of Q
        g = Q @ a + h
        lam = g @ a
        assert np.abs(g - lam * a).max() < 1e-9 and lam >= np.linalg.eigvalsh(Q).max() - 1e-9


def test_sphere_max_special_cases(O):
    rng = np.random.default_rng(6)
    A = _sphere_samples(rng, 200000)
    # h = 0: the top eigenvector
    Q = np.diag([0.5, 2.0, -1.0, 1.0])
    a = O.sphere_max(Q, np.zeros(4))
    assert abs(abs(a[1]) - 1) < 1e-13 and abs(_f(Q, np.zeros(4), a) - 2.0) < 1e-13
    # h orthogonal to the top eigenvector and small: the maximiser leaves the eigenvector plane
    Q = np.diag([3.0, 1.0, 0.0, -1.0])
    h = np.array([0.0, 0.5, 0.2, 0.0])
    a = O.sphere_max(Q, h)
    best = (np.einsum("ni,ij,nj->n", A, Q, A) + 2 * A @ h).max()
    assert abs(np.linalg.norm(a) - 1) < 1e-13 and _f(Q, h, a) >= best - 1e-12
    want = np.array([np.sqrt(1 - 0.25 ** 2 - (0.2 / 3) ** 2), 0.25, 0.2 / 3, 0.0])
    assert np.abs(np.abs(a) - want).max() < 1e-12


def test_exact_hits_never_lower_the_functional_and_converge(O, S):
    rng = np.random.default_rng(7)
    for _ in range(10):
        M = rand_m(rng)
        prev = F(np.eye(3), M)
        for h in range(1, 6):
            g = O.site_g_exact(M, 1.0, h)
            f = F(g, M)
            assert f >= prev - 1e-10 * max(prev, 1.0)
            assert np.abs(g @ g.conj().T - np.eye(3)).max() < 1e-13
            prev = f
    # one link: the centre maximum 9; many hits: a stationary point of the local problem
    U = rand_m(None, 1, True, S)[0]
    M = np.zeros((8, 3, 3), np.complex128)
    M[0] = U
    assert abs(F(O.site_g_exact(M, 1.0, 200), M) - 9.0) < 1e-9
    M = rand_m(None, 8, True, S)
    g = O.site_g_exact(M, 1.0, 400)
    Y = g @ sum(np.conj(np.trace(g @ m)) * m for m in M)
    A = (Y - Y.conj().T) / 2
    A -= np.trace(A) / 3 * np.eye(3)
    assert np.abs(A).max() < 1e-9 * np.abs(Y).max()


def test_exact_first_step_beats_the_linearised_one(O):
    """With one hit and omega = 1 the exact update maximises each subgroup in
    turn, so on random links it ends higher than the linearised update
    (statistically: in most trials and on average)."""
    rng = np.random.default_rng(8)
    wins, gain = 0, 0.0
    for _ in range(40):
        M = rand_m(rng)
        fe, fl = F(O.site_g_exact(M, 1.0, 1), M), F(O.site_g(M, 1.0), M)
        wins += fe >= fl
        gain += fe - fl
    assert wins >= 30 and gain > 0


def test_fix_with_exact_steps(O, S):
    L = (4, 4, 4, 4)
    U = S.heatbath_field(L, S.sub_seed(6003), 5.7, 3)
    G = S.haar_gauge(L, S.sub_seed(6004))
    W = O.apply_gauge(U, G)
    r = O.functional(W)
    for par in (0, 1, 0, 1):
        W, G = O.halfsweep(W, G, par, 1.0, exact=True)
        r2 = O.functional(W)
        assert r2 >= r - 1e-14
        r = r2
    assert np.abs(O.apply_gauge(U, G) - W).max() < 1e-12
    Ge, ie, te = O.mcg_fix(U, tol=1e-9, max_sweeps=3000, omega=1.0, want_traj=True, exact=True)
    assert ie["status"] == 0 and (np.diff(te) > -1e-14).all() and ie["theta"] < 1e-6
