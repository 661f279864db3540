"""Pins of the oracle's MCG functional and fixing (Sec. II.A, II.B)."""
import numpy as np
import pytest

from helpers import (center_links, dag, gauge_transform, identity_gauge, planted_field,
                     random_su3, unitarity_error)

L4 = (4, 4, 4, 4)


@pytest.fixture(scope="module")
def U(S):
    return S.heatbath_field(L4, S.sub_seed(201), 5.7, 20)


def test_functional_range_and_haar_mean(O, S):
    """R in [0, 1]; for Haar-random links E|tr U|^2 = 1, so E[R] = 1/9."""
    L = (8, 8, 8, 8)
    U = S.haar_links(L, S.sub_seed(202))
    R = O.functional(U)
    n = 4 * 8 ** 4
    # |tr U|^2 for Haar SU(3) has variance 1: 5 standard errors
    assert abs(R - 1 / 9) < 5 * (1 / 9) / np.sqrt(n)
    assert O.functional(center_links(np.zeros((2, 2, 2, 2, 4)))) == 1.0


def test_functional_is_invariant_under_z3_gauge_transforms(O, S, U):
    a = S.z3_links(L4, S.sub_seed(203))[..., 0]
    g = np.exp(2j * np.pi * a / 3)[..., None, None] * np.eye(3)
    assert abs(O.functional(gauge_transform(U, g)) - O.functional(U)) < 1e-15


def test_site_step_never_lowers_local_functional(O):
    """Minorise-maximise: F(g) = sum_k |tr(g M_k)|^2 >= F(1) for the g built
    by one local update, for arbitrary (even non-unitary) M_k and any omega
    in [0, 2]."""
    rng = np.random.default_rng(9)
    for omega in (0.0, 0.5, 1.0, 1.7, 2.0):
        for _ in range(200):
            M = rng.normal(size=(8, 3, 3)) + 1j * rng.normal(size=(8, 3, 3))
            g = O.site_g(M, omega)
            F1 = np.sum(np.abs(np.trace(M, axis1=1, axis2=2)) ** 2)
            Fg = np.sum(np.abs(np.trace(g @ M, axis1=1, axis2=2)) ** 2)
            assert Fg >= F1 * (1 - 1e-14)
            assert unitarity_error(g) < 1e-14


def test_subgroup_step_is_argmax_of_linear_minorant(O):
    """For X supported on the (0,1) block and omega = 1, the local update
    reaches at least max over SU(2)_(0,1) of Re tr(s X), found here by a dense
    random sample of S^3 (the first subgroup step attains that maximum and
    the later steps cannot lower Re tr(g X))."""
    rng = np.random.default_rng(13)
    a = rng.normal(size=(200000, 4))
    a /= np.linalg.norm(a, axis=1, keepdims=True)
    s = np.zeros((len(a), 2, 2), complex)
    s[:, 0, 0] = a[:, 0] + 1j * a[:, 3]
    s[:, 0, 1] = a[:, 2] + 1j * a[:, 1]
    s[:, 1, 0] = -a[:, 2] + 1j * a[:, 1]
    s[:, 1, 1] = a[:, 0] - 1j * a[:, 3]
    for _ in range(5):
        M = np.zeros((8, 3, 3), complex)
        M[:, :2, :2] = rng.normal(size=(8, 2, 2)) + 1j * rng.normal(size=(8, 2, 2))
        X = np.einsum("k,kij->ij", np.conj(np.trace(M, axis1=1, axis2=2)), M)
        grid = np.max(np.real(np.einsum("nij,ji->n", s, X[:2, :2])))
        g = O.site_g(M, 1.0)
        got = np.real(np.trace(g @ X))
        assert got >= grid - 1e-12
        assert got >= np.real(np.trace(X)) - 1e-12


@pytest.mark.parametrize("omega", [1.0, 1.7, 1.9])
def test_r_never_decreases_per_halfsweep(O, U, omega):
    W, G = U.copy(), identity_gauge(L4)
    R = O.functional(W)
    for it in range(30):
        for p in (0, 1):
            W, G = O.halfsweep(W, G, p, omega)
            Rn = O.functional(W)
            assert Rn >= R - 1e-15
            R = Rn
    # W stays equal to U^G
    assert np.abs(W - O.apply_gauge(U, G)).max() < 1e-13


def test_fix_converges_to_stationary_local_maximum(O, S, U):
    G, info, traj = O.mcg_fix(U, tol=1e-12, max_sweeps=5000, omega=1.7, want_traj=True)
    assert info["status"] == 0
    assert np.all(np.diff(traj) >= -1e-15)
    assert info["theta"] < 1e-8
    assert unitarity_error(G) < 1e-13
    # local maximum: random small per-site perturbations of G never raise R
    rng = np.random.default_rng(4)
    R0 = O.functional(O.apply_gauge(U, G))
    for _ in range(10):
        X = random_su3(rng, 256, 1e-3).reshape(G.shape)
        Gp = np.einsum("...ij,...jk->...ik", np.array([O.exp_taylor(x) for x in X.reshape(-1, 3, 3)]).reshape(G.shape), G)
        assert O.functional(O.apply_gauge(U, Gp)) <= R0 + 1e-12


def test_gauge_invariants_unchanged_by_fixing(O, U):
    G, info, _ = O.mcg_fix(U, tol=1e-9, max_sweeps=2000)
    W = O.apply_gauge(U, G)
    assert abs(O.plaquette(W) - O.plaquette(U)) < 1e-12
    for r, t in ((1, 1), (2, 1), (2, 2)):
        assert abs(O.wilson_loop(W, r, t) - O.wilson_loop(U, r, t)) < 1e-12
    assert np.abs(O.polyakov(W) - O.polyakov(U)).max() < 1e-12


def test_planted_center_field_fixes_to_one(O, S):
    """U = g Z g^dag: the global maximum R = 1 is reached from at least one of
    a few Haar-random starting transforms (here: from the identity)."""
    Up, g, m = planted_field(S, L4, 301)
    best = 0
    for copy in range(4):
        G0 = None if copy == 0 else S.haar_gauge(L4, S.sub_seed(302), copy)
        G, info, _ = O.mcg_fix(Up, G0=G0, tol=1e-12, max_sweeps=5000, omega=1.7)
        best = max(best, info["R"])
        if best > 1 - 1e-10:
            break
    assert best > 1 - 1e-10


def test_precondition_identity(O, S, U):
    """Fixing U from G_s is fixing U^{G_s} from the identity, composed with G_s."""
    Gs = S.haar_gauge(L4, S.sub_seed(303))
    G1, i1, t1 = O.mcg_fix(U, G0=Gs, tol=1e-9, max_sweeps=120, want_traj=True)
    G2, i2, t2 = O.mcg_fix(O.apply_gauge(U, Gs), tol=1e-9, max_sweeps=120, want_traj=True)
    assert i1["sweeps"] == i2["sweeps"]
    assert np.abs(t1 - t2).max() < 1e-13
    assert np.abs(G1 - np.einsum("...ij,...jk->...ik", G2, Gs)).max() < 1e-12


def test_resume_from_block_boundary_is_bitwise(O, U):
    """Stopping after a multiple of reunit_every sweeps and resuming with
    start_sweep gives the bits of an uninterrupted run."""
    Ga, ia, _ = O.mcg_fix(U, tol=-1.0, max_sweeps=100, reunit_every=50)
    Gb, ib, _ = O.mcg_fix(U, tol=-1.0, max_sweeps=50, reunit_every=50)
    assert ib["status"] == 1
    Gc, ic, _ = O.mcg_fix(U, G0=Gb, tol=-1.0, max_sweeps=50, reunit_every=50, start_sweep=50)
    assert np.array_equal(Ga, Gc)
    assert ia["R"] == ic["R"]


def test_max_sweeps_reports_not_converged(O, U):
    G, info, _ = O.mcg_fix(U, tol=1e-12, max_sweeps=1)
    assert info["status"] == 1 and info["sweeps"] == 1
    assert unitarity_error(G) < 1e-14


def _one_link_field(L, x0, alpha, beta):
    """Unit links except U_0 at site x0 = diag(e^{i a}, e^{i b}, e^{-i(a+b)})."""
    U = np.zeros(tuple(L[::-1]) + (4, 3, 3), np.complex128)
    U[..., :, 0, 0] = U[..., :, 1, 1] = U[..., :, 2, 2] = 1
    d = np.exp(1j * np.array([alpha, beta, -alpha - beta]))
    U[x0[3], x0[2], x0[1], x0[0], 0] = np.diag(d)
    return U, d


def test_theta_closed_form_one_link(O):
    """theta = (1/V) sum_x |TA X(x)|^2.  With every link 1 except one diagonal D = U_0(x0), X is a
    multiple of 1 except at x0 (X = 21 + conj(t) D, t = tr D) and at x0 + 0 (X = 21 + t D^dagger);
    TA of a diagonal A is i(Im A_kk - mean_j Im A_jj) on the diagonal, and Im(t conj d_k) =
    -Im(conj(t) d_k), so theta = (2/V) sum_k (Im(conj(t) d_k) - mean)^2."""
    L = (4, 2, 2, 2)
    U, d = _one_link_field(L, (1, 0, 1, 0), 0.7, -0.2)
    t = d.sum()
    im = (np.conj(t) * d).imag
    want = 2 * np.sum((im - im.mean()) ** 2) / np.prod(L)
    assert abs(O.theta(U) - want) < 1e-15 and want > 0.1
    # a pure centre field is stationary
    assert O.theta(center_links(np.ones((2, 2, 2, 2, 4)))) == 0.0


def test_site_g_at_closed_form(O, S):
    """A unit field with one site x0 transformed by h^dagger: the eight links the update gathers at
    x0 are all M_k = h^dagger (forward g(x0) 1, backward (1 g(x0)^dagger)^dagger), so the
    linearisation is X = 8 tr(h) h^dagger.  For h in the (0, 1) subgroup with tr h > 0 the (0, 1)
    step at omega = 1 maximises Re tr(s X) at s = h, and the other two steps then see a multiple of
    1: the update is g = h exactly, which takes the site back to the unit field."""
    L = (4, 4, 2, 2)
    a = np.array([0.6, 0.3, -0.5, 0.2])
    a /= np.linalg.norm(a)
    h = np.eye(3, dtype=np.complex128)
    h[:2, :2] = [[a[0] + 1j * a[3], a[2] + 1j * a[1]], [-a[2] + 1j * a[1], a[0] - 1j * a[3]]]
    g = np.tile(np.eye(3, dtype=np.complex128), tuple(L[::-1]) + (1, 1))
    x0 = (2, 1, 1, 0)
    g[x0[3], x0[2], x0[1], x0[0]] = dag(h)
    U = gauge_transform(center_links(np.zeros(tuple(L[::-1]) + (4,))), g)
    i = x0[0] + L[0] * (x0[1] + L[1] * (x0[2] + L[2] * x0[3]))
    assert np.abs(O.site_g_at(U, i, 1.0) - h).max() < 1e-14
