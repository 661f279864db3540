"""Pins of the oracle's centre projection and P-vortex count (Sec. II.A)."""
import numpy as np
import pytest

from helpers import center_links, gauge_transform, identity_gauge, planted_field

L4 = (4, 4, 4, 4)


def test_projection_of_center_field_is_exact(O, S):
    m = S.z3_links(L4, S.sub_seed(401))
    Z, margin = O.center_project(center_links(m))
    assert np.array_equal(Z, m)
    assert np.abs(margin - np.pi / 3).max() < 1e-14


def test_projection_through_G_matches_transformed_field(O, S):
    U = S.heatbath_field(L4, S.sub_seed(402), 5.7, 5)
    G = S.haar_gauge(L4, S.sub_seed(403))
    Z1, m1 = O.center_project(U, G)
    Z2, m2 = O.center_project(gauge_transform(U, G))
    ok = m1 > 1e-12
    assert np.array_equal(Z1[ok], Z2[ok])
    assert np.all((m1 >= 0) & (m1 <= np.pi / 3 + 1e-15))


def test_zero_trace_gives_m0(O):
    w = np.exp(2j * np.pi / 3)
    U = np.zeros((2, 2, 2, 2, 4, 3, 3), complex)
    U[...] = np.diag([1, w, w * w])  # tr = 1 + w + w^2 = 0 up to rounding
    Z, margin = O.center_project(U)
    # |t| ~ 1e-16: the phase is arbitrary, but margin and m stay in range
    assert np.all(np.isin(Z, (-1, 0, 1)))
    U[...] = 0
    Z, margin = O.center_project(U)
    assert np.all(Z == 0) and np.all(margin == 0)


def test_nearest_phase_rule(O):
    """For t = r e^{i phi}, m is the centre phase nearest to phi and the
    margin is pi/3 minus the distance to it."""
    rng = np.random.default_rng(2)
    phis = rng.uniform(-np.pi, np.pi, 64)
    U = np.zeros((2, 2, 2, 2, 4, 3, 3), complex)
    flat = U.reshape(64, 3, 3)
    for k, ph in enumerate(phis):
        flat[k, 0, 0] = 3 * np.exp(1j * ph)  # t = 3 e^{i phi}
    Z, margin = O.center_project(U)
    cands = np.array([0, 1, -1])
    for k, ph in enumerate(phis):
        d = np.abs(np.angle(np.exp(1j * (ph - 2 * np.pi * cands / 3))))
        assert Z.reshape(-1)[k] == cands[np.argmin(d)]
        assert abs(margin.reshape(-1)[k] - (np.pi / 3 - d.min())) < 1e-14


def test_center_phases_evenly_distributed(O, S):
    """The phases of the fixed links stay evenly spread over m = -1, 0, 1."""
    U = S.heatbath_field((6, 6, 6, 6), S.sub_seed(404), 5.7, 20)
    G, info, _ = O.mcg_fix(U, tol=1e-7, max_sweeps=3000)
    Z, _ = O.center_project(U, G)
    frac = np.array([(Z == m).mean() for m in (-1, 0, 1)])
    assert np.abs(frac - 1 / 3).max() < 0.03


def test_z3_gauge_transform_shifts_m(O, S):
    m = S.z3_links(L4, S.sub_seed(405))
    a = S.z3_links(L4, S.sub_seed(406))[..., 0]
    g = np.exp(2j * np.pi * a / 3)[..., None, None] * np.eye(3)
    Z, _ = O.center_project(gauge_transform(center_links(m), g))
    for mu in range(4):
        want = (m[..., mu] + a - np.roll(a, -1, axis=3 - mu) + 1) % 3 - 1
        assert np.array_equal(Z[..., mu], want)


def _bianchi_residual(n):
    """For every 3-cube (mu < nu < la): the oriented sum of the six face
    fluxes, mod 3.  Faces: F_{mu nu}, F_{nu la}, F_{la mu} = -F_{mu la}."""
    planes = [(0, 1), (0, 2), (0, 3), (1, 2), (1, 3), (2, 3)]
    idx = {p: k for k, p in enumerate(planes)}
    sh = lambda a, d: np.roll(a, -1, axis=3 - d)  # noqa: E731
    res = []
    for mu, nu, la in ((0, 1, 2), (0, 1, 3), (0, 2, 3), (1, 2, 3)):
        Fmn = n[..., idx[(mu, nu)]].astype(int)
        Fnl = n[..., idx[(nu, la)]].astype(int)
        Fml = n[..., idx[(mu, la)]].astype(int)
        r = (sh(Fmn, la) - Fmn) + (sh(Fnl, mu) - Fnl) - (sh(Fml, nu) - Fml)
        res.append(r % 3)
    return np.array(res)


def test_vortex_bianchi_and_counts(O, S):
    m = S.z3_links(L4, S.sub_seed(407))
    out = O.count_vortices(m, want_n=True)
    assert np.all(_bianchi_residual(out["n"]) == 0)
    assert out["total"] == sum(out["per_plane"]) == sum(out["per_charge"])
    assert out["total"] == int(np.count_nonzero(out["n"]))


def test_random_z3_density_two_thirds(O, S):
    m = S.z3_links((8, 8, 8, 8), S.sub_seed(408))
    out = O.count_vortices(m)
    nplaq = 6 * 8 ** 4
    d = out["total"] / nplaq
    assert abs(d - 2 / 3) < 5 * np.sqrt(2 / 9 / nplaq)


def test_pure_gauge_has_no_vortices_and_one_flip_makes_six(O, S):
    a = S.z3_links(L4, S.sub_seed(409))[..., 0].astype(int)
    m = np.stack([(a - np.roll(a, -1, axis=3 - mu) + 1) % 3 - 1 for mu in range(4)], axis=-1).astype(np.int8)
    assert O.count_vortices(m)["total"] == 0
    m2 = m.copy()
    m2[1, 2, 3, 0, 2] = (m2[1, 2, 3, 0, 2] + 2) % 3 - 1
    out = O.count_vortices(m2)
    assert out["total"] == 6  # a link lies on 2 x 3 plaquettes in 4D
    assert out["per_plane"][1] == 2 and out["per_plane"][3] == 2 and out["per_plane"][5] == 2


def test_planted_pipeline(O, S):
    """Planted U = g Z g^dag: after fixing, the projected field equals the
    planted m up to a Z3 gauge transform, and the vortex count equals the
    count of the planted integers."""
    Up, g, m = planted_field(S, L4, 410)
    G, info, _ = O.mcg_fix(Up, tol=1e-12, max_sweeps=5000)
    assert info["R"] > 1 - 1e-10
    Z, margin = O.center_project(Up, G)
    assert margin.min() > 1.0
    assert O.count_vortices(Z)["total"] == O.count_vortices(m)["total"]
    # Z - m = a(x) - a(x+mu) mod 3: recover a by walking a spanning tree
    d = (Z.astype(int) - m.astype(int)) % 3
    a = np.zeros(d.shape[:4], int)
    for t in range(L4[3]):
        for z in range(L4[2]):
            for y in range(L4[1]):
                for x in range(L4[0]):
                    if x > 0:
                        a[t, z, y, x] = (a[t, z, y, x - 1] - d[t, z, y, x - 1, 0]) % 3
                    elif y > 0:
                        a[t, z, y, x] = (a[t, z, y - 1, x] - d[t, z, y - 1, x, 1]) % 3
                    elif z > 0:
                        a[t, z, y, x] = (a[t, z - 1, y, x] - d[t, z - 1, y, x, 2]) % 3
                    elif t > 0:
                        a[t, z, y, x] = (a[t - 1, z, y, x] - d[t - 1, z, y, x, 3]) % 3
    for mu in range(4):
        assert np.array_equal(d[..., mu], (a - np.roll(a, -1, axis=3 - mu)) % 3)
