"""Pins of the oracle's Wilson loops and vortex-only / vortex-removed fields
(Sec. III.B) against closed forms and lattice symmetries.

- an abelian field with constant, quantised flux through every (j, t) plane
  gives every contractible loop the phase Phi = sum_j 2 pi n_j D_j T / (L_j L_t)
  (Stokes), whatever the staircase shape, so Re tr/3 is known exactly;
- on a centre (Z3) field a planar loop carries the product of the centre
  fluxes of the plaquettes it encloses;
- loops are gauge invariant, and their orbit averages are invariant under a
  reflection or a permutation of the lattice axes;
- U^G = Z (Z^dagger U^G), the vortex-removed field projects to m = 0 on
  every link, the vortex-only field projects back onto Z.
"""
import itertools

import numpy as np
import pytest


def flux_field(L, n):
    """U(1) links diag(e^{i th}, e^{i th}, e^{-2 i th}) with flux 2 pi n_j / (L_j L_t)
    through every plaquette of the (j, t) planes and none through spatial planes."""
    Lx, Ly, Lz, Lt = L
    t, z, y, x = np.meshgrid(range(Lt), range(Lz), range(Ly), range(Lx), indexing="ij")
    c = [x, y, z]
    th = np.zeros((Lt, Lz, Ly, Lx, 4))
    for j in range(3):
        th[..., j] = np.where(c[j] == L[j] - 1, -2 * np.pi * n[j] * t / Lt, 0.0)
        th[..., 3] += 2 * np.pi * n[j] * c[j] / (L[j] * Lt)
    U = np.zeros(th.shape + (3, 3), np.complex128)
    U[..., 0, 0] = U[..., 1, 1] = np.exp(1j * th)
    U[..., 2, 2] = np.exp(-2j * th)
    return U


def flux_value(L, n, D, T):
    phi = sum(2 * np.pi * n[j] * D[j] * T / (L[j] * L[3]) for j in range(3))
    return (2 * np.cos(phi) + np.cos(2 * phi)) / 3


L_FLUX = (6, 4, 8, 10)
N_FLUX = (1, -2, 3)


@pytest.mark.parametrize("d", [(1, 0, 0), (0, -1, 0), (0, 0, 1), (1, 1, 0), (-1, 1, 0), (2, 1, 0),
                               (1, -1, 1), (2, 1, 1), (-2, -1, 1), (1, 2, 2)])
def test_single_path_abelian_flux_closed_form(O, d):
    U = flux_field(L_FLUX, N_FLUX)
    for k in (1, 2):
        D = [k * v for v in d]
        if any(abs(D[j]) >= L_FLUX[j] for j in range(3)):
            continue
        for T in (1, 2, 5):
            got = O.wilson_path(U, O.staircase(d) * k, T)
            assert abs(got - flux_value(L_FLUX, N_FLUX, D, T)) < 1e-13, (d, k, T)


def test_staircase_reaches_target_and_orbit_sizes(O):
    for d in [(1, 0, 0), (2, 1, 0), (-2, 1, 1), (2, -2, 1), (3, 1, 2)]:
        st = O.staircase(d)
        disp = [sum((1 if s > 0 else -1) for s in st if abs(s) == a + 1) for a in range(3)]
        assert disp == list(d) and len(st) == sum(map(abs, d))
    # distinct images of the staircases under the cubic group: x; x,y; x,y,z; x,y,x; x,y,z,x
    assert [len(O.path_images(O.staircase(v))) for v in [(1, 0, 0), (1, 1, 0), (1, 1, 1), (2, 1, 0), (2, 1, 1)]] \
        == [6, 24, 48, 24, 48]


def test_orbit_average_abelian_flux(O):
    U = flux_field(L_FLUX, N_FLUX)
    vecs = [(1, 0, 0), (1, 1, 0), (2, 1, 0)]
    W = O.wilson_loops(U, vecs, 1, 3)
    for i, v in enumerate(vecs):
        # the displacements of the distinct images of the path, with multiplicity
        st = O.staircase(v)
        paths = {tuple(sg[abs(q) - 1] * np.sign(q) * (p[abs(q) - 1] + 1) for q in st)
                 for p in itertools.permutations(range(3)) for sg in itertools.product((1, -1), repeat=3)}
        disp = [[sum(np.sign(q) for q in path if abs(q) == a + 1) for a in range(3)] for path in paths]
        for T in (1, 2, 3):
            want = np.mean([flux_value(L_FLUX, N_FLUX, D, T) for D in disp])
            assert abs(W[i, 0, T - 1] - want) < 1e-13


def test_onaxis_matches_three_direction_loop(O, S):
    L = (4, 4, 6, 8)
    U = S.heatbath_field(L, S.sub_seed(4000), 5.7, 3)
    W = O.wilson_loops(U, [(1, 0, 0)], 2, 3)
    for r in (1, 2):
        for t in (1, 2, 3):
            assert abs(W[0, r - 1, t - 1] - O.wilson_loop(U, r, t)) < 1e-14
    # the 1x1 loop is the mean space-time plaquette
    P = O.plaquette(U)
    assert 0.2 < W[0, 0, 0] < 0.9 and 0 < P < 1


def test_gauge_invariance(O, S):
    L = (4, 4, 4, 6)
    U = S.heatbath_field(L, S.sub_seed(4001), 5.7, 3)
    G = S.haar_gauge(L, S.sub_seed(4002))
    vecs = [(1, 0, 0), (1, 1, 0), (1, 1, 1), (2, 1, 0)]
    a = O.wilson_loops(U, vecs, 1, 2)
    b = O.wilson_loops(O.apply_gauge(U, G), vecs, 1, 2)
    assert np.abs(a - b).max() < 1e-13


def reflect_x(U):
    """x -> -x: U'_0(x') = U_0(-x'-1)^dagger, U'_mu(x') = U_mu(-x') otherwise."""
    Lx = U.shape[3]
    idx = (-np.arange(Lx)) % Lx
    idx0 = (-np.arange(Lx) - 1) % Lx
    out = U[:, :, :, idx].copy()
    out[..., 0, :, :] = np.conj(np.swapaxes(U[:, :, :, idx0][..., 0, :, :], -1, -2))
    return out


def swap_xy(U):
    out = np.swapaxes(U, 2, 3).copy()
    out[..., [0, 1], :, :] = out[..., [1, 0], :, :]
    return out


def test_orbit_average_is_invariant_under_reflection_and_axis_swap(O, S):
    L = (4, 4, 4, 6)
    U = S.heatbath_field(L, S.sub_seed(4003), 5.7, 3)
    vecs = [(1, 1, 0), (2, 1, 0), (1, 1, 1)]
    a = O.wilson_loops(U, vecs, 1, 2)
    # a single image is not invariant: the pins below would pass trivially otherwise
    one = [O.wilson_path(U, O.staircase((2, 1, 0)), 1), O.wilson_path(reflect_x(U), O.staircase((2, 1, 0)), 1)]
    assert abs(one[0] - one[1]) > 1e-6
    assert np.abs(O.wilson_loops(reflect_x(U), vecs, 1, 2) - a).max() < 1e-13
    assert np.abs(O.wilson_loops(swap_xy(U), vecs, 1, 2) - a).max() < 1e-13
    # reflection and swap are exact symmetries of the plaquette too
    assert abs(O.plaquette(reflect_x(U)) - O.plaquette(U)) < 1e-14


def test_center_field_loops_carry_enclosed_vortex_flux(O, S):
    L = (4, 6, 4, 8)
    m = S.z3_links(L, S.sub_seed(4004))
    Zf = O.vortex_field(np.zeros(m.shape + (3, 3), np.complex128), None, m, O.VORTEX_ONLY)
    n = O.count_vortices(m, want_n=True)["n"].astype(np.int64)  # [t, z, y, x, plane]
    plane_t = {0: 2, 1: 4, 2: 5}  # planes (0,3), (1,3), (2,3)
    ax = {0: 3, 1: 2, 2: 1}  # array axis of spatial direction j
    for r in (1, 2):
        for T in (1, 3):
            vals = []
            for j in range(3):
                M = np.zeros(L[::-1], np.int64)
                for a in range(r):
                    for b in range(T):
                        M += np.roll(np.roll(n[..., plane_t[j]], -a, axis=ax[j]), -b, axis=0)
                vals.append(np.cos(2 * np.pi * M / 3).mean())
            want = np.mean(vals)
            got = O.wilson_loops(Zf, [(1, 0, 0)], r, T)[0, r - 1, T - 1]
            assert abs(got - want) < 1e-13, (r, T)


def test_vortex_fields(O, S):
    L = (4, 4, 4, 6)
    U = S.heatbath_field(L, S.sub_seed(4005), 5.7, 3)
    G = S.haar_gauge(L, S.sub_seed(4006))
    Z, _ = O.center_project(U, G)
    Zf = O.vortex_field(U, G, Z, O.VORTEX_ONLY)
    Vr = O.vortex_field(U, G, Z, O.VORTEX_REMOVED)
    UG = O.apply_gauge(U, G)
    assert np.abs(Zf @ Vr - UG).max() < 1e-14
    z = np.exp(2j * np.pi * Z / 3)
    assert np.abs(Zf - z[..., None, None] * np.eye(3)).max() == 0
    Zr, _ = O.center_project(Vr, None)
    assert not Zr.any() and O.count_vortices(Zr)["total"] == 0
    Zz, _ = O.center_project(Zf, None)
    assert np.array_equal(Zz, Z)
    assert O.count_vortices(Zz)["total"] == O.count_vortices(Z)["total"] > 0
    # without G the removal acts on U itself
    Z0, _ = O.center_project(U, None)
    assert np.abs(O.vortex_field(U, None, Z0, O.VORTEX_REMOVED) - np.conj(np.exp(2j * np.pi * Z0 / 3))[..., None, None] * U).max() < 1e-15


def test_polyakov_abelian_flux_closed_form(O):
    """The time-like links of the flux field are diag(e^{i th}, e^{i th}, e^{-2 i th}) with
    th = sum_j 2 pi n_j c_j / (L_j L_t) at every t, so the line through spatial site
    (x, y, z) has phase phi = sum_j 2 pi n_j c_j / L_j and tr/3 = (2 e^{i phi} + e^{-2 i phi}) / 3.
    A walk along a spatial axis, a wrong site index or a daggered product fails it (the
    value is complex and differs from site to site)."""
    L, n = L_FLUX, N_FLUX
    P = O.polyakov(flux_field(L, n))
    for z in range(L[2]):
        for y in range(L[1]):
            for x in range(L[0]):
                phi = 2 * np.pi * (n[0] * x / L[0] + n[1] * y / L[1] + n[2] * z / L[2])
                want = (2 * np.exp(1j * phi) + np.exp(-2j * phi)) / 3
                assert abs(P[x + L[0] * (y + L[1] * z)] - want) < 1e-13, (x, y, z)
    assert np.abs(P.imag).max() > 0.1


def test_polyakov_pure_gauge_line_telescopes(O, S):
    """Time-like links g(t) g(t+1)^dagger (Haar g, spatial links random) multiply to
    g(0) g(0)^dagger = 1 only when the factors are taken in the order of increasing t:
    the line is 1 at every spatial site.  Multiplied by a centre element z_t per time
    slice, the line is the product of the z_t."""
    L = (4, 2, 2, 6)
    U = S.haar_links(L, S.sub_seed(4007))
    g = S.haar_gauge(L, S.sub_seed(4008))
    gn = np.roll(g, -1, axis=0)
    U[..., 3, :, :] = g @ np.conj(np.swapaxes(gn, -1, -2))
    P = O.polyakov(U)
    assert np.abs(P - 1).max() < 1e-13
    m = np.array([1, 0, 2, 1, 1, 0])
    U[..., 3, :, :] *= np.exp(2j * np.pi * m / 3)[:, None, None, None, None, None]
    want = np.exp(2j * np.pi * m.sum() / 3)
    assert np.abs(O.polyakov(U) - want).max() < 1e-13
