"""Parity of the gfx950 path with the FP64 oracle, element by element, on
seeded inputs: lattices spanning several blocks with ragged tails, plus the
smallest (2^4) case.  FP64 to 1e-12 (relative where stated), FP32 to 1e-5
(the oracle is fed the FP32-rounded values); centre integers and vortex
counts bit-exact wherever the centre-phase margin exceeds 1e-4."""
import numpy as np
import pytest

from helpers import center_links, gauge_transform, planted_field

pytestmark = pytest.mark.gpu

LATS = [(4, 4, 4, 4), (6, 4, 4, 8), (6, 6, 6, 10), (2, 2, 2, 2)]
PRECS = [0, 1]
TOL = {0: 1e-12, 1: 1e-5}


@pytest.fixture(scope="module")
def g():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import gpu_util
    return gpu_util


@pytest.fixture(scope="module")
def api(g):
    from paper_0807_0264_amd import api as a
    for prec in (0, 1):
        a.set_variant(prec, 2)
    return a


def field(S, L, seed, sweeps=5):
    return S.heatbath_field(L, S.sub_seed(seed), 5.7, sweeps)


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("L", LATS)
def test_pack_roundtrip(S, g, api, L, prec):
    U = field(S, L, 1000)
    W = g.links(U, prec)
    back = g.host_links(W)
    assert np.array_equal(back, g.rounded(U, prec))
    G = S.haar_gauge(L, S.sub_seed(1001))
    assert np.array_equal(g.host_gauge(g.gauge(G)), G)


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("L", LATS)
def test_apply_gauge_functional_plaquette(S, O, g, api, L, prec):
    U = g.rounded(field(S, L, 1002), prec)
    G = S.haar_gauge(L, S.sub_seed(1003))
    Wd = api.apply_gauge(g.links(U, prec), g.gauge(G))
    want = O.apply_gauge(U, G)
    assert np.abs(g.host_links(Wd) - want).max() < (1e-14 if prec == 0 else 1e-6)
    assert abs(api.functional(Wd) - O.functional(want)) <= TOL[prec] * O.functional(want)
    assert abs(api.plaquette(g.links(U, prec)) - O.plaquette(U)) <= TOL[prec] * abs(O.plaquette(U))
    assert np.array_equal(g.host_gauge(api.gauge_identity(L)), np.broadcast_to(np.eye(3), G.shape))


@pytest.mark.parametrize("eps", [1.0, -0.25])
@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("L", LATS)
def test_smear(S, O, g, api, L, prec, eps):
    U = g.rounded(field(S, L, 1004), prec)
    rho = 0.1 if eps == 1.0 else 0.06
    got = g.host_links(api.smear(g.links(U, prec), rho, eps, 3))
    want = O.smear(U, rho, eps, 3)
    assert np.abs(got - want).max() < (1e-13 if prec == 0 else 1e-5)


# t-slices of 720 and 500 half-sites: several 128-site tiles per slice with a ragged last one, and
# 6 and 12 slices, so the last group of up to eight slices that the smearing kernel walks with the
# slice index fastest is a short one
RAGGED = [(12, 12, 10, 6), (10, 10, 10, 12)]


@pytest.mark.parametrize("eps", [1.0, -0.25])
@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("L", RAGGED)
def test_smear_ragged_tiles(S, O, g, api, L, prec, eps):
    U = g.rounded(field(S, L, 1006), prec)
    rho = 0.1 if eps == 1.0 else 0.06
    got = g.host_links(api.smear(g.links(U, prec), rho, eps, 3))
    want = O.smear(U, rho, eps, 3)
    assert np.abs(got - want).max() < (1e-13 if prec == 0 else 1e-5)


@pytest.mark.parametrize("prec", PRECS)
def test_smear_zero_steps_and_zero_rho(S, g, api, prec):
    L = (6, 4, 4, 8)
    U = g.rounded(field(S, L, 1005), prec)
    assert np.array_equal(g.host_links(api.smear(g.links(U, prec), 0.1, 1.0, 0)), U)
    # rho = 0: C = 0, exp(0) = 1 exactly
    assert np.array_equal(g.host_links(api.smear(g.links(U, prec), 0.0, -0.25, 2)), U)


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("L", LATS)
def test_halfsweeps(S, O, g, api, L, prec):
    U = g.rounded(field(S, L, 1006), prec)
    G0 = S.haar_gauge(L, S.sub_seed(1007))
    W = g.links(U, prec)
    Gd = g.gauge(G0)
    Wo, Go = U.copy(), G0.copy()
    for par in (0, 1, 0):
        api.halfsweep(W, Gd, par, 1.7)
        Wo, Go = O.halfsweep(Wo, Go, par, 1.7)
    assert np.abs(g.host_links(W) - Wo).max() < (1e-13 if prec == 0 else 2e-5)
    assert np.abs(g.host_gauge(Gd) - Go).max() < (1e-13 if prec == 0 else 2e-5)


@pytest.mark.parametrize("two_row", [True, False])
@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("L", [(6, 6, 6, 10), (2, 2, 2, 2)])
def test_sweeps_every_variant_and_form(S, O, g, api, L, prec, two_row):
    """Raw sweeps at every launch variant, in both storage forms of the
    working field, against the oracle's half-sweeps."""
    U = g.rounded(field(S, L, 1010), prec)
    G0 = S.haar_gauge(L, S.sub_seed(1011))
    Wo, Go = U.copy(), G0.copy()
    for par in (0, 1, 0, 1, 0, 1):
        Wo, Go = O.halfsweep(Wo, Go, par, 1.7)
    api.set_two_row(two_row)
    try:
        for v in range(6):
            api.set_variant(prec, v)
            W, Gd = g.links(U, prec), g.gauge(G0)
            api.sweeps(W, Gd, 3)
            assert np.abs(g.host_links(W) - Wo).max() < (1e-13 if prec == 0 else 3e-5), v
            assert np.abs(g.host_gauge(Gd) - Go).max() < (1e-13 if prec == 0 else 3e-5), v
        api.set_variant(prec, 2)
    finally:
        api.set_two_row(True)


@pytest.mark.parametrize("two_row", [True, False])
@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("L", LATS)
def test_fix_trajectory(S, O, g, api, L, prec, two_row):
    """40 sweeps with re-unitarisation every 7: R after every sweep matches,
    with the working field kept as two rows or as full matrices."""
    U = g.rounded(field(S, L, 1008), prec)
    api.set_two_row(two_row)
    try:
        G, info = api.fix(g.links(U, prec), None, tol=-1.0, max_sweeps=40, reunit_every=7,
                          check_every=9, want_traj=True)
    finally:
        api.set_two_row(True)
    Go, io, to = O.mcg_fix(U, tol=-1.0, max_sweeps=40, reunit_every=7, want_traj=True)
    assert info["sweeps"] == io["sweeps"] == 40 and info["status"] == io["status"] == 1
    rel = np.abs(info["traj"] - to) / to
    assert rel.max() < TOL[prec]
    assert abs(info["R"] - io["R"]) <= TOL[prec] * io["R"]
    if prec == 0:
        assert np.abs(g.host_gauge(G) - Go).max() < 1e-11
        assert abs(info["theta"] - io["theta"]) <= 1e-9 * max(io["theta"], 1e-12)


@pytest.mark.parametrize("L", [(4, 4, 4, 4), (6, 4, 4, 8), (6, 6, 6, 10)])
def test_fix_to_convergence_fp64(S, O, g, api, L):
    U = field(S, L, 1009, 20)
    G, info = api.fix(g.links(U, 0), None, tol=1e-9, max_sweeps=3000, want_traj=True)
    Go, io, to = O.mcg_fix(U, tol=1e-9, max_sweeps=3000, want_traj=True)
    assert info["status"] == io["status"] == 0
    # the stop sweep can differ only if some dR lies within rounding of tol
    assert abs(info["sweeps"] - io["sweeps"]) <= 1
    n = min(info["sweeps"], io["sweeps"]) + 1
    assert (np.abs(info["traj"][:n] - to[:n]) / to[:n]).max() < 1e-12
    if info["sweeps"] == io["sweeps"]:
        assert abs(info["R"] - io["R"]) < 1e-12 * io["R"]
        assert np.abs(g.host_gauge(G) - Go).max() < 1e-10


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("L", LATS)
def test_center_project_and_vortices(S, O, g, api, L, prec):
    U = g.rounded(field(S, L, 1010), prec)
    G0 = S.haar_gauge(L, S.sub_seed(1011))
    Gfix, _ = api.fix(g.links(U, prec), g.gauge(G0), tol=-1.0, max_sweeps=15)
    G = g.host_gauge(Gfix)
    Zd, mmin = api.center_project(g.links(U, prec), Gfix)
    Z = g.z_interchange(Zd, L)
    Zo, margin = O.center_project(U, G)
    safe = margin > 1e-4
    assert np.array_equal(Z[safe], Zo[safe])
    assert abs(mmin - margin.min()) < 1e-9
    # vortex counting is exact integer work: compare on the GPU's own Z
    vd = api.count_vortices(Zd, L)
    vo = O.count_vortices(Z)
    assert vd == {k: vo[k] for k in ("total", "per_plane", "per_charge")}
    # and on uniformly random Z3 integers
    m = S.z3_links(L, S.sub_seed(1012))
    import torch
    Zr = torch.from_numpy(np.ascontiguousarray(np.moveaxis(m, -1, 0).reshape(4, -1))).cuda()
    vo = O.count_vortices(m)
    assert api.count_vortices(Zr, L) == {k: vo[k] for k in ("total", "per_plane", "per_charge")}


def test_center_project_without_gauge(S, O, g, api):
    L = (6, 4, 4, 8)
    m = S.z3_links(L, S.sub_seed(1013))
    U = center_links(m)
    Zd, mmin = api.center_project(g.links(U, 0), None)
    assert np.array_equal(g.z_interchange(Zd, L), m)
    assert abs(mmin - np.pi / 3) < 1e-12


@pytest.mark.parametrize("prec", PRECS)
def test_planted_pipeline(S, O, g, api, prec):
    """Planted U = g Z g^dag (4^4): 10 stout steps at rho = 0.1 leave it
    unchanged, fixing reaches R = 1, and the projected field has exactly
    the planted vortex count."""
    L = (4, 4, 4, 4)
    Up, gp, m = planted_field(S, L, 1014)
    U = g.links(Up, prec)
    out = api.precondition_and_fix(U, rho=0.1, eps=1.0, n=10, tol=1e-10 if prec == 0 else 1e-7,
                                   max_sweeps=5000)
    # stopping at dR < 1e-10 leaves 1 - R of order 1e-10
    assert out["R_smeared"] > 1 - (1e-9 if prec == 0 else 1e-5)
    assert out["R"] > 1 - (1e-9 if prec == 0 else 1e-5)
    assert out["vortices"]["total"] == O.count_vortices(m)["total"]
    assert out["min_margin"] > 1.0


@pytest.mark.parametrize("prec", PRECS)
def test_batch_equals_single(S, g, api, prec):
    """Each field of a batch (unequal lattices and Gribov copies) gets the bits
    of its standalone fix."""
    Ls = [(4, 4, 4, 4), (6, 6, 6, 10), (6, 4, 4, 8), (6, 6, 6, 10)]
    Us = [g.rounded(field(S, L, 1015 + i), prec) for i, L in enumerate(Ls)]
    Us[3] = Us[1]  # a second Gribov copy of field 1
    G0s = [S.haar_gauge(L, S.sub_seed(1020), copy=i) for i, L in enumerate(Ls)]
    tols = [1e-9, 1e-9, 1e-8, 1e-9] if prec == 0 else [1e-6] * 4
    Fs = [g.links(U, prec) for U in Us]
    Gs, infos = api.fix_batch(Fs, [g.gauge(G0) for G0 in G0s], tol=tols, max_sweeps=[400, 300, 400, 250],
                              reunit_every=20, check_every=25, want_traj=True)
    for b in range(4):
        Gb, ib = api.fix(g.links(Us[b], prec), g.gauge(G0s[b]), tol=tols[b],
                         max_sweeps=[400, 300, 400, 250][b], reunit_every=20, check_every=25,
                         want_traj=True)
        assert ib["sweeps"] == infos[b]["sweeps"]
        assert ib["R"] == infos[b]["R"] and ib["theta"] == infos[b]["theta"]
        assert np.array_equal(ib["traj"], infos[b]["traj"])
        assert np.array_equal(g.host_gauge(Gb), g.host_gauge(Gs[b]))


def test_resume_is_bitwise(S, g, api):
    L = (6, 4, 4, 8)
    U = field(S, L, 1030)
    Ga, ia = api.fix(g.links(U, 0), None, tol=-1.0, max_sweeps=60, reunit_every=30)
    Gb, ib = api.fix(g.links(U, 0), None, tol=-1.0, max_sweeps=30, reunit_every=30)
    assert ib["status"] == 1
    Gc, ic = api.fix(g.links(U, 0), Gb, tol=-1.0, max_sweeps=30, reunit_every=30, start_sweep=30)
    assert np.array_equal(g.host_gauge(Ga), g.host_gauge(Gc))
    assert ia["R"] == ic["R"]


def test_invalid_arguments_raise(S, g, api):
    import torch
    from paper_0807_0264_amd.api import MCGError, Links
    L = (4, 4, 4, 4)
    U = g.links(field(S, L, 1031), 0)
    bad = Links((5, 4, 4, 4), 0, U.data)
    with pytest.raises(ValueError, match="even"):
        api.functional(bad)
    # the C library rejects it too when called directly
    import ctypes
    from paper_0807_0264_amd import _abi
    f = _abi.Field()
    f.d = api._dims((5, 4, 4, 4))
    f.prec = 0
    f.ptr = U.data.data_ptr()
    v = ctypes.c_double()
    st = _abi.load().mcg_functional(api.context(), ctypes.byref(f), ctypes.byref(v), None)
    assert st == _abi.MCG_EINVAL
    assert b"even" in _abi.load().mcg_last_error(api.context())
    with pytest.raises(MCGError, match="alias"):
        api.smear(U, 0.1, 1.0, 2, out=U)
    with pytest.raises(MCGError, match="omega"):
        api.fix(U, None, omega=2.5)
    with pytest.raises(MCGError, match="parity"):
        api.halfsweep(U, api.gauge_identity(L), 2)
    # the context stays usable after an error
    assert 0 < api.functional(U) < 1


def test_max_sweeps_zero_and_warning(S, g, api):
    L = (4, 4, 4, 4)
    U = g.links(field(S, L, 1032), 0)
    G, info = api.fix(U, None, tol=1e-12, max_sweeps=0)
    assert info["sweeps"] == 0 and info["status"] == 1
    G, info = api.fix(U, None, tol=1e-12, max_sweeps=3)
    assert info["sweeps"] == 3 and info["status"] == 1 and info["blocks50"] == 1


def test_autotune_keeps_results_valid(S, g, api):
    L = (6, 6, 6, 10)
    U = field(S, L, 1033)
    best, ms = api.autotune(g.links(U, 1))
    assert 0 <= best < 6 and all(t > 0 for t in ms)
    G, info = api.fix(g.links(g.rounded(U, 1), 1), None, tol=-1.0, max_sweeps=10, want_traj=True)
    api.set_variant(1, 2)
    G2, info2 = api.fix(g.links(g.rounded(U, 1), 1), None, tol=-1.0, max_sweeps=10, want_traj=True)
    assert np.abs(info["traj"] - info2["traj"]).max() < 1e-6


def test_autotune_batch(S, g, api):
    """The batched tuner times launches over the whole batch, keeps its
    choice for the precision and storage form, and a batched fix afterwards
    gives the bits of the same fix at a fixed variant (results do not depend
    on the launch shape)."""
    Ls = [(6, 6, 6, 10), (4, 4, 4, 4), (8, 8, 8, 16)]
    Us = [g.rounded(field(S, L, 1034 + i), 1) for i, L in enumerate(Ls)]
    try:
        best, ms = api.autotune_batch([g.links(U, 1) for U in Us])
        assert 0 <= best < 6 and all(t > 0 for t in ms)
        assert api.get_variant(1) == best
        _, a = api.fix_batch([g.links(U, 1) for U in Us], None, tol=-1.0, max_sweeps=12, want_traj=True)
        api.set_variant(1, (best + 1) % 6)
        _, b = api.fix_batch([g.links(U, 1) for U in Us], None, tol=-1.0, max_sweeps=12, want_traj=True)
        for x, y in zip(a, b):
            assert np.array_equal(x["traj"], y["traj"])
    finally:
        api.set_variant(1, 2)


@pytest.mark.parametrize("prec", PRECS)
def test_tune_batch(S, g, api, prec):
    """The schedule tuner (variant x tile order x paired sweeps x slabs, timed as whole sweeps over
    the batch) keeps its choice for the batch shape; the fix of that batch afterwards, in the tuned
    schedule, gives the bits of the untuned fix (every schedule visits independent sites in another
    order, nothing else), G and trajectory, across a re-unitarisation and a graph replay."""
    Ls = [(6, 6, 6, 10), (4, 4, 4, 4), (8, 8, 8, 16)]
    Us = [g.rounded(field(S, L, 1036 + i), prec) for i, L in enumerate(Ls)]
    kw = dict(tol=-1.0, max_sweeps=12, reunit_every=5, want_traj=True)
    try:
        Ga, a = api.fix_batch([g.links(U, prec) for U in Us], None, **kw)
        c = api.tune_batch([g.links(U, prec) for U in Us])
        print(f"prec {prec}: tuned {c}")
        assert 0 <= c["variant"] < 6 and 0 <= c["order"] <= 2 and c["slabs"] in (1, 2, 4)
        assert c["paired"] in ((0, 1) if prec == 1 else (0, 2))
        assert c["ms_per_sweep"] > 0 and c["ms_default"] > 0
        # the schedule in use is kept unless another is more than 1 % faster in the same passes
        assert c["ms_per_sweep"] <= c["ms_default"]
        Gb, b = api.fix_batch([g.links(U, prec) for U in Us], None, **kw)
        for x, y, ga, gb in zip(a, b, Ga, Gb):
            assert np.array_equal(x["traj"], y["traj"])
            assert np.array_equal(g.host_gauge(ga), g.host_gauge(gb))
    finally:
        api.clear_tuning()


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("rho,eps,n", [(0.1, 1.0, 4), (0.06, -0.25, 3), (0.1, 1.0, 0)])
def test_precondition_batch_equals_its_calls(S, g, api, prec, rho, eps, n):
    """The whole path of a batch in one library call gives, field by field, the bits of the calls it
    is made of: smear, fix_batch of the smeared fields, fix_batch of the originals from their
    transforms, centre projection and vortex count."""
    Ls = [(6, 6, 6, 10), (4, 4, 4, 4), (8, 4, 4, 8)]
    Us = [g.links(g.rounded(field(S, L, 1050 + i), prec), prec) for i, L in enumerate(Ls)]
    kw = dict(tol=1e-9 if prec == 0 else 1e-6, max_sweeps=400, omega=1.7, reunit_every=50, check_every=50)
    Gs, Zs, res = api.precondition_batch(Us, rho, eps, n, **kw)
    Sm = [api.smear(U, rho, eps, n) for U in Us]
    G1, i1 = api.fix_batch(Sm, None, **kw)
    G2, i2 = api.fix_batch(Us, G1, **kw)
    for b, L in enumerate(Ls):
        assert res[b]["smeared"]["R"] == i1[b]["R"] and res[b]["smeared"]["sweeps"] == i1[b]["sweeps"]
        assert res[b]["fixed"]["R"] == i2[b]["R"] and res[b]["fixed"]["sweeps"] == i2[b]["sweeps"]
        assert np.array_equal(g.host_gauge(Gs[b]), g.host_gauge(G2[b]))
        Z, m = api.center_project(Us[b], G2[b])
        assert np.array_equal(Zs[b].cpu().numpy(), Z.cpu().numpy()) and res[b]["min_margin"] == m
        assert res[b]["vortices"] == api.count_vortices(Z, L)


def test_synth_gpu_is_bitwise_cpu(S, g):
    for L, n in (((4, 4, 4, 4), 4), ((6, 4, 4, 8), 3)):
        a = S.heatbath_field(L, S.sub_seed(1040), 5.7, n)
        b = S.heatbath_field_gpu(L, S.sub_seed(1040), 5.7, n).cpu().numpy()
        assert np.array_equal(a, b)
        assert np.array_equal(S.haar_gauge(L, 5, 3), S.haar_gauge_gpu(L, 5, 3).cpu().numpy())
    # the Luscher-Weisz heatbath (eight-colour schedule)
    for L, n in (((4, 4, 4, 4), 3), ((8, 4, 4, 4), 2)):
        a = S.heatbath_lw_field(L, S.sub_seed(1041), 4.52, n, 0.884)
        b = S.heatbath_lw_field_gpu(L, S.sub_seed(1041), 4.52, n, 0.884).cpu().numpy()
        assert np.array_equal(a, b)


@pytest.mark.parametrize("prec", PRECS)
def test_slab_pipelined_sweeps_are_bitwise(S, g, api, prec):
    """Half-sweeps run slab by slab (several slab counts, a batch mixing a
    split and an unsplit field), odd half-sweeps in reverse tile order (also
    with contiguous tile ranges per XCD), and paired or plain sweeps (FP64
    paired too), give the bits of whole forward half-sweeps."""
    L1, L2 = (8, 8, 8, 32), (6, 6, 6, 10)
    U1 = g.rounded(field(S, L1, 1050), prec)
    U2 = g.rounded(field(S, L2, 1051), prec)
    G1 = S.haar_gauge(L1, S.sub_seed(1052))
    ref = None
    try:
        for n, order, paired in ((1, False, 1), (2, False, 1), (5, False, 1), (8, False, 1), (1, True, 1),
                                 (5, True, 1), (1, 2, 1), (5, 2, 1), (5, 2, 2), (1, 1, 0)):
            api.set_slabs(n)
            api.set_sweep_order(order)
            api.set_paired(paired)
            assert api.get_sweep_order() == order
            G, info = api.fix(g.links(U1, prec), g.gauge(G1), tol=-1.0, max_sweeps=60, reunit_every=25,
                              check_every=20, want_traj=True)
            Gb, infos = api.fix_batch([g.links(U2, prec), g.links(U1, prec)], [api.gauge_identity(L2), g.gauge(G1)],
                                      tol=-1.0, max_sweeps=[40, 60],
                                      reunit_every=25, check_every=20, want_traj=True)
            W, Gd = g.links(U1, prec), g.gauge(G1)
            api.sweeps(W, Gd, 3)
            got = [g.host_gauge(G), info["traj"], infos[0]["traj"], infos[1]["traj"], g.host_gauge(Gb[1]),
                   g.host_links(W), g.host_gauge(Gd)]
            if ref is None:
                ref = got
                assert np.array_equal(got[1], got[3]) and np.array_equal(got[0], got[4])
            else:
                for a, b in zip(got, ref):
                    assert np.array_equal(a, b), (n, order, paired)
    finally:
        api.set_slabs(1)
        api.set_sweep_order(2)
        api.set_paired(1)


@pytest.mark.parametrize("two_row", [True, False])
def test_transform_ring_is_bitwise(S, g, api, two_row):
    """FP32: each half-sweep's g kept in the ring and folded into G later gives
    the bits of updating G in every half-sweep, and paired sweeps (the even
    half-sweep leaves the links to the odd one, which applies the even g as it
    loads them) the bits of plain ones: a batch where one field stops early,
    blocks of 30 sweeps replayed from a captured graph (ring of 15: a fold
    inside each block and one at its start), a standalone fix (ring of 25, 37
    sweeps) and raw sweeps."""
    prec = 1
    L1, L2 = (8, 8, 8, 32), (6, 6, 6, 10)
    U1 = g.rounded(field(S, L1, 1055), prec)
    U2 = g.rounded(field(S, L2, 1056), prec)
    G1 = S.haar_gauge(L1, S.sub_seed(1057))
    got = []
    try:
        api.set_two_row(two_row)
        for defer, paired in ((True, True), (True, False), (False, True)):
            api.set_defer_g(defer)
            api.set_paired(paired)
            assert api.get_defer_g() == defer and api.get_paired() == paired
            Gb, infos = api.fix_batch([g.links(U2, prec), g.links(U1, prec)],
                                      [api.gauge_identity(L2), g.gauge(G1)], tol=[1e-4, -1.0],
                                      max_sweeps=[130, 130], reunit_every=30, check_every=5, want_traj=True)
            G, info = api.fix(g.links(U1, prec), g.gauge(G1), tol=-1.0, max_sweeps=37, reunit_every=50,
                              check_every=9, want_traj=True)
            W, Gd = g.links(U1, prec), g.gauge(G1)
            api.sweeps(W, Gd, 35)
            got.append([infos[0]["traj"], infos[1]["traj"], infos[0]["sweeps"], g.host_gauge(Gb[0]),
                        g.host_gauge(Gb[1]), info["traj"], g.host_gauge(G), g.host_links(W), g.host_gauge(Gd)])
    finally:
        api.set_paired(True)
        api.set_defer_g(True)
        api.set_two_row(True)
    assert got[0][2] < 130
    for m in (1, 2):
        for k, (a, b) in enumerate(zip(got[0], got[m])):
            assert np.array_equal(a, b), (m, k)


def test_paired_sweeps_fp64(S, g, api):
    """FP64 links with MCG_OPT_PAIRED = 2: paired sweeps (the even g handed to
    the odd half-sweep in a one-slot buffer, G updated in place) give the bits
    of plain ones: a batch where one field stops early, a standalone fix and
    raw sweeps."""
    prec = 0
    L1, L2 = (8, 8, 8, 16), (6, 6, 6, 10)
    U1 = field(S, L1, 1062)
    U2 = field(S, L2, 1063)
    G1 = S.haar_gauge(L1, S.sub_seed(1064))
    got = []
    try:
        for paired in (2, 1):
            api.set_paired(paired)
            assert api.get_paired() == paired
            Gb, infos = api.fix_batch([g.links(U2, prec), g.links(U1, prec)],
                                      [api.gauge_identity(L2), g.gauge(G1)], tol=[1e-4, -1.0],
                                      max_sweeps=[120, 120], reunit_every=30, check_every=5, want_traj=True)
            G, info = api.fix(g.links(U1, prec), g.gauge(G1), tol=-1.0, max_sweeps=37, reunit_every=50,
                              check_every=9, want_traj=True)
            W, Gd = g.links(U1, prec), g.gauge(G1)
            api.sweeps(W, Gd, 9)
            got.append([infos[0]["traj"], infos[1]["traj"], infos[0]["sweeps"], g.host_gauge(Gb[0]),
                        g.host_gauge(Gb[1]), info["traj"], g.host_gauge(G), g.host_links(W), g.host_gauge(Gd)])
    finally:
        api.set_paired(True)
    assert got[0][2] < 120
    for k, (a, b) in enumerate(zip(*got)):
        assert np.array_equal(a, b), k


def test_paired_sweeps_with_hits_and_exact_steps(S, g, api):
    """FP32 with the ring: paired sweeps give the bits of plain ones also for
    re-linearisation hits and exact subgroup steps (their own 256-thread
    instantiations of both halves), in a fix and in raw sweeps."""
    prec = 1
    L = (8, 8, 8, 16)
    U = g.rounded(field(S, L, 1058), prec)
    G0 = S.haar_gauge(L, S.sub_seed(1059))
    try:
        for hits, exact in ((3, False), (1, True), (2, True)):
            api.set_update_variant(hits, 1, exact)
            got = []
            for paired in (True, False):
                api.set_paired(paired)
                G, info = api.fix(g.links(U, prec), g.gauge(G0), tol=-1.0, max_sweeps=30, reunit_every=20,
                                  check_every=7, want_traj=True)
                W, Gd = g.links(U, prec), g.gauge(G0)
                api.sweeps(W, Gd, 3)
                got.append((g.host_gauge(G), info["traj"], g.host_links(W), g.host_gauge(Gd)))
            for k, (a, b) in enumerate(zip(*got)):
                assert np.array_equal(a, b), (hits, exact, k)
    finally:
        api.set_paired(True)
        api.set_update_variant(1, 1)


@pytest.mark.parametrize("prec", PRECS)
def test_sweeps_timed(S, g, api, prec):
    """mcg_sweeps_timed leaves W and G exactly as mcg_sweeps does (ring folds
    included for FP32) and returns the half-sweeps' own duration: positive and
    within the wall time of the call."""
    import time

    import torch
    L = (8, 8, 8, 32)
    U = g.rounded(field(S, L, 1058), prec)
    G0 = S.haar_gauge(L, S.sub_seed(1059))
    W1, G1 = g.links(U, prec), g.gauge(G0)
    api.sweeps(W1, G1, 30)
    W2, G2 = g.links(U, prec), g.gauge(G0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ms = api.sweeps_timed(W2, G2, 30)
    wall = 1000 * (time.perf_counter() - t0)
    assert np.array_equal(g.host_links(W1), g.host_links(W2))
    assert np.array_equal(g.host_gauge(G1), g.host_gauge(G2))
    assert 0 < ms < wall


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("L", [(4, 4, 4, 4), (6, 6, 6, 10)])
def test_update_variants(S, O, g, api, L, prec):
    """Re-linearisation hits and the block-wise stop test against the oracle."""
    U = g.rounded(field(S, L, 1060), prec)
    G0 = S.haar_gauge(L, S.sub_seed(1061))
    try:
        for hits, stop_every in ((2, 1), (3, 1), (1, 25), (2, 10)):
            api.set_update_variant(hits, stop_every)
            for two_row in (True, False):
                api.set_two_row(two_row)
                G, info = api.fix(g.links(U, prec), g.gauge(G0), tol=1e-6, max_sweeps=60, reunit_every=20,
                                  check_every=7, want_traj=True)
                Go, io, to = O.mcg_fix(U, G0, tol=1e-6, max_sweeps=60, reunit_every=20, want_traj=True, hits=hits,
                                       stop_every=stop_every)
                n = min(info["sweeps"], io["sweeps"]) + 1
                # FP32 links: the ~1e-7 rounding of every sweep accumulates over the 20 sweeps between
                # re-derivations of W from the FP64 G (extra hits amplify it), reaching ~1e-5 by sweep 60
                tol = TOL[0] if prec == 0 else 3e-5
                assert (np.abs(info["traj"][:n] - to[:n]) / to[:n]).max() < tol
                if prec == 0:
                    assert info["status"] == io["status"] and info["sweeps"] == io["sweeps"]
                    assert np.abs(g.host_gauge(G) - Go).max() < 1e-10
                if info["status"] == 0:
                    assert info["sweeps"] % stop_every == 0
            W, Gd = g.links(U, prec), g.gauge(G0)
            api.sweeps(W, Gd, 2)
            Wo, Ho = U.copy(), G0.copy()
            for par in (0, 1, 0, 1):
                Wo, Ho = O.halfsweep(Wo, Ho, par, 1.7, hits=hits)
            assert np.abs(g.host_links(W) - Wo).max() < (1e-13 if prec == 0 else 3e-5)
    finally:
        api.set_update_variant(1, 1)
        api.set_two_row(True)


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("L", [(4, 4, 4, 4), (6, 6, 6, 10)])
def test_exact_update(S, O, g, api, L, prec):
    """Exact maximisation over each SU(2) subgroup (omega = 1 and over-relaxed,
    one and two rounds of the three subgroups, with a block-wise stop) against
    the oracle: trajectory, stop sweep and transform, and two sweeps of W.

    The exact step is worse conditioned than the linearised one: where the
    root of the secular equation lies close to the second eigenvalue of the
    4x4 form, rounding of the form rotates the maximiser.  Measured on the
    oracle itself (FP64) on these inputs: relative noise of 1e-15 on U moves
    W by up to 7e-12 after two sweeps (linearised update: 2e-13), hence the
    FP64 bound 2e-11 on W, and noise of 6e-8 by up to 3e-5 (linearised:
    1.5e-6), hence the FP32 bound 1e-4; with omega = 1.7 a relative 1e-7
    grows to 2e-6 of R by sweep 20 and 2e-4 by sweep 60 (linearised: 6e-7),
    so over-relaxed FP32 trajectories are compared element-wise over the
    first 20 sweeps and at the end within 1e-3.  Over a 60-sweep fix, noise
    of 1e-15 moves the oracle's transform by up to 2.6e-9 and its relative
    trajectory by 8e-13 (omega = 1.7 on 6x6x6x10), hence the FP64 bounds
    2e-8 on G and 1e-11 on R."""
    U = g.rounded(field(S, L, 1065), prec)
    G0 = S.haar_gauge(L, S.sub_seed(1066))
    try:
        for hits, stop_every, omega in ((1, 1, 1.0), (1, 1, 1.7), (2, 10, 1.0)):
            api.set_update_variant(hits, stop_every, exact=True)
            assert api.get_update_variant() == (hits, stop_every, True)
            Go, io, to = O.mcg_fix(U, G0, tol=1e-6, max_sweeps=60, omega=omega, reunit_every=20,
                                   want_traj=True, hits=hits, stop_every=stop_every, exact=True)
            for two_row in (True, False):
                api.set_two_row(two_row)
                G, info = api.fix(g.links(U, prec), g.gauge(G0), tol=1e-6, max_sweeps=60, omega=omega,
                                  reunit_every=20, check_every=7, want_traj=True)
                n = min(info["sweeps"], io["sweeps"]) + 1
                tol = 1e-11 if prec == 0 else 3e-5
                m = n if prec == 0 or omega == 1.0 else min(n, 21)
                assert (np.abs(info["traj"][:m] - to[:m]) / to[:m]).max() < tol, (hits, omega)
                assert abs(info["traj"][n - 1] - to[n - 1]) / to[n - 1] < (tol if prec == 0 else 1e-3)
                if prec == 0:
                    assert info["status"] == io["status"] and info["sweeps"] == io["sweeps"]
                    assert np.abs(g.host_gauge(G) - Go).max() < 2e-8
                if info["status"] == 0:
                    assert info["sweeps"] % stop_every == 0
            W, Gd = g.links(U, prec), g.gauge(G0)
            api.sweeps(W, Gd, 2, omega)
            Wo, Ho = U.copy(), G0.copy()
            for par in (0, 1, 0, 1):
                Wo, Ho = O.halfsweep(Wo, Ho, par, omega, hits=hits, exact=True)
            assert np.abs(g.host_links(W) - Wo).max() < (2e-11 if prec == 0 else 1e-4)
    finally:
        api.set_update_variant(1, 1)
        api.set_two_row(True)


@pytest.mark.parametrize("prec", PRECS)
def test_fix_is_bitwise_across_launch_variants(S, g, api, prec):
    """The FP64 partial sums of R are per 64-site wavefront in index order, so
    the block size and occupancy of the launch do not change any bit of the
    trajectory, the stop sweep or the transform."""
    L = (6, 6, 6, 10)
    U = g.rounded(field(S, L, 1070), prec)
    ref = None
    try:
        for two_row in (True, False):
            api.set_two_row(two_row)
            for v in range(6):
                api.set_variant(prec, v)
                G, info = api.fix(g.links(U, prec), None, tol=1e-6, max_sweeps=120, reunit_every=25,
                                  check_every=10, want_traj=True)
                got = (g.host_gauge(G), info["traj"], info["sweeps"])
                if ref is None or ref[0] != two_row:
                    ref = (two_row, got)
                else:
                    assert np.array_equal(got[0], ref[1][0]) and np.array_equal(got[1], ref[1][1]), v
                    assert got[2] == ref[1][2]
    finally:
        api.set_two_row(True)
        api.set_variant(prec, 2)
