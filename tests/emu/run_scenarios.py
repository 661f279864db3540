"""Run the library's kernels and driver, built for the host against the
emulated HIP runtime (libmcg_emu.so, AddressSanitizer + UBSan), through the
C ABI on small seeded lattices, and compare with the FP64 oracle.  Any
out-of-bounds access aborts the process.  Started by tests/test_emu.py in a
subprocess with libasan preloaded.  Test infrastructure only."""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path[:0] = [ROOT, os.path.dirname(HERE), HERE]

import emu_api as E  # noqa: E402
from helpers import center_links, planted_field  # noqa: E402
from oracle import oracle as O  # noqa: E402
from paper_0807_0264_amd import synth as S  # noqa: E402

TOL = {0: 1e-12, 1: 1e-5}


def rounded(U, prec):
    return U if prec == 0 else U.astype(np.complex64).astype(np.complex128)


def field(L, seed, sweeps=3):
    return S.heatbath_field(L, S.sub_seed(seed), 5.7, sweeps)


def check(cond, what):
    if not cond:
        raise AssertionError(what)


def scenario_fields(L, prec):
    U = rounded(field(L, 2000), prec)
    G = S.haar_gauge(L, S.sub_seed(2001))
    W = E.links(U, prec)
    check(np.array_equal(E.host_links(W), U), "pack/unpack")
    check(np.array_equal(E.host_gauge(E.gauge(G)), G), "gauge pack/unpack")
    Wd = E.apply_gauge(W, E.gauge(G))
    want = O.apply_gauge(U, G)
    check(np.abs(E.host_links(Wd) - want).max() < (1e-14 if prec == 0 else 1e-6), "apply_gauge")
    check(abs(E.functional(Wd) - O.functional(want)) <= TOL[prec] * O.functional(want), "functional")
    check(abs(E.plaquette(W) - O.plaquette(U)) <= TOL[prec] * abs(O.plaquette(U)), "plaquette")
    check(np.array_equal(E.host_gauge(E.gauge_identity(L)), np.broadcast_to(np.eye(3), G.shape)), "identity")


def scenario_smear(L, prec):
    U = rounded(field(L, 2002), prec)
    for eps, rho in ((1.0, 0.1), (-0.25, 0.06)):
        got = E.host_links(E.smear(E.links(U, prec), rho, eps, 2))
        want = O.smear(U, rho, eps, 2)
        check(np.abs(got - want).max() < (1e-13 if prec == 0 else 1e-5), f"smear eps={eps}")


def scenario_halfsweep(L, prec):
    U = rounded(field(L, 2003), prec)
    G0 = S.haar_gauge(L, S.sub_seed(2004))
    W, Gd = E.links(U, prec), E.gauge(G0)
    Wo, Go = U.copy(), G0.copy()
    for par in (0, 1):
        E.halfsweep(W, Gd, par)
        Wo, Go = O.halfsweep(Wo, Go, par, 1.7)
    check(np.abs(E.host_links(W) - Wo).max() < (1e-13 if prec == 0 else 2e-5), "halfsweep links")
    check(np.abs(E.host_gauge(Gd) - Go).max() < (1e-13 if prec == 0 else 2e-5), "halfsweep gauge")


def scenario_fix(L, prec):
    U = rounded(field(L, 2005), prec)
    Go, io, to = O.mcg_fix(U, tol=-1.0, max_sweeps=9, reunit_every=4, want_traj=True)
    for two_row in (True, False):
        E.set_two_row(two_row)
        G, info = E.fix(E.links(U, prec), None, tol=-1.0, max_sweeps=9, reunit_every=4, check_every=3)
        check(info["sweeps"] == io["sweeps"] == 9, "sweep count")
        check((np.abs(info["traj"] - to) / to).max() < TOL[prec], f"trajectory two_row={two_row}")
        check(abs(info["R"] - io["R"]) <= TOL[prec] * io["R"], "final R")
        if prec == 0:
            check(np.abs(E.host_gauge(G) - Go).max() < 1e-11, "final G")
            check(abs(info["theta"] - io["theta"]) <= 1e-9 * max(io["theta"], 1e-12), "theta")
    E.set_two_row(True)
    # raw sweeps in both forms agree with the oracle's half-sweeps
    G0 = S.haar_gauge(L, S.sub_seed(2009))
    Wo, Gh = U.copy(), G0.copy()
    for par in (0, 1, 0, 1):
        Wo, Gh = O.halfsweep(Wo, Gh, par, 1.7)
    for two_row in (True, False):
        E.set_two_row(two_row)
        W, Gd = E.links(U, prec), E.gauge(G0)
        E.sweeps(W, Gd, 2)
        check(np.abs(E.host_links(W) - Wo).max() < (1e-13 if prec == 0 else 2e-5), f"sweeps two_row={two_row}")
        check(np.abs(E.host_gauge(Gd) - Gh).max() < (1e-13 if prec == 0 else 2e-5), "sweeps gauge")
    E.set_two_row(True)


def scenario_project(L, prec):
    U = rounded(field(L, 2006), prec)
    G0 = S.haar_gauge(L, S.sub_seed(2007))
    Gf, _ = E.fix(E.links(U, prec), E.gauge(G0), tol=-1.0, max_sweeps=4)
    G = E.host_gauge(Gf)
    Zd, mmin = E.center_project(E.links(U, prec), Gf)
    Z = E.z_interchange(Zd, L)
    # the allocation-free entry point: the same integers and margin from the library's static scratch
    Zn, mn = E.center_project_noalloc(E.links(U, prec), Gf)
    check(np.array_equal(Zn, Zd) and mn == mmin, "allocation-free projection")
    Zn2, none = E.center_project_noalloc(E.links(U, prec), None, want_margin=False)
    check(none is None and np.array_equal(Zn2, E.center_project(E.links(U, prec), None)[0]),
          "allocation-free projection without G or margin")
    Zo, margin = O.center_project(U, G)
    safe = margin > 1e-4
    check(np.array_equal(Z[safe], Zo[safe]), "centre integers")
    check(abs(mmin - margin.min()) < 1e-9, "min margin")
    vo = O.count_vortices(Z)
    check(E.count_vortices(Zd, L) == {k: vo[k] for k in ("total", "per_plane", "per_charge")}, "vortices")
    m = S.z3_links(L, S.sub_seed(2008))
    Zr = np.ascontiguousarray(np.moveaxis(m, -1, 0).reshape(4, -1))
    vo = O.count_vortices(m)
    check(E.count_vortices(Zr, L) == {k: vo[k] for k in ("total", "per_plane", "per_charge")}, "random Z3")
    Zc, mc = E.center_project(E.links(center_links(m), 0), None)
    check(np.array_equal(E.z_interchange(Zc, L), m) and abs(mc - np.pi / 3) < 1e-12, "centre field")


def scenario_batch(prec):
    Ls = [(4, 4, 4, 4), (6, 4, 4, 2), (2, 2, 2, 2)]
    Us = [rounded(field(L, 2010 + i), prec) for i, L in enumerate(Ls)]
    G0s = [S.haar_gauge(L, S.sub_seed(2020), copy=i) for i, L in enumerate(Ls)]
    maxs, tols = [9, 7, 5], [1e-12, 1e-12, 1e-12]
    infos = E.fix_batch([E.links(U, prec) for U in Us], [E.gauge(G) for G in G0s], tols, maxs,
                        reunit_every=3, check_every=2)
    for b in range(3):
        _, ib = E.fix(E.links(Us[b], prec), E.gauge(G0s[b]), tol=tols[b], max_sweeps=maxs[b],
                      reunit_every=3, check_every=2)
        check(ib["sweeps"] == infos[b]["sweeps"], "batch sweeps")
        check(ib["R"] == infos[b]["R"] and np.array_equal(ib["traj"], infos[b]["traj"]), "batch bits")
    # the batched tuner: launches over the whole batch, its choice kept; the fields are not modified
    Ws = [E.links(U, prec) for U in Us]
    before = [E.host_links(W) for W in Ws]
    best, ms = E.autotune_batch(Ws)
    check(0 <= best < 6 and all(t > 0 for t in ms) and E.get_variant(prec) == best, f"autotune_batch {best}")
    check(all(np.array_equal(a, E.host_links(W)) for a, W in zip(before, Ws)), "autotune leaves U alone")
    E.set_variant(prec, 2)
    # the schedule tuner: its choice is kept for this batch shape and gives the bits of the defaults
    Gref = [E.gauge(G) for G in G0s]
    ref = E.fix_batch([E.links(U, prec) for U in Us], Gref, tols, maxs, reunit_every=3, check_every=2)
    c = E.tune_batch(Ws)
    check(0 <= c["variant"] < 6 and 0 <= c["order"] <= 2 and c["paired"] in ((0, 1) if prec else (0, 2))
          and c["slabs"] in (1, 2, 4) and 0 < c["ms_per_sweep"] <= c["ms_default"], f"tune_batch {c}")
    check(all(np.array_equal(a, E.host_links(W)) for a, W in zip(before, Ws)), "tune_batch leaves U alone")
    Gt = [E.gauge(G) for G in G0s]
    got = E.fix_batch([E.links(U, prec) for U in Us], Gt, tols, maxs, reunit_every=3, check_every=2)
    check(all(np.array_equal(a["traj"], b["traj"]) and a["R"] == b["R"] for a, b in zip(ref, got)) and
          all(np.array_equal(E.host_gauge(a), E.host_gauge(b)) for a, b in zip(Gref, Gt)),
          f"tuned schedule gives the default bits ({c})")
    E.clear_tuning()
    # the whole path of the batch in one call: the bits of its calls made one by one
    for rho, eps, n in ((0.1, 1.0, 2), (0.06, -0.25, 1)):
        Gp = [E.gauge(G) for G in G0s]
        Zs, rp = E.precondition_batch([E.links(U, prec) for U in Us], Gp, rho, eps, n, 1e-12, 6, reunit_every=3,
                                      check_every=2)
        Sm = [E.smear(E.links(U, prec), rho, eps, n) for U in Us]
        Gq = [E.gauge(G) for G in G0s]
        i1 = E.fix_batch(Sm, Gq, [1e-12] * 3, [6] * 3, reunit_every=3, check_every=2)
        i2 = E.fix_batch([E.links(U, prec) for U in Us], Gq, [1e-12] * 3, [6] * 3, reunit_every=3, check_every=2)
        for b in range(3):
            Zq, mq = E.center_project(E.links(Us[b], prec), Gq[b])
            check(rp[b]["Rs"] == i1[b]["R"] and rp[b]["R"] == i2[b]["R"] and rp[b]["s"] == i2[b]["sweeps"] and
                  np.array_equal(E.host_gauge(Gp[b]), E.host_gauge(Gq[b])) and np.array_equal(Zs[b], Zq) and
                  rp[b]["m"] == mq and rp[b]["v"] == E.count_vortices(Zq, Ls[b])["total"],
                  f"precondition_batch field {b} ({rho}, {eps}, {n})")


def scenario_planted():
    L = (4, 4, 4, 4)
    Up, gp, m = planted_field(S, L, 2030)
    G, info = E.fix(E.links(Up, 0), None, tol=1e-12, max_sweeps=200, check_every=20)
    check(info["R"] > 1 - 1e-10, f"planted R {info['R']}")
    Zd, _ = E.center_project(E.links(Up, 0), G)
    check(E.count_vortices(Zd, L)["total"] == O.count_vortices(m)["total"], "planted vortex count")


def scenario_backward(L, prec):
    U = rounded(field(L, 2040), prec)
    G = S.haar_gauge(L, S.sub_seed(2041))
    for rho, eps, n, ck in ((0.1, 1.0, 3, 2), (0.06, -0.25, 3, 1), (0.06, -0.25, 2, 0), (0.06, -0.25, 5, 2),
                            (0.06, -0.25, 1, 0)):
        gd, loss, dr, de = E.smear_mcg_backward(E.links(U, prec), rho, eps, n, E.gauge(G), ck)
        go, dro, deo, losso = O.smear_loss_grad(U, rho, eps, n, G, ckpt_every=ck)
        tol = 1e-12 if prec == 0 else 1e-5
        scale = np.abs(go).max()
        check(np.abs(E.host_links(gd) - go).max() < tol * max(scale, 1e-3) * 10, f"gradU eps={eps}")
        check(abs(loss - losso) < tol * losso, "loss")
        check(abs(dr - dro) < tol * max(abs(dro), 1e-3) * 10, f"dRho {dr} {dro}")
        check(abs(de - deo) < tol * max(abs(deo), 1e-3) * 10, f"dEps {de} {deo}")


def scenario_loops(L, prec):
    U = rounded(field(L, 2050), prec)
    G = S.haar_gauge(L, S.sub_seed(2051))
    Zd, _ = E.center_project(E.links(U, prec), E.gauge(G))
    Z = E.z_interchange(Zd, L)
    tol = 1e-14 if prec == 0 else 1e-6
    for mode in (0, 1):
        got = E.host_links(E.vortex_field(E.links(U, prec), E.gauge(G), Zd, mode))
        want = O.vortex_field(U, G, Z, mode)
        check(np.abs(got - want).max() < tol, f"vortex field mode {mode}")
    got = E.host_links(E.vortex_field(E.links(U, prec), None, Zd, 1))
    check(np.abs(got - O.vortex_field(U, None, Z, 1)).max() < tol, "vortex removal without G")
    # every lane is a host thread here: a few loop shapes only (the GPU tests take many more)
    cases = ([(1, 0, 0)], 2), ([(2, 1, 0)], 1)
    if L == (2, 2, 2, 2):
        cases += (([(1, 1, 1)], 1),)
    for vecs, rmax in cases:
        tmax = min(L[3], 3)
        got = E.wilson_loops(E.links(U, prec), vecs, rmax, tmax)
        want = O.wilson_loops(U, vecs, rmax, tmax)
        check(np.abs(got - want).max() < (1e-13 if prec == 0 else 2e-6), f"wilson loops {vecs}")


def scenario_slabs(prec):
    """Slab-pipelined half-sweeps, and odd half-sweeps in reverse tile order,
    give the bits of whole forward half-sweeps."""
    L1, L2 = (4, 4, 4, 16), (2, 2, 2, 2)
    U1, U2 = rounded(field(L1, 2060), prec), rounded(field(L2, 2061), prec)
    G1 = S.haar_gauge(L1, S.sub_seed(2062))
    E.set_variant(prec, 0)  # 64-thread blocks: 8 blocks per half-sweep of L1, split into 2 or 3 slabs
    ref = None
    for n, order, paired in ((1, 0, 1), (2, 0, 1), (3, 0, 1), (1, 1, 1), (3, 1, 1), (3, 1, 0), (1, 0, 0),
                             (1, 2, 1), (3, 2, 1), (3, 2, 2), (1, 1, 2)):
        E.set_slabs(n)
        E.set_sweep_order(order)
        E.set_paired(paired)
        G, info = E.fix(E.links(U1, prec), E.gauge(G1), tol=-1.0, max_sweeps=5, reunit_every=2, check_every=2)
        infos = E.fix_batch([E.links(U2, prec), E.links(U1, prec)], [E.gauge_identity(L2), E.gauge(G1)],
                            [-1.0, -1.0], [4, 5], reunit_every=2, check_every=2)
        W, Gd = E.links(U1, prec), E.gauge(G1)
        E.sweeps(W, Gd, 2)
        got = (E.host_gauge(G), info["traj"], infos[0]["traj"], infos[1]["traj"], E.host_links(W), E.host_gauge(Gd))
        if ref is None:
            ref = got
            check(np.array_equal(got[1], got[3]), "batch equals single")
        else:
            check(all(np.array_equal(a, b) for a, b in zip(got, ref)),
                  f"slabs {n} order {order} paired {paired} differ from whole forward half-sweeps")
    E.set_slabs(1)
    E.set_paired(True)
    # 20 blocks of 64 sites per half-sweep: residue classes mod 8 of three and two blocks
    L3 = (4, 4, 4, 40)
    U3 = rounded(field(L3, 2063), prec)
    got = []
    for order in (0, 1, 2):
        E.set_sweep_order(order)
        G, info = E.fix(E.links(U3, prec), None, tol=-1.0, max_sweeps=4, reunit_every=2, check_every=2)
        got.append((E.host_gauge(G), info["traj"]))
    for m in (1, 2):
        check(all(np.array_equal(a, b) for a, b in zip(got[0], got[m])), f"tile order {m} differs on 20 blocks")
    E.set_sweep_order(2)
    E.set_variant(prec, 2)


def scenario_variants(prec):
    """Re-linearisation hits, exact subgroup maximisation and the block-wise
    stop test against the oracle."""
    L = (4, 4, 4, 4)
    U = rounded(field(L, 2070), prec)
    for hits, stop_every, exact, omega in ((2, 1, False, 1.7), (3, 4, False, 1.7), (1, 1, True, 1.0),
                                           (2, 3, True, 1.7)):
        E.set_update_variant(hits, stop_every, exact)
        what = f"hits={hits} exact={exact}"
        for two_row in (True, False):
            E.set_two_row(two_row)
            G, info = E.fix(E.links(U, prec), None, tol=1e-4, max_sweeps=9, omega=omega, reunit_every=4,
                            check_every=3)
            Go, io, to = O.mcg_fix(U, tol=1e-4, max_sweeps=9, omega=omega, reunit_every=4, want_traj=True,
                                   hits=hits, stop_every=stop_every, exact=exact)
            check(info["sweeps"] == io["sweeps"], f"sweeps {info['sweeps']} {io['sweeps']} {what}")
            check((np.abs(info["traj"] - to) / to).max() < TOL[prec], f"trajectory {what}")
            if prec == 0:
                check(np.abs(E.host_gauge(G) - Go).max() < 1e-11, f"final G {what}")
        W, Gd = E.links(U, prec), E.gauge_identity(L)
        E.halfsweep(W, Gd, 1, omega)
        Wo, Ho = O.halfsweep(U, np.broadcast_to(np.eye(3), (L[3], L[2], L[1], L[0], 3, 3)).copy(),
                             1, omega, hits=hits, exact=exact)
        check(np.abs(E.host_links(W) - Wo).max() < (1e-13 if prec == 0 else 2e-5), f"halfsweep {what}")
    E.set_update_variant(1, 1)
    E.set_two_row(True)


def scenario_defer(parts=("rows", "full", "fp64")):
    """FP32: the transform ring (each half-sweep's g folded into G later) gives
    the bits of updating G in every half-sweep, and paired sweeps (the first
    half-sweep leaves the links to the second) the bits of plain ones: a batch
    where one field stops early, blocks replayed from a captured graph, more
    sweeps than the ring holds, both storage forms, raw sweeps."""
    prec = 1
    L1, L2 = (4, 4, 4, 16), (4, 2, 2, 4)
    U1, U2 = rounded(field(L1, 2090), prec), rounded(field(L2, 2091), prec)
    G1 = S.haar_gauge(L1, S.sub_seed(2092))
    for two_row in [t for t, name in ((True, "rows"), (False, "full")) if name in parts]:
        E.set_two_row(two_row)
        got = []
        for defer, paired in ((True, True), (True, False), (False, True)):
            E.set_defer_g(defer)
            E.set_paired(paired)
            Gs = [E.gauge_identity(L2), E.gauge(G1)]
            infos = E.fix_batch([E.links(U2, prec), E.links(U1, prec)], Gs, [1e-5, -1.0], [70, 70],
                                reunit_every=30, check_every=5)
            G, info = E.fix(E.links(U1, prec), E.gauge(G1), tol=-1.0, max_sweeps=37, reunit_every=50,
                            check_every=9)
            W, Gd = E.links(U1, prec), E.gauge(G1)
            E.sweeps(W, Gd, 35)
            got.append([infos[0]["traj"], infos[1]["traj"], infos[0]["sweeps"], info["traj"], E.host_gauge(G),
                        E.host_links(W), E.host_gauge(Gd)] + [E.host_gauge(x) for x in Gs])
        check(got[0][2] < 70, f"the small field stops early ({got[0][2]} sweeps)")
        for m in (1, 2):
            for k, (a, b) in enumerate(zip(got[0], got[m])):
                check(np.array_equal(a, b), f"mode {m} differs from paired sweeps with the ring "
                                            f"(item {k}, two_row={two_row})")
    E.set_paired(True)
    E.set_defer_g(True)
    E.set_two_row(True)
    if "fp64" not in parts:
        return
    # FP64 with paired = 2: the even g is handed over in a one-slot buffer, G updated in place
    U0 = field(L1, 2093)
    got = []
    for paired in (2, 1):
        E.set_paired(paired)
        Gs = [E.gauge_identity(L2), E.gauge(G1)]
        infos = E.fix_batch([E.links(field(L2, 2094), 0), E.links(U0, 0)], Gs, [1e-9, -1.0], [40, 40],
                            reunit_every=30, check_every=5)
        W, Gd = E.links(U0, 0), E.gauge(G1)
        E.sweeps(W, Gd, 7)
        got.append([infos[0]["traj"], infos[1]["traj"], E.host_links(W), E.host_gauge(Gd)]
                   + [E.host_gauge(x) for x in Gs])
    for k, (a, b) in enumerate(zip(*got)):
        check(np.array_equal(a, b), f"FP64 paired sweeps differ from plain ones (item {k})")
    E.set_paired(True)


def expect_error(fn, status_word, what):
    try:
        fn()
    except E.MCGError as e:
        check(f"(status {status_word})" in str(e), f"{what}: {e}")
        return str(e)
    raise AssertionError(f"{what}: no error")


def scenario_checks(prec):
    """Input validation (check mode) and the scratch limit."""
    L = (4, 4, 4, 4)
    U = rounded(field(L, 2080), prec)
    G = S.haar_gauge(L, S.sub_seed(2081))
    du, dg = E.unitarity(E.links(U, prec), E.gauge(G))
    check(du < (1e-6 if prec == 1 else 1e-13) and dg < 1e-13, f"unitary inputs {du} {dg}")
    bad = U.copy()
    bad[1, 2, 3, 0, 2] *= 1.001
    check(abs(E.unitarity(E.links(bad, prec))[0] - 0.002001) < 1e-4, "deviation of a scaled link")
    nan = U.copy()
    nan[0, 0, 0, 1, 3, 1, 2] = np.nan
    check(E.unitarity(E.links(nan, prec))[0] == np.inf, "NaN reads as inf")
    Gbad = G.copy()
    Gbad[0, 1, 0, 0] *= 1 + 1e-8
    check(E.unitarity(None, E.gauge(Gbad))[1] > 1e-9, "perturbed G")
    E.set_check(True)
    try:
        for Ub in (bad, nan):
            msg = expect_error(lambda: E.smear(E.links(Ub, prec), 0.1, 1.0, 1), -4, "smear")
            check("not unitary" in msg, msg)
            expect_error(lambda: E.fix(E.links(Ub, prec), None, tol=-1.0, max_sweeps=2), -4, "fix")
        expect_error(lambda: E.fix(E.links(U, prec), E.gauge(Gbad), tol=-1.0, max_sweeps=2), -4, "fix G")
        expect_error(lambda: E.apply_gauge(E.links(U, prec), E.gauge(Gbad)), -4, "apply_gauge")
        expect_error(lambda: E.center_project(E.links(bad, prec), None), -4, "center_project")
        expect_error(lambda: E.wilson_loops(E.links(bad, prec), [(1, 0, 0)], 1, 1), -4, "wilson_loops")
        # valid inputs pass in check mode and give the unchecked results
        a = E.host_links(E.smear(E.links(U, prec), 0.1, 1.0, 2))
    finally:
        E.set_check(False)
    check(np.array_equal(a, E.host_links(E.smear(E.links(U, prec), 0.1, 1.0, 2))), "check mode changes nothing")
    check(E.host_links(E.smear(E.links(bad, prec), 0.1, 1.0, 1)).shape == U.shape, "unchecked call runs")
    # the scratch limit: a fix of this size needs a larger working field than any before it (>1 MiB)
    L8 = (8, 8, 8, 8) if prec == 0 else (12, 12, 8, 8)
    U8 = rounded(field(L8, 2082, 1), prec)
    E.set_scratch_limit_mib(1)
    try:
        msg = expect_error(lambda: E.fix(E.links(U8, prec), None, tol=-1.0, max_sweeps=1), -2, "scratch limit")
        check("scratch limit" in msg, msg)
    finally:
        E.set_scratch_limit_mib(0)
    _, info = E.fix(E.links(U8, prec), None, tol=-1.0, max_sweeps=1)
    check(info["sweeps"] == 1, "usable after the limit")
    # option values out of range: the tile order and paired sweeps take 0-2, the ring 0 or 1
    for opt, val in ((8, 3), (8, -1), (10, 3), (10, -1), (9, 2)):
        check(E.lib().mcg_set_option(E.ctx(), opt, val) == -1, f"option {opt} = {val} rejected")
    import ctypes
    v = ctypes.c_int32()
    for opt, want in ((8, 2), (9, 1), (10, 1)):
        check(E.lib().mcg_get_option(E.ctx(), opt, ctypes.byref(v)) == 0 and v.value == want,
              f"option {opt} keeps its default {want}")


def main():
    lat = [(4, 4, 4, 4), (6, 4, 2, 4), (2, 2, 2, 2)]
    names = sys.argv[1:] or ["fields", "smear", "halfsweep", "fix", "project", "batch", "planted", "backward",
                             "loops", "slabs", "variants", "checks", "defer"]
    for arg in names:
        # "group" runs all of it; "group:part" one part (a precision, or a part of defer), so that
        # the long groups can run side by side
        name, _, part = arg.partition(":")
        precs = (int(part),) if part in ("0", "1") else (0, 1)
        if name == "batch":
            for prec in precs:
                scenario_batch(prec)
        elif name == "planted":
            scenario_planted()
        elif name == "checks":
            for prec in precs:
                scenario_checks(prec)
        elif name == "defer":
            scenario_defer((part,) if part else ("rows", "full", "fp64"))
        elif name == "variants":
            for prec in precs:
                scenario_variants(prec)
        elif name == "slabs":
            for prec in precs:
                scenario_slabs(prec)
        elif name == "loops":
            for L in ((4, 4, 4, 4), (2, 2, 2, 2)):
                for prec in (0, 1):
                    scenario_loops(L, prec)
        elif name == "backward":
            for L in ((4, 4, 4, 4), (2, 2, 2, 2)):
                for prec in (0, 1):
                    scenario_backward(L, prec)
        else:
            for L in lat:
                for prec in (0, 1):
                    globals()["scenario_" + name](L, prec)
        print("ok", arg, flush=True)


if __name__ == "__main__":
    main()
