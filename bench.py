"""Benchmark of the stout-preconditioned MCG hot path on one MI355X.

Workload (one "step" = the whole path over one batch of synthetic fields):
  four lattices 32^3x64, 24^3x48, 20^3x40 and 16^4, each a Haar start plus
  50 Cabibbo-Marinari heatbath sweeps of the Wilson action at beta = 5.7
  (seeded), links in FP32 with FP64 gauge transforms and reductions;
  per step: 10 stout steps (rho = 0.1) of every field, MCG fixing of the
  smeared fields to dR < 1e-7 (one batched, graph-captured sweep loop), the
  carried-back fix of the original fields (batched again), centre
  projection and P-vortex counting of every field.
Metric: MCG site-updates per second over the timed steps (site-updates =
  sum over fields of sweeps x V), plus the roofline of the half-sweep
  kernel at 32^3x64, the FP64 CPU oracle timed on a bounded sample, and
  Gribov copies per second of the 20^3x40 field: 16 Haar copies batched with
  FP32 links against the same copies fixed one by one with FP64 links, per
  smearing level, with the copies whose final R agree to 1e-6 counted.

    python bench.py [--steps K] [--warmup W] [--gpus 1] [--no-cpu-baseline] [--no-gribov]
    python bench.py --profile      # short fixed-work run for rocprofv3
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "MCG site-updates/s and % HBM peak at 32^3x64; batched FP32 vs plain at equal R"
LATTICES = [(32, 32, 32, 64), (24, 24, 24, 48), (20, 20, 20, 40), (16, 16, 16, 16)]
HBM_PEAK_GBS = 8000.0
# algorithmic bytes of one half-sweep site-update with FP32 links, keyed by
# (two-row form, transform ring): the 8 links read and written, plus G(x) read
# and written (FP64) or, with the ring, the site's g written once (two FP32
# rows, 48 B; the fold kernel reads it later).  In the two-row form (the
# default) a link is 6 complex FP32 (48 B) and G(x) 6 complex FP64 (96 B); as
# full matrices 72 B and 144 B.
BYTES_PER_SITE_UPDATE = {(True, True): 8 * 48 * 2 + 48, (True, False): 8 * 48 * 2 + 2 * 96,
                         (False, True): 8 * 72 * 2 + 48, (False, False): 8 * 72 * 2 + 2 * 144}
# paired sweeps (two-row form with the ring): the even half-sweep reads the 8 links and writes g
# (8 * 48 + 48 B per site), the odd one reads the 8 links and the even g of its neighbours (each
# g needed once: 48 B per site), writes the 8 links and its own g (8 * 48 * 2 + 48 + 48); per
# site-update the mean of the two
BYTES_PER_SITE_UPDATE_PAIRED = (8 * 48 + 48 + 8 * 48 * 2 + 48 + 48) // 2
# the model of a site-update with full 3x3 FP32 links and an FP64 G read and written in every
# half-sweep: 8 * 72 * 2 + 2 * 144 B
SURVEY_BYTES_PER_SITE_UPDATE = 8 * 72 * 2 + 2 * 144
# the fold kernel's bytes per site-update it folds, with 25 sweeps per fold (raw sweeps, and
# fixes re-unitarising every 50): g read once (48 B) + G(x) read and written once per 25
FOLD_BYTES_PER_SITE_UPDATE = {True: 48 + 2 * 96 / 25, False: 48 + 2 * 144 / 25}
PMC_FILE = os.path.join(ROOT, "profiles", "halfsweep_pmc_32x32x32x64_fp32.json")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_hash():
    h = hashlib.sha256()
    for f in ("mcg_kernels.hpp", "common.hpp", "fix_types.hpp", "k_mcg.hip"):
        h.update(open(os.path.join(ROOT, "paper_0807_0264_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


def make_inputs(api, synth, torch):
    fields = []
    for i, L in enumerate(LATTICES):
        t0 = time.time()
        U64 = synth.heatbath_field_gpu(L, synth.sub_seed(5, i), 5.7, 50)
        U = api.to_links(U64, 1)  # FP32 links
        torch.cuda.synchronize()
        log(f"input {L}: heatbath on the GPU in {time.time() - t0:.1f} s, "
            f"plaquette {api.plaquette(U):.5f}")
        fields.append((L, U, U64 if i == 0 else None))
    return fields


def gribov_copies(api, synth, torch, U, ncopies=16, rho=0.1, nsmear=20, tol=1e-6, max_sweeps=5000,
                  r_match=1e-6, deep_tol=1e-10):
    """Gribov copies of one field: Haar-random start transforms g_c, each copy
    fixed without smearing and with nsmear stout steps (then carried back and
    re-fixed), centre-projected and vortex-counted.  Every level runs once with
    all copies batched in FP32 links and once copy by copy with FP64 links
    (the same FP32-rounded input); both stop on the same criterion
    dR < tol = 1e-6.  "Equal final R" is read three ways:
    (a) the same stop test, R distributions compared (rounding steers a copy
        to a different local maximum after enough over-relaxed sweeps, so the
        two paths' copies are different maxima: means, standard errors, Welch
        t, and the sweep at which each copy's two R trajectories first differ
        by more than r_match);
    (b) every batched FP32 copy polished by a batched FP64 fix from its own G
        to the same dR < tol, timed as part of the FP32 path: a copy counts
        when its FP32 R lies within r_match of the polished FP64 R;
    (c) both paths' copies polished in FP64 to dR < deep_tol (untimed): a copy
        counts when its R lies within r_match of the maximum it converges to."""
    import numpy as np

    L = U.L
    U64 = api.to_links(api.from_links(U).to(torch.complex128), 0)
    G0 = [api.to_gauge(synth.haar_gauge_gpu(L, synth.sub_seed(7), c)) for c in range(ncopies)]
    V = api.volume(L)
    fix_kw = dict(tol=tol, max_sweeps=max_sweeps, omega=1.7, check_every=50)

    def finish(W, G, infos, infos_s):
        out = []
        for c in range(ncopies):
            Z, _ = api.center_project(W, G[c])
            v = api.count_vortices(Z, L)
            sw = infos[c]["sweeps"] + (infos_s[c]["sweeps"] if infos_s else 0)
            first = (infos_s or infos)[c]  # the first fix of the level
            out.append(dict(R=infos[c]["R"], sweeps=sw, vf=v["total"] / (6 * V), status=infos[c]["status"],
                            traj=first["traj"][:first["sweeps"] + 1]))
        return out

    def polish(G, ptol):
        """batched FP64 fix of every copy from its own transform to dR < ptol: final R and sweeps"""
        _, inf = api.fix_batch([U64] * ncopies, [g.clone() for g in G],
                               **dict(fix_kw, tol=ptol, max_sweeps=20000))
        return [x["R"] for x in inf], [x["sweeps"] for x in inf]

    def batched(n):
        G = [g.clone() for g in G0]
        infos_s = None
        if n:
            S = api.smear(U, rho, 1.0, n)
            G, infos_s = api.fix_batch([S] * ncopies, G, want_traj=True, **fix_kw)
            del S
        G, infos = api.fix_batch([U] * ncopies, G, want_traj=True, **fix_kw)
        out = finish(U, G, infos, infos_s)
        torch.cuda.synchronize()
        t0 = time.time()
        Rp, sw = polish(G, tol)  # (b): part of the FP32 path
        torch.cuda.synchronize()
        dt = time.time() - t0
        for x, r, k, g in zip(out, Rp, sw, G):
            x.update(R_polished=r, polish_sweeps=k, polish_s=dt, G=g)
        return out

    def plain(n):
        S = api.smear(U64, rho, 1.0, n) if n else None
        G, infos, infos_s = [], [], [] if n else None
        for c in range(ncopies):
            g = G0[c].clone()
            if n:
                g, i_s = api.fix(S, g, want_traj=True, **fix_kw)
                infos_s.append(i_s)
            g, i = api.fix(U64, g, want_traj=True, **fix_kw)
            G.append(g)
            infos.append(i)
        out = finish(U64, G, infos, infos_s)
        for x, g in zip(out, G):
            x["G"] = g
        return out

    def mean_sem(x):
        x = np.asarray(x, dtype=float)
        return float(x.mean()), float(x.std(ddof=1) / np.sqrt(len(x)))

    def diverge(ta, tb):
        n = min(len(ta), len(tb))
        d = np.nonzero(np.abs(ta[:n] - tb[:n]) > r_match)[0]
        return int(d[0]) if len(d) else None

    best64, _ = api.autotune(U64)
    best32, _ = api.autotune_batch([U] * ncopies)  # the batch the FP32 path fixes
    sched32 = api.tune_batch([U] * ncopies)
    levels = []
    for n in (0, nsmear):
        runs = {}
        for name, fn in (("fp32_batched", batched), ("fp64_plain", plain)):
            torch.cuda.synchronize()
            t0 = time.time()
            runs[name] = fn(n)
            torch.cuda.synchronize()
            runs[name + "_s"] = time.time() - t0
            log(f"gribov copies n={n} {name}: {runs[name + '_s']:.2f} s")
        a, b = runs["fp32_batched"], runs["fp64_plain"]
        # (c): both paths' copies polished to deep_tol, untimed
        t0 = time.time()
        deep32, dsw32 = polish([x.pop("G") for x in a], deep_tol)
        deep64, dsw64 = polish([y.pop("G") for y in b], deep_tol)
        log(f"gribov copies n={n}: FP64 polish of both paths to dR < {deep_tol}: {time.time() - t0:.2f} s")
        dR = [abs(x["R"] - y["R"]) for x, y in zip(a, b)]
        matched = [c for c in range(ncopies) if dR[c] <= r_match]
        pol = [abs(x["R"] - x["R_polished"]) for x in a]
        own32 = [abs(x["R"] - r) for x, r in zip(a, deep32)]
        own64 = [abs(y["R"] - r) for y, r in zip(b, deep64)]
        (ma, sa), (mb, sb) = mean_sem([x["R"] for x in a]), mean_sem([x["R"] for x in b])
        (va, vsa), (vb, vsb) = mean_sem([x["vf"] for x in a]), mean_sem([x["vf"] for x in b])
        div = [diverge(x["traj"], y["traj"]) for x, y in zip(a, b)]
        t_polish = a[0]["polish_s"]
        levels.append(dict(
            smear=f"stout rho={rho} n={n}" if n else "none",
            copies_per_s_fp32_batched=round(ncopies / runs["fp32_batched_s"], 3),
            copies_per_s_fp64_plain=round(ncopies / runs["fp64_plain_s"], 3),
            speedup=round(runs["fp64_plain_s"] / runs["fp32_batched_s"], 3),
            fp32_polish_s=round(t_polish, 3), fp32_polish_sweeps=[x["polish_sweeps"] for x in a],
            speedup_without_polish=round(runs["fp64_plain_s"] / (runs["fp32_batched_s"] - t_polish), 3),
            matched_copies_polished=sum(d <= r_match for d in pol), max_abs_dR_polished=max(pol),
            matched_copies_converged_fp32=sum(d <= r_match for d in own32),
            matched_copies_converged_fp64=sum(d <= r_match for d in own64),
            max_abs_dR_converged_fp32=max(own32), max_abs_dR_converged_fp64=max(own64),
            deep_polish_sweeps_fp32=dsw32, deep_polish_sweeps_fp64=dsw64,
            matched_copies_same_copy=len(matched),
            max_abs_dR_matched=max([dR[c] for c in matched], default=None),
            R_mean_sem_fp32=[round(ma, 7), round(sa, 7)], R_mean_sem_fp64=[round(mb, 7), round(sb, 7)],
            R_welch_t=round((ma - mb) / np.hypot(sa, sb), 3),
            vortex_fraction_mean_sem_fp32=[round(va, 6), round(vsa, 6)],
            vortex_fraction_mean_sem_fp64=[round(vb, 6), round(vsb, 6)],
            trajectories_differ_by_r_match_at_sweep=div,
            R_fp32=[round(x["R"], 7) for x in a], R_fp64=[round(x["R"], 7) for x in b],
            sweeps_fp32=[x["sweeps"] for x in a], sweeps_fp64=[x["sweeps"] for x in b],
            vortex_fraction_fp32=[round(x["vf"], 5) for x in a],
            vortex_fraction_fp64=[round(x["vf"], 5) for x in b],
            not_converged=sum(x["status"] != 0 for x in a + b)))
    return dict(workload=f"{ncopies} Haar Gribov copies of one {'x'.join(map(str, L))} field, "
                         f"tol {tol}, all copies batched (FP32 links, then a batched FP64 polish to the "
                         f"same tol, timed) vs one by one (FP64 links)",
                readings=dict(polished="FP32 R within r_match of the FP64 polish of the same copy (timed)",
                              converged=f"R within r_match of the copy's maximum (FP64 polish to dR < "
                                        f"{deep_tol}, untimed), for each path",
                              same_copy="FP32 and FP64 final R of one copy within r_match",
                              r_match=r_match),
                fp64_variant=best64, fp32_variant=best32,
                fp32_schedule={k: (round(v, 4) if isinstance(v, float) else v) for k, v in sched32.items()},
                levels=levels)


# Wilson loops of the static-potential measurement (Sec. III.B) on the 20^3x40
# field: on-axis and off-axis spatial directions with R up to about L/2, T <= 10
LOOP_VECS = [((1, 0, 0), 10), ((1, 1, 0), 7), ((2, 1, 0), 5), ((1, 1, 1), 5), ((2, 1, 1), 5), ((2, 2, 1), 5)]
LOOP_TMAX = 10


def wilson_loop_run(api, torch, U, G=None, reps=3):
    """W(R, T) of the fixed field, its vortex-only and its vortex-removed
    parts (the three fields whose potentials the paper compares), timed."""
    fields = [("original", U)]
    if G is not None:
        Z, _ = api.center_project(U, G)
        fields += [("vortex-only", api.vortex_field(U, G, Z, 0)), ("vortex-removed", api.vortex_field(U, G, Z, 1))]
    out = {}
    for name, F in fields:
        for v, r in LOOP_VECS:
            api.wilson_loops(F, [v], r, LOOP_TMAX)  # warm-up (scratch allocation)
        torch.cuda.synchronize()
        t0 = time.time()
        for _ in range(reps):
            W = [api.wilson_loops(F, [v], r, LOOP_TMAX)[0] for v, r in LOOP_VECS]
        dt = (time.time() - t0) / reps
        out[name] = dict(ms=round(1000 * dt, 2), W_R1=[round(float(w[0, 0]), 6) for w in W],
                         W_onaxis_T1=[round(float(x), 6) for x in W[0][:, 0]])
    n_loops = sum(r for _, r in LOOP_VECS) * LOOP_TMAX
    return dict(workload=f"W(R, T) for spatial directions {[v for v, _ in LOOP_VECS]} with k = 1..rmax "
                         f"{[r for _, r in LOOP_VECS]} copies of the staircase path, T = 1..{LOOP_TMAX}, averaged "
                         f"over sites and cubic images; {n_loops} (R, T) entries per field",
                fields=out)


# Algorithmic FP32 flop per link of one smearing step, every staple path evaluated by itself: stout =
# 12 staple products + C U^dag + Q^2 + exp(iQ) U = 15 complex 3x3 products (198 flop each) plus sums
# and the exponential's scalar series (~0.3 kflop); over-improved adds the 18 rectangle paths per link,
# 66 products with the plaquettes' two-link prefixes reused (81 products).  The kernel shares the last
# product of rectangles that end on the same link and executes 70 of the 81.
SMEAR_FLOP_PER_LINK = {"stout": 15 * 198 + 300, "over-improved": 81 * 198 + 300}
SMEAR_PRODUCTS_EXECUTED = {"stout": 15, "over-improved": 70}
FP32_VECTOR_PEAK = 157.3e12


def smear_run(api, torch, U, nsteps=10, reps=3):
    """One smearing step of the 32^3x64 field, stout (rho 0.1) and
    over-improved (rho 0.06, eps -0.25), timed with HIP events."""
    out = {}
    for name, rho, eps in (("stout", 0.1, 1.0), ("over-improved", 0.06, -0.25)):
        S = api.smear(U, rho, eps, 1)  # warm-up and output allocation
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            api.smear(U, rho, eps, nsteps, out=S)
        e1.record()
        e1.synchronize()
        ms = e0.elapsed_time(e1) / (reps * nsteps)
        links = 4 * api.volume(U.L)
        tf = links * SMEAR_FLOP_PER_LINK[name] / (ms * 1e-3) / 1e12
        out[name] = dict(ms_per_step=round(ms, 4), flop_per_link=SMEAR_FLOP_PER_LINK[name],
                         products_executed_per_link=SMEAR_PRODUCTS_EXECUTED[name],
                         tflops=round(tf, 2), frac_fp32_peak=round(tf * 1e12 / FP32_VECTOR_PEAK, 4))
        del S
    return out


def backward_run(api, torch, synth, reps=3):
    """Gradient of R(S_20(U)^{G*}) (over-improved, rho 0.06, eps -0.25,
    checkpoint every 5 steps) on a 16^4 heatbath field, FP32 links."""
    L = (16, 16, 16, 16)
    U = api.to_links(synth.heatbath_field_gpu(L, synth.sub_seed(1, 0), 5.7, 50), 1)
    G, _ = api.fix(api.smear(U, 0.06, -0.25, 20), None, tol=1e-7, max_sweeps=5000)
    api.smear_mcg_backward(U, 0.06, -0.25, 20, G, 5)  # warm-up and scratch allocation
    torch.cuda.synchronize()
    t0 = time.time()
    for _ in range(reps):
        api.smear_mcg_backward(U, 0.06, -0.25, 20, G, 5)
    torch.cuda.synchronize()
    ms = 1000 * (time.time() - t0) / reps
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    api.smear(U, 0.06, -0.25, 20)
    e1.record()
    e1.synchronize()
    fwd = e0.elapsed_time(e1)
    return dict(workload="16^4, over-improved rho=0.06 eps=-0.25, n=20, checkpoint every 5, FP32",
                ms=round(ms, 3), forward_smear_ms=round(fwd, 3), ratio_to_forward=round(ms / fwd, 2))


def copy_ceiling(torch, nbytes=1 << 30, reps=10):
    """Device-to-device copy rate of the runtime's copy kernel (bytes read +
    written), the practical ceiling that an HBM-bound kernel is compared with."""
    a = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    e1.synchronize()
    return round(2 * nbytes * reps / (e0.elapsed_time(e1) * 1e-3) / 1e9, 1)


def one_step(api, fields, tol=1e-7, max_sweeps=5000):
    """The whole path over the batch in one library call (mcg_precondition_batch): 10 stout steps of
    every field, the batched fix of the smeared fields, the batched carried-back re-fix, projection
    and counting."""
    Us = [U for _, U, _ in fields]
    _, _, res = api.precondition_batch(Us, 0.1, 1.0, 10, tol=tol, max_sweeps=max_sweeps, omega=1.7,
                                       check_every=50)
    out = []
    for (L, U, _), r in zip(fields, res):
        V = api.volume(L)
        a, b = r["smeared"], r["fixed"]
        out.append(dict(L=L, sweeps_smeared=a["sweeps"], sweeps=b["sweeps"], R_smeared=a["R"], R=b["R"],
                        vortex_fraction=r["vortices"]["total"] / (6 * V), min_margin=r["min_margin"],
                        site_updates=(a["sweeps"] + b["sweeps"]) * V))
    return out


def roofline(api, torch, U, nsweeps=200, runs=5):
    """Average duration of the half-sweep kernel at 32^3x64 (FP32 links, FP64
    G), from HIP events that the library records on the stream the kernels
    are launched on (torch's current stream) around each sweep's two
    half-sweep launches (api.sweeps_timed): the folds of the transform ring
    and the storage-form conversions fall outside.  The median over `runs`
    calls of nsweeps sweeps each (a multiple of the ring's 25, so every call
    has the same folds between its sweeps), after 25 warm-up sweeps."""
    W = U.clone()
    G = api.gauge_identity(U.L)
    api.sweeps(W, G, 25)  # warm-up
    torch.cuda.synchronize()

    import statistics
    ms = statistics.median(api.sweeps_timed(W, G, nsweeps) / (2 * nsweeps) for _ in range(runs))
    two_row, defer = api.get_two_row(), api.get_defer_g()
    paired = two_row and defer and api.get_paired()
    bps = BYTES_PER_SITE_UPDATE_PAIRED if paired else BYTES_PER_SITE_UPDATE[(two_row, defer)]
    site_updates = api.volume(U.L) // 2
    achieved = site_updates * bps / (ms * 1e-3) / 1e9
    traffic = None
    if os.path.exists(PMC_FILE):
        pmc = json.load(open(PMC_FILE))
        if pmc.get("kernel_source_hash") == kernel_source_hash():
            traffic = pmc.get("hbm_bytes_per_launch")
    # the whole sweep loop, folds included: half-sweep and fold bytes over the plain sweeps' time
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    api.sweeps(W, G, nsweeps)
    e1.record()
    e1.synchronize()
    loop_ms = e0.elapsed_time(e1) / (2 * nsweeps)
    loop_bps = bps + (FOLD_BYTES_PER_SITE_UPDATE[two_row] if defer else 0)
    return dict(bound="hbm", achieved=round(achieved, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                frac=round(achieved / HBM_PEAK_GBS, 4), traffic=traffic,
                kernel="k_halfsweep<float,%s> (one parity of 32^3x64, %s, %s)" % (
                    "two-row" if two_row else "full",
                    {0: "forward tile order", 1: "alternating tile order",
                     2: "alternating tile order, XCD ranges per field"}[api.get_sweep_order()],
                    ("paired sweeps, g to the transform ring" if paired else "g to the transform ring")
                    if defer else "G updated in place"),
                ms_per_launch=round(ms, 4), bytes_per_launch=site_updates * bps, bytes_per_site_update=bps,
                **({"plain_equivalent": dict(
                    bytes_per_site_update=BYTES_PER_SITE_UPDATE[(two_row, defer)],
                    GBps=round(site_updates * BYTES_PER_SITE_UPDATE[(two_row, defer)] / (ms * 1e-3) / 1e9, 1),
                    frac=round(site_updates * BYTES_PER_SITE_UPDATE[(two_row, defer)] / (ms * 1e-3) / 1e9
                               / HBM_PEAK_GBS, 4),
                    note="context only: the same time per site-update against the bytes a plain half-sweep "
                         "with the ring needs (each link written in both half-sweeps)")} if paired else {}),
                survey_model=dict(
                    bytes_per_site_update=SURVEY_BYTES_PER_SITE_UPDATE,
                    GBps=round(site_updates * SURVEY_BYTES_PER_SITE_UPDATE / (ms * 1e-3) / 1e9, 1),
                    frac=round(site_updates * SURVEY_BYTES_PER_SITE_UPDATE / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                    note="effective rate: the same time per site-update against the bytes of the plain "
                         "full-matrix form (8 FP32 links read and written, FP64 G read and written); "
                         "above 1 because the two-row form, the ring and paired sweeps move fewer bytes"),
                sweep_loop=dict(ms_per_half_sweep=round(loop_ms, 4), bytes_per_site_update=loop_bps,
                                GBps=round(site_updates * loop_bps / (loop_ms * 1e-3) / 1e9, 1),
                                note="api.sweeps end to end (conversions of W and G to and from the "
                                     "storage form included), fold kernel bytes added"))


def cpu_baseline(U64, target_s=15.0):
    """The FP64 oracle's half-sweep on the host, on the same 32^3x64 field
    (FP32-rounded values), sized to about target_s seconds."""
    import numpy as np

    from oracle import oracle as O
    W = U64.to(dtype=__import__("torch").complex64).cpu().numpy().astype(np.complex128)
    L = O.dims_of(W)
    G = O.identity_gauge(L)
    V = int(np.prod(L))
    t0 = time.time()
    O.halfsweep_inplace(W, G, 0, 1.7)
    t1 = time.time() - t0
    n = max(1, min(1000, int(target_s / max(t1, 1e-3)) - 1))
    t0 = time.time()
    for k in range(n):
        O.halfsweep_inplace(W, G, (k + 1) & 1, 1.7)
    dt = time.time() - t0
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    # the same half-sweep on one thread (the oracle's OpenMP runtime is libgomp)
    import ctypes
    gomp = ctypes.CDLL("libgomp.so.1")
    gomp.omp_set_num_threads(1)
    t0 = time.time()
    n1 = 0
    while n1 < 2 or time.time() - t0 < 3.0:
        O.halfsweep_inplace(W, G, n1 & 1, 1.7)
        n1 += 1
    dt1 = time.time() - t0
    gomp.omp_set_num_threads(cores)
    model = ""
    try:
        model = next(ln.split(":", 1)[1].strip() for ln in open("/proc/cpuinfo") if ln.startswith("model name"))
    except (OSError, StopIteration):
        pass
    return dict(value=round(n * (V // 2) / dt, 1), unit="site-updates/s", cores=cores, kind="oracle",
                sample=f"{n} FP64 oracle half-sweeps of the 32^3x64 field ({V // 2} site-updates each), "
                       f"{dt:.1f} s, {cores} OpenMP threads on {os.cpu_count()} visible CPUs ({model})",
                single_thread_value=round(n1 * (V // 2) / dt1, 1))


def profile_run(api, torch, synth, variant=None):
    """Fixed work for rocprofv3: plain device copies of known size (to
    calibrate the byte counters), 25 warm-up sweeps, then 20 measured sweeps
    (the last 40 half-sweep launches and the last fold) at 32^3x64 FP32 in the
    benchmark's launch configuration: the variant autotuned on a batch of
    the benchmark's four shapes (the half-sweep's cost does not depend on
    the link values, so the three smaller fields are Haar-random)."""
    L = LATTICES[0]
    U = api.to_links(synth.heatbath_field_gpu(L, synth.sub_seed(5, 0), 5.7, 50), 1)
    others = [api.to_links(synth.haar_links_gpu(Lb, synth.sub_seed(5, 10 + i)), 1)
              for i, Lb in enumerate(LATTICES[1:])]
    if variant is None:
        best, _ = api.autotune_batch([U] + others)
    else:
        api.set_variant(1, variant)
        best = variant
    del others
    nbytes = 1 << 30
    a = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)  # 1 GiB read + 1 GiB written per copy
    W, G = U.clone(), api.gauge_identity(L)
    api.sweeps(W, G, 25)  # warm-up (one full ring)
    api.sweeps(W, G, 20)  # the measured 40 half-sweeps and their fold
    torch.cuda.synchronize()
    print(json.dumps(dict(profile="done", copy_bytes_each_way=nbytes, halfsweeps=40, lattice=L,
                          variant=best)))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-gribov", action="store_true", help="skip the Gribov-copy comparison")
    ap.add_argument("--profile", action="store_true")
    ap.add_argument("--profile-loops", action="store_true", help="short Wilson-loop run for rocprofv3")
    ap.add_argument("--profile-step", action="store_true", help="one benchmark step for rocprofv3")
    ap.add_argument("--profile-smear", action="store_true", help="smearing steps at 32^3x64 for rocprofv3")
    ap.add_argument("--profile-backward", action="store_true", help="one backward pass at 16^4 for rocprofv3")
    ap.add_argument("--profile-roofline", action="store_true",
                    help="the roofline measurement alone (batch-tuned variant), for rocprofv3")
    ap.add_argument("--variant", type=int, default=None,
                    help="with --profile / --profile-roofline: this half-sweep variant instead of the tuned one "
                         "(so that separate counter runs time the same instantiations)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU: the workload is one MI355X's share of the job, and "
              "runs on several GPUs are not part of this benchmark.")
        sys.exit(2)

    import torch

    from paper_0807_0264_amd import api, synth
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.profile:
        profile_run(api, torch, synth, args.variant)
        return
    if args.profile_step:
        fields = make_inputs(api, synth, torch)
        api.autotune_batch([U for _, U, _ in fields])
        api.tune_batch([U for _, U, _ in fields])
        r = one_step(api, fields)
        torch.cuda.synchronize()
        print(json.dumps(dict(profile="done", sweeps=[(x["sweeps_smeared"], x["sweeps"]) for x in r])))
        return
    if args.profile_smear:
        L = LATTICES[0]
        U = api.to_links(synth.heatbath_field_gpu(L, synth.sub_seed(5, 0), 5.7, 50), 1)
        print(json.dumps(dict(profile="done", lattice=L, smear=smear_run(api, torch, U, reps=1))))
        return
    if args.profile_roofline:
        L = LATTICES[0]
        U = api.to_links(synth.heatbath_field_gpu(L, synth.sub_seed(5, 0), 5.7, 50), 1)
        others = [api.to_links(synth.haar_links_gpu(Lb, synth.sub_seed(5, 10 + i)), 1)
                  for i, Lb in enumerate(LATTICES[1:])]
        if args.variant is None:
            best, _ = api.autotune_batch([U] + others)
        else:
            api.set_variant(1, args.variant)
            best = args.variant
        del others
        print(json.dumps(dict(profile="done", variant=best, roofline=roofline(api, torch, U))))
        return
    if args.profile_backward:
        print(json.dumps(dict(profile="done", backward=backward_run(api, torch, synth, reps=1))))
        return
    if args.profile_loops:
        L = LATTICES[2]
        U = api.to_links(synth.heatbath_field_gpu(L, synth.sub_seed(5, 2), 5.7, 50), 1)
        r = wilson_loop_run(api, torch, U, None, reps=1)
        print(json.dumps(dict(profile="done", lattice=L, **r)))
        return

    fields = make_inputs(api, synth, torch)
    # tuned on the batch the step fixes: every timed launch covers all four fields; first the
    # variant alone (kept as the context's variant: the raw sweeps of the roofline use it), then
    # variant and schedule together (kept for the batch's shape: the step's fixes use it)
    best, ms = api.autotune_batch([U for _, U, _ in fields])
    log(f"autotuned half-sweep variant {best}: ms per batched half-sweep {[round(x, 3) for x in ms]}")
    sched = api.tune_batch([U for _, U, _ in fields])
    log(f"tuned sweep schedule of the batch: {sched}")

    for w in range(args.warmup):
        t0 = time.time()
        r = one_step(api, fields)
        log(f"warm-up step {w}: {time.time() - t0:.2f} s, sweeps "
            f"{[(x['sweeps_smeared'], x['sweeps']) for x in r]}")
    torch.cuda.synchronize()
    t0 = time.time()
    results = []
    for k in range(args.steps):
        results.append(one_step(api, fields))
        log(f"step {k} done at {time.time() - t0:.2f} s")
    torch.cuda.synchronize()
    elapsed = time.time() - t0
    total = sum(x["site_updates"] for r in results for x in r)
    value = total / elapsed

    roof = roofline(api, torch, fields[0][1])
    # the same kernel inside the batch: the tuner's median over three passes of 8 launches, each one
    # half-sweep over all four fields, HIP events (no stop flags, no folds)
    su_batch = sum(api.volume(L) for L, _, _ in fields) // 2
    bps = roof["bytes_per_site_update"]
    gbps = su_batch * bps / (ms[best] * 1e-3) / 1e9
    roof["in_batch"] = dict(ms_per_launch=round(ms[best], 4), site_updates_per_launch=su_batch,
                            bytes_per_launch=su_batch * bps, GBps=round(gbps, 1),
                            frac=round(gbps / HBM_PEAK_GBS, 4),
                            note="one half-sweep over the four fields of the step (autotuner timing)")
    roof["copy_ceiling_GBps"] = copy_ceiling(torch)
    log(f"roofline: {roof}")
    gribov = None if args.no_gribov else gribov_copies(api, synth, torch, fields[2][1])
    smear = smear_run(api, torch, fields[0][1])
    log(f"smear: {smear}")
    backward = backward_run(api, torch, synth)
    log(f"backward: {backward}")
    G20, _ = api.fix(fields[2][1], None, tol=1e-7, max_sweeps=5000)
    loops = wilson_loop_run(api, torch, fields[2][1], G20)
    log(f"wilson loops: {loops['fields']}")
    line = dict(metric=METRIC, value=round(value, 1), unit="site-updates/s", n_gpus=1,
                steps=args.steps, warmup=args.warmup, ms_per_step=round(1000 * elapsed / args.steps, 2),
                higher_is_better=True, scaling="weak", vs_baseline=None, dtype="f32",
                data="synthetic (seeded beta=5.7 Wilson heatbath fields, 50 sweeps from Haar)",
                config=dict(workload="batch 32^3x64 + 24^3x48 + 20^3x40 + 16^4: stout rho=0.1 n=10, "
                                     "batched MCG fix to dR<1e-7 (omega=1.7), carried-back batched "
                                     "re-fix, centre projection, vortex count (one mcg_precondition_batch "
                                     "call per step)",
                            links="fp32", gauge="fp64", reductions="fp64", half_sweep_variant=best,
                            tuned_schedule=dict(sched, ms_per_sweep=round(sched["ms_per_sweep"], 4),
                                                ms_default=round(sched["ms_default"], 4)),
                            sweep_order={0: "forward", 1: "odd half-sweeps in reverse tile order",
                                         2: "odd half-sweeps in reverse tile order; each XCD a "
                                            "contiguous range of every field's tiles"}[sched["order"]],
                            transform="per-half-sweep g in a ring, folded into G every 25 sweeps"
                            if api.get_defer_g() else "G updated in every half-sweep",
                            sweeps=("paired: the even half-sweep leaves the links to the odd one"
                                    if api.get_defer_g() and sched["paired"] else "plain half-sweeps")
                            + (f", {sched['slabs']} slabs per half-sweep" if sched["slabs"] > 1 else ""),
                            per_field=[dict(L=x["L"], sweeps_smeared=x["sweeps_smeared"], sweeps=x["sweeps"],
                                            R_smeared=round(x["R_smeared"], 7), R=round(x["R"], 7),
                                            vortex_fraction=round(x["vortex_fraction"], 5))
                                       for x in results[-1]]),
                roofline=roof)
    if gribov is not None:
        line["gribov_copies"] = gribov
    line["wilson_loops"] = loops
    line["smear"] = smear
    line["backward"] = backward
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(fields[0][2])
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
