"""Preconditioning levels and the statistics across them (Sec. III, Tables
I-III).

A *level* is one preconditioning: n stout steps (rho = 0.1) or n over-improved
stout steps (rho = 0.06, eps = -0.25) of the original field, the MCG fix of
that smeared field, the carry-back of its transform to the original field and
the re-fix there, then centre projection and P-vortex counting.  Levels are
independent of each other (each starts from the unsmeared field and the same
start transform); n = 0 is plain MCG fixing.

run_levels() drives the GPU library for one field and all levels (every
smeared field of a level series is produced from the previous one by further
steps, which gives the same bits as smearing from scratch; the fixes of all
levels run as one batch).  table1() and transitions() are host statistics over
the per-configuration results, in the form of Tables I, II and III.
"""
from dataclasses import dataclass

import numpy as np


@dataclass(frozen=True)
class Level:
    name: str
    rho: float
    eps: float
    n: int


# the preconditioning levels of Sec. III: stout rho = 0.1 with 0..20 steps in
# steps of 4, and 80 over-improved steps with rho = 0.06, eps = -0.25
PAPER_LEVELS = tuple([Level(str(n), 0.1, 1.0, n) for n in range(0, 21, 4)] + [Level("OI 80", 0.06, -0.25, 80)])
# a wider range of stout steps (0, 10, 50, 100 at rho = 0.1) against the same over-improved level
WIDE_LEVELS = tuple([Level(str(n), 0.1, 1.0, n) for n in (0, 10, 50, 100)] + [Level("OI 80", 0.06, -0.25, 80)])


def run_levels(U, levels=PAPER_LEVELS, G0=None, tol=1e-7, max_sweeps=5000, omega=1.7, reunit_every=50,
               check_every=50):
    """All preconditioning levels of one field U (api.Links) on the GPU.

    G0 (api.GaugeField or None = identity) is the start transform of every
    level, so a Haar G0 selects a Gribov copy.  Returns one dict per level:
    R_smeared (None at n = 0), R, sweeps_smeared, sweeps, blocks (blocks of 50
    sweeps of both fixes, each rounded up), vortices (total P-vortex count),
    plaquettes (6V), min_margin, status (worst of the two fixes)."""
    from . import api

    L = U.L
    start = G0 if G0 is not None else api.gauge_identity(L, U.data.device.index)
    smeared = []  # (level index, smeared field)
    last = {}  # (rho, eps) -> (n, field): continue a series instead of restarting it
    for i, lv in enumerate(levels):
        if lv.n < 0:
            raise ValueError(f"level {lv.name}: n must be >= 0")
        if lv.n == 0:
            continue
        n0, S0 = last.get((lv.rho, lv.eps), (0, U))
        if n0 > lv.n:
            n0, S0 = 0, U
        S = api.smear(S0, lv.rho, lv.eps, lv.n - n0) if lv.n > n0 else S0.clone()
        last[(lv.rho, lv.eps)] = (lv.n, S)
        smeared.append((i, S))
    kw = dict(tol=tol, max_sweeps=max_sweeps, omega=omega, reunit_every=reunit_every, check_every=check_every)
    Gs = [start.clone() for _ in levels]
    info_s = [None] * len(levels)
    if smeared:
        G_sm, inf = api.fix_batch([S for _, S in smeared], [Gs[i] for i, _ in smeared], **kw)
        for (i, _), g, f in zip(smeared, G_sm, inf):
            Gs[i], info_s[i] = g, f
    del smeared, last
    G, info = api.fix_batch([U] * len(levels), Gs, **kw)
    nplaq = 6 * api.volume(L)
    out = []
    for lv, g, a, b in zip(levels, G, info_s, info):
        Z, margin = api.center_project(U, g)
        v = api.count_vortices(Z, L)
        sw_s = a["sweeps"] if a else 0
        out.append(dict(level=lv.name, n=lv.n, rho=lv.rho, eps=lv.eps,
                        R_smeared=a["R"] if a else None, R=b["R"], sweeps_smeared=sw_s, sweeps=b["sweeps"],
                        blocks=-(-sw_s // 50) + -(-b["sweeps"] // 50), vortices=v["total"],
                        plaquettes=nplaq, min_margin=margin,
                        status=max(b["status"], a["status"] if a else 0)))
    return out


def _stack(results, key):
    """results: list over configurations of lists over levels -> array [cfg, level]."""
    return np.array([[r[key] if r[key] is not None else np.nan for r in cfg] for cfg in results], dtype=float)


def table1(results):
    """Table I analogue: per level, the mean and standard deviation over
    configurations of the total blocks of 50 sweeps, and the mean and its
    standard error of the smeared-field maximum, the final maximum R and the
    P-vortex percentage."""
    blocks = _stack(results, "blocks")
    Rs = _stack(results, "R_smeared")
    R = _stack(results, "R")
    vp = 100.0 * _stack(results, "vortices") / _stack(results, "plaquettes")
    n = blocks.shape[0]

    def sem(a):
        return np.std(a, ddof=1) / np.sqrt(len(a)) if len(a) > 1 else float("nan")

    rows = []
    for k, lv in enumerate(results[0]):
        rs = Rs[:, k]
        rows.append(dict(level=lv["level"], blocks_mean=float(blocks[:, k].mean()),
                         blocks_std=float(np.std(blocks[:, k], ddof=1)) if n > 1 else float("nan"),
                         R_smeared_mean=None if np.isnan(rs).all() else float(rs.mean()),
                         R_smeared_sem=None if np.isnan(rs).all() else float(sem(rs)),
                         R_mean=float(R[:, k].mean()), R_sem=float(sem(R[:, k])),
                         vortex_pct_mean=float(vp[:, k].mean()), vortex_pct_sem=float(sem(vp[:, k]))))
    return rows


def transitions(results):
    """Tables II and III: for every ordered pair of levels i < j (rows and
    columns in level order), over configurations,

    vortex_reduced[i][j]   % of configurations whose P-vortex count at j is
                           below that at i                    (Table II, upper)
    reduction_pct[j][i]    mean and standard deviation of the percentage
                           reduction 100 (n_i - n_j) / n_i over those
                           configurations                    (Table II, lower)
    higher_max[i][j]       % of configurations whose final R at j exceeds
                           that at i                         (Table III, upper)
    lower_given_higher[j][i] % of the configurations with the higher maximum
                           whose P-vortex count at j is below that at i
                                                             (Table III, lower)

    Entries with no configuration to average over are None; diagonals are None."""
    nv = _stack(results, "vortices")
    R = _stack(results, "R")
    ncfg, nl = nv.shape
    names = [lv["level"] for lv in results[0]]
    t2 = [[None] * nl for _ in range(nl)]
    t3 = [[None] * nl for _ in range(nl)]
    for i in range(nl):
        for j in range(i + 1, nl):
            red = nv[:, j] < nv[:, i]
            t2[i][j] = 100.0 * red.sum() / ncfg
            if red.any():
                pct = 100.0 * (nv[red, i] - nv[red, j]) / nv[red, i]
                t2[j][i] = (float(pct.mean()), float(np.std(pct, ddof=1)) if red.sum() > 1 else 0.0)
            hi = R[:, j] > R[:, i]
            t3[i][j] = 100.0 * hi.sum() / ncfg
            if hi.any():
                t3[j][i] = 100.0 * (nv[hi, j] < nv[hi, i]).sum() / hi.sum()
    return dict(levels=names, configurations=ncfg, table2=t2, table3=t3)


def format_tables(results):
    """Plain-text rendering of table1() and transitions()."""
    t1 = table1(results)
    tr = transitions(results)
    lines = [f"{'level':>6} {'blocks':>12} {'smeared max':>16} {'max':>16} {'vortices %':>14}"]
    for r in t1:
        sm = "-" if r["R_smeared_mean"] is None else f"{r['R_smeared_mean']:.5f}({r['R_smeared_sem']:.1e})"
        lines.append(f"{r['level']:>6} {r['blocks_mean']:7.1f}+-{r['blocks_std']:<4.1f} {sm:>16} "
                     f"{r['R_mean']:.5f}({r['R_sem']:.1e}) {r['vortex_pct_mean']:7.3f}({r['vortex_pct_sem']:.1e})")
    for key, title in (("table2", "vortex reduction: % of configurations (upper) / mean % reduction (lower)"),
                       ("table3", "higher maximum: % of configurations (upper) / % of those with fewer vortices "
                                  "(lower)")):
        lines += ["", title, " " * 7 + "".join(f"{n:>12}" for n in tr["levels"])]
        for i, n in enumerate(tr["levels"]):
            cells = []
            for j in range(len(tr["levels"])):
                v = tr[key][i][j]
                cells.append("\\" if i == j else "-" if v is None else
                             f"{v[0]:.1f}+-{v[1]:.1f}" if isinstance(v, tuple) else f"{v:.1f}")
            lines.append(f"{n:>7}" + "".join(f"{c:>12}" for c in cells))
    return "\n".join(lines)


def main(argv=None):
    """Synthetic stand-in for the paper's study: configurations from a seeded
    heatbath (Wilson, or the Luscher-Weisz action of the paper's ensemble),
    all preconditioning levels per configuration."""
    import argparse
    import json

    import torch

    from . import api, synth
    ap = argparse.ArgumentParser(description=main.__doc__)
    ap.add_argument("--configs", type=int, default=8)
    ap.add_argument("--lattice", default="20,20,20,40")
    ap.add_argument("--action", choices=("wilson", "lw"), default="wilson",
                    help="input fields: Wilson heatbath, or Luscher-Weisz (plaquette + rectangle) heatbath")
    ap.add_argument("--beta", type=float, default=None, help="coupling (default 5.7 Wilson, 4.52 Luscher-Weisz)")
    ap.add_argument("--u0", type=float, default=0.884, help="tadpole factor of the Luscher-Weisz rectangle weight")
    ap.add_argument("--therm", type=int, default=None, help="heatbath sweeps from the Haar start (50 / 100)")
    ap.add_argument("--prec", choices=("fp32", "fp64"), default="fp32")
    ap.add_argument("--tol", type=float, default=1e-7)
    ap.add_argument("--levels", choices=("paper", "wide"), default="paper",
                    help="paper: stout 0..20 in steps of 4 and OI 80; wide: stout 0, 10, 50, 100 and OI 80")
    ap.add_argument("--compare", action="store_true",
                    help="run every configuration in both precisions and report the FP32 - FP64 differences")
    ap.add_argument("--json", action="store_true", help="print the raw per-configuration results as JSON")
    ap.add_argument("--first", type=int, default=0,
                    help="index of the first configuration (seeds follow the index, so runs can be split)")
    ap.add_argument("--jsonl", default=None,
                    help="append each configuration's results (first precision) to this file, one JSON line each")
    ap.add_argument("--tables", nargs="+", default=None, metavar="JSONL",
                    help="print the tables of the configurations recorded in these files and exit (no GPU)")
    a = ap.parse_args(argv)
    if a.tables:
        rows = [json.loads(ln) for f in a.tables for ln in open(f) if ln.strip()]
        seen = {}
        for r in rows:  # one entry per configuration index, the last one recorded
            seen[r["config"]] = r["levels"]
        print(f"{len(seen)} configurations", flush=True)
        print(format_tables([seen[k] for k in sorted(seen)]), flush=True)
        return
    L = tuple(int(v) for v in a.lattice.split(","))
    precs = (1, 0) if a.compare else ((1,) if a.prec == "fp32" else (0,))
    results = {p: [] for p in precs}
    lw = a.action == "lw"
    beta = a.beta if a.beta is not None else (4.52 if lw else 5.7)
    therm = a.therm if a.therm is not None else (100 if lw else 50)
    for c in range(a.first, a.first + a.configs):
        if lw:
            U64 = synth.heatbath_lw_field_gpu(L, synth.sub_seed(12, c), beta, therm, a.u0)
        else:
            U64 = synth.heatbath_field_gpu(L, synth.sub_seed(11, c), beta, therm)
        # both precisions start from the same (FP32-rounded when comparing) values
        if a.compare:
            U64 = U64.to(torch.complex64).to(torch.complex128)
        for p in precs:
            levels = PAPER_LEVELS if a.levels == "paper" else WIDE_LEVELS
            results[p].append(run_levels(api.to_links(U64, p), levels, tol=a.tol))
        torch.cuda.synchronize()
        print(f"configuration {c}: " + ", ".join(f"{r['level']}: R {r['R']:.5f} v {r['vortices']}"
                                                 for r in results[precs[0]][-1]), flush=True)
        if a.jsonl:
            with open(a.jsonl, "a") as fh:
                fh.write(json.dumps(dict(config=c, action=a.action, lattice=list(L), beta=beta,
                                         levels=results[precs[0]][-1])) + "\n")
    for p in precs:
        print(f"\n{'FP32' if p == 1 else 'FP64'} links", flush=True)
        print(json.dumps(results[p]) if a.json else format_tables(results[p]), flush=True)
    if a.compare:
        print("\nFP32 - FP64 per result (mean |difference| over configurations; sweeps: mean signed difference)")
        for k, lv in enumerate(results[1][0]):
            d = [(x[k], y[k]) for x, y in zip(results[1], results[0])]
            dRs = [abs(x["R_smeared"] - y["R_smeared"]) for x, y in d if x["R_smeared"] is not None]
            print(f"{lv['level']:>6}: |dR| {sum(abs(x['R'] - y['R']) for x, y in d) / len(d):.2e}"
                  + (f"  |dR_smeared| {sum(dRs) / len(dRs):.2e}" if dRs else "")
                  + f"  |d vortex %| {sum(abs(x['vortices'] - y['vortices']) for x, y in d) / len(d) / lv['plaquettes'] * 100:.3f}"
                  + f"  d sweeps {sum(x['sweeps'] + x['sweeps_smeared'] - y['sweeps'] - y['sweeps_smeared'] for x, y in d) / len(d):+.1f}",
                  flush=True)


if __name__ == "__main__":
    main()
