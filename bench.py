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
  kernel at 32^3x64 and the FP64 CPU oracle timed on a bounded sample.

    python bench.py [--steps K] [--warmup W] [--gpus 1] [--no-cpu-baseline]
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
# algorithmic bytes of one site-update with FP32 links and an FP64 transform:
# 8 links read and written + G(x) read and written.  In the two-row form (the
# default) a link is 6 complex FP32 (48 B) and G(x) 6 complex FP64 (96 B); as
# full matrices 72 B and 144 B.
BYTES_PER_SITE_UPDATE = {True: 8 * 48 * 2 + 2 * 96, False: 8 * 72 * 2 + 2 * 144}
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


def one_step(api, fields, tol=1e-7, max_sweeps=5000):
    Us = [U for _, U, _ in fields]
    S = [api.smear(U, 0.1, 1.0, 10) for U in Us]
    Gs, info_s = api.fix_batch(S, None, tol=tol, max_sweeps=max_sweeps, omega=1.7, check_every=50)
    del S
    G, info = api.fix_batch(Us, Gs, tol=tol, max_sweeps=max_sweeps, omega=1.7, check_every=50)
    out = []
    for (L, U, _), g, a, b in zip(fields, G, info_s, info):
        Z, margin = api.center_project(U, g)
        v = api.count_vortices(Z, L)
        V = api.volume(L)
        out.append(dict(L=L, sweeps_smeared=a["sweeps"], sweeps=b["sweeps"], R_smeared=a["R"], R=b["R"],
                        vortex_fraction=v["total"] / (6 * V), min_margin=margin,
                        site_updates=(a["sweeps"] + b["sweeps"]) * V))
    return out


def roofline(api, torch, U, nsweeps=100):
    """Average duration of the half-sweep kernel at 32^3x64 (FP32 links, FP64
    G), from HIP events on the stream the kernels are launched on (the
    library launches on torch's current stream).  A call of api.sweeps also
    converts W and G to and from the storage form; timing n + 20 and 20
    sweeps and taking the difference leaves 2n half-sweep launches alone."""
    W = U.clone()
    G = api.gauge_identity(U.L)
    api.sweeps(W, G, 5)  # warm-up
    torch.cuda.synchronize()

    def timed(n):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        api.sweeps(W, G, n)
        e1.record()
        e1.synchronize()
        return e0.elapsed_time(e1)

    ms = (timed(nsweeps + 20) - timed(20)) / (2 * nsweeps)
    two_row = api.get_two_row()
    bps = BYTES_PER_SITE_UPDATE[two_row]
    site_updates = api.volume(U.L) // 2
    achieved = site_updates * bps / (ms * 1e-3) / 1e9
    traffic = None
    if os.path.exists(PMC_FILE):
        pmc = json.load(open(PMC_FILE))
        if pmc.get("kernel_source_hash") == kernel_source_hash():
            traffic = pmc.get("hbm_bytes_per_launch")
    return dict(bound="hbm", achieved=round(achieved, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                frac=round(achieved / HBM_PEAK_GBS, 4), traffic=traffic,
                kernel="k_halfsweep<float,%s> (one parity of 32^3x64)" % ("two-row" if two_row else "full"),
                ms_per_launch=round(ms, 4), bytes_per_launch=site_updates * bps, bytes_per_site_update=bps)


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
    return dict(value=round(n * (V // 2) / dt, 1), unit="site-updates/s", cores=cores, kind="oracle",
                sample=f"{n} FP64 oracle half-sweeps of the 32^3x64 field ({V // 2} site-updates each), "
                       f"{dt:.1f} s")


def profile_run(api, torch, synth):
    """Fixed work for rocprofv3: plain device copies of known size (to
    calibrate the byte counters), then 20 sweeps at 32^3x64 FP32 in the
    benchmark's launch configuration (autotuned variant)."""
    L = LATTICES[0]
    U = api.to_links(synth.heatbath_field_gpu(L, synth.sub_seed(5, 0), 5.7, 50), 1)
    best, _ = api.autotune(U)
    nbytes = 1 << 30
    a = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)  # 1 GiB read + 1 GiB written per copy
    W, G = U.clone(), api.gauge_identity(L)
    api.sweeps(W, G, 20)
    torch.cuda.synchronize()
    print(json.dumps(dict(profile="done", copy_bytes_each_way=nbytes, halfsweeps=40, lattice=L,
                          variant=best)))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--profile", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU: the workload is one MI355X's share of the job, and "
              "runs on several GPUs are not part of this benchmark.")
        sys.exit(2)

    import torch

    from paper_0807_0264_amd import api, synth
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.profile:
        profile_run(api, torch, synth)
        return

    fields = make_inputs(api, synth, torch)
    best, ms = api.autotune(fields[0][1])
    log(f"autotuned half-sweep variant {best}: ms per half-sweep {[round(x, 3) for x in ms]}")

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
    log(f"roofline: {roof}")
    line = dict(metric=METRIC, value=round(value, 1), unit="site-updates/s", n_gpus=1,
                steps=args.steps, warmup=args.warmup, ms_per_step=round(1000 * elapsed / args.steps, 2),
                higher_is_better=True, scaling="weak", vs_baseline=None, dtype="f32",
                data="synthetic (seeded beta=5.7 Wilson heatbath fields, 50 sweeps from Haar)",
                config=dict(workload="batch 32^3x64 + 24^3x48 + 20^3x40 + 16^4: stout rho=0.1 n=10, "
                                     "batched MCG fix to dR<1e-7 (omega=1.7), carried-back batched "
                                     "re-fix, centre projection, vortex count",
                            links="fp32", gauge="fp64", reductions="fp64", half_sweep_variant=best,
                            per_field=[dict(L=x["L"], sweeps_smeared=x["sweeps_smeared"], sweeps=x["sweeps"],
                                            R_smeared=round(x["R_smeared"], 7), R=round(x["R"], 7),
                                            vortex_fraction=round(x["vortex_fraction"], 5))
                                       for x in results[-1]]),
                roofline=roof)
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(fields[0][2])
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
