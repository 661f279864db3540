"""The library (unchanged kernel and driver sources) built for the host
against an emulated HIP runtime, run under AddressSanitizer and UBSan, and
compared with the oracle on small lattices (tests/emu/run_scenarios.py).
Catches out-of-bounds indexing and wrong results without a GPU."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
EMU = os.path.join(ROOT, "tests", "emu")
# the long groups split by precision (or, for defer, by part) so that they run side by side
GROUPS = ["fields", "smear", "halfsweep", "fix", "project", "batch:0", "batch:1", "planted", "backward", "loops",
          "slabs:0", "slabs:1", "variants:0", "variants:1", "checks", "defer:rows", "defer:full", "defer:fp64"]


def _stale(lib, srcdirs):
    if not os.path.exists(lib):
        return True
    t = os.path.getmtime(lib)
    for d in srcdirs:
        for f in os.listdir(d):
            if os.path.getmtime(os.path.join(d, f)) > t:
                return True
    return False


@pytest.fixture(scope="module")
def emu_lib():
    sys.path.insert(0, EMU)
    import build_emu
    csrc = os.path.join(ROOT, "paper_0807_0264_amd", "csrc")
    if _stale(build_emu.LIB, [csrc, os.path.join(EMU, "include", "hip")]):
        build_emu.build()
    return build_emu.LIB


def test_emulated_kernels_match_oracle(emu_lib):
    asan = subprocess.check_output(["gcc", "-print-file-name=libasan.so"], text=True).strip()
    env = dict(os.environ, LD_PRELOAD=asan, ASAN_OPTIONS="detect_leaks=0", OMP_NUM_THREADS="1")
    procs = {g: subprocess.Popen([sys.executable, os.path.join(EMU, "run_scenarios.py"), g], env=env,
                                 stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
             for g in GROUPS}
    failed = {}
    for g, p in procs.items():
        out, _ = p.communicate(timeout=900)
        if p.returncode != 0:
            failed[g] = out[-3000:]
    assert not failed, failed
