"""gfx950 (MI355X) library for stout-preconditioned Maximal Center Gauge
fixing in SU(3) (O Cais et al., arXiv:0807.0264).

The compute path is libmcg.so (HIP kernels behind the C ABI of
include/mcg.h); `paper_0807_0264_amd.api` is its Python binding, and the
names below are re-exported from it on first use.  `paper_0807_0264_amd.synth`
generates seeded synthetic input fields.
"""
import importlib


def __getattr__(name):
    if name.startswith("__") or name in ("api", "synth", "_abi", "build", "autograd"):
        raise AttributeError(name)
    return getattr(importlib.import_module(__name__ + ".api"), name)
