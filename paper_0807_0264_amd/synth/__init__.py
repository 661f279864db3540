"""Seeded synthetic gauge fields (inputs only).

The paper's ensemble (quenched Luscher-Weisz configurations) is not
available, so every input is generated here from a seed:

* Haar-random SU(3) links and per-site gauge transforms,
* uniform Z3 integers (for planted centre configurations),
* standard normals (for random su(3) tangent directions),
* thermalised-like fields: a Haar start followed by Cabibbo-Marinari
  heatbath sweeps of the Wilson plaquette action.

Nothing in this module smears, gauge-fixes, projects or counts.  The host
build (synth_cpu.c) and the gfx950 build (synth_gpu.hip) of the same
generator produce bit-identical fields; the GPU build is used for large
lattices.

Arrays are numpy complex128 in the interchange layout
[Lt, Lz, Ly, Lx, 4, 3, 3] (links) or [Lt, Lz, Ly, Lx, 3, 3] (gauge).
"""
import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
CPU_LIB = os.path.join(HERE, "libsynth_cpu.so")
GPU_LIB = os.path.join(HERE, "libsynth_gpu.so")

MASTER_SEED = 8070264

_cpu = None
_gpu = None


def build(verbose=False):
    """Compile both builds of the generator (host and gfx950)."""
    cmds = [
        ["gcc", "-std=c11", "-O2", "-fopenmp", "-ffp-contract=off", "-fPIC", "-shared",
         "-Wall", os.path.join(HERE, "synth_cpu.c"), "-o", CPU_LIB + ".tmp"],
        ["/opt/rocm/bin/hipcc", "--offload-arch=gfx950", "-O2", "-ffp-contract=off",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-fPIC", "-shared", os.path.join(HERE, "synth_gpu.hip"), "-o", GPU_LIB + ".tmp"],
    ]
    for cmd, lib in zip(cmds, (CPU_LIB, GPU_LIB)):
        if verbose:
            print(" ".join(cmd))
        subprocess.check_call(cmd, stderr=subprocess.DEVNULL if not verbose else None)
        os.replace(lib + ".tmp", lib)


def _I4(L):
    return (C.c_int32 * 4)(*[int(v) for v in L])


def cpu():
    global _cpu
    if _cpu is None:
        if not os.path.exists(CPU_LIB):
            build()
        l = C.CDLL(CPU_LIB)
        P, I4 = C.c_void_p, C.POINTER(C.c_int32)
        l.sy_cpu_haar_links.argtypes = [I4, C.c_uint64, P]
        l.sy_cpu_haar_gauge.argtypes = [I4, C.c_uint64, C.c_uint64, P]
        l.sy_cpu_z3.argtypes = [I4, C.c_uint64, P]
        l.sy_cpu_gauss.argtypes = [C.c_uint64, C.c_uint64, C.c_int64, P]
        l.sy_cpu_heatbath.argtypes = [I4, C.c_uint64, C.c_double, C.c_int, P]
        l.sy_cpu_heatbath_lw.argtypes = [I4, C.c_uint64, C.c_double, C.c_double, C.c_int, P]
        l.sy_cpu_lw_staple.argtypes = [I4, P, C.c_int64, C.c_int, C.c_double, C.c_double, P]
        l.sy_cpu_lw_colour.argtypes = [I4, C.c_int64, C.c_int]
        l.sy_cpu_lw_colour.restype = C.c_int
        for f in ("sy_cpu_log", "sy_cpu_sqrt", "sy_cpu_recip"):
            getattr(l, f).argtypes = [C.c_double]
            getattr(l, f).restype = C.c_double
        l.sy_cpu_sincos_turn.argtypes = [C.c_double, C.POINTER(C.c_double), C.POINTER(C.c_double)]
        _cpu = l
    return _cpu


def gpu():
    global _gpu
    if _gpu is None:
        if not os.path.exists(GPU_LIB):
            raise RuntimeError("libsynth_gpu.so is not built; run __graft_entry__.build()")
        l = C.CDLL(GPU_LIB)
        P, I4 = C.c_void_p, C.POINTER(C.c_int32)
        l.sy_gpu_haar_links.argtypes = [I4, C.c_uint64, P, P]
        l.sy_gpu_haar_gauge.argtypes = [I4, C.c_uint64, C.c_uint64, P, P]
        l.sy_gpu_heatbath.argtypes = [I4, C.c_uint64, C.c_double, C.c_int, P, P]
        l.sy_gpu_heatbath_lw.argtypes = [I4, C.c_uint64, C.c_double, C.c_double, C.c_int, P, P]
        for f in ("sy_gpu_haar_links", "sy_gpu_haar_gauge", "sy_gpu_heatbath", "sy_gpu_heatbath_lw"):
            getattr(l, f).restype = C.c_int
        _gpu = l
    return _gpu


def link_shape(L):
    return (L[3], L[2], L[1], L[0], 4, 3, 3)


def gauge_shape(L):
    return (L[3], L[2], L[1], L[0], 3, 3)


def sub_seed(*parts, master=MASTER_SEED):
    """A 64-bit seed derived from the master seed and integer parts."""
    z = master & 0xFFFFFFFFFFFFFFFF
    for p in parts:
        z = (z * 0x100000001B3 ^ (int(p) & 0xFFFFFFFFFFFFFFFF)) & 0xFFFFFFFFFFFFFFFF
        z ^= z >> 29
        z = (z * 0xBF58476D1CE4E5B9) & 0xFFFFFFFFFFFFFFFF
        z ^= z >> 32
    return z


# ---- host generator ---------------------------------------------------------------
def haar_links(L, seed):
    out = np.empty(link_shape(L), np.complex128)
    cpu().sy_cpu_haar_links(_I4(L), seed, out.ctypes.data_as(C.c_void_p))
    return out


def haar_gauge(L, seed, copy=0):
    out = np.empty(gauge_shape(L), np.complex128)
    cpu().sy_cpu_haar_gauge(_I4(L), seed, copy, out.ctypes.data_as(C.c_void_p))
    return out


def z3_links(L, seed):
    out = np.empty(link_shape(L)[:5], np.int8)
    cpu().sy_cpu_z3(_I4(L), seed, out.ctypes.data_as(C.c_void_p))
    return out


def gaussians(n, seed, stream=0):
    out = np.empty(int(n), np.float64)
    cpu().sy_cpu_gauss(seed, stream, int(n), out.ctypes.data_as(C.c_void_p))
    return out


def heatbath_field(L, seed, beta=5.7, nsweeps=50):
    out = np.empty(link_shape(L), np.complex128)
    cpu().sy_cpu_heatbath(_I4(L), seed, beta, int(nsweeps), out.ctypes.data_as(C.c_void_p))
    return out


def _check_lw(L):
    if any(int(v) % 4 for v in L):
        raise ValueError(f"Luscher-Weisz heatbath needs extents divisible by 4, got {tuple(L)}")


def heatbath_lw_field(L, seed, beta=4.52, nsweeps=50, u0=1.0):
    """Haar start, then nsweeps heatbath sweeps of the Luscher-Weisz action
    (plaquette weight 5/3, rectangle weight -1/(12 u0^2))."""
    _check_lw(L)
    out = np.empty(link_shape(L), np.complex128)
    cpu().sy_cpu_heatbath_lw(_I4(L), seed, beta, float(u0), int(nsweeps), out.ctypes.data_as(C.c_void_p))
    return out


# ---- gfx950 generator (torch tensors on the GPU; bit-identical output) --------------
def _stream_ptr(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def heatbath_field_gpu(L, seed, beta=5.7, nsweeps=50, device="cuda", stream=None):
    import torch
    out = torch.empty(link_shape(L), dtype=torch.complex128, device=device)
    rc = gpu().sy_gpu_heatbath(_I4(L), seed, beta, int(nsweeps), C.c_void_p(out.data_ptr()),
                               _stream_ptr(stream))
    if rc != 0:
        raise RuntimeError(f"sy_gpu_heatbath failed with HIP error {rc}")
    return out


def heatbath_lw_field_gpu(L, seed, beta=4.52, nsweeps=50, u0=1.0, device="cuda", stream=None):
    import torch
    _check_lw(L)
    out = torch.empty(link_shape(L), dtype=torch.complex128, device=device)
    rc = gpu().sy_gpu_heatbath_lw(_I4(L), seed, beta, float(u0), int(nsweeps), C.c_void_p(out.data_ptr()),
                                  _stream_ptr(stream))
    if rc != 0:
        raise RuntimeError(f"sy_gpu_heatbath_lw failed with HIP error {rc}")
    return out


def haar_links_gpu(L, seed, device="cuda", stream=None):
    import torch
    out = torch.empty(link_shape(L), dtype=torch.complex128, device=device)
    rc = gpu().sy_gpu_haar_links(_I4(L), seed, C.c_void_p(out.data_ptr()), _stream_ptr(stream))
    if rc != 0:
        raise RuntimeError(f"sy_gpu_haar_links failed with HIP error {rc}")
    return out


def haar_gauge_gpu(L, seed, copy=0, device="cuda", stream=None):
    import torch
    out = torch.empty(gauge_shape(L), dtype=torch.complex128, device=device)
    rc = gpu().sy_gpu_haar_gauge(_I4(L), seed, copy, C.c_void_p(out.data_ptr()),
                                 _stream_ptr(stream))
    if rc != 0:
        raise RuntimeError(f"sy_gpu_haar_gauge failed with HIP error {rc}")
    return out


# ---- small helpers for tests (no method arithmetic) ---------------------------------
GELL_MANN = np.array([
    [[0, 1, 0], [1, 0, 0], [0, 0, 0]],
    [[0, -1j, 0], [1j, 0, 0], [0, 0, 0]],
    [[1, 0, 0], [0, -1, 0], [0, 0, 0]],
    [[0, 0, 1], [0, 0, 0], [1, 0, 0]],
    [[0, 0, -1j], [0, 0, 0], [1j, 0, 0]],
    [[0, 0, 0], [0, 0, 1], [0, 1, 0]],
    [[0, 0, 0], [0, 0, -1j], [0, 1j, 0]],
    [[1 / np.sqrt(3), 0, 0], [0, 1 / np.sqrt(3), 0], [0, 0, -2 / np.sqrt(3)]],
], dtype=np.complex128)


def su3_tangent(L, seed, stream=0):
    """Random su(3) field X = i sum_a c_a lambda_a / 2 with Gaussian c_a,
    normalised so that sum over links of |X|_F^2 = 1."""
    n = L[0] * L[1] * L[2] * L[3] * 4
    c = gaussians(8 * n, seed, stream).reshape(link_shape(L)[:5] + (8,))
    X = 0.5j * np.einsum("...a,aij->...ij", c, GELL_MANN)
    return X / np.sqrt(np.sum(np.abs(X) ** 2))
