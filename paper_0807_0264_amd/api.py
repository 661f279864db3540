"""Thin Python binding of libmcg.so: argument marshalling only.

Device memory comes from torch tensors on a ROCm device; every computation
runs in the gfx950 kernels behind the C ABI (include/mcg.h).  Names follow
the C calls: smear, fix, apply_gauge, center_project, count_vortices, ...

Fields handed to the library are `Links` (internal even/odd
structure-of-arrays layout, FP64 or FP32) and `GaugeField` (FP64).  Use
`to_links` / `from_links` and `to_gauge` / `from_gauge` to convert from and
to the interchange layout complex [Lt, Lz, Ly, Lx, 4, 3, 3] / [Lt, Lz, Ly, Lx, 3, 3].
"""
import ctypes as C
from dataclasses import dataclass

import torch

from . import _abi as A


class MCGError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"{message} (status {status})")
        self.status = status


_ctx_cache = {}


def context(device=None):
    """The (per-device, per-process) library context."""
    dev = torch.device("cuda", torch.cuda.current_device() if device is None else device)
    idx = dev.index
    if idx not in _ctx_cache:
        lib = A.load()
        h = C.c_void_p()
        with torch.cuda.device(idx):
            st = lib.mcg_create(C.byref(h), idx)
        if st != A.MCG_OK:
            raise MCGError(st, f"mcg_create(device={idx}) failed")
        _ctx_cache[idx] = h
    return _ctx_cache[idx]


def _check(st, ctx, allow_warn=False):
    if st == A.MCG_OK or (allow_warn and st == A.MCG_WNOTCONV):
        return st
    lib = A.load()
    msg = lib.mcg_last_error(ctx).decode() if ctx else lib.mcg_status_string(st).decode()
    raise MCGError(st, msg)


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dims(L):
    d = A.Dims()
    for k in range(4):
        d.L[k] = int(L[k])
    return d


def volume(L):
    return int(L[0]) * int(L[1]) * int(L[2]) * int(L[3])


@dataclass
class Links:
    """Link field in the internal layout: `data` is a flat torch tensor."""
    L: tuple
    prec: int  # A.MCG_F64 or A.MCG_F32
    data: torch.Tensor

    def abi(self):
        need = A.load().mcg_field_bytes(_dims(self.L), self.prec)
        have = self.data.numel() * self.data.element_size()
        if need == 0:
            raise ValueError(f"invalid extents {self.L}: each must be even and >= 2, with fewer than 53,687,092 sites")
        if have < need:
            raise ValueError(f"link buffer of {have} bytes, the field needs {need}")
        f = A.Field()
        f.d = _dims(self.L)
        f.prec = self.prec
        f.ptr = self.data.data_ptr()
        return f

    @property
    def dtype(self):
        return torch.float64 if self.prec == A.MCG_F64 else torch.float32

    def clone(self):
        return Links(self.L, self.prec, self.data.clone())


@dataclass
class GaugeField:
    L: tuple
    data: torch.Tensor  # float64, V * 18 reals

    def abi(self):
        need = A.load().mcg_gauge_bytes(_dims(self.L))
        have = self.data.numel() * self.data.element_size()
        if need == 0:
            raise ValueError(f"invalid extents {self.L}: each must be even and >= 2, with fewer than 53,687,092 sites")
        if have < need:
            raise ValueError(f"gauge buffer of {have} bytes, the field needs {need}")
        g = A.Gauge()
        g.d = _dims(self.L)
        g.ptr = self.data.data_ptr()
        return g

    def clone(self):
        return GaugeField(self.L, self.data.clone())


def _prec_of(dtype):
    if dtype in (torch.float64, torch.complex128, "f64", A.MCG_F64):
        return A.MCG_F64
    if dtype in (torch.float32, torch.complex64, "f32", A.MCG_F32):
        return A.MCG_F32
    raise ValueError(f"unsupported precision {dtype}")


def empty_links(L, prec, device=None):
    prec = _prec_of(prec)
    dt = torch.float64 if prec == A.MCG_F64 else torch.float32
    dev = torch.device("cuda", torch.cuda.current_device() if device is None else device)
    nbytes = A.load().mcg_field_bytes(_dims(L), prec)
    if nbytes == 0:
        raise ValueError(f"invalid extents {tuple(L)}: each must be even and >= 2, with fewer than 53,687,092 sites")
    return Links(tuple(int(v) for v in L), prec,
                 torch.empty(nbytes // torch.empty((), dtype=dt).element_size(), dtype=dt, device=dev))


def empty_gauge(L, device=None):
    dev = torch.device("cuda", torch.cuda.current_device() if device is None else device)
    nbytes = A.load().mcg_gauge_bytes(_dims(L))
    if nbytes == 0:
        raise ValueError(f"invalid extents {tuple(L)}: each must be even and >= 2, with fewer than 53,687,092 sites")
    return GaugeField(tuple(int(v) for v in L), torch.empty(nbytes // 8, dtype=torch.float64, device=dev))


def dims_of_interchange(U):
    return (U.shape[3], U.shape[2], U.shape[1], U.shape[0])


def to_links(U, prec=None):
    """Interchange complex tensor [Lt, Lz, Ly, Lx, 4, 3, 3] on the GPU -> Links."""
    if not U.is_cuda:
        raise ValueError("to_links expects a GPU tensor")
    U = U.contiguous()
    src_prec = _prec_of(U.dtype)
    out = empty_links(dims_of_interchange(U), src_prec if prec is None else prec, U.device.index)
    ctx = context(U.device.index)
    f = out.abi()
    _check(A.load().mcg_pack_links(ctx, C.c_void_p(U.data_ptr()), src_prec, C.byref(f), _stream()), ctx)
    return out


def from_links(W, dtype=None):
    dt = dtype or (torch.complex128 if W.prec == A.MCG_F64 else torch.complex64)
    out = torch.empty((W.L[3], W.L[2], W.L[1], W.L[0], 4, 3, 3), dtype=dt, device=W.data.device)
    ctx = context(W.data.device.index)
    f = W.abi()
    _check(A.load().mcg_unpack_links(ctx, C.byref(f), C.c_void_p(out.data_ptr()), _prec_of(dt), _stream()), ctx)
    return out


def to_gauge(G):
    """Interchange complex128 tensor [Lt, Lz, Ly, Lx, 3, 3] on the GPU -> GaugeField."""
    G = G.contiguous().to(torch.complex128)
    L = (G.shape[3], G.shape[2], G.shape[1], G.shape[0])
    out = empty_gauge(L, G.device.index)
    ctx = context(G.device.index)
    g = out.abi()
    _check(A.load().mcg_pack_gauge(ctx, C.c_void_p(G.data_ptr()), C.byref(g), _stream()), ctx)
    return out


def from_gauge(G):
    out = torch.empty((G.L[3], G.L[2], G.L[1], G.L[0], 3, 3), dtype=torch.complex128, device=G.data.device)
    ctx = context(G.data.device.index)
    g = G.abi()
    _check(A.load().mcg_unpack_gauge(ctx, C.byref(g), C.c_void_p(out.data_ptr()), _stream()), ctx)
    return out


def gauge_identity(L, device=None):
    G = empty_gauge(L, device)
    ctx = context(G.data.device.index)
    g = G.abi()
    _check(A.load().mcg_gauge_identity(ctx, C.byref(g), _stream()), ctx)
    return G


def gauge_reunit(G):
    ctx = context(G.data.device.index)
    g = G.abi()
    _check(A.load().mcg_gauge_reunit(ctx, C.byref(g), _stream()), ctx)
    return G


# ---- the method's calls -----------------------------------------------------------------
def smear(U, rho, eps=1.0, n=1, out=None):
    """n stout (eps = 1) or over-improved stout steps (Sec. II.B)."""
    out = out if out is not None else empty_links(U.L, U.prec, U.data.device.index)
    ctx = context(U.data.device.index)
    fu, fo = U.abi(), out.abi()
    _check(A.load().mcg_smear(ctx, C.byref(fu), C.byref(fo), float(rho), float(eps), int(n), _stream()), ctx)
    return out


def apply_gauge(U, G, out=None):
    out = out if out is not None else empty_links(U.L, U.prec, U.data.device.index)
    ctx = context(U.data.device.index)
    fu, g, fo = U.abi(), G.abi(), out.abi()
    _check(A.load().mcg_apply_gauge(ctx, C.byref(fu), C.byref(g), C.byref(fo), _stream()), ctx)
    return out


def _scalar(fn, U):
    ctx = context(U.data.device.index)
    f = U.abi()
    v = C.c_double()
    _check(fn(ctx, C.byref(f), C.byref(v), _stream()), ctx)
    return v.value


def functional(U):
    """R = (1/N_l) sum |tr U / 3|^2 of the field as given (Sec. II.A)."""
    return _scalar(A.load().mcg_functional, U)


def plaquette(U):
    return _scalar(A.load().mcg_plaquette, U)


def theta(W):
    return _scalar(A.load().mcg_theta, W)


def halfsweep(W, G, parity, omega=1.7):
    ctx = context(W.data.device.index)
    f, g = W.abi(), G.abi()
    _check(A.load().mcg_halfsweep(ctx, C.byref(f), C.byref(g), int(parity), float(omega), _stream()), ctx)


def sweeps(W, G, n, omega=1.7):
    """n raw sweeps (even then odd half-sweep) in place: no stop test, no R,
    no re-unitarisation.  For throughput measurements."""
    ctx = context(W.data.device.index)
    f, g = W.abi(), G.abi()
    _check(A.load().mcg_sweeps(ctx, C.byref(f), C.byref(g), int(n), float(omega), _stream()), ctx)


def sweeps_timed(W, G, n, omega=1.7):
    """sweeps() that returns the summed duration (ms) of the half-sweep
    launches alone, timed with HIP events on the launch stream (the ring folds
    and form conversions excluded).  Synchronises."""
    ctx = context(W.data.device.index)
    f, g = W.abi(), G.abi()
    ms = C.c_double()
    _check(A.load().mcg_sweeps_timed(ctx, C.byref(f), C.byref(g), int(n), float(omega), C.byref(ms), _stream()),
           ctx)
    return ms.value


def _opts(tol, max_sweeps, omega, reunit_every, start_sweep, check_every, traj):
    o = A.FixOpts()
    o.tol = float(tol)
    o.omega = float(omega)
    o.max_sweeps = int(max_sweeps)
    o.reunit_every = int(reunit_every)
    o.start_sweep = int(start_sweep)
    o.check_every = int(check_every)
    o.traj = traj.ctypes.data_as(C.POINTER(C.c_double)) if traj is not None else None
    return o


def _result(r, traj):
    out = dict(R=r.R, dR=r.dR, theta=r.theta, sweeps=r.sweeps, blocks50=r.blocks50, status=r.status)
    if traj is not None:
        out["traj"] = traj[: r.sweeps + 1].copy()
    return out


def fix(U, G=None, tol=1e-7, max_sweeps=5000, omega=1.7, reunit_every=50, start_sweep=0,
        check_every=50, want_traj=False):
    """MCG-fix U starting from G (identity if None); G is updated in place to the
    total transform.  Returns (G, info)."""
    import numpy as np
    G = G if G is not None else gauge_identity(U.L, U.data.device.index)
    traj = np.zeros(int(max_sweeps) + 1) if want_traj else None
    o = _opts(tol, max_sweeps, omega, reunit_every, start_sweep, check_every, traj)
    r = A.FixResult()
    ctx = context(U.data.device.index)
    fu, g = U.abi(), G.abi()
    _check(A.load().mcg_fix(ctx, C.byref(fu), C.byref(g), C.byref(o), C.byref(r), _stream()), ctx,
           allow_warn=True)
    return G, _result(r, traj)


def fix_batch(Us, Gs=None, tol=1e-7, max_sweeps=5000, omega=1.7, reunit_every=50, start_sweep=0,
              check_every=50, want_traj=False):
    """Fix several fields (copies and/or lattices of unequal sizes, one precision)
    in one batched, graph-captured sweep loop.  tol and max_sweeps may be lists."""
    import numpy as np
    B = len(Us)
    Gs = Gs if Gs is not None else [gauge_identity(U.L, U.data.device.index) for U in Us]
    tols = tol if isinstance(tol, (list, tuple)) else [tol] * B
    maxs = max_sweeps if isinstance(max_sweeps, (list, tuple)) else [max_sweeps] * B
    trajs = [np.zeros(int(m) + 1) if want_traj else None for m in maxs]
    F = (A.Field * B)(*[U.abi() for U in Us])
    GG = (A.Gauge * B)(*[G.abi() for G in Gs])
    O = (A.FixOpts * B)(*[_opts(tols[b], maxs[b], omega, reunit_every, start_sweep, check_every, trajs[b])
                          for b in range(B)])
    R = (A.FixResult * B)()
    ctx = context(Us[0].data.device.index)
    _check(A.load().mcg_fix_batch(ctx, B, F, GG, O, R, _stream()), ctx, allow_warn=True)
    return Gs, [_result(R[b], trajs[b]) for b in range(B)]


def precondition_batch(Us, rho=0.1, eps=1.0, n=10, Gs=None, tol=1e-7, max_sweeps=5000, omega=1.7,
                       reunit_every=50, check_every=50):
    """The whole preconditioned path (Sec. II.B) for a batch of fields in one library call: smear,
    fix the smeared fields, fix the originals from their transforms, project and count.  Gs: start
    transforms (identity if None), updated in place to the totals.  Returns (Gs, Zs, results), each
    result a dict with the two fixes' results, the minimum margin and the vortex counts."""
    B = len(Us)
    Gs = Gs if Gs is not None else [gauge_identity(U.L, U.data.device.index) for U in Us]
    Zs = [torch.empty((4, volume(U.L)), dtype=torch.int8, device=U.data.device) for U in Us]
    F = (A.Field * B)(*[U.abi() for U in Us])
    GG = (A.Gauge * B)(*[G.abi() for G in Gs])
    O = (A.FixOpts * B)(*[_opts(tol, max_sweeps, omega, reunit_every, 0, check_every, None) for _ in range(B)])
    Zp = (C.c_void_p * B)(*[Z.data_ptr() for Z in Zs])
    R = (A.PrecondResult * B)()
    ctx = context(Us[0].data.device.index)
    _check(A.load().mcg_precondition_batch(ctx, B, F, float(rho), float(eps), int(n), O, GG, Zp, R, _stream()),
           ctx, allow_warn=True)
    out = [dict(smeared=_result(r.smeared, None), fixed=_result(r.fixed, None), min_margin=r.min_margin,
                vortices=dict(total=r.vortices, per_plane=list(r.per_plane), per_charge=list(r.per_charge)))
           for r in R]
    return Gs, Zs, out


def center_project(U, G=None):
    """Centre integers Z (int8 tensor [4, V], lexicographic sites) of U^G and the
    minimum centre-phase margin (Sec. II.A)."""
    Z = torch.empty((4, volume(U.L)), dtype=torch.int8, device=U.data.device)
    ctx = context(U.data.device.index)
    f = U.abi()
    g = G.abi() if G is not None else None
    mm = C.c_double()
    _check(A.load().mcg_center_project(ctx, C.byref(f), C.byref(g) if g is not None else None,
                                       C.c_void_p(Z.data_ptr()), C.byref(mm), _stream()), ctx)
    return Z, mm.value


def center_project_noalloc(U, G=None, Z=None, want_margin=True):
    """center_project through the allocation-free entry point (lattices of up to 2^25 sites): Z
    (int8 [4, V], allocated here unless given) and the minimum margin, or None when want_margin is
    False (then the stream is not synchronised)."""
    if Z is None:
        Z = torch.empty((4, volume(U.L)), dtype=torch.int8, device=U.data.device)
    ctx = context(U.data.device.index)
    f = U.abi()
    g = G.abi() if G is not None else None
    mm = C.c_double()
    _check(A.load().mcg_center_project_noalloc(ctx, C.byref(f), C.byref(g) if g is not None else None,
                                               C.c_void_p(Z.data_ptr()), C.byref(mm) if want_margin else None,
                                               _stream()), ctx)
    return Z, (mm.value if want_margin else None)


def count_vortices(Z, L):
    ctx = context(Z.device.index)
    tot = C.c_int64()
    pp = (C.c_int64 * 6)()
    pc = (C.c_int64 * 2)()
    _check(A.load().mcg_count_vortices(ctx, C.c_void_p(Z.data_ptr()), _dims(L), C.byref(tot), pp, pc,
                                       _stream()), ctx)
    return dict(total=tot.value, per_plane=list(pp), per_charge=list(pc))


def vortex_field(U, G, Z, mode, out=None):
    """Vortex-only field (mode A.MCG_VORTEX_ONLY: z(m) 1 on every link) or
    vortex-removed field (A.MCG_VORTEX_REMOVED: conj(z(m)) U^G), with Z from
    center_project(U, G) (Sec. III.B).  out may be U itself."""
    out = out if out is not None else empty_links(U.L, U.prec, U.data.device.index)
    ctx = context(U.data.device.index)
    fu, fo = U.abi(), out.abi()
    g = G.abi() if G is not None else None
    if Z.dtype != torch.int8 or Z.numel() != 4 * volume(U.L) or not Z.is_contiguous():
        raise ValueError("Z must be a contiguous int8 tensor of 4 V entries")
    _check(A.load().mcg_vortex_field(ctx, C.byref(fu), C.byref(g) if g is not None else None,
                                     C.c_void_p(Z.data_ptr()), int(mode), C.byref(fo), _stream()), ctx)
    return out


def wilson_loops(U, vecs, rmax, tmax):
    """W[i, k-1, T-1] (numpy): Wilson loops of time extent T whose spatial side
    is k copies of the staircase path of vecs[i], averaged over all sites and
    the cubic images of the path."""
    import numpy as np
    v = np.ascontiguousarray(np.asarray(vecs, dtype=np.int32).reshape(-1, 3))
    W = np.zeros((len(v), int(rmax), int(tmax)))
    ctx = context(U.data.device.index)
    f = U.abi()
    _check(A.load().mcg_wilson_loops(ctx, C.byref(f), len(v), v.ctypes.data_as(C.POINTER(C.c_int32)), int(rmax),
                                     int(tmax), W.ctypes.data_as(C.POINTER(C.c_double)), _stream()), ctx)
    return W


def smear_mcg_backward(U, rho, eps, n, Gstar, ckpt_every=5):
    """Gradient of L = R(S_n(U; rho, eps)^{G*}) at fixed G*: returns
    (gradU Links (ambient), L, dL/drho, dL/deps)."""
    grad = empty_links(U.L, U.prec, U.data.device.index)
    ctx = context(U.data.device.index)
    fu, g, fg = U.abi(), Gstar.abi(), grad.abi()
    loss, dr, de = C.c_double(), C.c_double(), C.c_double()
    _check(A.load().mcg_smear_mcg_backward(ctx, C.byref(fu), float(rho), float(eps), int(n), C.byref(g),
                                           int(ckpt_every), C.byref(fg), C.byref(loss), C.byref(dr),
                                           C.byref(de), _stream()), ctx)
    return grad, loss.value, dr.value, de.value


def autotune(U):
    """Time every half-sweep variant on a copy of U; keep and return the fastest
    (median of three interleaved passes)."""
    ctx = context(U.data.device.index)
    f = U.abi()
    best = C.c_int32()
    ms = (C.c_double * A.MCG_NUM_VARIANTS)()
    _check(A.load().mcg_autotune(ctx, C.byref(f), C.byref(best), ms, _stream()), ctx)
    return best.value, list(ms)


def autotune_batch(Us):
    """Time every half-sweep variant on copies of the fields Us (one
    precision), each launch covering the whole batch as fix_batch runs it;
    keep and return the fastest (median of three interleaved passes)."""
    ctx = context(Us[0].data.device.index)
    B = len(Us)
    F = (A.Field * B)(*[U.abi() for U in Us])
    best = C.c_int32()
    ms = (C.c_double * A.MCG_NUM_VARIANTS)()
    _check(A.load().mcg_autotune_batch(ctx, B, F, C.byref(best), ms, _stream()), ctx)
    return best.value, list(ms)


def tune_batch(Us):
    """Tune the half-sweep variant and the sweep schedule (tile order, paired sweeps, slabs) on the
    batch Us, as fix_batch runs it; the choice is kept for batches of this shape.  Returns it as a
    dict (variant, order, paired, slabs, ms_per_sweep, ms_default)."""
    ctx = context(Us[0].data.device.index)
    B = len(Us)
    F = (A.Field * B)(*[U.abi() for U in Us])
    c = A.TuneChoice()
    _check(A.load().mcg_tune_batch(ctx, B, F, C.byref(c), _stream()), ctx)
    return {k: getattr(c, k) for k, _ in A.TuneChoice._fields_}


def clear_tuning(device=None):
    ctx = context(device)
    _check(A.load().mcg_clear_tuning(ctx), ctx)


def set_variant(prec, variant, device=None):
    ctx = context(device)
    _check(A.load().mcg_set_variant(ctx, _prec_of(prec), int(variant)), ctx)


def set_two_row(on=True, device=None):
    """Keep the fixing iteration's working field and transform as two rows."""
    ctx = context(device)
    _check(A.load().mcg_set_option(ctx, A.MCG_OPT_TWO_ROW, 1 if on else 0), ctx)


def set_slabs(n, device=None):
    """Run every half-sweep of the fixing loop in n slabs of time slices,
    pipelined so that a slab is re-read soon after it was written (results
    are bit-identical for every n)."""
    ctx = context(device)
    _check(A.load().mcg_set_option(ctx, A.MCG_OPT_SLABS, int(n)), ctx)


def set_sweep_order(alternate, device=None):
    """alternate=True (1): odd half-sweeps visit the lattice tiles in reverse
    order, starting where the even half-sweep ended; 2 (the default): the
    same, with each XCD taking a contiguous range of every field's tiles
    (bit-identical results)."""
    ctx = context(device)
    v = 2 if (not isinstance(alternate, bool) and alternate == 2) else (1 if alternate else 0)
    _check(A.load().mcg_set_option(ctx, A.MCG_OPT_ORDER, v), ctx)


def set_defer_g(on, device=None):
    """FP32 fixes and raw sweeps: keep each half-sweep's transform in a ring
    and fold it into G later (bit-identical, fewer bytes per site-update)."""
    ctx = context(device)
    _check(A.load().mcg_set_option(ctx, A.MCG_OPT_DEFER_G, 1 if on else 0), ctx)


def get_defer_g(device=None):
    ctx = context(device)
    v = C.c_int32()
    _check(A.load().mcg_get_option(ctx, A.MCG_OPT_DEFER_G, C.byref(v)), ctx)
    return bool(v.value)


def set_paired(on, device=None):
    """With the transform ring (FP32, two-row form): the first half-sweep of
    each sweep only records its transform, the second applies it to the links
    as it loads them (bit-identical, each link written once per sweep); 2:
    FP64 sweeps paired too (slower on MI355X)."""
    ctx = context(device)
    v = 2 if (not isinstance(on, bool) and on == 2) else (1 if on else 0)
    _check(A.load().mcg_set_option(ctx, A.MCG_OPT_PAIRED, v), ctx)


def get_paired(device=None):
    ctx = context(device)
    v = C.c_int32()
    _check(A.load().mcg_get_option(ctx, A.MCG_OPT_PAIRED, C.byref(v)), ctx)
    return v.value


def get_sweep_order(device=None):
    ctx = context(device)
    v = C.c_int32()
    _check(A.load().mcg_get_option(ctx, A.MCG_OPT_ORDER, C.byref(v)), ctx)
    return v.value


def unitarity(U=None, G=None):
    """(max |U U^dag - 1|, max |G G^dag - 1|) over all links / matrices (inf for NaN)."""
    if U is None and G is None:
        raise ValueError("need U or G")
    ref = U if U is not None else G
    ctx = context(ref.data.device.index)
    f = U.abi() if U is not None else None
    g = G.abi() if G is not None else None
    du, dg = C.c_double(), C.c_double()
    _check(A.load().mcg_unitarity(ctx, C.byref(f) if f is not None else None, C.byref(g) if g is not None else None,
                                  C.byref(du), C.byref(dg), _stream()), ctx)
    return du.value, dg.value


def set_check(on=True, device=None):
    """Validate input links and transforms in every call (MCG_EINPUT when not unitary or NaN)."""
    ctx = context(device)
    _check(A.load().mcg_set_option(ctx, A.MCG_OPT_CHECK, 1 if on else 0), ctx)


def set_scratch_limit_mib(mib, device=None):
    """Cap the device scratch the context may hold (0: no cap)."""
    ctx = context(device)
    _check(A.load().mcg_set_option(ctx, A.MCG_OPT_SCRATCH_LIMIT_MIB, int(mib)), ctx)


def set_update_variant(hits=1, stop_every=1, exact=False, device=None):
    """Update-rule variants of the fixing loop: `hits` re-linearisation hits
    per site visit, the stop test only after sweeps numbered by multiples of
    `stop_every`, and exact maximisation over each SU(2) subgroup (1, 1,
    False: the plain method)."""
    ctx = context(device)
    _check(A.load().mcg_set_option(ctx, A.MCG_OPT_HITS, int(hits)), ctx)
    _check(A.load().mcg_set_option(ctx, A.MCG_OPT_STOP_EVERY, int(stop_every)), ctx)
    _check(A.load().mcg_set_option(ctx, A.MCG_OPT_EXACT, 1 if exact else 0), ctx)


def get_update_variant(device=None):
    """(hits, stop_every, exact) as set by set_update_variant."""
    ctx = context(device)
    h, s, e = C.c_int32(), C.c_int32(), C.c_int32()
    _check(A.load().mcg_get_option(ctx, A.MCG_OPT_HITS, C.byref(h)), ctx)
    _check(A.load().mcg_get_option(ctx, A.MCG_OPT_STOP_EVERY, C.byref(s)), ctx)
    _check(A.load().mcg_get_option(ctx, A.MCG_OPT_EXACT, C.byref(e)), ctx)
    return h.value, s.value, bool(e.value)


def get_slabs(device=None):
    ctx = context(device)
    v = C.c_int32()
    _check(A.load().mcg_get_option(ctx, A.MCG_OPT_SLABS, C.byref(v)), ctx)
    return v.value


def get_two_row(device=None):
    ctx = context(device)
    v = C.c_int32()
    _check(A.load().mcg_get_option(ctx, A.MCG_OPT_TWO_ROW, C.byref(v)), ctx)
    return bool(v.value)


def get_variant(prec, device=None):
    ctx = context(device)
    v = C.c_int32()
    _check(A.load().mcg_get_variant(ctx, _prec_of(prec), C.byref(v)), ctx)
    return v.value


# ---- the paper's pipeline (Sec. II.B) ----------------------------------------------------
def precondition_and_fix(U, rho=0.1, eps=1.0, n=10, tol=1e-7, max_sweeps=5000, omega=1.7,
                         reunit_every=50, check_every=50):
    """Smear U, fix the smeared field, carry its transform back to U and fix
    again, then centre-project and count P-vortices."""
    S = smear(U, rho, eps, n)
    Gs, info_s = fix(S, None, tol, max_sweeps, omega, reunit_every, 0, check_every)
    R_smeared = info_s["R"]
    del S
    G, info = fix(U, Gs, tol, max_sweeps, omega, reunit_every, 0, check_every)
    Z, margin = center_project(U, G)
    vort = count_vortices(Z, U.L)
    nplaq = 6 * volume(U.L)
    return dict(G=G, Z=Z, R_smeared=R_smeared, R=info["R"], sweeps_smeared=info_s["sweeps"],
                sweeps=info["sweeps"], blocks50=(info_s["sweeps"] + info["sweeps"] + 49) // 50,
                min_margin=margin, vortices=vort, vortex_fraction=vort["total"] / nplaq,
                info_smeared=info_s, info=info)
