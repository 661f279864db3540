"""The library's C ABI driven with numpy buffers as device memory, for the
host-emulation build (libmcg_emu.so).  Mirrors paper_0807_0264_amd.api.
Test infrastructure only."""
import ctypes as C
import os

import numpy as np

from paper_0807_0264_amd import _abi as A

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "libmcg_emu.so")

_lib = None
_ctx = None


def lib():
    global _lib, _ctx
    if _lib is None:
        A._lib = None
        _lib = A.load(LIB)
        h = C.c_void_p()
        assert _lib.mcg_create(C.byref(h), 0) == 0
        _ctx = h
    return _lib


def ctx():
    lib()
    return _ctx


class MCGError(RuntimeError):
    pass


def check(st, allow_warn=False):
    if st == 0 or (allow_warn and st == 1):
        return st
    raise MCGError(f"{lib().mcg_last_error(ctx()).decode()} (status {st})")


def ptr(a):
    return C.c_void_p(a.ctypes.data) if a is not None else None


def dims(L):
    d = A.Dims()
    for k in range(4):
        d.L[k] = int(L[k])
    return d


def V(L):
    return int(L[0] * L[1] * L[2] * L[3])


class Links:
    def __init__(self, L, prec, data=None):
        self.L, self.prec = tuple(L), prec
        self.data = data if data is not None else np.zeros(V(L) * 72, np.float64 if prec == 0 else np.float32)

    def abi(self):
        f = A.Field()
        f.d = dims(self.L)
        f.prec = self.prec
        f.ptr = self.data.ctypes.data
        return f


class Gauge:
    def __init__(self, L, data=None):
        self.L = tuple(L)
        self.data = data if data is not None else np.zeros(V(L) * 18, np.float64)

    def abi(self):
        g = A.Gauge()
        g.d = dims(self.L)
        g.ptr = self.data.ctypes.data
        return g


def L_of(U):
    return (U.shape[3], U.shape[2], U.shape[1], U.shape[0])


def links(U, prec):
    U = np.ascontiguousarray(U, np.complex128)
    out = Links(L_of(U), prec)
    f = out.abi()
    check(lib().mcg_pack_links(ctx(), ptr(U), 0, C.byref(f), None))
    return out


def host_links(W):
    out = np.empty((W.L[3], W.L[2], W.L[1], W.L[0], 4, 3, 3), np.complex128)
    f = W.abi()
    check(lib().mcg_unpack_links(ctx(), C.byref(f), ptr(out), 0, None))
    return out


def gauge(G):
    G = np.ascontiguousarray(G, np.complex128)
    out = Gauge((G.shape[3], G.shape[2], G.shape[1], G.shape[0]))
    g = out.abi()
    check(lib().mcg_pack_gauge(ctx(), ptr(G), C.byref(g), None))
    return out


def host_gauge(Gd):
    out = np.empty((Gd.L[3], Gd.L[2], Gd.L[1], Gd.L[0], 3, 3), np.complex128)
    g = Gd.abi()
    check(lib().mcg_unpack_gauge(ctx(), C.byref(g), ptr(out), None))
    return out


def gauge_identity(L):
    G = Gauge(L)
    g = G.abi()
    check(lib().mcg_gauge_identity(ctx(), C.byref(g), None))
    return G


def apply_gauge(U, G):
    out = Links(U.L, U.prec)
    fu, g, fo = U.abi(), G.abi(), out.abi()
    check(lib().mcg_apply_gauge(ctx(), C.byref(fu), C.byref(g), C.byref(fo), None))
    return out


def _scalar(fn, U):
    f = U.abi()
    v = C.c_double()
    check(fn(ctx(), C.byref(f), C.byref(v), None))
    return v.value


def functional(U):
    return _scalar(lib().mcg_functional, U)


def plaquette(U):
    return _scalar(lib().mcg_plaquette, U)


def theta(U):
    return _scalar(lib().mcg_theta, U)


def smear(U, rho, eps, n):
    out = Links(U.L, U.prec)
    fu, fo = U.abi(), out.abi()
    check(lib().mcg_smear(ctx(), C.byref(fu), C.byref(fo), rho, eps, n, None))
    return out


def halfsweep(W, G, par, omega=1.7):
    f, g = W.abi(), G.abi()
    check(lib().mcg_halfsweep(ctx(), C.byref(f), C.byref(g), par, omega, None))


def _opts(tol, max_sweeps, omega, reunit_every, start_sweep, check_every, traj):
    o = A.FixOpts()
    o.tol, o.omega, o.max_sweeps = tol, omega, max_sweeps
    o.reunit_every, o.start_sweep, o.check_every = reunit_every, start_sweep, check_every
    o.traj = traj.ctypes.data_as(C.POINTER(C.c_double)) if traj is not None else None
    return o


def fix(U, G=None, tol=1e-7, max_sweeps=100, omega=1.7, reunit_every=50, start_sweep=0, check_every=10,
        want_traj=True):
    G = G if G is not None else gauge_identity(U.L)
    traj = np.zeros(max_sweeps + 1) if want_traj else None
    o = _opts(tol, max_sweeps, omega, reunit_every, start_sweep, check_every, traj)
    r = A.FixResult()
    fu, g = U.abi(), G.abi()
    check(lib().mcg_fix(ctx(), C.byref(fu), C.byref(g), C.byref(o), C.byref(r), None), allow_warn=True)
    info = dict(R=r.R, dR=r.dR, theta=r.theta, sweeps=r.sweeps, status=r.status)
    if traj is not None:
        info["traj"] = traj[: r.sweeps + 1].copy()
    return G, info


def fix_batch(Us, Gs, tols, maxs, omega=1.7, reunit_every=50, check_every=10):
    B = len(Us)
    trajs = [np.zeros(m + 1) for m in maxs]
    F = (A.Field * B)(*[U.abi() for U in Us])
    GG = (A.Gauge * B)(*[G.abi() for G in Gs])
    O = (A.FixOpts * B)(*[_opts(tols[b], maxs[b], omega, reunit_every, 0, check_every, trajs[b])
                          for b in range(B)])
    R = (A.FixResult * B)()
    check(lib().mcg_fix_batch(ctx(), B, F, GG, O, R, None), allow_warn=True)
    return [dict(R=R[b].R, theta=R[b].theta, sweeps=R[b].sweeps, status=R[b].status,
                 traj=trajs[b][: R[b].sweeps + 1].copy()) for b in range(B)]


def center_project(U, G=None):
    Z = np.zeros((4, V(U.L)), np.int8)
    f = U.abi()
    g = G.abi() if G is not None else None
    mm = C.c_double()
    check(lib().mcg_center_project(ctx(), C.byref(f), C.byref(g) if g is not None else None, ptr(Z),
                                   C.byref(mm), None))
    return Z, mm.value


def center_project_noalloc(U, G=None, want_margin=True):
    Z = np.zeros((4, V(U.L)), np.int8)
    f = U.abi()
    g = G.abi() if G is not None else None
    mm = C.c_double()
    check(lib().mcg_center_project_noalloc(ctx(), C.byref(f), C.byref(g) if g is not None else None, ptr(Z),
                                           C.byref(mm) if want_margin else None, None))
    return Z, (mm.value if want_margin else None)


def count_vortices(Z, L):
    tot = C.c_int64()
    pp = (C.c_int64 * 6)()
    pc = (C.c_int64 * 2)()
    check(lib().mcg_count_vortices(ctx(), ptr(np.ascontiguousarray(Z)), dims(L), C.byref(tot), pp, pc, None))
    return dict(total=tot.value, per_plane=list(pp), per_charge=list(pc))


def z_interchange(Z, L):
    z = Z.reshape(4, L[3], L[2], L[1], L[0])
    return np.ascontiguousarray(np.moveaxis(z, 0, -1))


def smear_mcg_backward(U, rho, eps, n, G, ckpt_every=2):
    grad = Links(U.L, U.prec)
    fu, g, fg = U.abi(), G.abi(), grad.abi()
    loss, dr, de = C.c_double(), C.c_double(), C.c_double()
    check(lib().mcg_smear_mcg_backward(ctx(), C.byref(fu), rho, eps, n, C.byref(g), ckpt_every, C.byref(fg),
                                       C.byref(loss), C.byref(dr), C.byref(de), None))
    return grad, loss.value, dr.value, de.value


def set_two_row(on):
    check(lib().mcg_set_option(ctx(), 1, 1 if on else 0))


def sweeps(W, G, n, omega=1.7):
    f, g = W.abi(), G.abi()
    check(lib().mcg_sweeps(ctx(), C.byref(f), C.byref(g), n, omega, None))


def vortex_field(U, G, Z, mode):
    out = Links(U.L, U.prec)
    f, fo = U.abi(), out.abi()
    g = G.abi() if G is not None else None
    check(lib().mcg_vortex_field(ctx(), C.byref(f), C.byref(g) if g is not None else None,
                                 ptr(np.ascontiguousarray(Z, dtype=np.int8)), mode, C.byref(fo), None))
    return out


def wilson_loops(U, vecs, rmax, tmax):
    v = np.ascontiguousarray(np.asarray(vecs, dtype=np.int32).reshape(-1, 3))
    W = np.zeros((len(v), rmax, tmax))
    f = U.abi()
    check(lib().mcg_wilson_loops(ctx(), C.byref(f), len(v), v.ctypes.data_as(C.POINTER(C.c_int32)), rmax, tmax,
                                 W.ctypes.data_as(C.POINTER(C.c_double)), None))
    return W


def set_slabs(n):
    check(lib().mcg_set_option(ctx(), 2, n))


def set_variant(prec, v):
    check(lib().mcg_set_variant(ctx(), prec, v))


def get_variant(prec):
    v = C.c_int32()
    check(lib().mcg_get_variant(ctx(), prec, C.byref(v)))
    return v.value


def autotune_batch(Us):
    B = len(Us)
    F = (A.Field * B)(*[U.abi() for U in Us])
    best = C.c_int32()
    ms = (C.c_double * 6)()
    check(lib().mcg_autotune_batch(ctx(), B, F, C.byref(best), ms, None))
    return best.value, list(ms)


def precondition_batch(Us, Gs, rho, eps, n, tol, max_sweeps, reunit_every=50, check_every=10):
    B = len(Us)
    Zs = [np.zeros((4, V(U.L)), np.int8) for U in Us]
    F = (A.Field * B)(*[U.abi() for U in Us])
    GG = (A.Gauge * B)(*[G.abi() for G in Gs])
    O = (A.FixOpts * B)(*[_opts(tol, max_sweeps, 1.7, reunit_every, 0, check_every, None) for _ in range(B)])
    Zp = (C.c_void_p * B)(*[Z.ctypes.data for Z in Zs])
    R = (A.PrecondResult * B)()
    check(lib().mcg_precondition_batch(ctx(), B, F, rho, eps, n, O, GG, Zp, R, None), allow_warn=True)
    return Zs, [dict(Rs=r.smeared.R, ss=r.smeared.sweeps, R=r.fixed.R, s=r.fixed.sweeps, m=r.min_margin,
                     v=r.vortices) for r in R]


def tune_batch(Us):
    B = len(Us)
    F = (A.Field * B)(*[U.abi() for U in Us])
    c = A.TuneChoice()
    check(lib().mcg_tune_batch(ctx(), B, F, C.byref(c), None))
    return {k: getattr(c, k) for k, _ in A.TuneChoice._fields_}


def clear_tuning():
    check(lib().mcg_clear_tuning(ctx()))


def set_update_variant(hits, stop_every, exact=False):
    check(lib().mcg_set_option(ctx(), 3, hits))
    check(lib().mcg_set_option(ctx(), 4, stop_every))
    check(lib().mcg_set_option(ctx(), 7, 1 if exact else 0))


def set_sweep_order(alternate):
    check(lib().mcg_set_option(ctx(), 8, int(alternate)))


def set_defer_g(on):
    check(lib().mcg_set_option(ctx(), 9, 1 if on else 0))


def set_paired(on):
    check(lib().mcg_set_option(ctx(), 10, int(on)))


def set_check(on):
    check(lib().mcg_set_option(ctx(), 5, 1 if on else 0))


def set_scratch_limit_mib(mib):
    check(lib().mcg_set_option(ctx(), 6, mib))


def status_of(fn, *a):
    """Run a library call that returns a status; give back (status, last error)."""
    st = fn(*a)
    return st, lib().mcg_last_error(ctx())


def unitarity(U=None, G=None):
    f = U.abi() if U is not None else None
    g = G.abi() if G is not None else None
    du, dg = C.c_double(), C.c_double()
    check(lib().mcg_unitarity(ctx(), C.byref(f) if f is not None else None, C.byref(g) if g is not None else None,
                              C.byref(du), C.byref(dg), None))
    return du.value, dg.value
