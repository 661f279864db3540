"""ctypes binding of the FP64 CPU oracle (oracle/mcg_oracle.c).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the benchmark's
CPU-baseline leg load this module; the library under paper_0807_0264_amd/
never does.

Array conventions (numpy, C order):
  links  U : complex128 [Lt, Lz, Ly, Lx, 4, 3, 3]
  gauge  G : complex128 [Lt, Lz, Ly, Lx, 3, 3]
  centre Z : int8       [Lt, Lz, Ly, Lx, 4]
so that the flat site index is x + Lx*(y + Ly*(z + Lz*t)).
"""
import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIBPATH = os.path.join(HERE, "libmcg_oracle.so")

_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIBPATH):
            from . import build as _b  # noqa: F401  (package-relative when imported as oracle.oracle)
            _b.build()
        _lib = C.CDLL(LIBPATH)
        _declare(_lib)
    return _lib


class FixResult(C.Structure):
    _fields_ = [("R", C.c_double), ("dR", C.c_double), ("theta", C.c_double),
                ("sweeps", C.c_int32), ("status", C.c_int32)]


_P = C.c_void_p
_I4 = C.POINTER(C.c_int32)


def _declare(l):
    sig = {
        "or_volume": (C.c_int64, [_I4]),
        "or_reunit": (None, [_P]),
        "or_exp_su3_eigen": (None, [_P, _P]),
        "or_exp_taylor": (None, [_P, C.c_int, _P]),
        "or_apply_gauge": (None, [_I4, _P, _P, _P]),
        "or_functional": (C.c_double, [_I4, _P]),
        "or_plaquette": (C.c_double, [_I4, _P]),
        "or_wilson_loop": (C.c_double, [_I4, _P, C.c_int, C.c_int]),
        "or_polyakov": (None, [_I4, _P, _P]),
        "or_staple_sum": (None, [_I4, _P, C.c_int64, C.c_int, C.c_double, C.c_double, _P]),
        "or_stout_staple_plain": (None, [_I4, _P, C.c_int64, C.c_int, C.c_double, _P]),
        "or_smear_link": (None, [_I4, _P, C.c_int64, C.c_int, C.c_double, C.c_double, _P]),
        "or_smear_step": (None, [_I4, _P, _P, C.c_double, C.c_double]),
        "or_smear": (None, [_I4, _P, _P, C.c_double, C.c_double, C.c_int]),
        "or_site_g": (None, [_P, C.c_double, _P]),
        "or_site_g_hits": (None, [_P, C.c_double, C.c_int, _P]),
        "or_halfsweep_hits": (None, [_I4, _P, _P, C.c_int, C.c_double, C.c_int]),
        "or_site_g_at": (None, [_I4, _P, C.c_int64, C.c_double, _P]),
        "or_halfsweep": (None, [_I4, _P, _P, C.c_int, C.c_double]),
        "or_theta": (C.c_double, [_I4, _P]),
        "or_mcg_fix": (C.c_int, [_I4, _P, _P, C.c_double, C.c_int32, C.c_double, C.c_int32,
                                 C.c_int32, _P, C.POINTER(FixResult)]),
        "or_mcg_fix_v": (C.c_int, [_I4, _P, _P, C.c_double, C.c_int32, C.c_double, C.c_int32,
                                   C.c_int32, C.c_int32, C.c_int32, C.c_int32, _P, C.POINTER(FixResult)]),
        "or_site_g_exact": (None, [_P, C.c_double, C.c_int, _P]),
        "or_sphere_max": (None, [_P, _P, _P]),
        "or_halfsweep_v": (None, [_I4, _P, _P, C.c_int, C.c_double, C.c_int, C.c_int]),
        "or_center_project": (None, [_I4, _P, _P, _P, _P]),
        "or_count_vortices": (None, [_I4, _P, _P, _P, _P, _P]),
        "or_vortex_field": (None, [_I4, _P, _P, _P, C.c_int, _P]),
        "or_wilson_path": (C.c_double, [_I4, _P, _P, C.c_int, C.c_int]),
        "or_smear_loss": (C.c_double, [_I4, _P, C.c_double, C.c_double, C.c_int, _P]),
        "or_smear_loss_grad": (None, [_I4, _P, C.c_double, C.c_double, C.c_int, _P, C.c_int,
                                      _P, _P, _P, _P, _P]),
        "or_step_jvp": (None, [_I4, _P, _P, C.c_double, C.c_double, _P]),
        "or_step_vjp": (None, [_I4, _P, _P, C.c_double, C.c_double, _P, _P, _P, _P]),
    }
    for name, (res, args) in sig.items():
        f = getattr(l, name)
        f.restype = res
        f.argtypes = args


def _dims(L):
    return (C.c_int32 * 4)(*[int(v) for v in L])


def _ptr(a):
    return a.ctypes.data_as(C.c_void_p) if a is not None else None


def _c128(a):
    return np.ascontiguousarray(a, dtype=np.complex128)


def dims_of(U):
    """(Lx, Ly, Lz, Lt) of a link array [Lt, Lz, Ly, Lx, 4, 3, 3]."""
    return (U.shape[3], U.shape[2], U.shape[1], U.shape[0])


# ---- small matrix helpers ---------------------------------------------------
def reunit(M):
    M = _c128(M).copy()
    lib().or_reunit(_ptr(M))
    return M


def exp_su3_eigen(A):
    A = _c128(A)
    E = np.empty((3, 3), np.complex128)
    lib().or_exp_su3_eigen(_ptr(A), _ptr(E))
    return E


def exp_taylor(A):
    A = _c128(A)
    n = A.shape[0]
    E = np.empty((n, n), np.complex128)
    lib().or_exp_taylor(_ptr(A), n, _ptr(E))
    return E


# ---- fields -------------------------------------------------------------------
def apply_gauge(U, G):
    U, G = _c128(U), _c128(G)
    out = np.empty_like(U)
    lib().or_apply_gauge(_dims(dims_of(U)), _ptr(U), _ptr(G), _ptr(out))
    return out


def functional(U):
    U = _c128(U)
    return lib().or_functional(_dims(dims_of(U)), _ptr(U))


def plaquette(U):
    U = _c128(U)
    return lib().or_plaquette(_dims(dims_of(U)), _ptr(U))


def wilson_loop(U, r, t):
    U = _c128(U)
    return lib().or_wilson_loop(_dims(dims_of(U)), _ptr(U), int(r), int(t))


def polyakov(U):
    U = _c128(U)
    L = dims_of(U)
    P = np.empty(L[0] * L[1] * L[2], np.complex128)
    lib().or_polyakov(_dims(L), _ptr(U), _ptr(P))
    return P


def site_index(L, x, y, z, t):
    return x + L[0] * (y + L[1] * (z + L[2] * t))


def staple_sum(U, site, mu, rho, eps):
    U = _c128(U)
    Cm = np.empty((3, 3), np.complex128)
    lib().or_staple_sum(_dims(dims_of(U)), _ptr(U), int(site), int(mu), rho, eps, _ptr(Cm))
    return Cm


def stout_staple_plain(U, site, mu, rho):
    U = _c128(U)
    Cm = np.empty((3, 3), np.complex128)
    lib().or_stout_staple_plain(_dims(dims_of(U)), _ptr(U), int(site), int(mu), rho, _ptr(Cm))
    return Cm


def smear_link(U, site, mu, rho, eps):
    U = _c128(U)
    out = np.empty((3, 3), np.complex128)
    lib().or_smear_link(_dims(dims_of(U)), _ptr(U), int(site), int(mu), rho, eps, _ptr(out))
    return out


def smear_step(U, rho, eps=1.0):
    U = _c128(U)
    out = np.empty_like(U)
    lib().or_smear_step(_dims(dims_of(U)), _ptr(U), _ptr(out), rho, eps)
    return out


def smear(U, rho, eps=1.0, n=1):
    U = _c128(U)
    out = np.empty_like(U)
    lib().or_smear(_dims(dims_of(U)), _ptr(U), _ptr(out), rho, eps, int(n))
    return out


# ---- MCG ----------------------------------------------------------------------
def site_g(M, omega):
    """M: complex [8, 3, 3] = (W_mu(x) for mu<4, W_mu(x-mu)^dag); returns g."""
    M = _c128(M)
    g = np.empty((3, 3), np.complex128)
    lib().or_site_g(_ptr(M), omega, _ptr(g))
    return g


def site_g_hits(M, omega, hits):
    """site_g with `hits` re-linearisation hits (hits = 1 is site_g)."""
    M = _c128(M)
    g = np.empty((3, 3), np.complex128)
    lib().or_site_g_hits(_ptr(M), omega, int(hits), _ptr(g))
    return g


def site_g_exact(M, omega, hits=1):
    """Site update with exact maximisation over each SU(2) subgroup."""
    M = _c128(M)
    g = np.empty((3, 3), np.complex128)
    lib().or_site_g_exact(_ptr(M), omega, int(hits), _ptr(g))
    return g


def sphere_max(Q, h):
    """argmax over the unit sphere in R^4 of a^T Q a + 2 h.a (Q symmetric)."""
    Q = np.ascontiguousarray(Q, dtype=np.float64)
    h = np.ascontiguousarray(h, dtype=np.float64)
    a = np.empty(4)
    lib().or_sphere_max(_ptr(Q), _ptr(h), _ptr(a))
    return a


def site_g_at(W, site, omega):
    W = _c128(W)
    g = np.empty((3, 3), np.complex128)
    lib().or_site_g_at(_dims(dims_of(W)), _ptr(W), int(site), omega, _ptr(g))
    return g


def halfsweep(W, G, parity, omega, hits=1, exact=False):
    """In place on copies; returns (W', G')."""
    W, G = _c128(W).copy(), _c128(G).copy()
    if hits == 1 and not exact:
        lib().or_halfsweep(_dims(dims_of(W)), _ptr(W), _ptr(G), int(parity), omega)
    else:
        lib().or_halfsweep_v(_dims(dims_of(W)), _ptr(W), _ptr(G), int(parity), omega, int(hits), int(exact))
    return W, G


def halfsweep_inplace(W, G, parity, omega):
    """One half-sweep applied in place to contiguous complex128 arrays."""
    assert W.dtype == np.complex128 and W.flags.c_contiguous and G.flags.c_contiguous
    lib().or_halfsweep(_dims(dims_of(W)), _ptr(W), _ptr(G), int(parity), omega)


def theta(W):
    W = _c128(W)
    return lib().or_theta(_dims(dims_of(W)), _ptr(W))


def identity_gauge(L):
    G = np.zeros((L[3], L[2], L[1], L[0], 3, 3), np.complex128)
    G[..., 0, 0] = G[..., 1, 1] = G[..., 2, 2] = 1
    return G


def mcg_fix(U, G0=None, tol=1e-7, max_sweeps=5000, omega=1.7, reunit_every=50,
            start_sweep=0, want_traj=False, hits=1, stop_every=1, exact=False):
    """Returns (G, result dict, trajectory or None).  hits: re-linearisation
    hits per site visit; stop_every: the stop test only after sweeps whose
    global number is a multiple of it."""
    U = _c128(U)
    L = dims_of(U)
    G = identity_gauge(L) if G0 is None else _c128(G0).copy()
    traj = np.zeros(max_sweeps + 1) if want_traj else None
    res = FixResult()
    if hits == 1 and stop_every == 1 and not exact:
        lib().or_mcg_fix(_dims(L), _ptr(U), _ptr(G), tol, int(max_sweeps), omega,
                         int(reunit_every), int(start_sweep), _ptr(traj), C.byref(res))
    else:
        lib().or_mcg_fix_v(_dims(L), _ptr(U), _ptr(G), tol, int(max_sweeps), omega, int(reunit_every),
                           int(start_sweep), int(hits), int(stop_every), int(exact), _ptr(traj), C.byref(res))
    info = dict(R=res.R, dR=res.dR, theta=res.theta, sweeps=res.sweeps, status=res.status)
    if traj is not None:
        traj = traj[: res.sweeps + 1].copy()
    return G, info, traj


def center_project(U, G=None):
    U = _c128(U)
    L = dims_of(U)
    Z = np.empty(U.shape[:5], np.int8)
    margin = np.empty(U.shape[:5], np.float64)
    Gc = _c128(G) if G is not None else None
    lib().or_center_project(_dims(L), _ptr(U), _ptr(Gc), _ptr(Z), _ptr(margin))
    return Z, margin


def count_vortices(Z, want_n=False):
    Z = np.ascontiguousarray(Z, dtype=np.int8)
    L = (Z.shape[3], Z.shape[2], Z.shape[1], Z.shape[0])
    tot = np.zeros(1, np.int64)
    pp = np.zeros(6, np.int64)
    pc = np.zeros(2, np.int64)
    n = np.empty(Z.shape[:4] + (6,), np.int8) if want_n else None
    lib().or_count_vortices(_dims(L), _ptr(Z), _ptr(tot), _ptr(pp), _ptr(pc), _ptr(n))
    out = dict(total=int(tot[0]), per_plane=pp.tolist(), per_charge=pc.tolist())
    if want_n:
        out["n"] = n
    return out


# ---- vortex-only / vortex-removed fields and Wilson loops (Sec. III.B) ----------
VORTEX_ONLY, VORTEX_REMOVED = 0, 1


def vortex_field(U, G, Z, mode):
    """mode VORTEX_ONLY: z(m) 1 per link; VORTEX_REMOVED: conj(z(m)) U^G."""
    U = _c128(U)
    out = np.empty_like(U)
    Gc = _c128(G) if G is not None else None
    Zc = np.ascontiguousarray(Z, dtype=np.int8)
    lib().or_vortex_field(_dims(dims_of(U)), _ptr(U), _ptr(Gc), _ptr(Zc), int(mode), _ptr(out))
    return out


def staircase(d):
    """Unit spatial steps (+-(axis+1)) from x to x + d: at each step the axis
    with steps left whose (taken + 1/2) / |d_axis| is smallest, ties to the
    lower axis, so the path stays close to the straight line."""
    taken = [0, 0, 0]
    steps = []
    for _ in range(sum(abs(v) for v in d)):
        best, key = None, None
        for a in range(3):
            if taken[a] < abs(d[a]):
                k = (taken[a] + 0.5) / abs(d[a])
                if key is None or k < key:
                    best, key = a, k
        taken[best] += 1
        steps.append((best + 1) if d[best] > 0 else -(best + 1))
    return steps


def path_images(steps):
    """The distinct images of a spatial step sequence under the 48 axis
    permutations and reflections of the cubic lattice (an image maps every
    step +-(a+1) to +-s_a (p_a + 1))."""
    import itertools
    out = set()
    for p in itertools.permutations(range(3)):
        for sg in itertools.product((1, -1), repeat=3):
            out.add(tuple((1 if st > 0 else -1) * sg[abs(st) - 1] * (p[abs(st) - 1] + 1) for st in steps))
    return sorted(out)


def wilson_path(U, spatial, t):
    U = _c128(U)
    st = np.ascontiguousarray(spatial, dtype=np.int32)
    return lib().or_wilson_path(_dims(dims_of(U)), _ptr(U), _ptr(st), len(st), int(t))


def wilson_loops(U, vecs, rmax, tmax):
    """W[i, k-1, T-1]: Wilson loops of time extent T whose spatial side is the
    staircase of v_i repeated k times, averaged over all sites and over the
    distinct cubic images of that spatial path."""
    U = _c128(U)
    W = np.zeros((len(vecs), rmax, tmax))
    for i, v in enumerate(vecs):
        imgs = path_images(staircase(v))
        for k in range(1, rmax + 1):
            for T in range(1, tmax + 1):
                W[i, k - 1, T - 1] = sum(wilson_path(U, list(p) * k, T) for p in imgs) / len(imgs)
    return W


# ---- loss and adjoint -----------------------------------------------------------
def smear_loss(U, rho, eps, n, Gstar):
    U, Gstar = _c128(U), _c128(Gstar)
    return lib().or_smear_loss(_dims(dims_of(U)), _ptr(U), rho, eps, int(n), _ptr(Gstar))


def smear_loss_grad(U, rho, eps, n, Gstar, ckpt_every=0, want_eps_scale=False):
    """(gradU, dL/drho, dL/deps, L); with want_eps_scale also the sum over steps
    and links of the magnitudes of the terms that add up to dL/deps."""
    U, Gstar = _c128(U), _c128(Gstar)
    g = np.empty_like(U)
    dr = np.zeros(1)
    de = np.zeros(1)
    loss = np.zeros(1)
    ae = np.zeros(1)
    lib().or_smear_loss_grad(_dims(dims_of(U)), _ptr(U), rho, eps, int(n), _ptr(Gstar),
                             int(ckpt_every), _ptr(g), _ptr(dr), _ptr(de), _ptr(loss), _ptr(ae))
    out = (g, float(dr[0]), float(de[0]), float(loss[0]))
    return out + (float(ae[0]),) if want_eps_scale else out


def step_jvp(U, dU, rho, eps):
    U, dU = _c128(U), _c128(dU)
    out = np.empty_like(U)
    lib().or_step_jvp(_dims(dims_of(U)), _ptr(U), _ptr(dU), rho, eps, _ptr(out))
    return out


def step_vjp(U, gOut, rho, eps):
    U, gOut = _c128(U), _c128(gOut)
    gU = np.empty_like(U)
    dr = np.zeros(1)
    de = np.zeros(1)
    lib().or_step_vjp(_dims(dims_of(U)), _ptr(U), _ptr(gOut), rho, eps, _ptr(gU),
                      _ptr(dr), _ptr(de), None)
    return gU, float(dr[0]), float(de[0])
