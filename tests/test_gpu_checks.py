"""Input validation on the GPU: the unitarity deviation against numpy, the
check mode's MCG_EINPUT on non-unitary or NaN links and transforms, and the
context's scratch limit (MCG_ENOMEM, context still usable)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def g():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import gpu_util
    return gpu_util


def deviation(M):
    M = M.reshape(-1, 3, 3)
    return np.abs(M @ np.conj(np.swapaxes(M, -1, -2)) - np.eye(3)).max()


@pytest.mark.parametrize("prec", [0, 1])
def test_unitarity_and_check_mode(S, g, prec):
    from paper_0807_0264_amd import api
    from paper_0807_0264_amd.api import MCGError
    L = (6, 4, 4, 8)
    U = g.rounded(S.heatbath_field(L, S.sub_seed(7000), 5.7, 3), prec)
    G = S.haar_gauge(L, S.sub_seed(7001))
    du, dg = api.unitarity(g.links(U, prec), g.gauge(G))
    assert du < (1e-6 if prec == 1 else 1e-13) and dg < 1e-13
    bad = U.copy()
    bad[3, 1, 2, 5, 1] *= 1.0005
    bad = g.rounded(bad, prec)
    # the deviation of the complex entries as numpy computes it (max over real and imaginary parts)
    M = bad.reshape(-1, 3, 3)
    P = M @ np.conj(np.swapaxes(M, -1, -2)) - np.eye(3)
    want = max(np.abs(P.real).max(), np.abs(P.imag).max())
    assert abs(api.unitarity(g.links(bad, prec))[0] - want) < 1e-6 * want + (1e-7 if prec else 1e-14)
    nan = U.copy()
    nan[0, 0, 1, 0, 2, 0, 0] = np.nan
    assert api.unitarity(g.links(nan, prec))[0] == np.inf
    Gbad = G.copy()
    Gbad[1, 0, 0, 0] *= 1 + 1e-8
    assert api.unitarity(None, g.gauge(Gbad))[1] > 1e-9
    api.set_check(True)
    try:
        for Ub in (bad, nan):
            with pytest.raises(MCGError, match="not unitary"):
                api.smear(g.links(Ub, prec), 0.1, 1.0, 1)
            with pytest.raises(MCGError, match="not unitary"):
                api.fix(g.links(Ub, prec), None, tol=-1.0, max_sweeps=2)
            with pytest.raises(MCGError, match="not unitary"):
                api.center_project(g.links(Ub, prec), None)
        with pytest.raises(MCGError, match="G is not unitary"):
            api.fix(g.links(U, prec), g.gauge(Gbad), tol=-1.0, max_sweeps=2)
        with pytest.raises(MCGError, match="G is not unitary"):
            api.apply_gauge(g.links(U, prec), g.gauge(Gbad))
        with pytest.raises(MCGError, match="not unitary"):
            api.wilson_loops(g.links(bad, prec), [(1, 0, 0)], 1, 1)
        a = g.host_links(api.smear(g.links(U, prec), 0.1, 1.0, 2))
        _, info = api.fix(g.links(U, prec), g.gauge(G), tol=-1.0, max_sweeps=3, want_traj=True)
    finally:
        api.set_check(False)
    assert np.array_equal(a, g.host_links(api.smear(g.links(U, prec), 0.1, 1.0, 2)))
    _, info2 = api.fix(g.links(U, prec), g.gauge(G), tol=-1.0, max_sweeps=3, want_traj=True)
    assert np.array_equal(info["traj"], info2["traj"])


def test_scratch_limit(S, g):
    """A fresh context (the shared one may already hold large buffers) with a
    4 MiB scratch cap: a fix needing a ~38 MB working field returns
    MCG_ENOMEM and the same context then works once the cap is lifted."""
    import ctypes as C

    import torch
    from paper_0807_0264_amd import _abi as A
    from paper_0807_0264_amd import api
    lib = A.load()
    L = (16, 16, 16, 32)
    U = api.to_links(S.haar_links_gpu(L, 11), 1)
    G = api.gauge_identity(L)
    ctx = C.c_void_p()
    assert lib.mcg_create(C.byref(ctx), torch.cuda.current_device()) == A.MCG_OK
    try:
        assert lib.mcg_set_option(ctx, A.MCG_OPT_SCRATCH_LIMIT_MIB, 4) == A.MCG_OK
        o = api._opts(-1.0, 1, 1.7, 50, 0, 50, None)
        r = A.FixResult()
        f, gg = U.abi(), G.abi()
        st = lib.mcg_fix(ctx, C.byref(f), C.byref(gg), C.byref(o), C.byref(r), api._stream())
        assert st == A.MCG_ENOMEM and b"scratch limit" in lib.mcg_last_error(ctx)
        assert lib.mcg_set_option(ctx, A.MCG_OPT_SCRATCH_LIMIT_MIB, 0) == A.MCG_OK
        st = lib.mcg_fix(ctx, C.byref(f), C.byref(gg), C.byref(o), C.byref(r), api._stream())
        assert st == A.MCG_WNOTCONV and r.sweeps == 1
    finally:
        assert lib.mcg_destroy(ctx) == A.MCG_OK


def test_ring_falls_back_under_the_scratch_limit(S, g):
    """A scratch limit that admits an FP32 fix but not its transform ring: the
    fix runs with G updated in place, gives the bits of a fix with the ring
    switched off, and leaves no error behind."""
    import ctypes as C

    import torch
    from paper_0807_0264_amd import _abi as A
    from paper_0807_0264_amd import api
    lib = A.load()
    L = (16, 16, 16, 32)
    U = api.to_links(S.haar_links_gpu(L, 13), 1)

    def run(ctx):
        G = api.gauge_identity(L)
        traj = np.zeros(41)
        o = api._opts(-1.0, 40, 1.7, 50, 0, 50, traj)
        r = A.FixResult()
        f, gg = U.abi(), G.abi()
        st = lib.mcg_fix(ctx, C.byref(f), C.byref(gg), C.byref(o), C.byref(r), api._stream())
        torch.cuda.synchronize()
        return st, g.host_gauge(G), traj

    ctxs = [C.c_void_p(), C.c_void_p()]
    for c in ctxs:
        assert lib.mcg_create(C.byref(c), torch.cuda.current_device()) == A.MCG_OK
    try:
        # W (25 MB) and G (13 MB) in the two-row form fit in 64 MiB, the ring of 25 sweeps (157 MB) does not
        assert lib.mcg_set_option(ctxs[0], A.MCG_OPT_SCRATCH_LIMIT_MIB, 64) == A.MCG_OK
        st, Ga, ta = run(ctxs[0])
        assert st == A.MCG_WNOTCONV and lib.mcg_last_error(ctxs[0]) == b""
        assert lib.mcg_set_option(ctxs[1], A.MCG_OPT_DEFER_G, 0) == A.MCG_OK
        st, Gb, tb = run(ctxs[1])
        assert st == A.MCG_WNOTCONV
        assert np.array_equal(Ga, Gb) and np.array_equal(ta, tb)
    finally:
        for c in ctxs:
            assert lib.mcg_destroy(c) == A.MCG_OK


def test_backward_falls_back_under_the_scratch_limit(S, g):
    """A scratch limit that admits the backward's checkpoints and segment fields but not the staple
    sums it keeps for the adjoint: the adjoint forms the staples itself, and the gradient and the
    scalars equal those of a context without a limit (the same staple arithmetic in either kernel),
    with no error left behind."""
    import ctypes as C

    import torch
    from paper_0807_0264_amd import _abi as A
    from paper_0807_0264_amd import api
    lib = A.load()
    L = (8, 8, 8, 8)
    U = api.to_links(S.heatbath_field_gpu(L, S.sub_seed(77, 0), 5.7, 20), 1)
    Gs = api.gauge_identity(L)

    def run(ctx):
        grad = api.empty_links(L, 1, torch.cuda.current_device())
        fu, gg, fg = U.abi(), Gs.abi(), grad.abi()
        loss, dr, de = C.c_double(), C.c_double(), C.c_double()
        st = lib.mcg_smear_mcg_backward(ctx, C.byref(fu), 0.06, -0.25, 6, C.byref(gg), 3, C.byref(fg),
                                        C.byref(loss), C.byref(dr), C.byref(de), api._stream())
        torch.cuda.synchronize()
        return st, g.host_links(grad), (loss.value, dr.value, de.value)

    ctxs = [C.c_void_p(), C.c_void_p()]
    for c in ctxs:
        assert lib.mcg_create(C.byref(c), torch.cuda.current_device()) == A.MCG_OK
    try:
        # a field is 1.18 MB: 9 of them (2 checkpoints, 2 segment fields, 5 temporaries) fit in 16 MiB,
        # the 17 with the staple sums do not
        assert lib.mcg_set_option(ctxs[0], A.MCG_OPT_SCRATCH_LIMIT_MIB, 16) == A.MCG_OK
        st, ga, sa = run(ctxs[0])
        assert st == A.MCG_OK and lib.mcg_last_error(ctxs[0]) == b""
        st, gb, sb = run(ctxs[1])
        assert st == A.MCG_OK
        rel = np.abs(ga - gb).max() / np.abs(gb).max()
        print(f"fallback vs stored staple sums: max rel {rel:.2e}, bitwise {np.array_equal(ga, gb)}")
        assert rel <= 1e-6
        for x, y in zip(sa, sb):
            assert abs(x - y) <= 1e-6 * abs(y)
    finally:
        for c in ctxs:
            assert lib.mcg_destroy(c) == A.MCG_OK


def test_destroy_returns_device_memory(S, g):
    """A context that ran an FP32 fix (working field, transform, transform
    ring, partial sums) and the batched tuner gives all of its device memory
    back when destroyed."""
    import ctypes as C

    import torch
    from paper_0807_0264_amd import _abi as A
    from paper_0807_0264_amd import api
    lib = A.load()
    L = (16, 16, 16, 32)
    U = api.to_links(S.haar_links_gpu(L, 12), 1)
    G = api.gauge_identity(L)
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    ctx = C.c_void_p()
    assert lib.mcg_create(C.byref(ctx), torch.cuda.current_device()) == A.MCG_OK
    try:
        f, gg = U.abi(), G.abi()
        best, ms = C.c_int32(), (C.c_double * A.MCG_NUM_VARIANTS)()
        assert lib.mcg_autotune_batch(ctx, 1, C.byref(f), C.byref(best), ms, api._stream()) == A.MCG_OK
        o = api._opts(-1.0, 30, 1.7, 50, 0, 50, None)
        r = A.FixResult()
        assert lib.mcg_fix(ctx, C.byref(f), C.byref(gg), C.byref(o), C.byref(r), api._stream()) == A.MCG_WNOTCONV
        torch.cuda.synchronize()
        held = free0 - torch.cuda.mem_get_info()[0]
        # at 16^3x32: W two-row 25 MB, G two-row 13 MB, ring of 25 sweeps 157 MB, identity 19 MB
        assert held > 150 << 20, held
    finally:
        assert lib.mcg_destroy(ctx) == A.MCG_OK
    torch.cuda.synchronize()
    assert free0 - torch.cuda.mem_get_info()[0] < 8 << 20
