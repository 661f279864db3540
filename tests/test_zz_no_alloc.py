"""The allocation-free centre projection (mcg_center_project_noalloc), for
callers that cannot allocate device memory, against mcg_center_project:
the same Z bit for bit and the same minimum margin, on two calls in a row,
the second on a smaller lattice (the static scratch keeps the first call's
contents), in FP64 and FP32, with and without a transform; without a margin
output the call does not synchronise; lattices beyond its limit are
rejected on the host."""
import ctypes as C

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import gpu_util
    from paper_0807_0264_amd import api
    return api, gpu_util, torch


@pytest.mark.parametrize("prec", [0, 1])
def test_noalloc_projection_matches_allocating_one(S, env, prec):
    api, g, torch = env
    for k, L in enumerate([(16, 16, 16, 32), (6, 4, 4, 8)]):  # the second call smaller
        U = g.links(S.heatbath_field_gpu(L, S.sub_seed(6000 + k), 5.7, 5).cpu().numpy(), prec)
        G = g.gauge(S.haar_gauge(L, S.sub_seed(6100 + k)))
        for gg in (G, None):
            Za, ma = api.center_project(U, gg)
            Zb, mb = api.center_project_noalloc(U, gg)
            torch.cuda.synchronize()
            print(f"prec {prec} {L} G {'yes' if gg is not None else 'no'}: min margin {ma:.6e} / {mb:.6e}",
                  flush=True)
            assert torch.equal(Za, Zb)
            assert ma == mb
            # without the margin: no copy back, no synchronisation; Z written all the same
            Zc = torch.full_like(Za, 7)
            _, none = api.center_project_noalloc(U, gg, Z=Zc, want_margin=False)
            torch.cuda.synchronize()
            assert none is None and torch.equal(Za, Zc)


def test_noalloc_projection_rejects_lattices_beyond_its_limit(env):
    api, g, torch = env
    from paper_0807_0264_amd import _abi as A
    ctx = api.context(0)
    buf = torch.zeros(64, dtype=torch.float32, device="cuda")
    Z = torch.zeros(64, dtype=torch.int8, device="cuda")
    f = A.Field()
    for k, n in enumerate((64, 64, 64, 130)):  # 34,078,720 sites > 2^25: rejected before any launch
        f.d.L[k] = n
    f.prec = 1
    f.ptr = buf.data_ptr()
    mm = C.c_double()
    st = A.load().mcg_center_project_noalloc(ctx, C.byref(f), None, C.c_void_p(Z.data_ptr()), C.byref(mm), None)
    assert st == -1 and b"2^25" in A.load().mcg_last_error(ctx)
    torch.cuda.synchronize()
    assert not Z.any()
