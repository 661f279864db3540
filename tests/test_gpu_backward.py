"""The hand-written adjoint of the smeared-field MCG functional on the GPU:
against the FP64 oracle adjoint, against central finite differences at the
16^4, 20-step over-improved configuration, checkpointing, and through
torch.autograd."""
import numpy as np
import pytest

from helpers import inner

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import gpu_util
    from paper_0807_0264_amd import api
    return api, gpu_util, torch


def _fd(f, h):
    """fourth-order central difference at 0"""
    return (-f(2 * h) + 8 * f(h) - 8 * f(-h) + f(-2 * h)) / (12 * h)


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("L", [(4, 4, 4, 4), (6, 4, 4, 8), (12, 12, 10, 6)])
@pytest.mark.parametrize("rho,eps,n,ck", [(0.1, 1.0, 3, 2), (0.06, -0.25, 3, 1)])
def test_backward_vs_oracle(S, O, env, L, prec, rho, eps, n, ck):
    api, g, torch = env
    U = g.rounded(S.heatbath_field(L, S.sub_seed(3000), 5.7, 5), prec)
    G = S.haar_gauge(L, S.sub_seed(3001))
    grad, loss, dr, de = api.smear_mcg_backward(g.links(U, prec), rho, eps, n, g.gauge(G), ck)
    go, dro, deo, losso, scale = O.smear_loss_grad(U, rho, eps, n, G, ckpt_every=ck, want_eps_scale=True)
    tol = 1e-11 if prec == 0 else 1e-5
    assert np.abs(g.host_links(grad) - go).max() < tol * np.abs(go).max()
    assert abs(loss - losso) < tol * losso
    assert abs(dr - dro) < tol * abs(dro)
    # dL/deps is a sum over steps and links of terms that cancel to 1/60 - 1/2400 of their summed
    # magnitude `scale` here.  FP64: relative to dL/deps itself.  FP32: every term to the FP32 bar,
    # i.e. the error within tol times the summed magnitude of the terms (rounding of a term is
    # relative to that term, and a sum cannot undo it).
    print(f"dL/deps {deo:.3e}, terms {scale:.3e}, |error| {abs(de - deo):.2e} "
          f"({abs(de - deo) / abs(deo):.2e} of dL/deps, {abs(de - deo) / scale:.2e} of the terms)")
    assert abs(de - deo) < (tol * abs(deo) if prec == 0 else tol * scale)


def test_backward_oi20_vs_oracle_6x4(S, O, env):
    """20 over-improved steps, checkpoint every 5, FP64: the oracle adjoint."""
    api, g, torch = env
    L = (6, 6, 6, 6)
    U = S.heatbath_field(L, S.sub_seed(3002), 5.7, 10)
    Sm = O.smear(U, 0.06, -0.25, 20)
    G, _, _ = O.mcg_fix(Sm, tol=1e-10, max_sweeps=3000)
    grad, loss, dr, de = api.smear_mcg_backward(g.links(U, 0), 0.06, -0.25, 20, g.gauge(G), 5)
    go, dro, deo, losso = O.smear_loss_grad(U, 0.06, -0.25, 20, G, ckpt_every=5)
    assert np.abs(g.host_links(grad) - go).max() < 1e-11 * np.abs(go).max()
    print(f"dL/drho {dro:.3e} dL/deps {deo:.3e}: relative errors {abs(dr - dro) / abs(dro):.2e}, "
          f"{abs(de - deo) / abs(deo):.2e}")
    assert abs(dr - dro) < 1e-11 * abs(dro) and abs(de - deo) < 1e-11 * abs(deo)


@pytest.fixture(scope="module")
def c4(S, env):
    """16^4 heatbath field, 20 over-improved steps (rho = 0.06, eps = -0.25),
    G* maximising R of the smeared field (FP64 fix to dR < 1e-9)."""
    api, g, torch = env
    L = (16, 16, 16, 16)
    U64 = S.heatbath_field_gpu(L, S.sub_seed(1, 0), 5.7, 50)
    U = api.to_links(U64, 0)
    Gs, info = api.fix(api.smear(U, 0.06, -0.25, 20), None, tol=1e-9, max_sweeps=6000)
    return L, U64, U, Gs


def _loss(api, U, rho, eps, n, G):
    return api.functional(api.apply_gauge(api.smear(U, rho, eps, n), G))


def test_c4_finite_differences_fp64(S, env, c4):
    api, g, torch = env
    L, U64, U, G = c4
    rho, eps, n, h = 0.06, -0.25, 20, 1e-4
    grad, loss, dr, de = api.smear_mcg_backward(U, rho, eps, n, G, 5)
    assert abs(loss - _loss(api, U, rho, eps, n, G)) < 1e-14
    fd_rho = _fd(lambda s: _loss(api, U, rho + s, eps, n, G), h)
    fd_eps = _fd(lambda s: _loss(api, U, rho, eps + s, n, G), h)
    print(f"C4: dL/drho {dr:.6e} (FD {fd_rho:.6e}), dL/deps {de:.6e} (FD {fd_eps:.6e}): relative "
          f"{abs(fd_rho - dr) / abs(dr):.2e}, {abs(fd_eps - de) / abs(de):.2e}")
    assert abs(fd_rho - dr) <= 1e-6 * abs(dr)
    assert abs(fd_eps - de) <= 1e-6 * abs(de)
    # random su(3) tangent: U_l -> exp(h X_l) U_l
    X = S.su3_tangent(L, S.sub_seed(3003))
    Uh = U64.cpu().numpy()
    w, V = np.linalg.eigh(-1j * X.reshape(-1, 3, 3))  # X = i H, H = V diag(w) V^dag

    def moved(s):
        E = (V * np.exp(1j * s * w)[:, None, :]) @ np.conj(np.swapaxes(V, -1, -2))
        return api.to_links(torch.from_numpy((E.reshape(Uh.shape) @ Uh)).cuda(), 0)

    # the derivative along a unit tangent spread over all 4V links is O(1/4V);
    # at h = 1e-4 the stencil's rounding floor (about 1.5 eps L / h) would be a
    # few 1e-6 of it, so the step is 1e-2 (each link then moves by ~1e-5, where
    # the h^4 truncation term is negligible)
    fd = _fd(lambda s: _loss(api, moved(s), rho, eps, n, G), 1e-2)
    an = inner(g.host_links(grad), X @ Uh)
    assert abs(fd - an) <= 1e-6 * abs(an)


def test_c4_checkpointing_is_bitwise_and_fp32_error(S, env, c4):
    api, g, torch = env
    L, U64, U, G = c4
    a = api.smear_mcg_backward(U, 0.06, -0.25, 20, G, 1)
    # every interval gives the bits of checkpointing each step: one that divides n, one whose last
    # segment is shorter (7, 7, 6), and one segment (20; 0 means n)
    for ck in (5, 7, 20, 0):
        b = api.smear_mcg_backward(U, 0.06, -0.25, 20, G, ck)
        assert torch.equal(a[0].data, b[0].data) and a[1:] == b[1:], ck
    # FP32 forward and adjoint against the FP64 adjoint (stated, loosely bounded)
    c = api.smear_mcg_backward(api.to_links(U64, 1), 0.06, -0.25, 20, G, 5)
    ga, gc = g.host_links(a[0]), g.host_links(c[0])
    rel = np.abs(gc - ga).max() / np.abs(ga).max()
    print(f"FP32 adjoint vs FP64: max rel {rel:.2e}, dRho {abs(c[2] - a[2]) / abs(a[2]):.2e}, "
          f"dEps {abs(c[3] - a[3]) / max(abs(a[3]), 1e-12):.2e}")
    assert rel < 1e-3
    assert abs(c[2] - a[2]) < 1e-3 * abs(a[2])


def test_autograd_function(S, env):
    api, g, torch = env
    from paper_0807_0264_amd.autograd import stout_mcg_loss
    L = (4, 4, 4, 4)
    U0 = S.heatbath_field(L, S.sub_seed(3004), 5.7, 5)
    G = g.gauge(S.haar_gauge(L, S.sub_seed(3005)))
    U = torch.from_numpy(U0).cuda().requires_grad_(True)
    rho = torch.tensor(0.06, dtype=torch.float64, requires_grad=True)
    eps = torch.tensor(-0.25, dtype=torch.float64, requires_grad=True)
    Lv = stout_mcg_loss(U, rho, eps, 3, G, 2)
    Lv.backward()
    grad, loss, dr, de = api.smear_mcg_backward(g.links(U0, 0), 0.06, -0.25, 3, G, 2)
    assert abs(float(Lv.detach()) - loss) < 1e-15
    assert torch.allclose(U.grad, api.from_links(grad, torch.complex128), rtol=0, atol=1e-15)
    assert abs(float(rho.grad) - dr) < 1e-15 and abs(float(eps.grad) - de) < 1e-15
