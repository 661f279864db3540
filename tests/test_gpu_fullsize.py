"""Parity at the benchmark's full size (32^3x64, FP32 links, FP64 transform)
in the launch configuration bench.py times (the autotuned half-sweep
variant): sampled outputs that the oracle computes one by one, a full
comparison of the centre projection and vortex count, and size-independent
properties of the fixing iteration."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

L = (32, 32, 32, 64)
NSAMPLE = 3000


@pytest.fixture(scope="module")
def big(S):
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_0807_0264_amd import api
    U64 = S.heatbath_field_gpu(L, S.sub_seed(5, 0), 5.7, 50)  # the benchmark's first field
    U = api.to_links(U64, 1)
    # the variant tuned on a batch of the benchmark's four shapes (Haar fields beside this one)
    others = [api.to_links(S.haar_links_gpu(Lb, S.sub_seed(5, 10 + i)), 1)
              for i, Lb in enumerate([(24, 24, 24, 48), (20, 20, 20, 40), (16, 16, 16, 16)])]
    best, _ = api.autotune_batch([U] + others)
    del others
    host = U64.to(torch.complex64).cpu().numpy().astype(np.complex128)
    del U64
    return api, U, host, best


def _site(Lt, i):
    x = i % Lt[0]
    r = i // Lt[0]
    y = r % Lt[1]
    r //= Lt[1]
    z = r % Lt[2]
    t = r // Lt[2]
    return x, y, z, t


def _sites_of_parity(rng, par, n):
    V = int(np.prod(L))
    out = []
    while len(out) < n:
        i = int(rng.integers(V))
        if sum(_site(L, i)) % 2 == par:
            out.append(i)
    return out


def test_halfsweep_sampled(O, big):
    import torch
    api, U, host, _ = big
    W = U.clone()
    G = api.gauge_identity(L)
    api.halfsweep(W, G, 0, 1.7)
    Wa = api.from_links(W, torch.complex128).cpu().numpy()
    Ga = api.from_gauge(G).cpu().numpy()
    rng = np.random.default_rng(1)
    for i in _sites_of_parity(rng, 0, NSAMPLE):
        x, y, z, t = _site(L, i)
        g = O.site_g_at(host, i, 1.7)
        assert np.abs(Ga[t, z, y, x] - g).max() < 1e-5
        for mu in range(4):
            assert np.abs(Wa[t, z, y, x, mu] - g @ host[t, z, y, x, mu]).max() < 1e-5
            c = [x, y, z, t]
            c[mu] = (c[mu] - 1) % L[mu]
            xb, yb, zb, tb = c
            want = host[tb, zb, yb, xb, mu] @ g.conj().T
            assert np.abs(Wa[tb, zb, yb, xb, mu] - want).max() < 1e-5
    # sites of the other parity are untouched by this half-sweep except through
    # their backward links; their gauge stays the identity
    for i in _sites_of_parity(rng, 1, 200):
        x, y, z, t = _site(L, i)
        assert np.array_equal(Ga[t, z, y, x], np.eye(3))


@pytest.mark.parametrize("rho,eps", [(0.1, 1.0), (0.06, -0.25)])
def test_smear_step_sampled(O, big, rho, eps):
    import torch
    api, U, host, _ = big
    Sm = api.from_links(api.smear(U, rho, eps, 1), torch.complex128).cpu().numpy()
    rng = np.random.default_rng(2)
    V = int(np.prod(L))
    for _ in range(NSAMPLE // 3):
        i, mu = int(rng.integers(V)), int(rng.integers(4))
        x, y, z, t = _site(L, i)
        assert np.abs(Sm[t, z, y, x, mu] - O.smear_link(host, i, mu, rho, eps)).max() < 1e-5


def test_project_and_count_full(O, big):
    import torch
    api, U, host, _ = big
    W = U.clone()
    G = api.gauge_identity(L)
    api.sweeps(W, G, 5, 1.7)
    api.gauge_reunit(G)
    Zd, mmin = api.center_project(U, G)
    Gh = api.from_gauge(G).cpu().numpy()
    Z = np.ascontiguousarray(np.moveaxis(Zd.cpu().numpy().reshape(4, L[3], L[2], L[1], L[0]), 0, -1))
    Zo, margin = O.center_project(host, Gh)
    safe = margin > 1e-4
    assert safe.mean() > 0.99
    assert np.array_equal(Z[safe], Zo[safe])
    assert abs(mmin - margin.min()) < 1e-9
    vd = api.count_vortices(Zd, L)
    vo = O.count_vortices(Z)
    assert vd == {k: vo[k] for k in ("total", "per_plane", "per_charge")}
    # a wrong decision on a low-margin link changes at most its 6 plaquettes
    vo2 = O.count_vortices(Zo)
    assert abs(vd["total"] - vo2["total"]) <= 6 * int((~safe).sum())


def test_fix_properties_full(O, big):
    import torch
    api, U, host, _ = big
    G, info = api.fix(U, None, tol=-1.0, max_sweeps=60, reunit_every=50, want_traj=True)
    traj = info["traj"]
    assert len(traj) == 61 and info["status"] == 1
    # R never decreases (up to FP32 rounding of the stored links)
    assert np.diff(traj).min() > -1e-6
    assert traj[-1] > traj[0] + 0.1
    assert np.isfinite(info["theta"]) and info["theta"] > 0
    # the transform is unitary and leaves the plaquette unchanged
    Gh = api.from_gauge(G).cpu().numpy().reshape(-1, 3, 3)
    rng = np.random.default_rng(3)
    idx = rng.integers(len(Gh), size=2000)
    M = Gh[idx]
    assert np.abs(M @ M.conj().transpose(0, 2, 1) - np.eye(3)).max() < 1e-12
    W = api.apply_gauge(U, G)
    assert abs(api.plaquette(W) - api.plaquette(U)) < 1e-5
    assert abs(api.functional(W) - info["R"]) < 1e-6


def test_order_and_ring_are_bitwise_at_full_size(big):
    """At the benchmark's size and launch variant, 60 sweeps (a re-unitarisation, two ring folds
    and the final one) with the default tile order (alternating, XCD ranges per field), the
    transform ring and paired sweeps give the bits of forward-order plain sweeps that update G in
    place, of the ring without paired sweeps, and of the alternating order without XCD ranges."""
    import torch
    api, U, host, best = big
    runs = []
    try:
        for order, defer, paired in ((2, True, True), (0, False, False), (2, True, False), (1, True, True)):
            api.set_sweep_order(order)
            api.set_defer_g(defer)
            api.set_paired(paired)
            G, info = api.fix(U, None, tol=-1.0, max_sweeps=60, want_traj=True)
            torch.cuda.synchronize()
            runs.append((G.data.cpu().numpy(), info["traj"]))
            del G
    finally:
        api.set_sweep_order(2)
        api.set_defer_g(True)
        api.set_paired(True)
    for m in (1, 2, 3):
        assert np.array_equal(runs[0][0], runs[m][0]) and np.array_equal(runs[0][1], runs[m][1]), m
