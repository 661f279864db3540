"""Preconditioning levels on the GPU (smear, fix the smeared field, carry back,
re-fix, project, count; all levels batched) against the same chain of oracle
calls, level by level."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

TOL = {0: 1e-12, 1: 1e-5}


@pytest.fixture(scope="module")
def g():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import gpu_util
    return gpu_util


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("L", [(4, 4, 4, 4), (6, 4, 4, 8)])
def test_run_levels_matches_oracle_chain(S, O, g, L, prec):
    from paper_0807_0264_amd import levels as LV
    U = g.rounded(S.heatbath_field(L, S.sub_seed(3000), 5.7, 5), prec)
    G0 = S.haar_gauge(L, S.sub_seed(3001), copy=2)
    lv = (LV.Level("0", 0.1, 1.0, 0), LV.Level("2", 0.1, 1.0, 2), LV.Level("5", 0.1, 1.0, 5),
          LV.Level("OI 3", 0.06, -0.25, 3))
    got = LV.run_levels(g.links(U, prec), lv, G0=g.gauge(G0), tol=-1.0, max_sweeps=30, reunit_every=20,
                        check_every=10)
    for lvl, r in zip(lv, got):
        Gs = G0
        if lvl.n:
            Sm = O.smear(U, lvl.rho, lvl.eps, lvl.n)
            Gs, i_s, _ = O.mcg_fix(Sm, G0, tol=-1.0, max_sweeps=30, reunit_every=20)
            assert abs(r["R_smeared"] - i_s["R"]) <= TOL[prec] * i_s["R"], lvl
        else:
            assert r["R_smeared"] is None
        Go, io, _ = O.mcg_fix(U, Gs, tol=-1.0, max_sweeps=30, reunit_every=20)
        assert abs(r["R"] - io["R"]) <= TOL[prec] * io["R"], lvl
        assert r["sweeps"] == 30 and r["sweeps_smeared"] == (30 if lvl.n else 0)
        assert r["blocks"] == (2 if lvl.n else 1) and r["status"] == 1
        Zo, margin = O.center_project(U, Go)
        if margin.min() > 1e-4:
            assert r["vortices"] == O.count_vortices(Zo)["total"], lvl
        assert r["plaquettes"] == 6 * int(np.prod(L))


def test_series_smearing_is_bitwise_restart(S, g):
    """Continuing a smearing series gives the bits of smearing from scratch."""
    from paper_0807_0264_amd import api
    L = (6, 4, 4, 8)
    U = g.links(S.heatbath_field(L, S.sub_seed(3002), 5.7, 5), 1)
    a = api.smear(api.smear(U, 0.1, 1.0, 4), 0.1, 1.0, 3)
    b = api.smear(U, 0.1, 1.0, 7)
    assert np.array_equal(g.host_links(a), g.host_links(b))
