"""Checks of the seeded input generator (inputs only, no method arithmetic)."""
import ctypes as C

import numpy as np

from helpers import dag, unitarity_error


def test_elementary_functions(S):
    xs = np.random.default_rng(0).uniform(1e-300, 1, 2000)
    lib = S.cpu()
    assert max(abs(lib.sy_cpu_log(float(x)) - np.log(x)) for x in xs) < 2e-15 * 700
    assert max(abs(lib.sy_cpu_log(float(x)) - np.log(x)) / abs(np.log(x)) for x in xs) < 1e-15
    assert max(abs(lib.sy_cpu_sqrt(float(x)) - np.sqrt(x)) / np.sqrt(x) for x in xs) < 1e-15
    assert max(abs(lib.sy_cpu_recip(float(x)) * x - 1) for x in xs) < 1e-15
    s, c = C.c_double(), C.c_double()
    for r in np.linspace(0, 1, 1001):
        lib.sy_cpu_sincos_turn(float(r), C.byref(s), C.byref(c))
        assert abs(s.value - np.sin(2 * np.pi * r)) < 1e-15
        assert abs(c.value - np.cos(2 * np.pi * r)) < 1e-15


def test_determinism_and_seeds(S):
    L = (4, 4, 4, 4)
    a = S.haar_links(L, 7)
    assert np.array_equal(a, S.haar_links(L, 7))
    assert not np.array_equal(a, S.haar_links(L, 8))
    h = S.heatbath_field(L, 3, 5.7, 2)
    assert np.array_equal(h, S.heatbath_field(L, 3, 5.7, 2))
    assert not np.array_equal(S.haar_gauge(L, 3, 0), S.haar_gauge(L, 3, 1))


def test_haar_moments(S):
    """Haar SU(3): E tr U = 0, E |tr U|^2 = 1, E |tr U|^4 = 2."""
    U = S.haar_links((8, 8, 8, 8), 11).reshape(-1, 3, 3)
    assert unitarity_error(U) < 1e-14
    assert np.abs(np.linalg.det(U) - 1).max() < 1e-14
    t = np.trace(U, axis1=1, axis2=2)
    n = len(t)
    assert abs(t.mean()) < 5 / np.sqrt(n)
    assert abs(np.mean(np.abs(t) ** 2) - 1) < 5 / np.sqrt(n)
    assert abs(np.mean(np.abs(t) ** 4) - 2) < 5 * np.sqrt(24 / n)


def test_gaussian_moments(S):
    z = S.gaussians(200000, 5)
    assert abs(z.mean()) < 5 / np.sqrt(len(z))
    assert abs(z.var() - 1) < 5 * np.sqrt(2 / len(z))


def test_z3_uniform(S):
    m = S.z3_links((8, 8, 8, 8), 9)
    assert set(np.unique(m)) == {-1, 0, 1}
    f = np.array([(m == k).mean() for k in (-1, 0, 1)])
    assert np.abs(f - 1 / 3).max() < 0.01


def test_heatbath_plaquette_beta_5p7(S, O):
    """50 sweeps from a Haar start at beta = 5.7: the plaquette approaches its
    equilibrium value (about 0.549 for the Wilson action)."""
    U = S.heatbath_field((8, 8, 8, 8), S.sub_seed(601), 5.7, 50)
    assert unitarity_error(U) < 1e-14
    P = O.plaquette(U)
    assert 0.53 < P < 0.56
