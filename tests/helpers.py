"""Small numpy helpers for the tests (independent of the oracle and of the HIP
library).  Arrays use the interchange layout [Lt, Lz, Ly, Lx, ...]."""
import numpy as np


def dag(a):
    return np.conj(np.swapaxes(a, -1, -2))


def shift(a, mu, step=1):
    """a(x + step*mu) as an array indexed by x (periodic)."""
    return np.roll(a, -step, axis=3 - mu)


def gauge_transform(U, g):
    """U^g_mu(x) = g(x) U_mu(x) g(x+mu)^dagger, written with numpy."""
    out = np.empty_like(U)
    for mu in range(4):
        out[..., mu, :, :] = g @ U[..., mu, :, :] @ dag(shift(g, mu))
    return out


def center_links(m):
    """Z3 links exp(2 pi i m / 3) * 1 from integers m [..., 4]."""
    z = np.exp(2j * np.pi * m / 3.0)
    return z[..., None, None] * np.eye(3)


def planted_field(S, L, seed):
    """U = g Z g^dag with uniform Z3 integers m and Haar g; returns (U, g, m)."""
    m = S.z3_links(L, S.sub_seed(seed, 1))
    g = S.haar_gauge(L, S.sub_seed(seed, 2))
    return gauge_transform(center_links(m), g), g, m


def identity_gauge(L):
    G = np.zeros((L[3], L[2], L[1], L[0], 3, 3), np.complex128)
    G[..., 0, 0] = G[..., 1, 1] = G[..., 2, 2] = 1
    return G


def unitarity_error(M):
    M = M.reshape(-1, 3, 3)
    return np.abs(M @ dag(M) - np.eye(3)).max()


def random_su3(rng, n, scale=1.0):
    """n random elements of su(3) (traceless anti-Hermitian), scaled."""
    H = rng.normal(size=(n, 3, 3)) + 1j * rng.normal(size=(n, 3, 3))
    H = 0.5 * (H + dag(H))
    H -= np.trace(H, axis1=1, axis2=2)[:, None, None] / 3 * np.eye(3)
    return 1j * H * scale


def inner(a, b):
    """Re tr(a^dagger b) summed over everything."""
    return float(np.sum(np.real(np.conj(a) * b)))
