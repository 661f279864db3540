"""Pins of the oracle's SU(3) building blocks against closed forms and
textbook routines (matrix exponential, Gram-Schmidt)."""
import numpy as np
import pytest

from helpers import dag, random_su3, unitarity_error


def test_exp_eigen_matches_taylor(O):
    """Two independent exponentials (Jacobi eigendecomposition of Q = -iA and
    scaled-and-squared Taylor series) agree to 1e-14 on su(3)."""
    rng = np.random.default_rng(11)
    for scale in (1e-6, 0.1, 0.7, 2.0, 4.0):
        for A in random_su3(rng, 20, scale):
            E1, E2 = O.exp_su3_eigen(A), O.exp_taylor(A)
            assert np.abs(E1 - E2).max() < 1e-14 * max(1.0, scale)
            assert unitarity_error(E1) < 1e-14
            assert abs(np.linalg.det(E1) - 1) < 1e-14


def test_exp_diagonal_closed_form(O):
    a, b = 0.37, -1.21
    A = 1j * np.diag([a, b, -a - b])
    want = np.diag(np.exp(1j * np.array([a, b, -a - b])))
    assert np.abs(O.exp_su3_eigen(A) - want).max() < 1e-15
    assert np.abs(O.exp_taylor(A) - want).max() < 1e-15


def test_exp_su2_embedding_closed_form(O):
    """exp(i theta n.sigma) = cos(theta) + i sin(theta) n.sigma in a 2x2 block."""
    sig = [np.array([[0, 1], [1, 0]]), np.array([[0, -1j], [1j, 0]]), np.array([[1, 0], [0, -1]])]
    n = np.array([0.3, -0.5, 0.8])
    n /= np.linalg.norm(n)
    th = 1.3
    ns = sum(n[k] * sig[k] for k in range(3))
    for (i, j) in ((0, 1), (1, 2), (0, 2)):
        A = np.zeros((3, 3), complex)
        A[np.ix_([i, j], [i, j])] = 1j * th * ns
        want = np.eye(3, dtype=complex)
        want[np.ix_([i, j], [i, j])] = np.cos(th) * np.eye(2) + 1j * np.sin(th) * ns
        assert np.abs(O.exp_su3_eigen(A) - want).max() < 1e-15
        assert np.abs(O.exp_taylor(A) - want).max() < 1e-15


def test_exp_zero_is_identity_bitwise(O):
    E = O.exp_su3_eigen(np.zeros((3, 3), complex))
    assert np.array_equal(E, np.eye(3, dtype=complex))


def test_exp_taylor_6x6_block_gives_frechet_derivative(O):
    """Upper-right block of exp([[A, E], [0, A]]) equals the directional
    derivative of exp at A along E (checked by central differences)."""
    rng = np.random.default_rng(5)
    A = random_su3(rng, 1, 0.8)[0]
    Ed = rng.normal(size=(3, 3)) + 1j * rng.normal(size=(3, 3))
    big = np.zeros((6, 6), complex)
    big[:3, :3] = big[3:, 3:] = A
    big[:3, 3:] = Ed
    Lb = O.exp_taylor(big)[:3, 3:]
    h = 1e-5
    fd = (O.exp_taylor(A + h * Ed) - O.exp_taylor(A - h * Ed)) / (2 * h)
    assert np.abs(Lb - fd).max() < 1e-9


def test_reunit(O):
    rng = np.random.default_rng(3)
    M = rng.normal(size=(3, 3)) + 1j * rng.normal(size=(3, 3))
    R = O.reunit(M)
    assert unitarity_error(R) < 1e-15
    assert abs(np.linalg.det(R) - 1) < 1e-15
    # first row keeps its direction; the row span of the first two rows is kept
    r0 = M[0] / np.linalg.norm(M[0])
    assert np.abs(R[0] - r0).max() < 1e-15
    proj = R[:2].T @ np.conj(R[:2])  # projector onto span(rows 0,1)
    assert np.abs(proj @ M[1] - M[1]).max() < 1e-14
    # idempotent on SU(3), up to rounding
    assert np.abs(O.reunit(R) - R).max() < 1e-15
    assert np.abs(R @ dag(R) - np.eye(3)).max() < 1e-15
