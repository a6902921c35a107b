"""Pins for the oracle's one-sided Jacobi SVD (Eq. 3/19) and spectrum sums (Eq. 4-5)."""
import math

import numpy as np
import pytest

import oracle
import synth

EPS = 2.0 ** -53


def _check_svd(A, c=16.0):
    S, U, V, sweeps, rc = oracle.svd(A)
    m, n = A.shape
    R = min(m, n)
    assert rc == 0
    tol = c * max(m, n) * EPS
    nrm = np.linalg.norm(A) or 1.0
    assert np.linalg.norm(U * S @ V.T - A) / nrm <= tol
    assert np.abs(U.T @ U - np.eye(R)).max() <= tol
    assert np.abs(V.T @ V - np.eye(R)).max() <= tol
    assert np.all(np.diff(S) <= 0) and np.all(S >= 0)
    # gauge: largest-magnitude entry of every left vector is positive
    for k in range(R):
        assert U[np.argmax(np.abs(U[:, k])), k] > 0
    return S, U, V


@pytest.mark.parametrize("m,n", [(1, 1), (2, 2), (7, 5), (5, 7), (33, 33), (64, 48), (40, 90), (1, 9), (9, 1)])
def test_random_invariants_and_library_spectrum(m, n):
    A = synth.random_matrix(m, n, 11 + m * 7 + n)
    S, _, _ = _check_svd(A)
    ref = np.linalg.svd(A, compute_uv=False)
    assert np.abs(S - ref).max() <= 16 * max(m, n) * EPS * ref[0]


def test_two_by_two_closed_form():
    a, b, c, d = 3.0, 1.0, -2.0, 0.5
    A = np.array([[a, b], [c, d]])
    S, _, _ = _check_svd(A)
    # sigma^2 are the roots of x^2 - (|A|_F^2) x + det(A)^2
    f2 = a * a + b * b + c * c + d * d
    det = a * d - b * c
    disc = math.sqrt(f2 * f2 - 4 * det * det)
    assert abs(S[0] - math.sqrt((f2 + disc) / 2)) <= 4 * EPS * S[0]
    assert abs(S[1] - math.sqrt((f2 - disc) / 2)) <= 8 * EPS * S[0]


def test_diagonal_and_orthogonal_and_rank1():
    d = np.array([0.3, -2.0, 0.0, 1.5, -0.7])
    S, _, _ = _check_svd(np.diag(d))
    assert np.array_equal(S, np.sort(np.abs(d))[::-1])
    Q, _ = np.linalg.qr(synth.random_matrix(12, 12, 5))
    S, _, _ = _check_svd(Q)
    assert np.abs(S - 1.0).max() <= 32 * EPS
    x, y = synth.random_matrix(9, 1, 1), synth.random_matrix(1, 6, 2)
    S, U, _ = _check_svd(x @ y)
    assert abs(S[0] - np.linalg.norm(x) * np.linalg.norm(y)) <= 16 * EPS * S[0]
    assert np.all(S[1:] <= 64 * EPS * S[0])


def test_zero_matrix_completion():
    S, U, V, _, rc = oracle.svd(np.zeros((4, 3)))
    assert np.all(S == 0)
    assert np.abs(U.T @ U - np.eye(3)).max() < 1e-15
    assert np.abs(V.T @ V - np.eye(3)).max() < 1e-15


@pytest.mark.parametrize("n,tau", [(64, 8.0), (128, 64.0)])
def test_prescribed_spectrum_recovered(n, tau):
    A = synth.svd_test_matrix(n, tau, seed=3)
    S, _, _ = _check_svd(A, c=32.0)
    sig = synth.svd_test_spectrum(n, tau)
    assert np.abs(S - sig).max() <= 32 * n * EPS


# ------------------------------------------------------------ entropy / tails
def test_entropy_special_cases():
    assert oracle.spectrum(np.array([1.0, 0.0, 0.0]), 3)[1] == 0.0
    s = 1 / math.sqrt(2)
    assert abs(oracle.spectrum(np.array([s, s]), 2)[1] - math.log(2)) <= 1e-15
    for chi in (3, 16, 257):
        ent = oracle.spectrum(np.full(chi, 0.37), chi)[1]
        assert abs(ent - math.log(chi)) <= 1e-13 * math.log(chi)  # S_max = ln chi


@pytest.mark.parametrize("n,tau", [(512, 8.0), (4096, 64.0)])
def test_geometric_entropy_closed_form(n, tau):
    # p_k = (1-q) q^k / (1 - q^n), q = exp(-2/tau): closed-form Shannon entropy.
    q = math.exp(-2.0 / tau)
    Zn = (1 - q ** n)
    mean_k = q / (1 - q) - n * q ** n / (1 - q ** n)
    ref = -math.log((1 - q) / Zn) - mean_k * math.log(q)
    ent = oracle.spectrum(synth.svd_test_spectrum(n, tau), n)[1]
    assert abs(ent - ref) <= 1e-12 * ref


@pytest.mark.parametrize("n,tau,k", [(512, 64.0, 256), (2048, 64.0, 1024), (64, 8.0, 5)])
def test_truncation_error_closed_form(n, tau, k):
    q = math.exp(-2.0 / tau)
    ref = math.sqrt(q ** k * (1 - q ** (n - k)) / (1 - q))
    Z, ent, eps, w = oracle.spectrum(synth.svd_test_spectrum(n, tau), k)
    assert abs(eps - ref) <= 1e-12 * ref
    assert abs(w - eps * eps / Z) <= 1e-15
