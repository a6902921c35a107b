"""Pins for the oracle's effective Hamiltonian (Eq. 18), environments and Lanczos.

H_eff is pinned by the brute-force identity H_eff = P^T H P, with H from the
matrix-free Hamiltonian (not the MPO) and P the isometry of a mixed-canonical
MPS; the Lanczos ground value is pinned by numpy's dense eigensolver on the
explicit H_eff matrix."""
import numpy as np
import pytest

import oracle
import synth
from _mps_util import block_left, block_right, left_isometries, right_isometries

d = 2


def _setup(model, params, N, b, chi_cap):
    dims = [min(chi_cap, d ** (i + 1), d ** (N - 1 - i)) for i in range(N - 1)]
    As = left_isometries(b, d, dims[:b], seed=7)
    Bs = right_isometries(N - b - 2, d, dims[b + 1:], seed=9)
    W = oracle.mpo(model, N, params)
    D = W.shape[1]
    L = np.zeros((1, D, 1)); L[0, D - 1, 0] = 1.0
    for i, A in enumerate(As):
        L = oracle.env_left(L, W[i], A)
    R = np.zeros((1, D, 1)); R[0, 0, 0] = 1.0
    for j, B in reversed(list(enumerate(Bs))):
        R = oracle.env_right(R, W[b + 2 + j], B)
    chl = 1 if b == 0 else dims[b - 1]
    chr_ = 1 if b == N - 2 else dims[b + 1]
    return As, Bs, W, L, R, chl, chr_


def _project(As, Bs, theta):
    PL, PR = block_left(As), block_right(Bs)
    chl, _, _, chr_ = theta.shape
    psi = np.einsum("xa,astc,cy->xsty", PL, theta, PR)
    return psi.reshape(-1), PL, PR


@pytest.mark.parametrize("model,params,N,b,chi", [
    (0, [1.0, 1.0, 0.0], 8, 3, 16),
    (0, [0.8, 1.7, 0.2], 9, 0, 8),
    (0, [1.0, 1.0, 0.0], 8, 6, 4),
    (1, [1.0, 0.241], 9, 4, 6),
    (2, [1.0, 0.6], 8, 2, 5),
])
def test_heff_equals_projected_hamiltonian(model, params, N, b, chi):
    As, Bs, W, L, R, chl, chr_ = _setup(model, params, N, b, chi)
    theta = synth.random_matrix(chl * d * d, chr_, 21).reshape(chl, d, d, chr_)
    out = oracle.heff_apply(L, W[b], W[b + 1], R, theta)
    psi, PL, PR = _project(As, Bs, theta)
    Hpsi = oracle.ed_apply(model, N, params, psi).reshape(PL.shape[0], d, d, PR.shape[1])
    ref = np.einsum("xa,xsty,cy->astc", PL, Hpsi, PR)
    assert np.abs(out - ref).max() <= 1e-13 * max(1.0, np.abs(ref).max())


def test_heff_symmetric():
    As, Bs, W, L, R, chl, chr_ = _setup(1, [1.0, 0.3], 9, 3, 8)
    x = synth.random_matrix(chl * 4, chr_, 1).reshape(chl, 2, 2, chr_)
    y = synth.random_matrix(chl * 4, chr_, 2).reshape(chl, 2, 2, chr_)
    hx = oracle.heff_apply(L, W[3], W[4], R, x)
    hy = oracle.heff_apply(L, W[3], W[4], R, y)
    assert abs(np.vdot(y, hx) - np.vdot(hy, x)) <= 1e-12 * np.abs(hx).max() * np.abs(y).sum()


def test_heff_two_sites_is_singlet_operator():
    W = oracle.mpo(0, 2, [1.0, 1.0, 0.0])
    L = np.zeros((1, 5, 1)); L[0, 4, 0] = 1
    R = np.zeros((1, 5, 1)); R[0, 0, 0] = 1
    H = np.stack([oracle.heff_apply(L, W[0], W[1], R, e.reshape(1, 2, 2, 1)).reshape(4) for e in np.eye(4)], 1)
    S = {"z": np.diag([0.5, -0.5]), "x": np.array([[0, 0.5], [0.5, 0]]), "y": np.array([[0, -0.5j], [0.5j, 0]])}
    ref = sum(np.kron(S[a], S[a]) for a in "xyz").real
    assert np.abs(H - ref).max() == 0.0


def test_env_right_canonical_identity_channel():
    # Canonical sites leave the identity-carrying MPO channels as identities:
    # channel 0 ("all terms closed") on the right, channel D-1 ("none opened") on the left.
    N, b = 8, 2
    As, Bs, W, L, R, chl, chr_ = _setup(0, [1, 1, 0], N, b, 8)
    assert np.abs(R[:, 0, :] - np.eye(chr_)).max() <= 1e-14
    assert np.abs(L[:, 4, :] - np.eye(chl)).max() <= 1e-14


@pytest.mark.parametrize("model,params,N,b,chi", [(0, [1, 1, 0], 10, 4, 8), (1, [1, 0.241], 9, 3, 6),
                                                 (0, [1, 1, 0], 6, 0, 4)])
def test_lanczos_ground_equals_dense_eigen(model, params, N, b, chi):
    As, Bs, W, L, R, chl, chr_ = _setup(model, params, N, b, chi)
    dim = chl * 4 * chr_
    H = np.stack([oracle.heff_apply(L, W[b], W[b + 1], R, e.reshape(chl, 2, 2, chr_)).reshape(dim)
                  for e in np.eye(dim)], 1)
    ref = np.linalg.eigvalsh(0.5 * (H + H.T))[0]
    th0 = synth.random_matrix(dim, 1, 5).reshape(chl, 2, 2, chr_)
    E, th, it, rc = oracle.lanczos_heff(L, W[b], W[b + 1], R, th0, tol=1e-12)
    assert rc == 0
    assert abs(E - ref) <= 1e-12 * max(1.0, abs(ref))
    v = th.reshape(dim)
    assert abs(np.linalg.norm(v) - 1) < 1e-14
    assert np.linalg.norm(H @ v - E * v) <= 1e-6


def test_sym_eig_jacobi_against_numpy():
    A = synth.random_matrix(30, 30, 4)
    A = A + A.T
    w, V, rc = oracle.sym_eig(A)
    assert rc == 0
    assert np.abs(np.sort(w) - np.linalg.eigvalsh(A)).max() <= 1e-13 * np.abs(w).max()
    assert np.abs(V.T @ V - np.eye(30)).max() <= 1e-14


def test_heff_element_equals_full_product():
    """The one-element form used for large-chi spot checks agrees with the full contraction (itself pinned
    against P^T H P above) on every element of a small random case."""
    rng = np.random.default_rng(3)
    chl, chr_, d, D = 7, 5, 2, 5
    W = oracle.mpo(oracle.MODEL_XXZ, 6, [1.0, 0.8, 0.0])
    L = rng.standard_normal((chl, D, chl))
    R = rng.standard_normal((chr_, D, chr_))
    th = rng.standard_normal((chl, d, d, chr_))
    full = oracle.heff_apply(L, W[2], W[3], R, th)
    for idx in np.ndindex(full.shape):
        assert abs(oracle.heff_element(L, W[2], W[3], R, th, idx) - full[idx]) <= 1e-13 * np.abs(full).max()


@pytest.mark.parametrize("k", [1, 3, 6, 10])
def test_fixed_iteration_lanczos_is_rayleigh_ritz_on_the_krylov_space(k):
    """After exactly k matvecs from theta0 (fixed-iteration mode, no restart), the Ritz value is the
    minimum of the Rayleigh quotient over span{theta0, H theta0, ..., H^(k-1) theta0}, and the returned
    vector is the minimiser.  The reference projects the explicit H_eff onto an orthonormal basis of
    that Krylov space made by numpy's QR of the power vectors."""
    As, Bs, W, L, R, chl, chr_ = _setup(0, [1, 1, 0], 10, 4, 8)
    dim = chl * 4 * chr_
    H = np.stack([oracle.heff_apply(L, W[4], W[5], R, e.reshape(chl, 2, 2, chr_)).reshape(dim)
                  for e in np.eye(dim)], 1)
    H = 0.5 * (H + H.T)
    th0 = synth.random_matrix(dim, 1, 17).reshape(dim)
    K = np.zeros((dim, k))
    x = th0 / np.linalg.norm(th0)
    for i in range(k):
        K[:, i] = x
        x = H @ x
        x /= np.linalg.norm(x)
    Q, _ = np.linalg.qr(K)
    w, Y = np.linalg.eigh(Q.T @ H @ Q)
    ref_E, ref_v = w[0], Q @ Y[:, 0]
    E, th, it, rc = oracle.lanczos_heff(L, W[4], W[5], R, th0.reshape(chl, 2, 2, chr_), tol=1e-300,
                                        restarts=0, fixed_iters=k)
    assert rc == 0 and it == k
    assert abs(E - ref_E) <= 1e-10 * abs(ref_E)
    v = th.reshape(dim)
    assert abs(abs(v @ ref_v) - 1.0) <= 1e-8
    if k > 1:  # more matvecs lower the Ritz value
        E1, _, _, _ = oracle.lanczos_heff(L, W[4], W[5], R, th0.reshape(chl, 2, 2, chr_), tol=1e-300,
                                          restarts=0, fixed_iters=k - 1)
        assert E < E1
