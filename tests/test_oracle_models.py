"""Pins for the oracle's Hamiltonians, MPOs and exact diagonalisation.

Each check is fixed by something other than the oracle: closed forms (singlet,
N=3/4 chains, free-fermion XX chain, critical Ising chain), values the paper
prints (tests/golden/paper_values.json), numpy's dense eigensolver applied to
an independently built matrix, and the Bethe-ansatz limit."""
import json
import math
import os

import numpy as np
import pytest

import oracle

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))
HEIS = [1.0, 1.0, 0.0]


@pytest.mark.parametrize("N,ref", [(2, -0.75), (3, -1.0), (4, -(3 + 2 * math.sqrt(3)) / 4)])
def test_ed_small_closed_forms(N, ref):
    E, _, _, rc = oracle.ed_ground(oracle.MODEL_XXZ, N, HEIS)
    assert rc == 0
    assert abs(E - ref) <= 1e-12 * abs(ref)


def test_singlet_spectrum_n2():
    H = np.stack([oracle.ed_apply(0, 2, HEIS, e) for e in np.eye(4)], 1)
    assert np.allclose(np.sort(np.linalg.eigvalsh(H)), [-0.75, 0.25, 0.25, 0.25], atol=1e-15)


@pytest.mark.parametrize("model,params", [(0, [1.0, 1.0, 0.0]), (0, [0.7, 1.6, 0.3]), (1, [1.0, 0.241]),
                                          (2, [1.0, 1.0]), (2, [1.0, 0.2])])
def test_mpo_matches_direct_hamiltonian(model, params):
    # The MPO contracted to a dense matrix equals the matrix-free Hamiltonian.
    N = 7
    W = oracle.mpo(model, N, params)
    H_mpo = oracle.mpo_dense(W)
    H_ed = np.stack([oracle.ed_apply(model, N, params, e) for e in np.eye(2 ** N)], 1)
    assert np.abs(H_mpo - H_ed).max() <= 1e-14
    assert np.abs(H_ed - H_ed.T).max() == 0.0


@pytest.mark.parametrize("model,params,N", [(0, HEIS, 10), (1, [1.0, 0.241], 10), (0, [1.0, 0.0, 0.0], 8)])
def test_ed_lanczos_matches_dense_eigensolver(model, params, N):
    H = np.stack([oracle.ed_apply(model, N, params, e) for e in np.eye(2 ** N)], 1)
    E, psi, _, rc = oracle.ed_ground(model, N, params)
    assert rc == 0
    assert abs(E - np.linalg.eigvalsh(H)[0]) <= 1e-12 * abs(E)
    assert np.linalg.norm(H @ psi - E * psi) <= 1e-6


@pytest.mark.parametrize("N", [2, 8, 12])
def test_xx_chain_free_fermions(N):
    # Delta = 0: hopping J/2, single-particle energies cos(k pi/(N+1)); fill the negative ones.
    E, _, _, rc = oracle.ed_ground(0, N, [1.0, 0.0, 0.0])
    ref = -sum(math.cos(k * math.pi / (N + 1)) for k in range(1, N // 2 + 1))
    assert abs(E - ref) <= 1e-10 * abs(ref)


def test_ed_n12_reference():
    E, _, _, _ = oracle.ed_ground(0, 12, HEIS)
    H_ref = -5.142090632840529  # independent sparse eigensolver value
    assert abs(E - H_ref) <= 1e-12 * abs(H_ref)


@pytest.mark.slow
def test_table4_energy_n20():
    # Table 4: E/N = -1.73649 in Pauli units (4 E0 / N with spin-1/2 operators).
    E, _, _, rc = oracle.ed_ground(0, 20, HEIS)
    g = GOLD["heisenberg_N20_E_per_site_pauli"]
    assert round(4 * E / 20, g["digits"]) == g["value"]


def test_bethe_trend():
    # E(N)/N approaches 1/4 - ln 2 from above; a fit E = aN + b + c/N recovers the bulk value.
    g = GOLD["bethe_limit_E_per_site"]
    assert abs(g["value"] - (0.25 - math.log(2))) < 1e-15
    Ns = [8, 10, 12, 14, 16]
    Es = [oracle.ed_ground(0, n, HEIS)[0] for n in Ns]
    per = [e / n for e, n in zip(Es, Ns)]
    assert all(p > g["value"] for p in per)
    assert all(per[i + 1] < per[i] for i in range(len(per) - 1))
    M = np.array([[n, 1.0, 1.0 / n] for n in Ns])
    a, b, c = np.linalg.lstsq(M, np.array(Es), rcond=None)[0]
    assert abs(a - g["value"]) <= 1e-3


def tfim_free_fermion_energy(N, J, h):
    """Ground energy of the open chain H = -J sum sz sz - h sum sx (Pauli) from its free-fermion form
    (Jordan-Wigner; Lieb, Schultz and Mattis 1961): quadratic form with A_ii = 2h, A_{i,i+1} = -J,
    B_{i,i+1} = -B_{i+1,i} = -J; E0 = -(1/2) sum_k Lambda_k with Lambda_k^2 the eigenvalues of
    (A - B)(A + B)."""
    A = np.zeros((N, N))
    B = np.zeros((N, N))
    for i in range(N):
        A[i, i] = 2.0 * h
    for i in range(N - 1):
        A[i, i + 1] = A[i + 1, i] = -J
        B[i, i + 1], B[i + 1, i] = -J, J
    lam2 = np.linalg.eigvalsh((A - B) @ (A + B))
    return -0.5 * float(np.sum(np.sqrt(np.abs(lam2))))


@pytest.mark.parametrize("N,J,h", [(6, 1.0, 0.7), (9, 0.6, 0.25), (10, 1.0, 1.3)])
def test_tfim_ed_equals_free_fermions(N, J, h):
    E = oracle.ed_ground(2, N, [J, h])[0]
    assert abs(E - tfim_free_fermion_energy(N, J, h)) <= 1e-10 * abs(E)


def test_tfim_critical_free_fermions_closed_form():
    # at J = h the single-particle energies are 4 sin((2k-1) pi / (2(2N+1))), k = 1..N, so
    # E0 = 1 - 1 / sin(pi / (2(2N+1))): checks the numerical free-fermion form itself
    import math
    for N in (5, 20, 40):
        assert abs(tfim_free_fermion_energy(N, 1.0, 1.0) - (1 - 1 / math.sin(math.pi / (2 * (2 * N + 1))))) < 1e-11


@pytest.mark.parametrize("N", [4, 6, 8, 10, 12, 14, 16])
def test_j1j2_majumdar_ghosh_point(N):
    # J2 = J1/2 on an open chain of even length: the dimer product state is the exact ground state,
    # E0 = -3N/8 (Majumdar-Ghosh)
    E, _, _, rc = oracle.ed_ground(oracle.MODEL_J1J2, N, [1.0, 0.5], tol=1e-13)
    assert rc == 0
    assert abs(E - (-3.0 * N / 8.0)) <= 1e-11 * N


def test_j1j2_mpo_at_majumdar_ghosh_point():
    # the J1-J2 MPO (not the matrix-free Hamiltonian) has the same ground energy
    N = 8
    H = oracle.mpo_dense(oracle.mpo(oracle.MODEL_J1J2, N, [1.0, 0.5]))
    assert abs(np.linalg.eigvalsh(H)[0] - (-3.0)) <= 1e-12
