"""Pins for the oracle's circuit simulation with adaptive bond dimensions (Sec. 8, circuit-level bond
dimension maps; the TEBD scheme of Sec. 2): the exact state-vector simulator against a dense Kronecker
construction and closed-form states, the MPS simulation against the state vector (untruncated) and
against the error bound of its truncations, its Schmidt values against a library SVD of the exact
state, and its controller decisions against a replay of the PID."""
import math

import numpy as np

import oracle
import synth

LN2 = math.log(2.0)
CNOT = np.array([[1.0, 0, 0, 0], [0, 1.0, 0, 0], [0, 0, 0, 1.0], [0, 0, 1.0, 0]])
I4 = np.eye(4)


def _dense_op(N, b, G):
    """2^N x 2^N matrix of the gate G on qubits (b, b+1), qubit 0 the most significant bit."""
    return np.kron(np.kron(np.eye(1 << b), G), np.eye(1 << (N - 2 - b)))


def test_statevector_against_dense_kronecker_products():
    N = 5
    rng_gates = synth.normal(7, 16 * 20).reshape(-1, 4, 4)  # arbitrary real 4 x 4 maps (not unitary)
    parity = [0, 1, 0, 1, 1]
    psi0 = synth.normal(8, 1 << N)
    psi = psi0.copy()
    gi = 0
    packed = []
    for p in parity:
        for b in range(p, N - 1, 2):
            psi = _dense_op(N, b, rng_gates[gi]) @ psi
            packed.append(rng_gates[gi].ravel())
            gi += 1
    got = oracle.circuit_statevector(N, parity, np.concatenate(packed), psi0=psi0)
    assert np.abs(got - psi).max() <= 1e-12 * np.abs(psi).max()


def test_bell_and_ghz_states():
    # RY(pi/2) on qubit 0 then CNOT(0 -> 1): (|00> + |11>) / sqrt 2
    G = CNOT @ np.kron(synth.ry(math.pi / 2), np.eye(2))
    psi = oracle.circuit_statevector(2, [0], G.ravel())
    assert np.allclose(psi, [1 / math.sqrt(2), 0, 0, 1 / math.sqrt(2)], atol=1e-15, rtol=0)
    # GHZ on 4 qubits: Bell pair on (0,1), then CNOT(1 -> 2), then CNOT(2 -> 3)
    ops = [0, 1, 0]
    gates = np.concatenate([G.ravel(), I4.ravel(), CNOT.ravel(), I4.ravel(), CNOT.ravel()])
    psi = oracle.circuit_statevector(4, ops, gates)
    want = np.zeros(16)
    want[0] = want[15] = 1 / math.sqrt(2)
    assert np.abs(psi - want).max() <= 1e-15
    r = oracle.circuit_run(4, ops, gates, oracle.pid_params(0.5, 0.05, 0.1, 0.3, 0.3, 2, 16))
    amp = oracle.mps_amplitudes(4, r["B"], r["chi"])
    assert np.abs(amp - want).max() <= 1e-14
    # every bond of a GHZ state carries one ebit: Schmidt values (1/sqrt 2, 1/sqrt 2)
    for lam in r["lam"]:
        assert np.allclose(lam[:2], [1 / math.sqrt(2)] * 2, atol=1e-15, rtol=0)
    assert all(abs(x["S"] - LN2) <= 1e-14 for x in r["log"][-1:])


def test_untruncated_mps_equals_statevector_and_library_schmidt_values():
    N, layers = 8, 4
    par, g, _ = synth.hea_circuit(N, layers, seed=2)
    psi = oracle.circuit_statevector(N, par, g)
    r = oracle.circuit_run(N, par, g, oracle.pid_params(0.5, 0.05, 0.1, 0.3, 0.3, 16, 16))
    amp = oracle.mps_amplitudes(N, r["B"], r["chi"])
    assert np.abs(amp - psi).max() <= 1e-12
    for b in range(N - 1):
        s = np.linalg.svd(psi.reshape(1 << (b + 1), -1), compute_uv=False)
        lam = r["lam"][b]
        k = len(lam)
        assert np.abs(lam - s[:k]).max() <= 1e-12
        assert np.all(s[k:] <= 1e-12)  # nothing of weight was discarded
    # the map: exact bond dimensions are bounded by 2^min(b+1, N-1-b)
    assert np.all(r["chimap"][-1] <= [min(2 ** (b + 1), 2 ** (N - 1 - b), 16) for b in range(N - 1)])


def test_truncated_mps_within_the_truncation_error_bound():
    """Each truncation replaces the state by its normalised projection: distance at most eps + eps^2
    per gate (eps of Eq. 4); the gates are orthogonal, so the distances add up."""
    N, layers = 10, 5
    par, g, _ = synth.hea_circuit(N, layers, seed=3)
    psi = oracle.circuit_statevector(N, par, g)
    pp = oracle.pid_params(2.0, 0.1, 0.5, 1.0, 0.3, 2, 6)
    r = oracle.circuit_run(N, par, g, pp)
    amp = oracle.mps_amplitudes(N, r["B"], r["chi"])
    bound = sum(x["eps"] + x["eps"] ** 2 for x in r["log"])
    dist = np.linalg.norm(amp - psi)
    assert bound > 1e-3  # the controller did truncate
    assert dist <= 2.0 * bound + 1e-12, (dist, bound)
    assert abs(np.linalg.norm(amp) - 1.0) <= 10 * bound  # renormalised at every cut


def test_controller_replay_and_the_map():
    """The entropies the run logs, fed to the PID of Algorithm 2 bond by bond in gate order, give the
    logged controller decisions; the kept rank is min(chi, rank); the map row of an op carries the new
    rank at the op's bonds and the previous one elsewhere."""
    N, layers = 9, 4
    par, g, _ = synth.hea_circuit(N, layers, seed=4)
    pp = oracle.pid_params(2.0, 0.1, 0.5, 0.5, 0.3, 2, 8)
    r = oracle.circuit_run(N, par, g, pp)
    states = [oracle.PidState(0, 0, 0, 0, pp.chi_min, 0) for _ in range(N - 1)]
    prev = np.ones(N - 1, dtype=int)
    it = iter(r["log"])
    for l, p in enumerate(par):
        row = prev.copy()
        for b in range(p, N - 1, 2):
            rec = next(it)
            assert int(rec["op"]) == l and int(rec["bond"]) == b
            chi, terms = oracle.pid_update(pp, states[b], rec["S"])
            assert chi == int(rec["chi_ctrl"]) and terms["sbar"] == rec["S_ema"] and terms["u"] == rec["u"]
            R = min(int(rec["m"]), int(rec["n"]))
            assert int(rec["k"]) == min(chi, R)
            row[b] = int(rec["k"])
        assert np.array_equal(r["chimap"][l], row)
        prev = row


def test_fixed_chi_and_product_state():
    N = 6
    par, g, _ = synth.hea_circuit(N, 3, seed=5)
    pp = oracle.pid_params(2.0, 0.1, 0.5, 0.5, 0.3, 1, 64)
    r = oracle.circuit_run(N, par, g, pp, fixed_chi=3)
    assert all(int(x["k"]) == min(3, int(x["m"]), int(x["n"])) for x in r["log"])
    # all angles zero: RY = identity and CNOT leaves |0...0> alone -> a product state throughout
    zero = np.concatenate([CNOT.ravel()] * len(g[::16]))
    rz = oracle.circuit_run(N, par, zero, pp)
    assert all(x["S"] == 0.0 and int(x["k"]) == 1 for x in rz["log"])
    amp = oracle.mps_amplitudes(N, rz["B"], rz["chi"])
    assert amp[0] == 1.0 and np.all(amp[1:] == 0.0)
