"""Circuit simulation with adaptive bond dimensions on the GPU (one grouped launch sequence per gate
layer) against the oracle: the controller's decisions and the kept ranks bit for bit, entropies and
truncation errors per gate, the bond-dimension map, and the final amplitudes against the oracle's MPS
and, untruncated, against the exact state vector."""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu


def _amplitudes(N, B, chi):
    """psi(s_0..s_{N-1}) of packed site tensors, contracted left to right with numpy."""
    cur = np.ones((1, 1))
    off = 0
    for i in range(N):
        cl = 1 if i == 0 else int(chi[i - 1])
        cr = 1 if i == N - 1 else int(chi[i])
        A = B[off:off + cl * 2 * cr].reshape(cl, 2 * cr)
        off += cl * 2 * cr
        cur = (cur @ A).reshape(-1, cr)
    return cur.ravel()


def _compare(gpu_recs, gpu_map, ora, N):
    """Gate by gate until the first ambiguous cut (oracle gap below 1e-8 with values discarded);
    returns the discarded weight of that cut (0 if none)."""
    assert len(gpu_recs) == len(ora["log"])
    amb = 0.0
    for g, o in zip(gpu_recs, ora["log"]):
        assert (g["layer"], g["bond"], g["m"], g["n"]) == (int(o["op"]), int(o["bond"]), int(o["m"]), int(o["n"]))
        if g["chi_ctrl"] != int(o["chi_ctrl"]) or g["k"] != int(o["k"]):
            assert o["gap"] < 1e-8, (g, o)
            return max(float(o["wdisc"]), 1e-300)
        assert abs(g["S"] - o["S"]) <= 1e-10 * max(1.0, o["S"]), (g, o)
        assert abs(g["eps"] - o["eps"]) <= 1e-10 * max(o["eps"], 1e-6), (g, o)
        if o["gap"] < 1e-8 and int(o["k"]) < min(int(o["m"]), int(o["n"])):
            amb = max(float(o["wdisc"]), 1e-300)
            break
    if amb == 0.0:
        assert np.array_equal(gpu_map, ora["chimap"])
    return amb


@pytest.mark.parametrize("N,layers,chi_min,chi_max,seed", [(8, 4, 16, 16, 2), (10, 5, 2, 6, 3), (12, 6, 4, 12, 6)])
def test_circuit_matches_oracle(N, layers, chi_min, chi_max, seed):
    import paper_2604_03960_amd as tna
    par, g, _ = synth.hea_circuit(N, layers, seed=seed)
    pp = (2.0, 0.1, 0.5, 1.0, 0.3, chi_min, chi_max)
    ora = oracle.circuit_run(N, par, g, oracle.pid_params(*pp))
    psi = oracle.circuit_statevector(N, par, g)
    ctx = tna.Context(0)
    circ = tna.Circuit(ctx, N, tna.pid_params(*pp))
    cmap, recs = circ.run(par, g)
    B, chi = circ.mps()
    amb = _compare(recs, cmap, ora, N)
    amp = _amplitudes(N, B, chi)
    amp_o = oracle.mps_amplitudes(N, ora["B"], ora["chi"])
    trunc = sum(float(o["eps"]) for o in ora["log"])
    print(f"N={N}: max chi {int(cmap.max())}, |psi_gpu - psi_oracle| {np.linalg.norm(amp - amp_o):.2e}, "
          f"|psi_gpu - psi_exact| {np.linalg.norm(amp - psi):.2e}, truncation sum {trunc:.2e}, ambiguous {amb:.1e}")
    assert np.linalg.norm(amp - amp_o) <= 1e-10 + 10.0 * np.sqrt(amb)
    if chi_min >= 2 ** (N // 2):  # untruncated: the exact state
        assert np.abs(amp - psi).max() <= 1e-12
    assert np.linalg.norm(amp - psi) <= 2.0 * sum(float(o["eps"]) + float(o["eps"]) ** 2 for o in ora["log"]) + 1e-10
    circ.close()


def test_batched_layer_equals_gates_one_at_a_time():
    """All gates of a layer through one grouped launch sequence (one group of SVDs) give what the same
    gates give one after another."""
    import paper_2604_03960_amd as tna
    N, layers = 14, 6
    par, g, _ = synth.hea_circuit(N, layers, seed=9)
    pp = tna.pid_params(2.0, 0.1, 0.5, 1.0, 0.3, 4, 24)
    ctx = tna.Context(0)
    a = tna.Circuit(ctx, N, pp)
    b = tna.Circuit(ctx, N, pp, one_at_a_time=True)
    ma, ra = a.run(par, g)
    mb, rb = b.run(par, g)
    for x, y in zip(ra, rb):
        assert (x["bond"], x["k"], x["chi_ctrl"]) == (y["bond"], y["k"], y["chi_ctrl"]) or x["gap"] < 1e-8
        assert abs(x["S"] - y["S"]) <= 1e-12 * max(1.0, x["S"])
    Ba, ca = a.mps()
    Bb, cb = b.mps()
    assert np.array_equal(ca, cb) and np.array_equal(ma, mb)
    assert np.linalg.norm(_amplitudes(N, Ba, ca) - _amplitudes(N, Bb, cb)) <= 1e-11
