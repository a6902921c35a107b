"""The other rank rules on the GPU vs the oracle: the standard threshold rule (keep the singular
values above eps_trunc, at most chi_max; Sec. 10) and Algorithm 1's entropy margin (Sec. 4), plus
the transverse-field Ising chain against its free-fermion ground energy."""
import math

import numpy as np
import pytest

import oracle
import synth
from gpu_common import ctx
from test_gpu_dmrg import _compare
from test_oracle_models import tfim_free_fermion_energy

pytestmark = pytest.mark.gpu


def _both_rule(N, chi_min, chi_max, sweeps, chi_rule, rule_param, model=0, params=(1.0, 1.0, 0.0), fixed_chi=0):
    import paper_2604_03960_amd as tna
    W = oracle.mpo(model, N, list(params))
    A, chi, _ = synth.random_mps(N, 2, chi_min, 0)
    gains = (0.5, 0.05, 0.1)
    ro = oracle.dmrg_run(W, A, chi, oracle.pid_params(*gains, 0.5, 0.3, chi_min, chi_max), sweeps,
                         fixed_chi=fixed_chi, chi_rule=chi_rule, rule_param=rule_param)
    dm = tna.Dmrg(ctx(), W, A, chi, tna.pid_params(*gains, 0.5, 0.3, chi_min, chi_max), fixed_chi=fixed_chi,
                  chi_rule=chi_rule, rule_param=rule_param)
    logs, Es = [], []
    for _ in range(sweeps):
        E, recs, st = dm.sweep()
        Es.append(E)
        logs += recs
    dm.close()
    return ro, np.array(Es), logs


@pytest.mark.parametrize("eps", [1e-10, 1e-4])
def test_threshold_rule_matches_oracle(eps):
    import paper_2604_03960_amd as tna
    ro, Es, logs = _both_rule(16, 4, 48, 3, tna.CHI_THRESHOLD, eps)
    _compare(ro, Es, logs, 1e-10)
    for g in logs:  # k = min(chi_max, #{sigma > eps}), and the last kept value is above eps
        assert g["k"] <= 48 and (g["k"] == min(g["m"], g["n"]) or g["k"] == 48 or g["sigma_last"] > eps)


@pytest.mark.parametrize("gamma", [1.5, 3.0])
def test_entropy_rule_matches_oracle(gamma):
    import paper_2604_03960_amd as tna
    ro, Es, logs = _both_rule(16, 4, 48, 3, tna.CHI_ENTROPY, gamma)
    _compare(ro, Es, logs, 1e-10)
    pp = oracle.pid_params(0.5, 0.05, 0.1, 0.5, 0.3, 4, 48)
    states = [oracle.PidState() for _ in range(15)]
    for g in logs:  # every GPU decision is Algorithm 1 replayed on the GPU's own entropies
        c, _ = oracle.entropy_chi_update(pp, gamma, states[g["bond"]], g["S"])
        assert c == g["chi_ctrl"]


def test_entropy_rule_binding_equals_oracle():
    import paper_2604_03960_amd as tna
    rng = np.random.default_rng(5)
    pg = tna.pid_params(0, 0, 0, 0, 0.25, 2, 500)
    po = oracle.pid_params(0, 0, 0, 0, 0.25, 2, 500)
    sg, so = tna.PidState(), oracle.PidState()
    for s in rng.uniform(0.0, 6.0, 200):
        assert tna.entropy_chi_update(pg, 1.3, sg, float(s)) == oracle.entropy_chi_update(po, 1.3, so, float(s))[0]
    with pytest.raises(Exception):
        tna.Dmrg(ctx(), oracle.mpo(0, 6, [1.0, 1.0, 0.0]), *synth.random_mps(6, 2, 4, 0)[:2],
                 tna.pid_params(0.5, 0.05, 0.1, 0.5, 0.3, 4, 16), chi_rule=tna.CHI_ENTROPY, rule_param=0.5)


@pytest.mark.parametrize("h", [1.0, 1.4, 2.0])
def test_tfim_matches_oracle_and_free_fermions(h):
    # critical and disordered chains (unique, gapped ground state), N = 16, chi fixed at 64: oracle
    # parity visit by visit, and the free-fermion energy
    ro, Es, logs = _both_rule(16, 8, 64, 3, 0, 0.0, model=2, params=(1.0, h), fixed_chi=64)
    _compare(ro, Es, logs, 1e-10)
    assert abs(Es[-1] - tfim_free_fermion_energy(16, 1.0, h)) <= 1e-9 * abs(Es[-1])


def test_tfim_paramagnet_low_rank_centre_chi128():
    # h = 4, N = 16, chi fixed at 128 from a random MPS of that bond dimension: the centre two-site
    # matrices are 256 x 256 (QR-started SVD) and, once the environments are good, numerically of low
    # rank, so the QR start stops early and the Jacobi sweeps work on the rows above the rounding level
    # only.  Oracle parity visit by visit, the free-fermion energy, and the stopped QR starts on record.
    import paper_2604_03960_amd as tna
    N, chi, h = 16, 128, 4.0
    W = oracle.mpo(2, N, [1.0, h])
    A, chis, _ = synth.random_mps(N, 2, chi, 0)
    pp = (0.5, 0.05, 0.1, 0.5, 0.3, chi, chi)
    ro = oracle.dmrg_run(W, A, chis, oracle.pid_params(*pp), 2, fixed_chi=chi)
    dm = tna.Dmrg(ctx(), W, A, chis, tna.pid_params(*pp), fixed_chi=chi)
    logs, Es = [], []
    for _ in range(2):
        E, recs, _st = dm.sweep()
        Es.append(E)
        logs += recs
    st = dm.stats()
    dm.close()
    _compare(ro, np.array(Es), logs, 1e-10)
    assert abs(Es[-1] - tfim_free_fermion_energy(N, 1.0, h)) <= 1e-9 * abs(Es[-1])
    print("svd rows", st["svd_rows"], "swept", st["svd_rows_swept"], "identity-channel steps", st["heff_ident_steps"])
    assert st["svd_rows_swept"] < st["svd_rows"]
    # canonical tensors: the grouped H_eff products left out the MPO's identity channels
    assert st["heff_ident_steps"] > 0


def test_tfim_ordered_phase_energy():
    # h = 0.6 < J: the two lowest states are split by ~ (h/J)^N, so the Lanczos vector may carry a
    # different tiny admixture of the partner state than the oracle's (entropies then differ at the
    # 1e-7 level); the energies, per sweep, agree with the oracle and the free-fermion value
    ro, Es, logs = _both_rule(16, 8, 64, 3, 0, 0.0, model=2, params=(1.0, 0.6), fixed_chi=64)
    assert np.all(np.abs(Es - ro["E"]) <= 1e-10 * np.abs(ro["E"]))
    assert abs(Es[-1] - tfim_free_fermion_energy(16, 1.0, 0.6)) <= 1e-9 * abs(Es[-1])


def test_tfim_n60_critical_closed_form():
    # N = 60 at the critical point under the PID: the energy is variational and within 1e-7 per site of
    # the closed form 1 - 1/sin(pi / (2(2N+1)))
    import paper_2604_03960_amd as tna
    N = 60
    W = oracle.mpo(2, N, [1.0, 1.0])
    A, chi, _ = synth.random_mps(N, 2, 16, 3)
    dm = tna.Dmrg(ctx(), W, A, chi, tna.pid_params(2.0, 0.1, 0.5, 0.5, 0.3, 16, 64))
    for _ in range(4):
        E, recs, st = dm.sweep()
    dm.close()
    closed = 1 - 1 / math.sin(math.pi / (2 * (2 * N + 1)))
    assert E >= closed - 1e-9 and (E - closed) / N < 1e-7, (E, closed)


def test_second_order_predictor_matches_oracle():
    # PID with the linear and second-order predictors (beta 0.4, beta2 0.3): visit-by-visit parity
    import paper_2604_03960_amd as tna
    N, gains = 16, (2.0, 0.1, 0.5)
    W = oracle.mpo(0, N, [1.0, 1.0, 0.0])
    A, chi, _ = synth.random_mps(N, 2, 4, 0)
    ro = oracle.dmrg_run(W, A, chi, oracle.pid_params(*gains, 0.5, 0.3, 4, 48, beta=0.4, beta2=0.3), 3)
    dm = tna.Dmrg(ctx(), W, A, chi, tna.pid_params(*gains, 0.5, 0.3, 4, 48, beta=0.4, beta2=0.3))
    logs, Es = [], []
    for _ in range(3):
        E, recs, st = dm.sweep()
        Es.append(E)
        logs += recs
    dm.close()
    _compare(ro, np.array(Es), logs, 1e-10)
    rng = np.random.default_rng(11)
    pg, po = tna.pid_params(*gains, 1.0, 0.3, 4, 256, beta=0.4, beta2=0.3), \
        oracle.pid_params(*gains, 1.0, 0.3, 4, 256, beta=0.4, beta2=0.3)
    sg, so = tna.PidState(), oracle.PidState()
    sg.chi = so.chi = 4
    for s in rng.uniform(0.0, 4.0, 200):
        assert tna.pid_chi_update(pg, sg, float(s))[0] == oracle.pid_update(po, so, float(s))[0]
