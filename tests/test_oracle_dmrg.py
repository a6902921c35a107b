"""Pins for the oracle's two-site DMRG sweep with the PID bond-dimension controller."""
import math

import numpy as np
import pytest

import oracle
import synth

HEIS = [1.0, 1.0, 0.0]
E12 = -5.142090632840529
S12 = [0.693147, 0.414031, 0.729338, 0.511429, 0.748112, 0.536833]


def _run(N, chi_init, chi_min, chi_max, sweeps, gains=(0.5, 0.05, 0.1), s_target=0.5, model=0, params=HEIS,
         fixed_chi=0):
    W = oracle.mpo(model, N, params)
    A, chi, _ = synth.random_mps(N, 2, chi_init, 0)
    pp = oracle.pid_params(*gains, s_target, 0.3, chi_min, chi_max)
    return oracle.dmrg_run(W, A, chi, pp, sweeps, fixed_chi=fixed_chi)


def test_untruncated_dmrg_equals_ed():
    r = _run(12, 8, 64, 64, 3)
    assert r["rc"] == 0
    assert abs(r["E"][-1] - E12) <= 1e-10 * abs(E12)
    last = r["log"][-11:][::-1]  # R->L visits of the last sweep, bonds 0..10
    ent = [rec["S"] for rec in last]
    assert np.allclose(ent[:6], S12, atol=1e-6)
    assert np.allclose(ent, ent[::-1], atol=1e-8)  # reflection symmetry of the chain
    # bond 0 of an SU(2) singlet: rho_1 = I/2, so S = ln 2 (up to the Lanczos residual)
    assert abs(ent[0] - math.log(2)) <= 1e-9


def test_c1_configuration_variational():
    # Heisenberg N=12, chi from 8, chi_max 32, PID (0.5, 0.05, 0.1), 4 sweeps.
    r = _run(12, 8, 8, 32, 4)
    assert r["rc"] == 0
    for rec in r["log"]:
        assert rec["E"] >= E12 - 1e-10
        assert rec["k"] <= min(rec["m"], rec["n"], rec["chi_ctrl"])
    assert abs(r["E"][-1] - E12) <= 1e-4  # truncated at chi <= 32
    assert all(8 <= st.chi <= 32 for st in r["pid"])
    assert all(c <= 32 for c in r["chi"])


def test_fixed_chi_energy_converges_above_ed():
    # Fixed chi = 8 (a clean SU(2) cluster end at N=12): every Ritz value is an upper
    # bound, and the sweep energies settle once the truncation pattern is fixed.
    r = _run(12, 8, 8, 8, 5, fixed_chi=8)
    E = r["E"]
    assert all(e >= E12 - 1e-12 for e in E)
    assert abs(E[-1] - E[-2]) <= 1e-10
    assert abs(E[-1] - E12) <= 1e-4


def test_controller_moves_chi_with_paper_gains():
    r = _run(12, 8, 8, 32, 3, gains=(2.0, 0.1, 0.5), s_target=0.3)
    chis = [rec["chi_ctrl"] for rec in r["log"]]
    assert max(chis) > 8
    # the controller chi follows Algorithm 2 step by step: replay it from the logged entropies
    pp = oracle.pid_params(2.0, 0.1, 0.5, 0.3, 0.3, 8, 32)
    states = [oracle.PidState() for _ in range(11)]
    for st in states:
        st.chi = 8
    for rec in r["log"]:
        c, _ = oracle.pid_update(pp, states[int(rec["bond"])], rec["S"])
        assert c == rec["chi_ctrl"]


def test_critical_ising_paper_value():
    # Sec. 13: critical Ising chain, N = 20, E/N = -1.25539; closed form 1 - 1/sin(pi/(2(2N+1))).
    W = oracle.mpo(2, 20, [1.0, 1.0])
    A, chi, _ = synth.random_mps(20, 2, 16, 0)
    pp = oracle.pid_params(0.5, 0.05, 0.1, 0.5, 0.3, 24, 24)
    r = oracle.dmrg_run(W, A, chi, pp, 3)
    e = r["E"][-1] / 20
    closed = (1 - 1 / math.sin(math.pi / (2 * (2 * 20 + 1)))) / 20
    assert abs(e - closed) <= 1e-8
    assert round(e, 5) == -1.25539


def _run_rule(N, chi_min, chi_max, sweeps, chi_rule, rule_param):
    W = oracle.mpo(0, N, HEIS)
    A, chi, _ = synth.random_mps(N, 2, chi_min, 0)
    pp = oracle.pid_params(0.5, 0.05, 0.1, 0.5, 0.3, chi_min, chi_max)
    return pp, oracle.dmrg_run(W, A, chi, pp, sweeps, chi_rule=chi_rule, rule_param=rule_param)


def test_threshold_rule_tiny_eps_is_exact():
    # standard rule chi_k = min(chi_max, r), r = #{sigma > eps_trunc} (Sec. 10): with eps_trunc far
    # below every nonzero value nothing is truncated, so the sweep reaches the exact ground state
    _, r = _run_rule(12, 8, 64, 3, 1, 1e-300)
    assert abs(r["E"][-1] - E12) <= 1e-10 * abs(E12)


def test_threshold_rule_keeps_values_above_eps():
    eps = 1e-3
    _, r = _run_rule(12, 8, 64, 3, 1, eps)
    for rec in r["log"]:
        if rec["k"] < min(rec["m"], rec["n"]) and rec["k"] < 64:
            assert rec["sigma_kept_last"] > eps  # every kept value exceeds eps_trunc
    assert r["E"][-1] >= E12 - 1e-12 and r["E"][-1] - E12 < 1e-4 * abs(E12)


def test_entropy_rule_large_margin_is_exact_and_decisions_replay():
    # gamma large enough that ceil(gamma e^S) >= chi_max = 64 >= every rank of N = 12: exact
    _, r = _run_rule(12, 8, 64, 3, 2, 64.0)
    assert abs(r["E"][-1] - E12) <= 1e-10 * abs(E12)
    # gamma = 2: every logged decision is Algorithm 1 replayed on the logged entropies
    pp, r = _run_rule(12, 4, 32, 3, 2, 2.0)
    states = [oracle.PidState() for _ in range(11)]
    for rec in r["log"]:
        c, _ = oracle.entropy_chi_update(pp, 2.0, states[int(rec["bond"])], rec["S"])
        assert c == rec["chi_ctrl"] and rec["k"] == min(c, rec["m"], rec["n"])
