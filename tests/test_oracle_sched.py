"""Pins for the oracle's learned-scheduler inputs, labels and fallback rule.

The network stands in for the predictive scheduler of Sec. 7 (Eq. 16-17); its
inputs are the bond's EMA entropy history (Eq. 8) and singular-value tail, its
label the smallest rank meeting the truncation-error target of Eq. (4).  The
pins are hand-computed values of those definitions and two limiting cases of
the fallback rule that reduce to runs without a scheduler."""
import math

import numpy as np

import oracle
import synth

HEIS = [1.0, 1.0, 0.0]


def test_features_by_hand():
    S = np.array([0.8, 0.6])
    f = oracle.sched_features([0.3, 0.5], S, bond=2, N=10)
    # fewer than 8 entropies: the oldest (0.3) fills the front
    assert list(f[:8]) == [0.3] * 7 + [0.5]
    assert f[8] == math.log(0.8) and f[9] == math.log(0.6)
    assert np.all(f[10:24] == math.log(1e-16))  # missing values count as the floor
    assert f[24] == 0.3  # (2 + 1) / 10
    # more than 8 entropies: the last 8, oldest first; tiny values are floored
    h = [0.1 * i for i in range(12)]
    f = oracle.sched_features(h, np.array([1.0, 1e-20, 0.0]), bond=0, N=4)
    assert np.allclose(f[:8], [0.4, 0.5, 0.6, 0.7, 0.8, 0.9, 1.0, 1.1], rtol=0, atol=1e-15)
    assert f[8] == 0.0 and f[9] == math.log(1e-16) and f[10] == math.log(1e-16)
    assert f[24] == 0.25


def test_labels_by_hand():
    S = np.array([0.9, 0.4, 0.1, 1e-5, 1e-9])
    # tails: k=1 -> sqrt(0.16+0.01+1e-10+1e-18) ~ 0.412; k=2 -> ~0.1; k=3 -> ~1e-5; k=4 -> 1e-9; k=5 -> 0
    assert oracle.k_needed(S, 1e-4) == 3
    assert oracle.k_needed(S, 1e-5) == 4  # sqrt(1e-10 + 1e-18) > 1e-5 by 5e-14 relative
    assert oracle.k_needed(S, 2e-5) == 3
    assert oracle.k_needed(S, 1e-9) == 4
    assert oracle.k_needed(S, 1e-10) == 5  # only the full rank meets it
    assert oracle.k_needed(S, 1.0) == 1   # k >= 1 always
    assert abs(oracle.trunc_error(S, 3) - math.sqrt(1e-10 + 1e-18)) <= 1e-22
    assert oracle.trunc_error(S, 5) == 0.0


def _chain(N, chi0, seed):
    W = oracle.mpo(oracle.MODEL_XXZ, N, HEIS)
    A, chi, _ = synth.random_mps(N, 2, chi0, seed)
    return W, A, chi


def test_proposals_at_full_rank_equal_fixed_chi():
    # with a target no normalised state misses (eps_target = 1), every proposal is used: proposals of
    # chi_max at every visit keep min(chi_max, R) everywhere, exactly as the fixed-chi rule does
    N, sweeps = 8, 2
    W, A, chi = _chain(N, 4, 3)
    pp = oracle.pid_params(0.5, 0.05, 0.1, 0.5, 0.3, 4, 12)
    nrec = sweeps * 2 * (N - 1)
    a = oracle.dmrg_run(W, A, chi, pp, sweeps, sched_pred=np.full(nrec, 12), eps_target=1.0)
    b = oracle.dmrg_run(W, A, chi, pp, sweeps, fixed_chi=12)
    assert [r["k"] for r in a["log"]] == [r["k"] for r in b["log"]]
    assert np.array_equal(a["E"], b["E"])
    # the proposal is used on every visit (no fallback)
    assert all(r["fallback"] == 0 and r["chi_sched"] == 12 for r in a["log"])


def test_proposals_that_always_miss_fall_back_to_the_controller():
    N, sweeps = 8, 2
    W, A, chi = _chain(N, 4, 5)
    pp = oracle.pid_params(0.5, 0.05, 0.1, 0.5, 0.3, 4, 12)
    nrec = sweeps * 2 * (N - 1)
    a = oracle.dmrg_run(W, A, chi, pp, sweeps, sched_pred=np.ones(nrec, dtype=np.int32), eps_target=1e-300)
    b = oracle.dmrg_run(W, A, chi, pp, sweeps)
    assert np.array_equal(a["E"], b["E"])
    assert [r["k"] for r in a["log"]] == [r["k"] for r in b["log"]]
    # a rank-1 proposal misses the target wherever the spectrum has more than one nonzero value
    for r in a["log"]:
        assert r["fallback"] == (1 if r["k_needed"] > 1 else 0)


def test_logged_inputs_follow_the_run():
    N, sweeps = 10, 3
    W, A, chi = _chain(N, 8, 11)
    run = oracle.dmrg_run(W, A, chi, oracle.pid_params(2.0, 0.1, 0.5, 0.5, 0.3, 8, 16), sweeps, eps_target=1e-6)
    hist = {}
    for r in run["log"]:
        b = int(r["bond"])
        hist.setdefault(b, []).append(r["S_ema"])
        h = hist[b][-8:]
        h = [h[0]] * (8 - len(h)) + h
        assert np.array_equal(r["feat"][:8], h)
        assert r["feat"][8] == math.log(r["sigma0"])
        assert r["feat"][24] == (b + 1) / N
        assert 1 <= r["k_needed"] <= min(r["m"], r["n"])
        # the kept rank meets the target exactly when it is at least the needed rank
        assert (r["eps"] <= 1e-6) == (r["k"] >= r["k_needed"])
