"""Batched chains (uneven N and anisotropy) swept together vs the oracle, chain by chain."""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu


def _chains(n, lengths, seed):
    out = []
    for (delta, N) in synth.xxz_chain_set(n, seed, lengths=lengths):
        W = oracle.mpo(oracle.MODEL_XXZ, N, [1.0, delta, 0.0])
        A, chi, _ = synth.random_mps(N, 2, 8, seed=N)
        out.append((delta, N, W, A, chi))
    return out


def _run(chains, sweeps, prec):
    import paper_2604_03960_amd as tna
    c = tna.Context(0)
    pid = tna.pid_params(2.0, 0.1, 0.5, 1.0, 0.3, 8, 24)
    bt = tna.DmrgBatch(c, [w for *_, w, a, chi in chains], [a for *_, a, chi in chains],
                       [chi for *_, chi in chains], pid, heff_prec=prec)
    Es, logs = [], [[] for _ in chains]
    for _ in range(sweeps):
        E, per, stats, st = bt.sweep()
        Es.append(E)
        for i, recs in enumerate(per):
            logs[i] += recs
    print("batch stats", stats)
    return np.array(Es), logs, stats


@pytest.mark.parametrize("prec", [0, 1])
def test_batched_chains_match_oracle(prec):
    chains = _chains(6, (8, 10, 12, 14), seed=3)
    sweeps = 2
    Es, logs, stats = _run(chains, sweeps, prec)
    assert stats["graph_launches"] > 0 and stats["autotune_entries"] > 0
    etol = 1e-10 if prec == 0 else 1e-7
    for i, (delta, N, W, A, chi) in enumerate(chains):
        ro = oracle.dmrg_run(W, A, chi, oracle.pid_params(2.0, 0.1, 0.5, 1.0, 0.3, 8, 24), sweeps)
        assert len(logs[i]) == len(ro["log"])
        for g, o in zip(logs[i], ro["log"]):
            assert (g["bond"], g["dir"]) == (int(o["bond"]), int(o["dir"]))
            if g["chi_ctrl"] != int(o["chi_ctrl"]) or g["k"] != int(o["k"]):
                assert o["gap"] < 1e-8, (i, g, o)  # ambiguous cut only
                break
            assert abs(g["E"] - o["E"]) <= etol * abs(o["E"]) * (1 if prec == 0 else N), (i, g["E"], o["E"])
        dEN = np.abs(Es[:, i] - ro["E"]) / N
        print(f"chain {i} delta={delta:.3f} N={N} dE/N={dEN.max():.2e}")
        assert np.all(dEN <= (1e-10 if prec == 0 else 1e-7) * max(1.0, np.abs(ro["E"]).max() / N))
