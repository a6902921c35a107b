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


def _run(chains, sweeps, prec, chi_max=24, chi_min=8):
    import paper_2604_03960_amd as tna
    c = tna.Context(0)
    pid = tna.pid_params(2.0, 0.1, 0.5, 1.0, 0.3, chi_min, chi_max)
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


def _check(chains, sweeps, prec, chi_max, Es, logs, chi_min=8):
    """Visit by visit against the oracle.  A truncation whose cut falls inside a (near) degenerate
    multiplet (oracle gap (s_{k-1} - s_k)/s_0 < 1e-8) keeps an arbitrary rotation of the multiplet on
    either side, so the comparison of that chain stops after such a visit, and its final energies may
    then differ by up to the discarded weight of the ambiguous truncation (times |E|); the per-site
    tolerance is 1e-10 (FP64 H_eff) or 1e-7 (FP32 H_eff) relative to max(1, |E|/N)."""
    etol = 1e-10 if prec == 0 else 1e-7
    for i, (delta, N, W, A, chi) in enumerate(chains):
        ro = oracle.dmrg_run(W, A, chi, oracle.pid_params(2.0, 0.1, 0.5, 1.0, 0.3, chi_min, chi_max), sweeps)
        assert len(logs[i]) == len(ro["log"])
        amb_w = 0.0
        for g, o in zip(logs[i], ro["log"]):
            assert (g["bond"], g["dir"]) == (int(o["bond"]), int(o["dir"]))
            if g["chi_ctrl"] != int(o["chi_ctrl"]) or g["k"] != int(o["k"]):
                assert o["gap"] < 1e-8, (i, g, o)  # ambiguous cut only
                amb_w = max(amb_w, float(o["wdisc"]), 1e-12)
                break
            assert abs(g["E"] - o["E"]) <= etol * abs(o["E"]) * (1 if prec == 0 else N), (i, g["E"], o["E"])
            if o["gap"] < 1e-8 and int(o["k"]) < min(int(o["m"]), int(o["n"])):
                amb_w = max(amb_w, float(o["wdisc"]), 1e-12)
                break
        dEN = np.abs(Es[:, i] - ro["E"]) / N
        print(f"chain {i} delta={delta:.3f} N={N} dE/N={dEN.max():.2e} ambiguous_w={amb_w:.1e}")
        tol = (1e-10 if prec == 0 else 1e-7) * max(1.0, np.abs(ro["E"]).max() / N)
        assert np.all(dEN <= tol + amb_w * np.abs(ro["E"]).max() / N)


@pytest.mark.parametrize("prec", [0, 1])
def test_batched_chains_match_oracle(prec):
    """Short theta throughout (chi <= 24): the single-workgroup Lanczos and fused Jacobi paths."""
    chains = _chains(6, (8, 10, 12, 14), seed=3)
    Es, logs, stats = _run(chains, 2, prec)
    assert stats["small_launches"] > 0
    assert (stats["heff_f32_iters"] >= stats["lanczos_iters"] > 0) if prec else stats["heff_f32_iters"] == 0
    _check(chains, 2, prec, 24, Es, logs)


@pytest.mark.parametrize("prec", [0, 1])
def test_batched_mixed_paths_match_oracle(prec):
    """chi pinned at 40 on N = 14..16: middle bonds exceed the short-theta limit (chi_l d^2 chi_r > 4096) and
    take the graph-replayed grouped path within the same steps as the short edge bonds; with prec 1 both
    paths run their FP32 H_eff (the grouped GEMMs, the mixing and the L/R copies in FP32)."""
    chains = _chains(4, (14, 16), seed=5)
    Es, logs, stats = _run(chains, 2, prec, chi_max=40, chi_min=40)
    assert stats["small_launches"] > 0 and stats["graph_launches"] > 0 and stats["autotune_entries"] > 0
    assert (stats["heff_f32_iters"] >= stats["lanczos_iters"] > 0) if prec else stats["heff_f32_iters"] == 0
    _check(chains, 2, prec, 40, Es, logs, chi_min=40)


@pytest.mark.parametrize("tile", [64, 128])
def test_forced_tiles_match_oracle(tile, tmp_path):
    """Every grouped GEMM on one tile size (autotuner table forced), chi pinned at 40 so that both the
    short-theta and the grouped H_eff paths run: both tile sizes must reproduce the oracle."""
    import paper_2604_03960_amd as tna
    table = tmp_path / "tiles.txt"
    table.write_text("".join(f"{op} {b} {tile}\n" for op in range(7) for b in range(64)))
    tna.autotune_clear()
    tna.autotune_load(str(table))
    try:
        chains = _chains(3, (14, 16), seed=7)
        Es, logs, stats = _run(chains, 2, 0, chi_max=40, chi_min=40)
        assert stats["graph_launches"] > 0 and stats["autotune_entries"] == 7 * 64
        _check(chains, 2, 0, 40, Es, logs, chi_min=40)
    finally:
        tna.autotune_clear()
