"""The learned scheduler, trained on the method's own sweeps, vs the PID alone.

Training data: PID-only runs of Heisenberg and XXZ chains.  Evaluation: a
J1-J2 chain (J2 = 0.241, not in the training set) run twice from the same
initial state, PID only and PID + learned scheduler (with PID fallback)."""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu
EPS_T = 1e-6
CHI = (8, 48)


def _run(ctx, model, params, N, sweeps, net=None):
    import paper_2604_03960_amd as tna
    W = oracle.mpo(model, N, params)
    A, chi, _ = synth.random_mps(N, 2, CHI[0], seed=N + model)
    dm = tna.Dmrg(ctx, W, A, chi, tna.pid_params(2.0, 0.1, 0.5, 1.0, 0.3, *CHI), eps_target=EPS_T)
    if net is not None:
        dm.set_scheduler(net)
    recs, E = [], None
    for _ in range(sweeps):
        E, r, st = dm.sweep()
        recs += r
    dm.close()
    return E, recs


def test_learned_scheduler_gain():
    import paper_2604_03960_amd as tna
    from paper_2604_03960_amd import scheduler
    ctx = tna.Context(0)
    runs = []
    for model, params, N in [(0, [1, 1, 0], 16), (0, [1, 1, 0], 20), (0, [1, 0.5, 0], 20), (0, [1, 1.5, 0], 18),
                             (0, [1, 0.8, 0], 22)]:
        _, recs = _run(ctx, model, params, N, 4)
        runs.append(recs)
    X, T = scheduler.build_dataset(runs, *CHI)
    assert X.shape[0] > 200
    net, losses = scheduler.train(ctx, X, T, epochs=150, batch=128, lr=2e-3, seed=1)
    print(f"dataset {X.shape[0]} samples; loss {losses[0]:.4f} -> {losses[-1]:.4f}")
    assert losses[-1] < 0.5 * losses[0]
    # held-out model: J1-J2 at J2 = 0.241
    E_pid, r_pid = _run(ctx, 1, [1.0, 0.241], 20, 4)
    E_ml, r_ml = _run(ctx, 1, [1.0, 0.241], 20, 4, net=net)
    E_ref, _ = _run(ctx, 1, [1.0, 0.241], 20, 3)  # same controller, for the drift check
    s_pid = scheduler.summarize(r_pid[-38:], EPS_T)  # last sweep
    s_ml = scheduler.summarize(r_ml[-38:], EPS_T)
    print("PID only   ", s_pid, "E", E_pid)
    print("PID+learned", s_ml, "E", E_ml)
    # the gain: the error target is met on more visits, and the energy is lower
    assert s_ml["frac_eps_ok"] > s_pid["frac_eps_ok"]
    assert E_ml <= E_pid + 1e-10
    assert s_ml["scheduler_visits"] > 0
