"""The whole sweep on the GPU vs the oracle: controller decisions bit for bit,
energies within 1e-10 relative (FP64 H_eff) or 1e-7 (FP32 H_eff)."""
import numpy as np
import pytest

import oracle
import synth
from gpu_common import ctx

pytestmark = pytest.mark.gpu
E12 = -5.142090632840529


def _both(N, chi_init, chi_min, chi_max, sweeps, gains, s_target, model=0, params=(1.0, 1.0, 0.0), prec=0,
          fixed_chi=0):
    import paper_2604_03960_amd as tna
    W = oracle.mpo(model, N, list(params))
    A, chi, _ = synth.random_mps(N, 2, chi_init, 0)
    ro = oracle.dmrg_run(W, A, chi, oracle.pid_params(*gains, s_target, 0.3, chi_min, chi_max), sweeps,
                         fixed_chi=fixed_chi)
    c = ctx()
    dm = tna.Dmrg(c, W, A, chi, tna.pid_params(*gains, s_target, 0.3, chi_min, chi_max), heff_prec=prec,
                  fixed_chi=fixed_chi)
    logs, Es = [], []
    for _ in range(sweeps):
        E, recs, st = dm.sweep()
        Es.append(E)
        logs += recs
    return ro, np.array(Es), logs


def _compare(ro, Es, logs, etol):
    assert len(logs) == len(ro["log"])
    amb = 0
    for g, o in zip(logs, ro["log"]):
        assert (g["bond"], g["dir"]) == (int(o["bond"]), int(o["dir"]))
        if g["chi_ctrl"] != int(o["chi_ctrl"]) or g["k"] != int(o["k"]):
            amb += 1
            assert o["gap"] < 1e-8, (g, o)  # only an ambiguous cut may differ
            break
        assert abs(g["E"] - o["E"]) <= etol * abs(o["E"]), (g["E"], o["E"])
        assert abs(g["S"] - o["S"]) <= 1e-8
    assert np.all(np.abs(Es - ro["E"]) <= etol * np.abs(ro["E"]))
    return amb


def test_c1_heisenberg_n12():
    # Heisenberg J=1, N=12, chi from 8 to 32, EMA 0.3, PID (0.5, 0.05, 0.1), 4 sweeps, Lanczos tol 1e-12
    ro, Es, logs = _both(12, 8, 8, 32, 4, (0.5, 0.05, 0.1), 0.5)
    print("c1 E gpu", Es, "oracle", ro["E"])
    _compare(ro, Es, logs, 1e-10)


def test_untruncated_equals_ed():
    ro, Es, logs = _both(12, 8, 64, 64, 3, (0.5, 0.05, 0.1), 0.5)
    assert abs(Es[-1] - E12) <= 1e-10 * abs(E12)
    _compare(ro, Es, logs, 1e-10)


def test_controller_moving_chi_paper_gains():
    ro, Es, logs = _both(14, 8, 8, 40, 3, (2.0, 0.1, 0.5), 0.3)
    assert max(g["chi_ctrl"] for g in logs) > 8
    _compare(ro, Es, logs, 1e-10)


def test_j1j2_and_xxz_models():
    ro, Es, logs = _both(12, 8, 8, 24, 2, (2.0, 0.1, 0.5), 0.5, model=1, params=(1.0, 0.241))
    _compare(ro, Es, logs, 1e-10)
    ro, Es, logs = _both(12, 8, 8, 24, 2, (2.0, 0.1, 0.5), 0.5, model=0, params=(1.0, 1.5, 0.0))
    _compare(ro, Es, logs, 1e-10)


def test_mixed_precision_energy():
    import paper_2604_03960_amd as tna
    ro, Es, logs = _both(12, 8, 16, 16, 3, (0.5, 0.05, 0.1), 0.5, prec=tna.HEFF_F32)
    print("f32 E", Es, "oracle", ro["E"], "dE/N", (Es - ro["E"]) / 12)
    assert np.all(np.abs(Es - ro["E"]) / 12 <= 1e-7)
