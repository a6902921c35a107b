"""The C-ABI library loads and exports every entry point include/tna.h declares.
Also compares the two host-only entry points (the MPO builder and the PID
controller, which touch no GPU) with the oracle, bit for bit."""
import os
import re
import subprocess

import numpy as np
import pytest

import oracle
import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "tna.h")


def _declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(tna_[a-z_0-9]+)\s*\(", txt)))


def test_library_exports_every_declared_symbol():
    import paper_2604_03960_amd as tna
    out = subprocess.run(["nm", "-D", "--defined-only", tna.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r" T (tna_\w+)", out))
    missing = [s for s in _declared() if s not in exported]
    assert not missing, missing
    assert set(tna.EXPORTED) <= exported


@pytest.mark.parametrize("model,params", [(0, [1.0, 1.0, 0.0]), (0, [0.8, 1.7, 0.25]), (1, [1.0, 0.241]),
                                          (2, [1.0, 0.6])])
def test_mpo_builder_matches_oracle(model, params):
    import paper_2604_03960_amd as tna
    W = tna.mpo_build(model, 6, params)
    Wo = oracle.mpo(model, 6, params)
    assert np.array_equal(W, Wo)


@pytest.mark.parametrize("seed", range(6))
def test_pid_host_function_bitwise_vs_oracle(seed):
    import paper_2604_03960_amd as tna
    rng_u = synth.uniform53(seed, 0, 64)
    gains = (0.5 + 2 * rng_u[0], 0.2 * rng_u[1], rng_u[2])
    args = dict(s_target=0.3 + rng_u[3], alpha=0.1 + 0.8 * rng_u[4], chi_min=4, chi_max=40,
                beta=0.8 * rng_u[5] if seed % 2 else 0.0, ema_init_zero=seed == 4)
    pp_g = tna.pid_params(*gains, args["s_target"], args["alpha"], args["chi_min"], args["chi_max"],
                          beta=args["beta"], ema_init_zero=args["ema_init_zero"])
    pp_o = oracle.pid_params(*gains, args["s_target"], args["alpha"], args["chi_min"], args["chi_max"],
                             beta=args["beta"], ema_init_zero=args["ema_init_zero"])
    sg, so = tna.PidState(), oracle.PidState()
    sg.chi = so.chi = 4
    for s in 3.0 * rng_u[8:64]:
        cg, tg = tna.pid_chi_update(pp_g, sg, s)
        co, to = oracle.pid_update(pp_o, so, s)
        assert cg == co
        for key in ("P", "I", "D", "u", "sbar", "e"):
            assert tg[key] == to[key]
        assert (sg.s_ema, sg.e_prev, sg.integ, sg.chi, sg.visits) == (so.s_ema, so.e_prev, so.integ, so.chi,
                                                                      so.visits)


def test_pid_rejects_bad_bounds():
    import paper_2604_03960_amd as tna
    with pytest.raises(tna.TnaError) as e:
        tna.pid_chi_update(tna.pid_params(1, 0, 0, 0, 0.5, 10, 5), tna.PidState(), 1.0)
    assert e.value.status == tna.TNA_ERR_ARG
