"""Pins for the EMA + PID controller (Eq. 8-11, Algorithm 2), traced by hand."""
import pytest

import oracle


def _run(pp, seq, chi0=None):
    st = oracle.PidState()
    st.chi = pp.chi_min if chi0 is None else chi0
    out = []
    for s in seq:
        chi, t = oracle.pid_update(pp, st, s)
        out.append((chi, t))
    return st, out


def test_hand_trace():
    # S_target = 1, alpha = 0.3, gains (0.5, 0.05, 0.1), chi in [8, 32].
    pp = oracle.pid_params(0.5, 0.05, 0.1, 1.0, 0.3, 8, 32)
    st, out = _run(pp, [3, 2, 0, 0, 0])
    sbar = [3.0, 2.7, 1.89, 1.323, 0.9261]
    u = [1.1, 1.005, 0.5935, 0.35045, 0.165315]
    assert [c for c, _ in out] == [9, 10, 11, 11, 11]
    for (c, t), sb, uu in zip(out, sbar, u):
        assert t["sbar"] == pytest.approx(sb, abs=1e-14)
        assert t["u"] == pytest.approx(uu, abs=1e-14)


def test_ema_init_zero_reading():
    pp = oracle.pid_params(0.5, 0.05, 0.1, 1.0, 0.3, 8, 32, ema_init_zero=True)
    _, out = _run(pp, [3])
    # Sbar = 0.3*3 = 0.9, e = -0.1 -> u = -0.055 -> chi stays 8 (and is not clamped)
    assert out[0][0] == 8
    assert out[0][1]["sbar"] == pytest.approx(0.9, abs=1e-15)


def test_anti_windup_at_chi_max():
    pp = oracle.pid_params(0.5, 0.05, 0.1, 1.0, 0.3, 8, 32)
    st, out = _run(pp, [3, 3, 3], chi0=32)
    assert [c for c, _ in out] == [32, 32, 32]
    assert st.integ == 0.0  # the integral step is undone every time the output clamps


def test_anti_windup_at_chi_min():
    pp = oracle.pid_params(2.0, 0.1, 0.5, 1.0, 0.3, 8, 32)
    st, out = _run(pp, [0.0, 0.0])
    assert [c for c, _ in out] == [8, 8]
    assert st.integ == 0.0


@pytest.mark.parametrize("u,delta", [(0.5, 0), (1.5, 2), (2.5, 2), (-0.5, 0), (-1.5, -2), (0.49, 0), (0.51, 1)])
def test_round_half_to_even(u, delta):
    # Kp = 1, Ki = Kd = 0, S_target = 0: u = e = Sbar = S on the first visit.
    pp = oracle.pid_params(1.0, 0.0, 0.0, 0.0, 0.3, 1, 100)
    _, out = _run(pp, [u], chi0=50)
    assert out[0][0] == 50 + delta


def test_predictor_beta():
    # Eq. (16): S_hat = Sbar + beta (Sbar - Sbar_prev), fed to the error in place of Sbar.
    pp = oracle.pid_params(1.0, 0.0, 0.0, 0.0, 0.5, 1, 100, beta=0.8)
    _, out = _run(pp, [1.0, 3.0], chi0=50)
    # visit 1: Sbar = 1, no trend -> u = 1; visit 2: Sbar = 2, S_hat = 2 + 0.8 = 2.8
    assert out[0][1]["u"] == pytest.approx(1.0)
    assert out[1][1]["e"] == pytest.approx(2.8)
    assert out[1][0] == 51 + 3


# ---- Algorithm 1 (Sec. 4, Eq. 6-8): chi = clamp(ceil(gamma exp(S_ema)), chi_min, chi_max)
def test_entropy_rule_hand_values():
    import math
    pp = oracle.pid_params(0.0, 0.0, 0.0, 0.0, 0.3, 4, 64)
    st = oracle.PidState()
    st.chi = 4
    chi, sbar = oracle.entropy_chi_update(pp, 1.5, st, 1.0)  # first visit seeds the EMA: 1.5 e = 4.08 -> 5
    assert sbar == 1.0 and chi == 5
    chi, sbar = oracle.entropy_chi_update(pp, 1.5, st, 2.0)  # 0.3*2 + 0.7*1 = 1.3; 1.5 e^1.3 = 5.50 -> 6
    assert abs(sbar - 1.3) < 1e-15 and chi == 6
    chi, sbar = oracle.entropy_chi_update(pp, 1.5, st, 12.0)  # 3.6 + 0.91 = 4.51; 1.5 e^4.51 = 136 -> 64
    assert abs(sbar - 4.51) < 1e-14 and chi == 64
    chi, _ = oracle.entropy_chi_update(pp, 2.5, oracle.PidState(), 0.0)  # product state: ceil(2.5) = 3 -> 4
    assert chi == 4
    # ten equal Schmidt weights: S = ln 10, so chi >= e^S = 10 (Eq. 6); margin 1.05 -> ceil(10.5) = 11
    chi, _ = oracle.entropy_chi_update(pp, 1.05, oracle.PidState(), math.log(10.0))
    assert chi == 11


def test_entropy_rule_ema_zero_seed_and_bad_margin():
    pp = oracle.pid_params(0.0, 0.0, 0.0, 0.0, 0.5, 1, 100, ema_init_zero=True)
    chi, sbar = oracle.entropy_chi_update(pp, 1.0, oracle.PidState(), 2.0)  # 0.5*2 + 0.5*0 = 1; ceil(e) = 3
    assert sbar == 1.0 and chi == 3
    with pytest.raises(ValueError):
        oracle.entropy_chi_update(pp, 0.9, oracle.PidState(), 1.0)  # the margin must be >= 1


def test_second_order_predictor():
    # Sec. 7: S_hat = Sbar + beta (Sbar - Sbar(t-1)) + beta2 (Sbar - 2 Sbar(t-1) + Sbar(t-2)), the
    # curvature from the third visit on.  alpha = 1 makes Sbar = S; S = t^2 is then extrapolated
    # exactly one visit ahead with beta = beta2 = 1 (Newton's backward form of the parabola).
    pp = oracle.pid_params(1.0, 0.0, 0.0, 0.0, 1.0, 1, 1000, beta=1.0, beta2=1.0)
    _, out = _run(pp, [0.0, 1.0, 4.0, 9.0], chi0=500)
    # visits: no trend (0); 1 + 1 (no curvature yet); 4 + 3 + 2 = 9; 9 + 5 + 2 = 16
    assert [o[1]["e"] for o in out] == pytest.approx([0.0, 2.0, 9.0, 16.0])


def test_second_order_off_is_linear():
    seq = [0.3, 0.9, 1.4, 1.6, 1.65]
    lin = _run(oracle.pid_params(2.0, 0.1, 0.5, 1.0, 0.3, 4, 64, beta=0.5), seq)[1]
    off = _run(oracle.pid_params(2.0, 0.1, 0.5, 1.0, 0.3, 4, 64, beta=0.5, beta2=0.0), seq)[1]
    on = _run(oracle.pid_params(2.0, 0.1, 0.5, 1.0, 0.3, 4, 64, beta=0.5, beta2=0.7), seq)[1]
    assert [o[1]["e"] for o in lin] == [o[1]["e"] for o in off]
    assert [o[1]["e"] for o in on][:2] == [o[1]["e"] for o in lin][:2]  # no curvature before visit 3
    assert [o[1]["e"] for o in on][2:] != [o[1]["e"] for o in lin][2:]
