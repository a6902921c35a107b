"""H_eff (Eq. 18) on the GPU vs the oracle, element by element."""
import numpy as np
import pytest

import oracle
from gpu_common import ctx, env_pair, to_dev

pytestmark = pytest.mark.gpu

SHAPES = [(1, 1), (1, 8), (8, 1), (7, 9), (16, 16), (33, 65), (64, 64), (130, 97), (200, 256)]


@pytest.mark.parametrize("chl,chr_", SHAPES)
@pytest.mark.parametrize("model,params", [(0, [1.0, 1.0, 0.0]), (1, [1.0, 0.241])])
def test_heff_f64_matches_oracle(chl, chr_, model, params):
    import paper_2604_03960_amd as tna
    W, L, R, th = env_pair(model, params, chl, chr_, 10 + chl + chr_)
    c = ctx()
    out = c.heff_apply(to_dev(L), to_dev(W[1]), to_dev(W[2]), to_dev(R), to_dev(th), prec=tna.HEFF_F64)
    ref = oracle.heff_apply(L, W[1], W[2], R, th)
    got = out.cpu().numpy()
    scale = np.abs(L).max() * np.abs(R).max() * np.abs(th).max() * max(chl, chr_) * 8
    print(f"heff f64 chl={chl} chr={chr_} model={model} max|d|={np.abs(got - ref).max():.3e} scale={scale:.3e}")
    assert np.abs(got - ref).max() <= 1e-14 * scale


@pytest.mark.parametrize("chl,chr_", [(16, 16), (64, 64), (130, 97)])
def test_heff_f32_error_bound(chl, chr_):
    import paper_2604_03960_amd as tna
    W, L, R, th = env_pair(0, [1.0, 1.0, 0.0], chl, chr_, 3)
    c = ctx()
    out = c.heff_apply(to_dev(L), to_dev(W[1]), to_dev(W[2]), to_dev(R), to_dev(th), prec=tna.HEFF_F32)
    ref = oracle.heff_apply(L, W[1], W[2], R, th)
    got = out.cpu().numpy()
    scale = np.abs(L).max() * np.abs(R).max() * np.abs(th).max() * max(chl, chr_) * 8
    err = np.abs(got - ref).max()
    print(f"heff f32 chl={chl} chr={chr_} max|d|={err:.3e} scale={scale:.3e}")
    assert err <= 2e-6 * scale
    assert err > 0.0  # it really ran in FP32


def test_heff_rejects_alias_and_bad_dims():
    import paper_2604_03960_amd as tna
    W, L, R, th = env_pair(0, [1.0, 1.0, 0.0], 4, 4, 1)
    c = ctx()
    t = to_dev(th)
    with pytest.raises(tna.TnaError) as e:
        c.heff_apply(to_dev(L), to_dev(W[1]), to_dev(W[2]), to_dev(R), t, out=t)
    assert e.value.status == tna.TNA_ERR_ARG


@pytest.mark.parametrize("prec,tol", [(0, 1e-12), (1, 1e-5)])
def test_heff_chi1024_sampled_against_oracle(prec, tol):
    """chi_l = chi_r = 1024 (the c2 throughput shape): 24 sampled output elements against the oracle's
    element-by-element definition; tolerance relative to the RMS of the output."""
    import torch

    import paper_2604_03960_amd as tna
    rng = np.random.default_rng(1024)
    chi, d, D = 1024, 2, 5
    W = oracle.mpo(oracle.MODEL_XXZ, 8, [1.0, 1.0, 0.0])
    L = rng.standard_normal((chi, D, chi)) / chi
    R = rng.standard_normal((chi, D, chi)) / chi
    th = rng.standard_normal((chi, d, d, chi))
    c = tna.Context(0)
    out = c.heff_apply(*(torch.from_numpy(np.ascontiguousarray(x)).cuda() for x in (L, W[3], W[4], R, th)),
                       prec=prec).cpu().numpy()
    rms = np.sqrt(np.mean(out ** 2))
    picks = [tuple(int(v) for v in (rng.integers(chi), rng.integers(d), rng.integers(d), rng.integers(chi)))
             for _ in range(22)] + [(0, 0, 0, 0), (chi - 1, d - 1, d - 1, chi - 1)]
    for idx in picks:
        ref = oracle.heff_element(L, W[3], W[4], R, th, idx)
        assert abs(out[idx] - ref) <= tol * rms, (idx, out[idx], ref)
