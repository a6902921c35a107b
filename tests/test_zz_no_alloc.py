"""The allocation-free H_eff entry point (tna_heff_apply_noalloc) against tna_heff_apply, through the
C ABI: identical kernels, so the outputs must agree bit for bit; two calls in a row, the second with a
smaller shape (the fixed scratch keeps the first call's contents), in FP64 and FP32; a shape beyond the
fixed scratch is refused before any launch."""
import numpy as np
import pytest

import oracle
import synth
from gpu_common import env_pair, to_dev

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("prec", [0, 1])
def test_noalloc_heff_equals_heff_apply(prec):
    import torch
    import paper_2604_03960_amd as tna
    c = tna.Context(0)
    for chl, chr_, seed in [(96, 80, 31), (20, 36, 32)]:  # the second call is the smaller one
        W, L, R, th = env_pair(oracle.MODEL_XXZ, [1.0, 1.0, 0.0], chl, chr_, seed)
        Ld, Rd, thd, W1, W2 = to_dev(L), to_dev(R), to_dev(th), to_dev(W[1]), to_dev(W[2])
        ref = c.heff_apply(Ld, W1, W2, Rd, thd, prec=prec)
        out = torch.full_like(thd, float("nan"))
        c.heff_apply_noalloc(Ld, W1, W2, Rd, thd, out, prec=prec)
        torch.cuda.synchronize()
        assert torch.equal(out, ref), (chl, chr_, (out - ref).abs().max().item())
        if prec == 0:  # and the definition, through the oracle, for the FP64 form
            o = oracle.heff_apply(L, W[1], W[2], R, th)
            assert np.abs(out.cpu().numpy() - o).max() <= 1e-13 * np.abs(o).max()
        assert tna.heff_apply_noalloc_bytes(chl, chr_, 2, 5, prec) <= tna.NOALLOC_SCRATCH_BYTES


def test_noalloc_rejects_oversized_shapes():
    import torch
    import paper_2604_03960_amd as tna
    c = tna.Context(0)
    chi = 1024  # X and Z alone need 2 * 5 * 4 * 1024^2 * 8 bytes = 320 MiB
    assert tna.heff_apply_noalloc_bytes(chi, chi, 2, 5, 0) > tna.NOALLOC_SCRATCH_BYTES
    L = torch.zeros((chi, 5, chi), dtype=torch.float64, device="cuda")
    W1 = torch.zeros((5, 5, 2, 2), dtype=torch.float64, device="cuda")
    th = torch.zeros((chi, 2, 2, chi), dtype=torch.float64, device="cuda")
    out = torch.empty_like(th)
    with pytest.raises(tna.TnaError) as e:
        c.heff_apply_noalloc(L, W1, W1, L, th, out)
    assert e.value.status == tna.TNA_ERR_ARG and "fixed array" in str(e.value)
