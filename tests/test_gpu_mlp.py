"""The learned scheduler's FP32 training/inference kernels vs the FP64 oracle."""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu


def _init(seed):
    p = synth.normal(seed, oracle.MLP_NPARAM) * 0.2
    return p


def _data(B, seed):
    x = synth.normal(seed, B * 25).reshape(B, 25)
    t = np.tanh(x[:, 0] - 0.5 * x[:, 3]) + 0.1 * x[:, 7]
    return x, t


@pytest.mark.parametrize("B", [1, 63, 64, 200])
def test_forward_matches_oracle(B):
    import torch
    import paper_2604_03960_amd as tna
    p = _init(1)
    x, _ = _data(B, 2)
    c = tna.Context(0)
    net = tna.Mlp(c, p.astype(np.float32))
    y = net.forward(torch.from_numpy(x.astype(np.float32)).cuda()).cpu().numpy()
    ref = oracle.mlp_forward(p.astype(np.float32).astype(np.float64), x.astype(np.float32).astype(np.float64))
    print(f"mlp fwd B={B} max rel {np.abs(y - ref).max() / np.abs(ref).max():.2e}")
    assert np.abs(y - ref).max() <= 1e-5 * max(1.0, np.abs(ref).max())


@pytest.mark.parametrize("B", [37, 256, 300])
def test_gradient_matches_oracle(B):
    import torch
    import paper_2604_03960_amd as tna
    p = _init(3).astype(np.float32)
    x, t = _data(B, 4)
    x32, t32 = x.astype(np.float32), t.astype(np.float32)
    c = tna.Context(0)
    net = tna.Mlp(c, p)
    loss, g = net.loss_grad(torch.from_numpy(x32).cuda(), torch.from_numpy(t32).cuda())
    lo, go = oracle.mlp_loss_grad(p.astype(np.float64), x32.astype(np.float64), t32.astype(np.float64))
    g = g.cpu().numpy()
    rel = np.abs(g - go).max() / np.abs(go).max()
    print(f"mlp grad B={B} max rel {rel:.2e} loss {loss.item():.6f} vs {lo:.6f}")
    assert rel <= 1e-4
    assert abs(loss.item() - lo) <= 1e-5 * max(1.0, lo)


def test_adam_and_training_track_oracle():
    import torch
    import paper_2604_03960_amd as tna
    p = _init(5).astype(np.float32)
    x, t = _data(256, 6)
    x32, t32 = x.astype(np.float32), t.astype(np.float32)
    c = tna.Context(0)
    net = tna.Mlp(c, p)
    X, T = torch.from_numpy(x32).cuda(), torch.from_numpy(t32).cuda()
    po = p.astype(np.float64).copy()
    m, v = np.zeros_like(po), np.zeros_like(po)
    for step in range(1, 21):
        _, g = net.loss_grad(X, T)
        net.adam_step(g, 3e-3)
        _, go = oracle.mlp_loss_grad(po, x32.astype(np.float64), t32.astype(np.float64))
        oracle.adam_step(po, go, m, v, step, lr=3e-3)
    pg = net.params()
    print("adam param drift", np.abs(pg - po).max())
    assert np.abs(pg - po).max() <= 2e-4
    # full training loop with device permutations reduces the loss
    perm = np.stack([np.argsort(synth.uniform53(100 + e, 0, 256)) for e in range(30)]).astype(np.int32)
    losses = net.train(X, T, torch.from_numpy(perm).cuda(), epochs=30, batch=64, lr=3e-3)
    assert losses[-1] < 0.5 * losses[0]
