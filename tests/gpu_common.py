"""Shared helpers of the GPU parity tests (inputs come from synth only)."""
import numpy as np


def ctx():
    import paper_2604_03960_amd as tna
    return tna.Context(0)


def to_dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def env_pair(model, params, chl, chr_, seed):
    """Random symmetric-in-(bra,ket) environments of the right shapes plus MPO tensors."""
    import oracle
    import synth
    W = oracle.mpo(model, 4, params)
    D = W.shape[1]
    L = synth.normal(seed, chl * D * chl).reshape(chl, D, chl)
    R = synth.normal(seed + 1, chr_ * D * chr_).reshape(chr_, D, chr_)
    L = 0.5 * (L + L.transpose(2, 1, 0))
    R = 0.5 * (R + R.transpose(2, 1, 0))
    th = synth.normal(seed + 2, chl * 4 * chr_).reshape(chl, 2, 2, chr_)
    return W, L, R, th
