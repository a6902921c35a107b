"""Truncated SVD + spectrum sums on the GPU vs the oracle and closed forms."""
import math

import numpy as np
import pytest

import oracle
import synth
from gpu_common import ctx, to_dev

pytestmark = pytest.mark.gpu
EPS = 2.0 ** -53


def _svd(c, A, k):
    S, U, Vt, spec, kk, sw, st = c.svd_truncate(to_dev(A), k)
    return S.cpu().numpy(), U.cpu().numpy(), Vt.cpu().numpy(), spec.cpu().numpy(), kk, sw, st


@pytest.mark.parametrize("m,n", [(1, 1), (2, 8), (8, 2), (5, 7), (33, 33), (64, 100), (100, 64), (130, 70),
                                 (97, 300), (256, 256), (300, 520), (600, 280)])
def test_svd_matches_oracle(m, n):
    """Shapes span the fused single-workgroup Jacobi (min(m, n) <= 64), the blocked path, and the
    pivoted-QR start (min(m, n) >= 256), with the rows of A and of A^T."""
    A = synth.random_matrix(m, n, 100 + m + 7 * n)
    c = ctx()
    R = min(m, n)
    k = max(1, (2 * R) // 3)
    S, U, Vt, spec, kk, sw, st = _svd(c, A, k)
    So, Uo, Vo, swo, rc = oracle.svd(A)
    print(f"svd {m}x{n} k={kk} sweeps gpu={sw} oracle={swo} max|dS|={np.abs(S - So).max():.3e}")
    assert st == 0 and kk == k
    assert np.abs(S - So).max() <= 1e-12 * So[0]
    # factors: reconstruction of the kept part, orthonormality, gauge-identical columns
    tol = 64 * max(m, n) * EPS
    assert np.abs(U.T @ U - np.eye(k)).max() <= tol
    assert np.abs(Vt @ Vt.T - np.eye(k)).max() <= tol
    assert np.abs((U * S[:k]) @ Vt - (Uo[:, :k] * So[:k]) @ Vo[:, :k].T).max() <= tol * So[0]
    gaps = np.abs(np.diff(So[:k + 1])) / So[0] if k < R else np.abs(np.diff(So[:k])) / So[0]
    if gaps.size == 0 or gaps.min() > 1e-6:
        assert np.abs(U - Uo[:, :k]).max() <= 1e-9
        assert np.abs(Vt - Vo[:, :k].T).max() <= 1e-9
    # spectrum sums vs the oracle's
    Z, ent, eps, w = oracle.spectrum(So, k)
    # Z and S follow from the spectrum, which matches to 1e-12 sigma_0: |dZ| <= 2 sum sigma |dsigma|
    assert abs(spec[0] - Z) <= 2e-12 * So[0] * So.sum()
    assert abs(spec[1] - ent) <= 1e-10 * max(1.0, ent)
    assert abs(spec[2] - eps) <= 1e-10 * max(eps, 1e-300) + 1e-14 * So[0]


@pytest.mark.parametrize("n,tau", [(512, 8.0), (512, 64.0)])
def test_prescribed_spectrum_c3_small(n, tau):
    A = synth.svd_test_matrix(n, tau, seed=0)
    c = ctx()
    S, U, Vt, spec, kk, sw, st = _svd(c, A, n // 2)
    sig = synth.svd_test_spectrum(n, tau)
    So = oracle.svd(A)[0]
    print(f"c3 n={n} tau={tau} sweeps={sw} max|S-sig|={np.abs(S - sig).max():.3e} max|S-So|={np.abs(S - So).max():.3e}")
    assert np.abs(S - sig).max() <= 64 * n * EPS
    big = So >= 1e-4 * So[0]
    assert np.all(np.abs(S[big] - So[big]) <= 1e-10 * So[big])
    q = math.exp(-2.0 / tau)
    ent = -math.log((1 - q) / (1 - q ** n)) - (q / (1 - q) - n * q ** n / (1 - q ** n)) * math.log(q)
    assert abs(spec[1] - ent) <= 1e-10


def test_svd_rank_deficient_and_zero():
    c = ctx()
    x, y = synth.random_matrix(40, 1, 1), synth.random_matrix(1, 24, 2)
    S, U, Vt, spec, kk, sw, st = _svd(c, x @ y, 5)
    assert abs(S[0] - np.linalg.norm(x) * np.linalg.norm(y)) <= 1e-13 * S[0]
    assert np.all(S[1:] <= 1e-13 * S[0])
    assert np.abs(U.T @ U - np.eye(5)).max() <= 1e-12
    assert np.abs(Vt @ Vt.T - np.eye(5)).max() <= 1e-12
    S, U, Vt, spec, kk, sw, st = _svd(c, np.zeros((6, 9)), 3)
    assert np.all(S == 0)
    assert np.abs(Vt @ Vt.T - np.eye(3)).max() <= 1e-14


@pytest.mark.parametrize("m,n,k", [(70, 90, 20), (270, 300, 100)])
def test_svd_batched_equals_single(m, n, k):
    c = ctx()
    As = np.stack([synth.random_matrix(m, n, 200 + i) for i in range(4)])
    S, U, Vt, spec, sw, st = c.svd_truncate_batched(to_dev(As), k)
    for i in range(4):
        S1, U1, Vt1, spec1, _, _, _ = _svd(c, As[i], k)
        assert np.abs(S[i].cpu().numpy() - S1).max() <= 1e-13 * S1[0]
        assert np.abs(U[i].cpu().numpy() - U1).max() <= 1e-10


def test_svd_f32_input():
    import torch
    c = ctx()
    A = synth.svd_test_matrix(128, 8.0, seed=1)
    A32 = A.astype(np.float32)
    S, U, Vt, spec, kk, sw, st = c.svd_truncate(torch.from_numpy(A32).cuda(), 64)
    So = oracle.svd(A32.astype(np.float64))[0]
    assert U.dtype == torch.float32
    assert np.abs(S.cpu().numpy() - So).max() <= 1e-12 * So[0]


def test_prescribed_spectrum_chi1024_closed_form():
    """2048 x 2048 (chi = 1024, the QR-started blocked path): sigma against the closed form exp(-k/64),
    the kept factors orthonormal and reconstructing the kept part."""
    import torch
    n, tau, k = 2048, 64.0, 1024
    A = synth.svd_test_matrix(n, tau, seed=0)
    c = ctx()
    S, U, Vt, spec, kk, sw, st = c.svd_truncate(torch.from_numpy(A).cuda(), k)
    sig = synth.svd_test_spectrum(n, tau)
    assert st == 0 and kk == k
    assert np.abs(S.cpu().numpy() - sig).max() <= 64 * n * EPS
    eye = torch.eye(k, dtype=torch.float64, device="cuda")
    assert (U.T @ U - eye).abs().max().item() <= 64 * n * EPS
    assert (Vt @ Vt.T - eye).abs().max().item() <= 64 * n * EPS
    # (U S_k) Vt equals A minus its discarded part: project A onto the kept left vectors
    Ad = torch.from_numpy(A).cuda()
    rec = (U * S[:k]) @ Vt
    assert (rec - U @ (U.T @ Ad)).abs().max().item() <= 64 * n * EPS


def test_svd_batched_c3_against_closed_form_and_oracle():
    """The isolated-SVD configuration at batch 16: sixteen 512 x 512 FP64 matrices (chi = 256) with
    spectra exp(-k/8) and exp(-k/64) alternating, one batched call.  Every member's sigma against the
    closed form, its kept factors orthonormal and reconstructing the kept part of A, its entropy
    against the closed form; member 1 (tau = 64) against the oracle's Jacobi SVD as well."""
    import torch
    n, k, B = 512, 256, 16
    taus = [8.0 if i % 2 == 0 else 64.0 for i in range(B)]
    As = np.stack([synth.svd_test_matrix(n, taus[i], seed=0, index=i) for i in range(B)])
    c = ctx()
    Ad = torch.from_numpy(As).cuda()
    S, U, Vt, spec, sw, st = c.svd_truncate_batched(Ad, k)
    assert st == 0
    eye = torch.eye(k, dtype=torch.float64, device="cuda")
    for i in range(B):
        sig = synth.svd_test_spectrum(n, taus[i])
        Si = S[i].cpu().numpy()
        assert np.abs(Si - sig).max() <= 64 * n * EPS, (i, np.abs(Si - sig).max())
        assert (U[i].T @ U[i] - eye).abs().max().item() <= 64 * n * EPS
        assert (Vt[i] @ Vt[i].T - eye).abs().max().item() <= 64 * n * EPS
        rec = (U[i] * S[i, :k]) @ Vt[i]
        assert (rec - U[i] @ (U[i].T @ Ad[i])).abs().max().item() <= 64 * n * EPS
        q = math.exp(-2.0 / taus[i])
        ent = -math.log((1 - q) / (1 - q ** n)) - (q / (1 - q) - n * q ** n / (1 - q ** n)) * math.log(q)
        assert abs(spec[i, 1].item() - ent) <= 1e-10
    So = oracle.svd(As[1])[0]
    big = So >= 1e-4 * So[0]
    S1 = S[1].cpu().numpy()
    assert np.all(np.abs(S1[big] - So[big]) <= 1e-10 * So[big])


@pytest.mark.parametrize("case", ["single_600x280", "batched_4x300x520", "decaying_1024"])
def test_qr_panel_cooperative_equals_per_column(case, monkeypatch):
    """The QR start's panel factorisation in one cooperative launch per panel (every workgroup
    resident, one grid barrier per column) against one launch per column: the same reflectors from
    the same additions in the same order, so sigma, U, Vt, the spectrum sums and the sweep counts
    agree bit for bit.  TNA_QR_PANEL=coop makes a refused cooperative launch an error, so the first
    call really ran the cooperative form."""
    import torch
    c = ctx()
    if case == "single_600x280":
        As, k = synth.random_matrix(600, 280, 17)[None], 180
    elif case == "batched_4x300x520":
        As, k = np.stack([synth.random_matrix(300, 520, 40 + i) for i in range(4)]), 200
    else:
        As, k = synth.svd_test_matrix(1024, 8.0, seed=3)[None], 512
    Ad = torch.from_numpy(np.ascontiguousarray(As)).cuda()
    outs = {}
    for mode in ("coop", "col"):
        monkeypatch.setenv("TNA_QR_PANEL", mode)
        S, U, Vt, spec, sw, st = c.svd_truncate_batched(Ad, k)
        assert st == 0, (mode, st)
        outs[mode] = [t.cpu().numpy().copy() for t in (S, U, Vt, spec)] + [np.array(sw).copy()]
    print(case, "sweeps", outs["coop"][4], "max sigma", outs["coop"][0].max())
    for a, b in zip(outs["coop"], outs["col"]):
        assert np.array_equal(a, b)
