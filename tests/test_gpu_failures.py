"""Failure modes of the boundary: non-finite inputs, iteration caps (the best result is still written),
object lifetimes and the order of single visits.  Every condition is forced from the host; every kernel
exits normally."""
import numpy as np
import pytest

import oracle
import synth
from gpu_common import to_dev

pytestmark = pytest.mark.gpu
HEIS = [1.0, 1.0, 0.0]


def _pid(chi_min=4, chi_max=16):
    import paper_2604_03960_amd as tna
    return tna.pid_params(2.0, 0.1, 0.5, 0.5, 0.3, chi_min, chi_max)


def test_nan_in_svd_input_is_reported():
    import paper_2604_03960_amd as tna
    c = tna.Context(0)
    for m, n in [(20, 30), (300, 280)]:  # single-workgroup Jacobi, QR-started blocked Jacobi
        A = synth.random_matrix(m, n, 5)
        A[3, 7] = np.nan
        with pytest.raises(tna.TnaError) as e:
            c.svd_truncate(to_dev(A), 10)
        assert e.value.status == tna.TNA_ERR_NONFINITE
        B = synth.random_matrix(m, n, 6)
        B[m - 1, n - 1] = np.inf
        with pytest.raises(tna.TnaError) as e:
            c.svd_truncate(to_dev(B), 10)
        assert e.value.status == tna.TNA_ERR_NONFINITE
    # the context stays usable
    S, U, Vt, spec, k, sw, st = c.svd_truncate(to_dev(synth.random_matrix(20, 30, 6)), 10)
    assert st == 0 and np.all(np.isfinite(S.cpu().numpy()))


def test_nan_in_initial_mps_is_reported():
    import paper_2604_03960_amd as tna
    c = tna.Context(0)
    N = 8
    W = oracle.mpo(oracle.MODEL_XXZ, N, HEIS)
    A, chi, _ = synth.random_mps(N, 2, 4, 0)
    A = A.copy()
    A[len(A) // 2] = np.nan
    with pytest.raises(tna.TnaError) as e:
        tna.Dmrg(c, W, A, chi, _pid())
    assert e.value.status == tna.TNA_ERR_NONFINITE


def test_svd_sweep_cap_returns_noconv_with_best_result():
    """svd_max_sweeps = 1: the first visit whose Jacobi needs a second sweep makes the sweep report NOCONV;
    the sweep still completes and writes its records, each visit's SVD stopped after one sweep.  (The
    factors of a stopped Jacobi are not both orthonormal, so the state after such a visit is no longer
    in canonical form: the energy is not checked here.)"""
    import paper_2604_03960_amd as tna
    c = tna.Context(0)
    N = 12
    W = oracle.mpo(oracle.MODEL_XXZ, N, HEIS)
    A, chi, _ = synth.random_mps(N, 2, 8, 0)
    dm = tna.Dmrg(c, W, A, chi, _pid(8, 32), svd_max_sweeps=1)
    E, recs, st = dm.sweep()
    assert st == tna.TNA_ERR_NOCONV
    assert len(recs) == 2 * (N - 1) and all(r["svd_sweeps"] <= 1 for r in recs)
    assert any(r["svd_sweeps"] == 1 and min(r["m"], r["n"]) > 1 for r in recs)


def test_lanczos_cap_returns_noconv_with_best_result():
    """lanczos_kmax = 1 with no restarts: one matvec per visit, NOCONV, and the energy written is the
    Rayleigh quotient of the start vector (finite, above the exact ground energy)."""
    import paper_2604_03960_amd as tna
    c = tna.Context(0)
    N = 12
    W = oracle.mpo(oracle.MODEL_XXZ, N, HEIS)
    A, chi, _ = synth.random_mps(N, 2, 8, 0)
    dm = tna.Dmrg(c, W, A, chi, _pid(8, 32), lanczos_kmax=1, lanczos_restarts=0)
    E, recs, st = dm.sweep()
    assert st == tna.TNA_ERR_NOCONV
    assert np.isfinite(E) and E >= -5.142090632840529 - 1e-9
    assert all(r["lanczos_iters"] == 1 and r["lanczos_ok"] == 0 for r in recs if r["m"] * r["n"] > 1)


def test_context_outlives_its_objects():
    """Destroying a context while a run or a network made from it is alive is refused (TNA_ERR_ARG,
    nothing freed); after they are destroyed it succeeds."""
    import paper_2604_03960_amd as tna
    c = tna.Context(0)
    N = 8
    W = oracle.mpo(oracle.MODEL_XXZ, N, HEIS)
    A, chi, _ = synth.random_mps(N, 2, 4, 0)
    dm = tna.Dmrg(c, W, A, chi, _pid())
    net = tna.Mlp(c, np.zeros(tna.MLP_NPARAM, dtype=np.float32))
    with pytest.raises(tna.TnaError) as e:
        c.close()
    assert e.value.status == tna.TNA_ERR_ARG and c.h is not None
    E, recs, st = dm.sweep()  # still usable
    assert np.isfinite(E)
    dm.close()
    with pytest.raises(tna.TnaError):
        c.close()
    net.close()
    c.close()
    assert c.h is None


def test_single_visits_follow_the_centre_and_equal_a_sweep():
    """A sweep made of single visits gives the same energies, ranks and controller decisions, bit for
    bit, as tna_dmrg_sweep from the same state; visits off the orthogonality centre are refused, and so
    is a sweep while the centre is elsewhere.  The environment getter returns the current ones only."""
    import paper_2604_03960_amd as tna
    c = tna.Context(0)
    N = 10
    W = oracle.mpo(oracle.MODEL_XXZ, N, HEIS)
    A, chi, _ = synth.random_mps(N, 2, 8, 1)
    a = tna.Dmrg(c, W, A, chi, _pid(8, 24))
    b = tna.Dmrg(c, W, A, chi, _pid(8, 24))
    Ea, ra, _ = a.sweep()
    rb = []
    for h in (0, 1):
        for step in range(N - 1):
            bond = step if h == 0 else N - 2 - step
            with pytest.raises(tna.TnaError) as e:
                b.visit(bond, 1 - h)  # the other direction needs the centre on the other site
            assert e.value.status == tna.TNA_ERR_ARG
            E, r, st = b.visit(bond, h)
            rb.append(r)
            if h == 0 and step == 3:
                with pytest.raises(tna.TnaError):
                    b.sweep()
                Lb = b.env(0, 4)
                assert Lb.shape[1] == 5 and Lb.shape[0] == Lb.shape[2] == b.state()[0][3]
                with pytest.raises(tna.TnaError):
                    b.env(0, 6)  # left of the centre only
                with pytest.raises(tna.TnaError):
                    b.env(1, 3)  # right of the centre only
    assert b.centre() == 0
    assert E == Ea
    for x, y in zip(ra, rb):
        for key in ("bond", "dir", "k", "chi_ctrl", "E", "S", "lanczos_iters"):
            assert x[key] == y[key], (key, x, y)
    Rb = b.env(1, N - 1).cpu().numpy()  # right boundary: selects MPO column 0
    assert Rb.shape == (1, 5, 1) and Rb.ravel().tolist() == [1.0, 0.0, 0.0, 0.0, 0.0]
