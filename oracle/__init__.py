"""Plain FP64 CPU oracle for the two-site DMRG step with the entropy-EMA-PID
bond-dimension controller (arXiv 2604.03960).

TEST INFRASTRUCTURE ONLY: only tests/, the smoke check in __graft_entry__ and
the CPU-baseline leg of bench.py may import this package.  The GPU library never
loads it.  The arithmetic lives in oracle.c (plain C, no BLAS/LAPACK); this file
only marshals arguments.  See oracle.c for the definitions and their citations.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_SRCS = [_SRC, os.path.join(_HERE, "circuit.c")]
# A checking build of the same sources (extra compiler flags, a library name of its own) is
# selected through the environment: TNA_ORACLE_EXTRA_CFLAGS and TNA_ORACLE_LIB_SUFFIX.
_EXTRA = os.environ.get("TNA_ORACLE_EXTRA_CFLAGS", "").split()
_LIB = os.path.join(_HERE, "liboracle%s.so" % os.environ.get("TNA_ORACLE_LIB_SUFFIX", ""))

CFLAGS = ["-O2", "-fPIC", "-shared", "-std=c11", "-ffp-contract=off", "-fno-fast-math"]

LOG_FIELDS = 50
LOG_NAMES = ["sweep", "dir", "bond", "m", "n", "k", "chi_ctrl", "E", "S", "S_ema", "eps", "wdisc", "gap",
             "lanczos_iters", "svd_sweeps", "P", "I", "D", "u", "lanczos_ok", "sigma0", "sigma_kept_last",
             "k_needed", "chi_sched", "fallback"]  # then 25 scheduler inputs ("feat")

MODEL_XXZ, MODEL_J1J2, MODEL_TFIM = 0, 1, 2


def build(force: bool = False) -> str:
    """Compile oracle.c into liboracle.so with gcc."""
    if force or _EXTRA or not os.path.exists(_LIB) or \
            os.path.getmtime(_LIB) < max(os.path.getmtime(f) for f in _SRCS):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", *CFLAGS, *_EXTRA, "-o", tmp, *_SRCS, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class PidParams(C.Structure):
    _fields_ = [("kp", C.c_double), ("ki", C.c_double), ("kd", C.c_double), ("s_target", C.c_double),
                ("alpha", C.c_double), ("beta", C.c_double), ("chi_min", C.c_int), ("chi_max", C.c_int),
                ("ema_init_zero", C.c_int), ("pad", C.c_int), ("beta2", C.c_double)]


class PidState(C.Structure):
    _fields_ = [("s_ema", C.c_double), ("s_ema_prev", C.c_double), ("e_prev", C.c_double),
                ("integ", C.c_double), ("chi", C.c_int), ("visits", C.c_int)]


class DmrgOpts(C.Structure):
    _fields_ = [("n_sweeps", C.c_int), ("lanczos_kmax", C.c_int), ("lanczos_restarts", C.c_int),
                ("fixed_iters", C.c_int), ("lanczos_tol", C.c_double), ("fixed_chi", C.c_int), ("pad", C.c_int),
                ("chi_rule", C.c_int), ("pad2", C.c_int), ("rule_param", C.c_double),
                ("eps_target", C.c_double), ("sched_pred", C.POINTER(C.c_int))]


class CircuitOpts(C.Structure):
    _fields_ = [("fixed_chi", C.c_int), ("pad", C.c_int)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        _lib = C.CDLL(build())
        dp, ip = C.POINTER(C.c_double), C.POINTER(C.c_int)
        _lib.or_mpo_build.argtypes = [C.c_int, C.c_int, dp, dp]
        _lib.or_mpo_dense.argtypes = [C.c_int, C.c_int, dp, dp]
        _lib.or_ed_apply.argtypes = [C.c_int, C.c_int, dp, dp, dp]
        _lib.or_ed_ground.argtypes = [C.c_int, C.c_int, dp, C.c_double, dp, dp, ip]
        _lib.or_sym_eig_jacobi.argtypes = [C.c_int, dp, dp, dp]
        _lib.or_svd_jacobi.argtypes = [C.c_int, C.c_int, dp, dp, dp, dp, ip]
        _lib.or_spectrum.argtypes = [C.c_int, dp, C.c_int, dp]
        _lib.or_spectrum.restype = None
        _lib.or_pid_update.argtypes = [C.POINTER(PidParams), C.POINTER(PidState), C.c_double, ip, dp]
        _lib.or_entropy_chi_update.argtypes = [C.POINTER(PidParams), C.c_double, C.POINTER(PidState), C.c_double,
                                               ip, dp]
        _lib.or_heff_apply.argtypes = [C.c_int] * 4 + [dp] * 6
        _lib.or_heff_element.argtypes = [C.c_int] * 4 + [dp] * 5 + [C.c_int] * 4
        _lib.or_heff_element.restype = C.c_double
        _lib.or_env_left.argtypes = [C.c_int] * 4 + [dp] * 4
        _lib.or_env_right.argtypes = [C.c_int] * 4 + [dp] * 4
        _lib.or_lanczos_heff.argtypes = [C.c_int] * 4 + [dp] * 5 + [C.c_double, C.c_int, C.c_int, C.c_int, dp, ip]
        _lib.or_dmrg_run.argtypes = [C.c_int, C.c_int, C.c_int, dp, dp, ip, C.POINTER(PidParams),
                                     C.POINTER(DmrgOpts), dp, dp, ip, C.POINTER(PidState)]
        _lib.or_right_canonical.argtypes = [C.c_int, C.c_int, dp, ip, dp, ip]
        _lib.or_sched_features.argtypes = [dp, C.c_int, dp, C.c_int, C.c_int, C.c_int, dp]
        _lib.or_sched_features.restype = None
        _lib.or_trunc_error.argtypes = [C.c_int, dp, C.c_int]
        _lib.or_trunc_error.restype = C.c_double
        _lib.or_k_needed.argtypes = [C.c_int, dp, C.c_double]
        _lib.or_mlp_forward.argtypes = [dp, C.c_int, dp, dp]
        _lib.or_mlp_forward.restype = None
        _lib.or_mlp_loss_grad.argtypes = [dp, C.c_int, dp, dp, dp]
        _lib.or_mlp_loss_grad.restype = C.c_double
        _lib.or_adam_step.argtypes = [C.c_int, dp, dp, dp, dp, C.c_int, C.c_double, C.c_double, C.c_double,
                                      C.c_double]
        _lib.or_adam_step.restype = None
        _lib.or_circuit_gates.argtypes = [C.c_int, C.c_int]
        _lib.or_circuit_statevector.argtypes = [C.c_int, C.c_int, ip, dp, dp]
        _lib.or_circuit_statevector.restype = None
        _lib.or_circuit_run.argtypes = [C.c_int, C.c_int, ip, dp, C.POINTER(PidParams), C.POINTER(CircuitOpts), dp, ip,
                                        dp, C.c_size_t, ip, dp, C.c_size_t]
        _lib.or_mps_amplitudes.argtypes = [C.c_int, dp, ip, dp]
        _lib.or_mps_amplitudes.restype = None
    return _lib


def _p(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _ip(a):
    return a.ctypes.data_as(C.POINTER(C.c_int))


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


# ---------------------------------------------------------------- models
def mpo(model: int, N: int, params) -> np.ndarray:
    """N bulk MPO tensors, shape (N, D, D, 2, 2); boundaries select row D-1 / column 0."""
    D = {MODEL_XXZ: 5, MODEL_J1J2: 8, MODEL_TFIM: 3}[model]
    p = _f64(list(params) + [0.0] * (3 - len(params)))
    W = np.zeros((N, D, D, 2, 2))
    rc = lib().or_mpo_build(model, N, _p(p), _p(W))
    assert rc == D
    return W


def mpo_dense(W: np.ndarray) -> np.ndarray:
    N, D = W.shape[0], W.shape[1]
    H = np.zeros((2 ** N, 2 ** N))
    assert lib().or_mpo_dense(N, D, _p(_f64(W)), _p(H)) == 0
    return H


def ed_apply(model: int, N: int, params, x: np.ndarray) -> np.ndarray:
    p = _f64(list(params) + [0.0] * (3 - len(params)))
    y = np.zeros(2 ** N)
    assert lib().or_ed_apply(model, N, _p(p), _p(_f64(x)), _p(y)) == 0
    return y


def ed_ground(model: int, N: int, params, tol: float = 1e-13):
    p = _f64(list(params) + [0.0] * (3 - len(params)))
    E = np.zeros(1)
    psi = np.zeros(2 ** N)
    psi[:] = 1.0 + 0.37 * np.sin(1.7 * np.arange(2 ** N) + 0.3) + 1e-3 * (np.arange(2 ** N) % 7)
    it = np.zeros(1, dtype=np.int32)
    rc = lib().or_ed_ground(model, N, _p(p), tol, _p(E), _p(psi), _ip(it))
    return float(E[0]), psi, int(it[0]), rc


# ---------------------------------------------------------------- linear algebra
def sym_eig(A: np.ndarray):
    n = A.shape[0]
    a = _f64(A).copy()
    w = np.zeros(n)
    V = np.zeros((n, n))
    rc = lib().or_sym_eig_jacobi(n, _p(a), _p(w), _p(V))
    return w, V, rc


def svd(A: np.ndarray):
    """One-sided Jacobi SVD: returns (S, U, V, sweeps, rc); A = U diag(S) V^T."""
    A = _f64(A)
    m, n = A.shape
    R = min(m, n)
    S, U, V = np.zeros(R), np.zeros((m, R)), np.zeros((n, R))
    info = np.zeros(1, dtype=np.int32)
    rc = lib().or_svd_jacobi(m, n, _p(A), _p(S), _p(U), _p(V), _ip(info))
    return S, U, V, int(info[0]), rc


def spectrum(S: np.ndarray, k: int):
    """(Z, entropy, eps, discarded weight) of Eq. (4)-(5)."""
    out = np.zeros(4)
    S = _f64(S)
    lib().or_spectrum(len(S), _p(S), int(k), _p(out))
    return tuple(float(v) for v in out)


def pid_params(kp, ki, kd, s_target, alpha, chi_min, chi_max, beta=0.0, ema_init_zero=False,
               beta2=0.0) -> PidParams:
    return PidParams(kp, ki, kd, s_target, alpha, beta, chi_min, chi_max, int(ema_init_zero), 0, beta2)


def pid_update(pp: PidParams, st: PidState, s_raw: float):
    chi = C.c_int(0)
    terms = np.zeros(6)
    rc = lib().or_pid_update(C.byref(pp), C.byref(st), float(s_raw), C.byref(chi), _p(terms))
    assert rc == 0
    return chi.value, dict(P=terms[0], I=terms[1], D=terms[2], u=terms[3], sbar=terms[4], e=terms[5])


def entropy_chi_update(pp: PidParams, gamma: float, st: PidState, s_raw: float):
    """Algorithm 1 (Sec. 4, Eq. 6-8): EMA of the entropy, chi = clamp(ceil(gamma exp(S_ema)))."""
    chi = C.c_int(0)
    terms = np.zeros(6)
    rc = lib().or_entropy_chi_update(C.byref(pp), C.c_double(gamma), C.byref(st), C.c_double(s_raw), C.byref(chi),
                                     _p(terms))
    if rc != 0:
        raise ValueError("entropy rule: bad arguments")
    return chi.value, float(terms[4])


def heff_apply(L, W1, W2, R, theta):
    chl, D, _ = L.shape
    chr_ = R.shape[0]
    d = W1.shape[2]
    out = np.zeros((chl, d, d, chr_))
    lib().or_heff_apply(chl, chr_, d, D, _p(_f64(L)), _p(_f64(W1)), _p(_f64(W2)), _p(_f64(R)),
                        _p(_f64(theta)), _p(out))
    return out


def heff_element(L, W1, W2, R, theta, idx):
    """One element (a, s, t, c) of H_eff theta from the definition (for large chi)."""
    chl, D, _ = L.shape
    chr_ = R.shape[0]
    d = W1.shape[2]
    a, s, t, c = (int(x) for x in idx)
    return lib().or_heff_element(chl, chr_, d, D, _p(_f64(L)), _p(_f64(W1)), _p(_f64(W2)), _p(_f64(R)),
                                 _p(_f64(theta)), a, s, t, c)


def env_left(L, W, A):
    chl, d, chn = A.shape
    D = W.shape[0]
    out = np.zeros((chn, D, chn))
    lib().or_env_left(chl, chn, d, D, _p(_f64(L)), _p(_f64(W)), _p(_f64(A)), _p(out))
    return out


def env_right(R, W, B):
    chn, d, chr_ = B.shape
    D = W.shape[0]
    out = np.zeros((chn, D, chn))
    lib().or_env_right(chn, chr_, d, D, _p(_f64(R)), _p(_f64(W)), _p(_f64(B)), _p(out))
    return out


def lanczos_heff(L, W1, W2, R, theta0, tol=1e-12, kmax=100, restarts=5, fixed_iters=0):
    chl, D, _ = L.shape
    chr_ = R.shape[0]
    d = W1.shape[2]
    th = _f64(theta0).copy()
    E = np.zeros(1)
    it = np.zeros(1, dtype=np.int32)
    rc = lib().or_lanczos_heff(chl, chr_, d, D, _p(_f64(L)), _p(_f64(W1)), _p(_f64(W2)), _p(_f64(R)), _p(th),
                               tol, kmax, restarts, fixed_iters, _p(E), _ip(it))
    return float(E[0]), th.reshape(chl, d, d, chr_), int(it[0]), rc


def right_canonical(N, d, A_packed, chi):
    A_out = np.zeros_like(_f64(A_packed))
    chi_out = np.zeros(N - 1, dtype=np.int32)
    lib().or_right_canonical(N, d, _p(_f64(A_packed)), _ip(np.asarray(chi, dtype=np.int32)), _p(A_out),
                             _ip(chi_out))
    return A_out, chi_out


def dmrg_run(W, A_packed, chi_init, pp: PidParams, n_sweeps, lanczos_tol=1e-12, kmax=100, restarts=5,
             fixed_iters=0, fixed_chi=0, chi_rule=0, rule_param=0.0, eps_target=1e-8, sched_pred=None):
    """Runs the two-site DMRG; returns dict(log=[records], E=[per sweep], chi=[final], pid=[states], rc).
    sched_pred: optional rank proposal per visit in run order (0 = none), applied with the scheduler's
    fallback rule (the proposals are inputs; no network runs here)."""
    W = _f64(W)
    N, D, _, d, _ = W.shape
    nrec = n_sweeps * 2 * (N - 1)
    pred = None
    if sched_pred is not None:
        pred = np.ascontiguousarray(sched_pred, dtype=np.int32)
        assert pred.shape == (nrec,)
    opts = DmrgOpts(n_sweeps, kmax, restarts, fixed_iters, lanczos_tol, fixed_chi, 0, chi_rule, 0, rule_param,
                    eps_target, _ip(pred) if pred is not None else None)
    log = np.zeros((nrec, LOG_FIELDS))
    E = np.zeros(n_sweeps)
    chi = np.zeros(N - 1, dtype=np.int32)
    pid = (PidState * (N - 1))()
    rc = lib().or_dmrg_run(N, d, D, _p(W), _p(_f64(A_packed)), _ip(np.asarray(chi_init, dtype=np.int32)),
                           C.byref(pp), C.byref(opts), _p(log), _p(E), _ip(chi), pid)
    recs = []
    for row in log:
        r = dict(zip(LOG_NAMES, row))
        r["feat"] = row[25:50].copy()
        recs.append(r)
    return dict(log=recs, log_array=log, E=E, chi=chi, pid=pid, rc=rc)


# ---------------------------------------------------------------- learned-scheduler inputs and labels
def sched_features(ema_hist, S, bond: int, N: int) -> np.ndarray:
    """The 25 scheduler inputs of one visit: last 8 EMA entropies of the bond (oldest first, front-padded
    with the oldest), ln of the 16 largest singular values floored at ln 1e-16, (bond + 1) / N."""
    h = _f64(ema_hist)
    S = _f64(S)
    f = np.zeros(25)
    lib().or_sched_features(_p(h), len(h), _p(S), len(S), int(bond), int(N), _p(f))
    return f


def trunc_error(S, k: int) -> float:
    """Eq. (4) with k values kept."""
    S = _f64(S)
    return float(lib().or_trunc_error(len(S), _p(S), int(k)))


def k_needed(S, eps_target: float) -> int:
    """Smallest k >= 1 whose truncation error (Eq. 4) is at most eps_target."""
    S = _f64(S)
    return int(lib().or_k_needed(len(S), _p(S), float(eps_target)))


# ---------------------------------------------------------------- learned scheduler (MLP)
MLP_IN, MLP_H = 25, 64
MLP_NPARAM = MLP_H * MLP_IN + MLP_H + MLP_H * MLP_H + MLP_H + MLP_H + 1


def mlp_forward(params, x):
    x = _f64(np.atleast_2d(x))
    y = np.zeros(x.shape[0])
    lib().or_mlp_forward(_p(_f64(params)), x.shape[0], _p(x), _p(y))
    return y


def mlp_loss_grad(params, x, t):
    x = _f64(np.atleast_2d(x))
    g = np.zeros(MLP_NPARAM)
    loss = lib().or_mlp_loss_grad(_p(_f64(params)), x.shape[0], _p(x), _p(_f64(t)), _p(g))
    return float(loss), g


def adam_step(params, g, m, v, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """In place on params, m, v (float64 arrays)."""
    lib().or_adam_step(len(params), _p(params), _p(_f64(g)), _p(m), _p(v), int(t), lr, b1, b2, eps)


# ---------------------------------------------------------------- circuits with adaptive bond dimensions (Sec. 8)
CIRC_LOG_NAMES = ["op", "bond", "m", "n", "k", "chi_ctrl", "S", "S_ema", "eps", "wdisc", "gap", "sigma0",
                  "sigma_last", "u", "svd_sweeps", "Z"]


def circuit_statevector(N: int, parity, gates, psi0=None) -> np.ndarray:
    """Exact state vector after the ops (qubit 0 the most significant bit); starts from |0...0>."""
    par = np.ascontiguousarray(parity, dtype=np.int32)
    psi = np.zeros(1 << N)
    if psi0 is None:
        psi[0] = 1.0
    else:
        psi[:] = psi0
    lib().or_circuit_statevector(N, len(par), _ip(par), _p(_f64(gates)), _p(psi))
    return psi


def circuit_run(N: int, parity, gates, pp: PidParams, fixed_chi: int = 0):
    """The adaptive-chi MPS simulation of the ops from |0...0>: dict(log=[per-gate records], chimap (ops x
    N-1), B (packed site tensors), chi (N-1), lam (list of Schmidt-value arrays))."""
    par = np.ascontiguousarray(parity, dtype=np.int32)
    ngate = sum(int(lib().or_circuit_gates(N, int(p))) for p in par)
    log = np.zeros((ngate, len(CIRC_LOG_NAMES)))
    chimap = np.zeros((len(par), N - 1), dtype=np.int32)
    cap = 2 * N * 4096 * 4096 if N > 24 else 2 * N * (1 << N)
    cap = min(cap, 1 << 26)
    B = np.zeros(cap)
    lam = np.zeros(N * 4096)
    chi = np.zeros(N - 1, dtype=np.int32)
    rc = lib().or_circuit_run(N, len(par), _ip(par), _p(_f64(gates)), C.byref(pp), C.byref(CircuitOpts(fixed_chi, 0)),
                              _p(log), _ip(chimap), _p(B), cap, _ip(chi), _p(lam), len(lam))
    if rc != 0:
        raise ValueError("circuit_run: output capacity too small")
    recs = [dict(zip(CIRC_LOG_NAMES, row)) for row in log]
    n_b = sum((1 if i == 0 else int(chi[i - 1])) * 2 * (1 if i == N - 1 else int(chi[i])) for i in range(N))
    lams, off = [], 0
    for b in range(N - 1):
        lams.append(lam[off:off + chi[b]].copy())
        off += chi[b]
    return dict(log=recs, chimap=chimap, B=B[:n_b].copy(), chi=chi, lam=lams)


def mps_amplitudes(N: int, A_packed, chi) -> np.ndarray:
    """psi(s_0..s_{N-1}) of an open-chain MPS (d = 2) by contraction, N <= 24."""
    psi = np.zeros(1 << N)
    lib().or_mps_amplitudes(N, _p(_f64(A_packed)), _ip(np.asarray(chi, dtype=np.int32)), _p(psi))
    return psi
