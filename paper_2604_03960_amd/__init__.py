"""Python binding of libtna: the MI355X (gfx950) two-site DMRG hot path with an
entropy-EMA-PID bond-dimension controller (arXiv 2604.03960).

Argument marshalling only: every numerical step runs in the HIP kernels behind
the C ABI declared in include/tna.h.  PyTorch provides device memory and
streams.  Importing this module fails loudly when libtna.so has not been
built (python -m paper_2604_03960_amd.build); there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libtna.so")

TNA_OK, TNA_ERR_ARG, TNA_ERR_NOMEM, TNA_ERR_DEVICE, TNA_ERR_NOCONV, TNA_ERR_NONFINITE, TNA_ERR_UNSUPPORTED = range(7)
F64, F32 = 0, 1
HEFF_F64, HEFF_F32, HEFF_BF16X3 = 0, 1, 2
MODEL_XXZ, MODEL_J1J2, MODEL_TFIM = 0, 1, 2
CHI_PID, CHI_THRESHOLD, CHI_ENTROPY = 0, 1, 2  # rank rules: Algorithm 2, singular values above eps_trunc, Algorithm 1

STATUS_NAMES = {0: "OK", 1: "ERR_ARG", 2: "ERR_NOMEM", 3: "ERR_DEVICE", 4: "ERR_NOCONV", 5: "ERR_NONFINITE",
                6: "ERR_UNSUPPORTED"}


class TnaError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"tna status {STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2604_03960_amd.build` "
                      "(the GPU path has no fallback)")

# torch is loaded before the library so that the process has one HIP runtime: the one torch
# ships, which libtna.so's libamdhip64 dependency then resolves to.  Loaded the other way round,
# a second runtime comes up beside torch's and may not see the device.
import torch  # noqa: E402,F401

_lib = C.CDLL(LIB_PATH)


class PidParams(C.Structure):
    _fields_ = [("kp", C.c_double), ("ki", C.c_double), ("kd", C.c_double), ("s_target", C.c_double),
                ("alpha", C.c_double), ("beta", C.c_double), ("chi_min", C.c_int), ("chi_max", C.c_int),
                ("ema_init_zero", C.c_int), ("pad", C.c_int), ("beta2", C.c_double)]


class PidState(C.Structure):
    _fields_ = [("s_ema", C.c_double), ("s_ema_prev", C.c_double), ("e_prev", C.c_double),
                ("integ", C.c_double), ("chi", C.c_int), ("visits", C.c_int)]


class DmrgOpts(C.Structure):
    _fields_ = [("lanczos_tol", C.c_double), ("lanczos_kmax", C.c_int), ("lanczos_restarts", C.c_int),
                ("lanczos_fixed_iters", C.c_int), ("heff_prec", C.c_int), ("fixed_chi", C.c_int),
                ("svd_max_sweeps", C.c_int), ("eps_target", C.c_double), ("chi_rule", C.c_int), ("pad_", C.c_int),
                ("rule_param", C.c_double)]


class VisitLog(C.Structure):
    _fields_ = [(n, C.c_int) for n in ("sweep", "dir", "bond", "m", "n", "k", "chi_ctrl", "lanczos_iters",
                                       "svd_sweeps", "lanczos_ok")] + \
               [(n, C.c_double) for n in ("E", "S", "S_ema", "eps", "wdisc", "gap", "P", "I", "D", "u", "sigma0",
                                          "sigma_last", "ms_lanczos", "ms_svd", "ms_other")] + \
               [(n, C.c_int) for n in ("k_needed", "chi_sched", "fallback", "pad")] + [("feat", C.c_float * 25)]


class BatchStats(C.Structure):
    _fields_ = [("ms_total", C.c_double), ("ms_lanczos", C.c_double), ("ms_svd", C.c_double), ("ms_env", C.c_double),
                ("lanczos_iters", C.c_long), ("graph_launches", C.c_long), ("small_launches", C.c_long),
                ("heff_f32_iters", C.c_long), ("svd_rows", C.c_long), ("svd_rows_swept", C.c_long),
                ("heff_ident_steps", C.c_long), ("heff_ident_dev", C.c_double),
                ("autotune_entries", C.c_int),
                ("steps", C.c_int)]


class CircuitOpts(C.Structure):
    _fields_ = [("fixed_chi", C.c_int), ("one_at_a_time", C.c_int), ("svd_max_sweeps", C.c_int), ("pad", C.c_int)]


class GateLog(C.Structure):
    _fields_ = [(n, C.c_int) for n in ("layer", "bond", "m", "n", "k", "chi_ctrl", "svd_sweeps", "pad")] + \
               [(n, C.c_double) for n in ("S", "S_ema", "eps", "wdisc", "gap", "sigma0", "sigma_last", "u")]


_vp, _dp, _ip = C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_int)
_SIGS = {
    "tna_create": ([C.POINTER(C.c_void_p), C.c_int, _vp], C.c_int),
    "tna_destroy": ([_vp], C.c_int),
    "tna_set_stream": ([_vp, _vp], C.c_int),
    "tna_synchronize": ([_vp], C.c_int),
    "tna_last_error": ([], C.c_char_p),
    "tna_set_timing": ([_vp, C.c_int, C.c_char_p], C.c_int),
    "tna_kernel_stats": ([_vp, C.c_char_p, C.c_size_t, C.c_int], C.c_int),
    "tna_mpo_build": ([C.c_int, C.c_int, _dp, _dp, _ip], C.c_int),
    "tna_heff_apply": ([_vp, C.c_int, C.c_int, C.c_int, C.c_int, _vp, _vp, _vp, _vp, _vp, _vp, C.c_int], C.c_int),
    "tna_heff_apply_noalloc": ([_vp, C.c_int, C.c_int, C.c_int, C.c_int, _vp, _vp, _vp, _vp, _vp, _vp, C.c_int],
                               C.c_int),
    "tna_heff_apply_noalloc_bytes": ([C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, C.POINTER(C.c_size_t)], C.c_int),
    "tna_svd_truncate": ([_vp, C.c_int, C.c_int, C.c_int, _vp, C.c_int, _vp, _vp, _vp, _vp, _ip, _ip], C.c_int),
    "tna_svd_truncate_batched": ([_vp, C.c_int, C.c_int, C.c_int, C.c_int, _vp, C.c_int64, C.c_int, _vp, C.c_int64,
                                  _vp, C.c_int64, _vp, C.c_int64, _vp, _ip], C.c_int),
    "tna_pid_chi_update": ([C.POINTER(PidParams), C.POINTER(PidState), C.c_double, _ip, _dp], C.c_int),
    "tna_entropy_chi_update": ([C.POINTER(PidParams), C.c_double, C.POINTER(PidState), C.c_double, _ip], C.c_int),
    "tna_dmrg_create": ([_vp, C.c_int, C.c_int, C.c_int, _dp, _dp, _ip, C.POINTER(PidParams), C.POINTER(DmrgOpts),
                         C.POINTER(C.c_void_p)], C.c_int),
    "tna_dmrg_sweep": ([_vp, _dp, C.POINTER(VisitLog)], C.c_int),
    "tna_dmrg_visit": ([_vp, C.c_int, C.c_int, _dp, C.POINTER(VisitLog)], C.c_int),
    "tna_dmrg_centre": ([_vp], C.c_int),
    "tna_dmrg_get_stats": ([_vp, C.POINTER(BatchStats)], C.c_int),
    "tna_dmrg_get_env": ([_vp, C.c_int, C.c_int, _vp, C.c_size_t, C.POINTER(C.c_size_t)], C.c_int),
    "tna_dmrg_get_state": ([_vp, _ip, C.POINTER(PidState)], C.c_int),
    "tna_dmrg_get_mps": ([_vp, _dp, C.c_size_t, C.POINTER(C.c_size_t)], C.c_int),
    "tna_dmrg_destroy": ([_vp], None),
    "tna_dmrg_save": ([_vp, C.c_char_p], C.c_int),
    "tna_dmrg_load": ([_vp, C.c_char_p, C.POINTER(C.c_void_p)], C.c_int),
    "tna_workspace_size": ([_vp, C.c_char_p, C.POINTER(C.c_int64), C.POINTER(C.c_size_t)], C.c_int),
    "tna_set_workspace": ([_vp, _vp, C.c_size_t], C.c_int),
    "tna_mlp_create": ([_vp, _vp, C.POINTER(C.c_void_p)], C.c_int),
    "tna_mlp_set_normalization": ([_vp, _vp, _vp], C.c_int),
    "tna_mlp_get_params": ([_vp, _vp], C.c_int),
    "tna_mlp_forward": ([_vp, C.c_int, _vp, _vp], C.c_int),
    "tna_mlp_loss_grad": ([_vp, C.c_int, _vp, _vp, _vp, _vp], C.c_int),
    "tna_mlp_adam_step": ([_vp, _vp, C.c_float], C.c_int),
    "tna_mlp_train": ([_vp, C.c_int, _vp, _vp, _vp, C.c_int, C.c_int, C.c_float, _vp], C.c_int),
    "tna_mlp_destroy": ([_vp], None),
    "tna_dmrg_set_scheduler": ([_vp, _vp], C.c_int),
    "tna_dmrg_batch_create": ([_vp, C.c_int, _ip, C.c_int, C.c_int, C.POINTER(_dp), C.POINTER(_dp), C.POINTER(_ip),
                               C.POINTER(PidParams), C.POINTER(DmrgOpts), C.POINTER(C.c_void_p)], C.c_int),
    "tna_dmrg_batch_sweep": ([_vp, _dp, C.POINTER(VisitLog), C.POINTER(C.c_int64), C.POINTER(BatchStats)], C.c_int),
    "tna_dmrg_batch_get_state": ([_vp, C.c_int, _ip, C.POINTER(PidState)], C.c_int),
    "tna_dmrg_batch_destroy": ([_vp], None),
    "tna_circuit_create": ([_vp, C.c_int, C.POINTER(PidParams), C.POINTER(CircuitOpts), C.POINTER(C.c_void_p)],
                           C.c_int),
    "tna_circuit_layer": ([_vp, C.c_int, _dp, C.POINTER(GateLog), _ip], C.c_int),
    "tna_circuit_get_mps": ([_vp, _dp, C.c_size_t, C.POINTER(C.c_size_t), _ip], C.c_int),
    "tna_circuit_destroy": ([_vp], None),
    "tna_autotune_save": ([C.c_char_p], C.c_int),
    "tna_autotune_load": ([C.c_char_p], C.c_int),
    "tna_autotune_entries": ([], C.c_int),
    "tna_autotune_clear": ([], None),
}
for _name, (_args, _res) in _SIGS.items():
    _f = getattr(_lib, _name)
    _f.argtypes = _args
    _f.restype = _res

EXPORTED = tuple(_SIGS)


def last_error() -> str:
    return _lib.tna_last_error().decode()


def _check(status, allow=()):
    if status != TNA_OK and status not in allow:
        raise TnaError(status, last_error())
    return status


def _ptr(t):
    return C.c_void_p(t.data_ptr())


NOALLOC_SCRATCH_BYTES = 64 << 20  # TNA_NOALLOC_SCRATCH_BYTES


def heff_apply_noalloc_bytes(chi_l, chi_r, d, D, prec=HEFF_F64) -> int:
    out = C.c_size_t(0)
    _check(_lib.tna_heff_apply_noalloc_bytes(chi_l, chi_r, d, D, prec, C.byref(out)))
    return out.value


# ------------------------------------------------------------------ host-only helpers
def mpo_build(model: int, N: int, params) -> np.ndarray:
    """Bulk MPO tensors (N, D, D, 2, 2) from the library's host builder."""
    p = np.zeros(3)
    p[:len(params)] = params
    D = {MODEL_XXZ: 5, MODEL_J1J2: 8, MODEL_TFIM: 3}[model]
    W = np.zeros((N, D, D, 2, 2))
    d_out = C.c_int(0)
    _check(_lib.tna_mpo_build(model, N, p.ctypes.data_as(_dp), W.ctypes.data_as(_dp), C.byref(d_out)))
    assert d_out.value == D
    return W


def pid_params(kp, ki, kd, s_target, alpha, chi_min, chi_max, beta=0.0, ema_init_zero=False,
               beta2=0.0) -> PidParams:
    return PidParams(kp, ki, kd, s_target, alpha, beta, chi_min, chi_max, int(ema_init_zero), 0, beta2)


def entropy_chi_update(pp: PidParams, gamma: float, st: PidState, s_raw: float) -> int:
    """Algorithm 1: EMA of the entropy, then clamp(ceil(gamma exp(S_ema)), chi_min, chi_max)."""
    chi = C.c_int(0)
    _check(_lib.tna_entropy_chi_update(C.byref(pp), float(gamma), C.byref(st), float(s_raw), C.byref(chi)))
    return chi.value


def pid_chi_update(pp: PidParams, st: PidState, s_raw: float):
    chi = C.c_int(0)
    terms = np.zeros(6)
    _check(_lib.tna_pid_chi_update(C.byref(pp), C.byref(st), float(s_raw), C.byref(chi), terms.ctypes.data_as(_dp)))
    return chi.value, dict(P=terms[0], I=terms[1], D=terms[2], u=terms[3], sbar=terms[4], e=terms[5])


# ------------------------------------------------------------------ device context
class Context:
    """One library context on a HIP device, enqueueing on a torch stream."""

    def __init__(self, device: int = 0, stream=None):
        import torch
        self.torch = torch
        self.device = device
        if stream is None:
            stream = torch.cuda.current_stream(device)
        h = C.c_void_p()
        _check(_lib.tna_create(C.byref(h), device, C.c_void_p(stream.cuda_stream)))
        self.h = h

    def close(self):
        """Destroys the context; raises TnaError (and keeps it) while runs or networks made from it live."""
        if getattr(self, "h", None):
            _check(_lib.tna_destroy(self.h))
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def synchronize(self):
        _check(_lib.tna_synchronize(self.h))

    def workspace_size(self, op: str, dims) -> int:
        """Device bytes of scratch one call needs: op "heff_apply" with dims (chi_l, chi_r, d, D, prec) or
        "svd_truncate" with dims (m, n, dtype, batch)."""
        arr = (C.c_int64 * 5)(*[int(x) for x in dims] + [0] * (5 - len(dims)))
        out = C.c_size_t(0)
        _check(_lib.tna_workspace_size(self.h, op.encode(), arr, C.byref(out)))
        return out.value

    def set_workspace(self, buf=None):
        """Caller-owned device scratch (e.g. a torch uint8 tensor, kept alive by this object); None returns to
        context-owned scratch."""
        self._ws = buf
        if buf is None:
            _check(_lib.tna_set_workspace(self.h, None, 0))
        else:
            _check(_lib.tna_set_workspace(self.h, _ptr(buf), buf.numel() * buf.element_size()))

    def set_timing(self, enable: bool, prefix: str = ""):
        """HIP-event timing of launches whose kernel name starts with prefix."""
        _check(_lib.tna_set_timing(self.h, int(enable), prefix.encode()))

    def kernel_stats(self, reset: bool = True):
        """[{name, count, ms, flops, bytes}] accumulated since the last reset (synchronises)."""
        import json
        buf = C.create_string_buffer(1 << 20)
        _check(_lib.tna_kernel_stats(self.h, buf, len(buf), int(reset)))
        return json.loads(buf.value.decode())

    def set_stream(self, stream):
        _check(_lib.tna_set_stream(self.h, C.c_void_p(stream.cuda_stream)))

    # -------------------------------------------------------------- H_eff
    def heff_apply(self, L, W1, W2, R, theta, prec=HEFF_F64, out=None):
        torch = self.torch
        chl, D, _ = L.shape
        chr_ = R.shape[0]
        d = W1.shape[2]
        for t in (L, W1, W2, R, theta):
            assert t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()
        assert theta.shape == (chl, d, d, chr_)
        if out is None:
            out = torch.empty_like(theta)
        _check(_lib.tna_heff_apply(self.h, chl, chr_, d, D, _ptr(L), _ptr(W1), _ptr(W2), _ptr(R), _ptr(theta),
                                   _ptr(out), prec))
        return out

    def heff_apply_noalloc(self, L, W1, W2, R, theta, out, prec=HEFF_F64):
        """tna_heff_apply on the library's fixed device scratch: no allocation (out is caller-provided)."""
        torch = self.torch
        chl, D, _ = L.shape
        chr_ = R.shape[0]
        d = W1.shape[2]
        for t in (L, W1, W2, R, theta, out):
            assert t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()
        assert theta.shape == (chl, d, d, chr_) and out.shape == theta.shape
        _check(_lib.tna_heff_apply_noalloc(self.h, chl, chr_, d, D, _ptr(L), _ptr(W1), _ptr(W2), _ptr(R),
                                           _ptr(theta), _ptr(out), prec))
        return out

    # -------------------------------------------------------------- SVD
    def svd_truncate(self, A, chi_keep: int):
        """Returns (S, U, Vt, spec, k, sweeps, status); spec = [Z, S_vN, eps, eps^2/Z, |S_k|, gap]."""
        torch = self.torch
        assert A.is_cuda and A.is_contiguous() and A.dim() == 2
        m, n = A.shape
        dt = F64 if A.dtype == torch.float64 else F32
        k = min(chi_keep, m, n)
        S = torch.empty(min(m, n), dtype=torch.float64, device=A.device)
        U = torch.empty((m, k), dtype=A.dtype, device=A.device)
        Vt = torch.empty((k, n), dtype=A.dtype, device=A.device)
        spec = torch.empty(6, dtype=torch.float64, device=A.device)
        k_out, sw = C.c_int(0), C.c_int(0)
        st = _check(_lib.tna_svd_truncate(self.h, m, n, dt, _ptr(A), chi_keep, _ptr(S), _ptr(U), _ptr(Vt),
                                          _ptr(spec), C.byref(k_out), C.byref(sw)), allow=(TNA_ERR_NOCONV,))
        return S, U, Vt, spec, k_out.value, sw.value, st

    def svd_truncate_batched(self, A, chi_keep: int):
        torch = self.torch
        assert A.is_cuda and A.is_contiguous() and A.dim() == 3
        B, m, n = A.shape
        dt = F64 if A.dtype == torch.float64 else F32
        k = min(chi_keep, m, n)
        R = min(m, n)
        S = torch.empty((B, R), dtype=torch.float64, device=A.device)
        U = torch.empty((B, m, k), dtype=A.dtype, device=A.device)
        Vt = torch.empty((B, k, n), dtype=A.dtype, device=A.device)
        spec = torch.empty((B, 6), dtype=torch.float64, device=A.device)
        sw = C.c_int(0)
        st = _check(_lib.tna_svd_truncate_batched(self.h, B, m, n, dt, _ptr(A), m * n, chi_keep, _ptr(S), R, _ptr(U),
                                                  m * k, _ptr(Vt), k * n, _ptr(spec), C.byref(sw)),
                    allow=(TNA_ERR_NOCONV,))
        return S, U, Vt, spec, sw.value, st


# ------------------------------------------------------------------ DMRG
class Dmrg:
    """Device-resident two-site DMRG with per-bond EMA+PID bond dimensions."""

    def __init__(self, ctx: Context, W: np.ndarray, A_packed: np.ndarray, chi_init, pid: PidParams,
                 lanczos_tol=1e-12, lanczos_kmax=100, lanczos_restarts=5, fixed_iters=0, heff_prec=HEFF_F64,
                 fixed_chi=0, svd_max_sweeps=60, eps_target=1e-8, chi_rule=CHI_PID, rule_param=0.0):
        W = np.ascontiguousarray(W, dtype=np.float64)
        N, D, _, d, _ = W.shape
        self.N, self.d, self.D = N, d, D
        self.ctx = ctx
        A = np.ascontiguousarray(A_packed, dtype=np.float64)
        chi = np.ascontiguousarray(chi_init, dtype=np.int32)
        self.opts = DmrgOpts(lanczos_tol, lanczos_kmax, lanczos_restarts, fixed_iters, heff_prec, fixed_chi,
                             svd_max_sweeps, eps_target, chi_rule, 0, rule_param)
        self.pid = pid
        h = C.c_void_p()
        _check(_lib.tna_dmrg_create(ctx.h, N, d, D, W.ctypes.data_as(_dp), A.ctypes.data_as(_dp),
                                    chi.ctypes.data_as(_ip), C.byref(pid), C.byref(self.opts), C.byref(h)))
        self.h = h

    def sweep(self):
        """One full sweep; returns (E, list of per-visit dicts, status)."""
        n = 2 * (self.N - 1)
        logs = (VisitLog * n)()
        E = C.c_double(0.0)
        st = _check(_lib.tna_dmrg_sweep(self.h, C.byref(E), logs), allow=(TNA_ERR_NOCONV,))
        recs = []
        for r in logs:
            d = {f: getattr(r, f) for f, _ in VisitLog._fields_ if f != "feat"}
            d["feat"] = np.array(r.feat[:], dtype=np.float32)
            recs.append(d)
        return E.value, recs, st

    def visit(self, bond: int, direction: int):
        """One bond visit (0: left to right, 1: right to left); returns (E, visit dict, status)."""
        log = VisitLog()
        E = C.c_double(0.0)
        st = _check(_lib.tna_dmrg_visit(self.h, bond, direction, C.byref(E), C.byref(log)), allow=(TNA_ERR_NOCONV,))
        d = {f: getattr(log, f) for f, _ in VisitLog._fields_ if f != "feat"}
        d["feat"] = np.array(log.feat[:], dtype=np.float32)
        return E.value, d, st

    def centre(self) -> int:
        return _lib.tna_dmrg_centre(self.h)

    def stats(self) -> dict:
        """Step-engine counters since create (Lanczos iterations, launches per path, FP32 H_eff iterations)."""
        st = BatchStats()
        _check(_lib.tna_dmrg_get_stats(self.h, C.byref(st)))
        return {f: getattr(st, f) for f, _ in BatchStats._fields_}

    def env(self, side: int, site: int):
        """Copy of the left (side 0) or right (side 1) environment of `site` as a device tensor (chi, D, chi)."""
        torch = self.ctx.torch
        cnt = C.c_size_t(0)
        _check(_lib.tna_dmrg_get_env(self.h, side, site, None, 0, C.byref(cnt)))
        chi = int(round((cnt.value / self.D) ** 0.5))
        out = torch.empty((chi, self.D, chi), dtype=torch.float64, device="cuda")
        _check(_lib.tna_dmrg_get_env(self.h, side, site, C.c_void_p(out.data_ptr()), cnt.value, C.byref(cnt)))
        return out

    def save(self, path: str):
        """Checkpoint (MPS, MPO, controller state) to a file; see tna_dmrg_save."""
        _check(_lib.tna_dmrg_save(self.h, path.encode()))

    @classmethod
    def load(cls, ctx: "Context", path: str) -> "Dmrg":
        """Resume a run saved with save()."""
        h = C.c_void_p()
        _check(_lib.tna_dmrg_load(ctx.h, path.encode(), C.byref(h)))
        self = cls.__new__(cls)
        self.h, self.ctx = h, ctx
        # N, d, D from the file header (magic, then int32 N, d, D)
        with open(path, "rb") as f:
            f.read(8)
            hdr = np.frombuffer(f.read(16), dtype=np.int32)
        self.N, self.d, self.D = int(hdr[0]), int(hdr[1]), int(hdr[2])
        return self

    def set_scheduler(self, net):
        """Attach a trained Mlp (None detaches); keeps a reference for the run's lifetime."""
        self._sched = net
        _check(_lib.tna_dmrg_set_scheduler(self.h, net.h if net is not None else None))

    def state(self):
        chi = np.zeros(self.N - 1, dtype=np.int32)
        pid = (PidState * (self.N - 1))()
        _check(_lib.tna_dmrg_get_state(self.h, chi.ctypes.data_as(_ip), pid))
        return chi, list(pid)

    def mps(self):
        cnt = C.c_size_t(0)
        _check(_lib.tna_dmrg_get_mps(self.h, None, 0, C.byref(cnt)))
        out = np.zeros(cnt.value)
        _check(_lib.tna_dmrg_get_mps(self.h, out.ctypes.data_as(_dp), cnt.value, C.byref(cnt)))
        return out

    def close(self):
        if getattr(self, "h", None):
            _lib.tna_dmrg_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ------------------------------------------------------------------ learned scheduler
MLP_IN, MLP_NPARAM = 25, 5889


class Mlp:
    """The learned bond-dimension scheduler network (FP32, library kernels)."""

    def __init__(self, ctx: Context, params: np.ndarray):
        p = np.ascontiguousarray(params, dtype=np.float32)
        assert p.size == MLP_NPARAM
        h = C.c_void_p()
        _check(_lib.tna_mlp_create(ctx.h, C.c_void_p(p.ctypes.data), C.byref(h)))
        self.h, self.ctx = h, ctx

    def set_normalization(self, mean=None, std=None):
        if mean is None:
            _check(_lib.tna_mlp_set_normalization(self.h, None, None))
            return
        m = np.ascontiguousarray(mean, dtype=np.float32)
        s = np.ascontiguousarray(std, dtype=np.float32)
        self._norm = (m, s)
        _check(_lib.tna_mlp_set_normalization(self.h, C.c_void_p(m.ctypes.data), C.c_void_p(s.ctypes.data)))

    def params(self) -> np.ndarray:
        out = np.zeros(MLP_NPARAM, dtype=np.float32)
        _check(_lib.tna_mlp_get_params(self.h, C.c_void_p(out.ctypes.data)))
        return out

    def forward(self, X):
        torch = self.ctx.torch
        assert X.is_cuda and X.dtype == torch.float32 and X.is_contiguous() and X.shape[1] == MLP_IN
        y = torch.empty(X.shape[0], dtype=torch.float32, device=X.device)
        _check(_lib.tna_mlp_forward(self.h, X.shape[0], _ptr(X), _ptr(y)))
        return y

    def loss_grad(self, X, T):
        torch = self.ctx.torch
        g = torch.empty(MLP_NPARAM, dtype=torch.float32, device=X.device)
        loss = torch.empty(1, dtype=torch.float32, device=X.device)
        _check(_lib.tna_mlp_loss_grad(self.h, X.shape[0], _ptr(X), _ptr(T), _ptr(g), _ptr(loss)))
        return loss, g

    def adam_step(self, g, lr=1e-3):
        _check(_lib.tna_mlp_adam_step(self.h, _ptr(g), float(lr)))

    def train(self, X, T, perm, epochs, batch=256, lr=1e-3):
        losses = np.zeros(epochs, dtype=np.float32)
        _check(_lib.tna_mlp_train(self.h, X.shape[0], _ptr(X), _ptr(T), _ptr(perm), epochs, batch, float(lr),
                                  C.c_void_p(losses.ctypes.data)))
        return losses

    def close(self):
        if getattr(self, "h", None):
            _lib.tna_mlp_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ------------------------------------------------------------------ many chains
class DmrgBatch:
    """Independent chains swept together through grouped launches."""

    def __init__(self, ctx: Context, Ws, As, chis, pid: PidParams, lanczos_tol=1e-12, lanczos_kmax=100,
                 lanczos_restarts=5, heff_prec=HEFF_F64, fixed_chi=0, svd_max_sweeps=60, eps_target=1e-8,
                 chi_rule=CHI_PID, rule_param=0.0):
        n = len(Ws)
        self.Ws = [np.ascontiguousarray(w, dtype=np.float64) for w in Ws]
        self.As = [np.ascontiguousarray(a, dtype=np.float64) for a in As]
        self.chis = [np.ascontiguousarray(c, dtype=np.int32) for c in chis]
        self.N = np.array([w.shape[0] for w in self.Ws], dtype=np.int32)
        D, d = self.Ws[0].shape[1], self.Ws[0].shape[3]
        Wp = (_dp * n)(*[w.ctypes.data_as(_dp) for w in self.Ws])
        Ap = (_dp * n)(*[a.ctypes.data_as(_dp) for a in self.As])
        Cp = (_ip * n)(*[c.ctypes.data_as(_ip) for c in self.chis])
        self.opts = DmrgOpts(lanczos_tol, lanczos_kmax, lanczos_restarts, 0, heff_prec, fixed_chi, svd_max_sweeps,
                             eps_target, chi_rule, 0, rule_param)
        self.pid = pid
        h = C.c_void_p()
        _check(_lib.tna_dmrg_batch_create(ctx.h, n, self.N.ctypes.data_as(_ip), d, D, Wp, Ap, Cp, C.byref(pid),
                                          C.byref(self.opts), C.byref(h)))
        self.h, self.n = h, n
        self.ctx = ctx  # the context must outlive the batch (its chains use its stream)
        self.offsets = np.concatenate([[0], np.cumsum(2 * (self.N - 1))]).astype(np.int64)

    def sweep(self):
        """One sweep of every chain: (E per chain, per-chain lists of visit dicts, stats dict, status)."""
        total = int(self.offsets[-1])
        logs = (VisitLog * total)()
        E = np.zeros(self.n)
        stats = BatchStats()
        off = self.offsets[:-1].copy()
        st = _check(_lib.tna_dmrg_batch_sweep(self.h, E.ctypes.data_as(_dp), logs,
                                              off.ctypes.data_as(C.POINTER(C.c_int64)), C.byref(stats)),
                    allow=(TNA_ERR_NOCONV,))
        per = []
        for c in range(self.n):
            recs = []
            for r in logs[int(self.offsets[c]):int(self.offsets[c + 1])]:
                d = {f: getattr(r, f) for f, _ in VisitLog._fields_ if f != "feat"}
                recs.append(d)
            per.append(recs)
        return E, per, {f: getattr(stats, f) for f, _ in BatchStats._fields_}, st

    def state(self, chain):
        chi = np.zeros(self.N[chain] - 1, dtype=np.int32)
        pid = (PidState * int(self.N[chain] - 1))()
        _check(_lib.tna_dmrg_batch_get_state(self.h, chain, chi.ctypes.data_as(_ip), pid))
        return chi, list(pid)

    def close(self):
        if getattr(self, "h", None):
            _lib.tna_dmrg_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Circuit:
    """Circuit simulation with adaptive bond dimensions: an MPS from |0...0> through layers of real
    two-qubit gates (one grouped launch sequence per layer)."""

    def __init__(self, ctx: Context, N: int, pid: PidParams, fixed_chi=0, one_at_a_time=False, svd_max_sweeps=60):
        self.ctx, self.N = ctx, N
        self.opts = CircuitOpts(fixed_chi, int(one_at_a_time), svd_max_sweeps, 0)
        self.pid = pid
        h = C.c_void_p()
        _check(_lib.tna_circuit_create(ctx.h, N, C.byref(pid), C.byref(self.opts), C.byref(h)))
        self.h = h

    def layer(self, parity: int, gates):
        """Applies one layer; returns (bond dimensions after it, list of per-gate dicts, status)."""
        g = np.ascontiguousarray(gates, dtype=np.float64).ravel()
        ng = len(range(parity, self.N - 1, 2))
        assert g.size == 16 * ng
        logs = (GateLog * max(ng, 1))()
        row = np.zeros(self.N - 1, dtype=np.int32)
        st = _check(_lib.tna_circuit_layer(self.h, parity, g.ctypes.data_as(_dp), logs, row.ctypes.data_as(_ip)),
                    allow=(TNA_ERR_NOCONV,))
        recs = [{f: getattr(r, f) for f, _ in GateLog._fields_} for r in logs[:ng]]
        return row, recs, st

    def run(self, parity, gates):
        """All ops of a circuit (parity list, packed gates); returns (map: ops x (N-1), records)."""
        g = np.ascontiguousarray(gates, dtype=np.float64).ravel()
        rows, recs, off = [], [], 0
        for p in parity:
            ng = len(range(p, self.N - 1, 2))
            row, r, _ = self.layer(p, g[off:off + 16 * ng])
            off += 16 * ng
            rows.append(row)
            recs += r
        return np.array(rows), recs

    def mps(self):
        cnt = C.c_size_t(0)
        chi = np.zeros(self.N - 1, dtype=np.int32)
        _check(_lib.tna_circuit_get_mps(self.h, None, 0, C.byref(cnt), chi.ctypes.data_as(_ip)))
        out = np.zeros(cnt.value)
        _check(_lib.tna_circuit_get_mps(self.h, out.ctypes.data_as(_dp), cnt.value, C.byref(cnt),
                                        chi.ctypes.data_as(_ip)))
        return out, chi

    def close(self):
        if getattr(self, "h", None):
            _lib.tna_circuit_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def autotune_save(path: str):
    _check(_lib.tna_autotune_save(path.encode()))


def autotune_load(path: str):
    _check(_lib.tna_autotune_load(path.encode()))


def autotune_entries() -> int:
    return _lib.tna_autotune_entries()


def autotune_clear():
    _lib.tna_autotune_clear()
