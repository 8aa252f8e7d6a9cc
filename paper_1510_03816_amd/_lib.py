"""ctypes binding of liblm.so (include/liblm.h).  Argument marshalling only.

Functions carry the C names and take torch tensors on the GPU (shape (dim, n), contiguous,
float64 or float32) plus an optional stream; every computation runs in the HIP library.
A non-OK status raises LmError with the library's message.
"""

from __future__ import annotations

import ctypes
import os

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "liblm.so")

LM_OK, LM_EINVAL, LM_ENOMEM, LM_EHIP, LM_ENOTCONV, LM_EDIVERGED, LM_ESINGULAR, LM_EUNSUPPORTED = (
    0, -1, -2, -3, -4, -5, -6, -7)
STATUS_NAMES = {0: "LM_OK", -1: "LM_EINVAL", -2: "LM_ENOMEM", -3: "LM_EHIP", -4: "LM_ENOTCONV",
                -5: "LM_EDIVERGED", -6: "LM_ESINGULAR", -7: "LM_EUNSUPPORTED"}
CONON, GAUSS = 0, 1
F64, F32 = 0, 1
SOLVE_AUTO, SOLVE_CG, SOLVE_DENSE = 0, 1, 2

# every symbol include/liblm.h declares
EXPORTS = ["lm_rhs", "lm_shoot", "lm_shoot_noalloc", "lm_hamiltonian", "lm_ksolve", "lm_feedback_match",
           "lm_feedback_step", "lm_velocity", "lm_flow_points", "lm_rhs_vjp", "lm_shoot_adjoint", "lm_energy_grad",
           "lm_lbfgs_match", "lm_batch_default_tuning", "lm_batch_autotune", "lm_rhs_batched",
           "lm_shoot_batched", "lm_feedback_match_batched", "lm_pair_plan", "lm_last_error", "lm_version"]
BATCH_BUCKETS = 4


class LmError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__("%s: %s" % (STATUS_NAMES.get(status, str(status)), message))
        self.status = status


class lm_params(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int32), ("kernel", ctypes.c_int32), ("dtype", ctypes.c_int32),
                ("flags", ctypes.c_int32), ("sigma", ctypes.c_double), ("tau", ctypes.c_double),
                ("cutoff", ctypes.c_double)]


class lm_match_opts(ctypes.Structure):
    _fields_ = [("h", ctypes.c_double), ("tol", ctypes.c_double), ("max_iter", ctypes.c_int32),
                ("steps", ctypes.c_int32), ("stop_rule", ctypes.c_int32), ("cg_max_iter", ctypes.c_int32),
                ("cg_rtol", ctypes.c_double), ("resid_hist", ctypes.POINTER(ctypes.c_double)),
                ("hist_len", ctypes.c_int32), ("solver", ctypes.c_int32), ("f32_switch", ctypes.c_double)]


class lm_match_info(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("cg_iters", ctypes.c_int32), ("resid_inf", ctypes.c_double),
                ("H", ctypes.c_double), ("shoot_ms", ctypes.c_double), ("solve_ms", ctypes.c_double),
                ("factor_ms", ctypes.c_double), ("shoots", ctypes.c_int32)]


class lm_plan_info(ctypes.Structure):
    _fields_ = [("symmetric", ctypes.c_int32), ("waves", ctypes.c_int32), ("workgroups", ctypes.c_int64),
                ("partial_slots", ctypes.c_int32), ("small", ctypes.c_int32), ("rows", ctypes.c_int32)]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


class lm_step_info(ctypes.Structure):
    _fields_ = [("resid_inf", ctypes.c_double), ("shoot_ms", ctypes.c_double), ("solve_ms", ctypes.c_double),
                ("converged", ctypes.c_int32), ("cg_iters", ctypes.c_int32)]


class lm_lbfgs_opts(ctypes.Structure):
    _fields_ = [("lam", ctypes.c_double), ("reg", ctypes.c_double), ("gtol", ctypes.c_double),
                ("match_tol", ctypes.c_double), ("max_iter", ctypes.c_int32), ("history", ctypes.c_int32),
                ("steps", ctypes.c_int32), ("ckpt_every", ctypes.c_int32)]


class lm_lbfgs_info(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("evals", ctypes.c_int32), ("E", ctypes.c_double),
                ("gnorm_inf", ctypes.c_double), ("resid_inf", ctypes.c_double)]


class lm_batch_tuning(ctypes.Structure):
    _fields_ = [("bucket_max", ctypes.c_int64 * BATCH_BUCKETS), ("split", ctypes.c_int32 * BATCH_BUCKETS),
                ("groups", ctypes.c_int32), ("graph_steps", ctypes.c_int32), ("sym_min", ctypes.c_int32),
                ("sym_waves", ctypes.c_int32), ("stage_us", ctypes.c_double)]

    def as_dict(self):
        return {"bucket_max": list(self.bucket_max), "split": list(self.split), "groups": self.groups,
                "graph_steps": self.graph_steps, "sym_min": self.sym_min, "sym_waves": self.sym_waves,
                "stage_us": self.stage_us}


_lib = None


def load():
    """Load the in-tree liblm.so.  Raises if it has not been built: there is no fallback.

    torch is imported first: its HIP runtime (the one that owns every tensor the binding
    passes in) must be the one the library binds to.  Loaded the other way round, the
    library would pull in the system runtime under the same soname and the process would
    hold two HIP runtimes, each blind to the other's device state.
    """
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("liblm.so is not built (run __graft_entry__.build() or "
                              "python paper_1510_03816_amd/build.py)")
        import torch  # noqa: F401  (loads torch's HIP runtime before liblm.so)
        L = ctypes.CDLL(LIB_PATH)
        P, i64, i32, d = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_double
        PP = ctypes.POINTER(lm_params)
        L.lm_rhs.argtypes = [PP, i64, P, P, P, P, P]
        L.lm_shoot.argtypes = [PP, i64, P, P, d, i32, P, P, P]
        L.lm_shoot_noalloc.argtypes = [PP, i64, P, P, d, i32, P, P, P]
        L.lm_hamiltonian.argtypes = [PP, i64, P, P, ctypes.POINTER(d), P]
        L.lm_ksolve.argtypes = [PP, i64, P, P, P, d, i32, i32, ctypes.POINTER(i32), P]
        L.lm_feedback_match.argtypes = [PP, ctypes.POINTER(lm_match_opts), i64, P, P, P, P,
                                        ctypes.POINTER(lm_match_info), P]
        L.lm_feedback_step.argtypes = [PP, ctypes.POINTER(lm_match_opts), i64, P, P, P, P,
                                       ctypes.POINTER(lm_step_info), P]
        L.lm_velocity.argtypes = [PP, i64, P, P, i64, P, P, P]
        L.lm_flow_points.argtypes = [PP, i64, P, P, i64, P, d, i32, P, P, P, P]
        L.lm_rhs_vjp.argtypes = [PP, i64, P, P, P, P, P, P, P]
        L.lm_shoot_adjoint.argtypes = [PP, i64, P, P, d, i32, i32, P, P, P, P, P, P, P]
        L.lm_energy_grad.argtypes = [PP, i64, P, P, P, d, d, i32, i32, ctypes.POINTER(d), P, P, P]
        L.lm_lbfgs_match.argtypes = [PP, ctypes.POINTER(lm_lbfgs_opts), i64, P, P, P, ctypes.POINTER(lm_lbfgs_info), P]
        PT = ctypes.POINTER(lm_batch_tuning)
        L.lm_batch_default_tuning.argtypes = [i32, P, PT]
        L.lm_batch_autotune.argtypes = [PP, i32, P, P, P, PT, P]
        L.lm_rhs_batched.argtypes = [PP, i32, P, P, P, P, P, PT, P]
        L.lm_shoot_batched.argtypes = [PP, i32, P, P, P, d, i32, P, P, PT, P]
        L.lm_feedback_match_batched.argtypes = [PP, ctypes.POINTER(lm_match_opts), i32, P, P, P, P, P,
                                                ctypes.POINTER(lm_match_info), P, PT, P]
        L.lm_pair_plan.argtypes = [PP, i64, ctypes.POINTER(lm_plan_info)]
        for name in ["lm_rhs", "lm_shoot", "lm_shoot_noalloc", "lm_hamiltonian", "lm_ksolve", "lm_feedback_match",
                     "lm_feedback_step", "lm_velocity", "lm_flow_points", "lm_rhs_vjp", "lm_shoot_adjoint", "lm_energy_grad",
                     "lm_lbfgs_match", "lm_batch_default_tuning", "lm_batch_autotune", "lm_rhs_batched",
                     "lm_shoot_batched", "lm_feedback_match_batched", "lm_pair_plan"]:
            getattr(L, name).restype = ctypes.c_int
        L.lm_last_error.restype = ctypes.c_char_p
        L.lm_last_error.argtypes = []
        L.lm_version.restype = ctypes.c_char_p
        L.lm_version.argtypes = []
        _lib = L
    return _lib


def last_error() -> str:
    return load().lm_last_error().decode()


def _check(status: int, allow=()):
    if status != LM_OK and status not in allow:
        raise LmError(status, last_error())
    return status


def make_params(dim: int, kernel: int, sigma: float, dtype: int = F64, tau: float = 0.0,
                cutoff: float = 0.0) -> lm_params:
    return lm_params(dim, kernel, dtype, 0, float(sigma), float(tau), float(cutoff))


def _stream(stream):
    if stream is None:
        import torch
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return ctypes.c_void_p(stream)
    return ctypes.c_void_p(stream.cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(0 if t is None else t.data_ptr())


def _check_tensor(t, dim, n, dtype, name):
    import torch
    if t.device.type != "cuda":
        raise ValueError("%s must be a GPU tensor" % name)
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    if tuple(t.shape) != (dim, n):
        raise ValueError("%s must have shape (%d, %d), got %s" % (name, dim, n, tuple(t.shape)))
    want = torch.float64 if dtype == F64 else torch.float32
    if t.dtype != want:
        raise ValueError("%s must be %s" % (name, want))


def lm_rhs(params: lm_params, q, p, dq, dp, stream=None):
    dim, n = q.shape
    for t, nm in [(q, "q"), (p, "p"), (dq, "dq"), (dp, "dp")]:
        _check_tensor(t, params.dim, n, params.dtype, nm)
    return _check(load().lm_rhs(ctypes.byref(params), n, _ptr(q), _ptr(p), _ptr(dq), _ptr(dp), _stream(stream)))


def lm_pair_plan(params: lm_params, n: int) -> dict:
    """The pair-sum launch plan for n points (host only): symmetric, waves, workgroups,
    partial_slots, small, rows."""
    info = lm_plan_info()
    _check(load().lm_pair_plan(ctypes.byref(params), int(n), ctypes.byref(info)))
    return info.as_dict()


def lm_shoot(params: lm_params, q0, p0, t1: float, steps: int, q1, p1, stream=None):
    dim, n = q0.shape
    for t, nm in [(q0, "q0"), (p0, "p0"), (q1, "q1"), (p1, "p1")]:
        _check_tensor(t, params.dim, n, params.dtype, nm)
    return _check(load().lm_shoot(ctypes.byref(params), n, _ptr(q0), _ptr(p0), float(t1), int(steps),
                                  _ptr(q1), _ptr(p1), _stream(stream)))


def lm_shoot_noalloc(params: lm_params, q0, p0, t1: float, steps: int, q1, p1, stream=None):
    """lm_shoot with the library's fixed scratch array instead of allocated workspace."""
    dim, n = q0.shape
    for t, nm in [(q0, "q0"), (p0, "p0"), (q1, "q1"), (p1, "p1")]:
        _check_tensor(t, params.dim, n, params.dtype, nm)
    return _check(load().lm_shoot_noalloc(ctypes.byref(params), n, _ptr(q0), _ptr(p0), float(t1), int(steps),
                                          _ptr(q1), _ptr(p1), _stream(stream)))


def lm_hamiltonian(params: lm_params, q, p, stream=None) -> float:
    dim, n = q.shape
    for t, nm in [(q, "q"), (p, "p")]:
        _check_tensor(t, params.dim, n, params.dtype, nm)
    H = ctypes.c_double(0.0)
    _check(load().lm_hamiltonian(ctypes.byref(params), n, _ptr(q), _ptr(p), ctypes.byref(H), _stream(stream)))
    return H.value


def lm_ksolve(params: lm_params, X, b, x, rtol: float = 1e-13, max_iter: int = 0, solver: int = SOLVE_AUTO,
              stream=None) -> int:
    """Solves (K(X) + tau I) x = b per component; returns the CG iteration count (0 if dense)."""
    dim, n = X.shape
    for t, nm in [(X, "X"), (b, "b"), (x, "x")]:
        _check_tensor(t, params.dim, n, F64, nm)
    it = ctypes.c_int32(0)
    mi = int(max_iter) if max_iter > 0 else min(20 * n + 100, 10000)
    _check(load().lm_ksolve(ctypes.byref(params), n, _ptr(X), _ptr(b), _ptr(x), float(rtol), mi, int(solver),
                            ctypes.byref(it), _stream(stream)))
    return it.value


def lm_feedback_match(params: lm_params, X, Y, p0, h: float, tol: float, steps: int, max_iter: int = 500,
                      q1=None, stop_rule: int = 0, cg_rtol: float = 0.0, cg_max_iter: int = 0,
                      hist_len: int = 1024, solver: int = SOLVE_AUTO, f32_switch: float = 0.0, stream=None,
                      raise_on=(LM_EINVAL, LM_ENOMEM, LM_EHIP, LM_EUNSUPPORTED)):
    """Runs Algorithm 1 in place on p0.  Returns (status, info, residual of every shoot).

    Statuses describing the iteration itself (not converged, diverged, singular K) are
    returned, not raised; argument and runtime errors raise LmError.
    """
    dim, n = X.shape
    for t, nm in [(X, "X"), (Y, "Y"), (p0, "p0")] + ([(q1, "q1")] if q1 is not None else []):
        _check_tensor(t, params.dim, n, F64, nm)
    nan = float("nan")
    hist = (ctypes.c_double * max(1, hist_len))(*([nan] * max(1, hist_len)))
    o = lm_match_opts(float(h), float(tol), int(max_iter), int(steps), int(stop_rule), int(cg_max_iter),
                      float(cg_rtol), ctypes.cast(hist, ctypes.POINTER(ctypes.c_double)), int(hist_len), int(solver),
                      float(f32_switch))
    info = lm_match_info()
    st = load().lm_feedback_match(ctypes.byref(params), ctypes.byref(o), n, _ptr(X), _ptr(Y), _ptr(p0),
                                  _ptr(q1), ctypes.byref(info), _stream(stream))
    if st in raise_on:
        raise LmError(st, last_error())
    shots = []
    for i in range(hist_len):
        if hist[i] != hist[i]:
            break
        shots.append(hist[i])
    return st, info, shots


def lm_feedback_step(params: lm_params, X, Y, p, h: float, tol: float, steps: int, q1=None,
                     cg_rtol: float = 0.0, cg_max_iter: int = 0, solver: int = SOLVE_CG, stream=None,
                     raise_on=(LM_EINVAL, LM_ENOMEM, LM_EHIP, LM_EUNSUPPORTED)):
    """One iteration of Algorithm 1 on p (in place).  Returns (status, lm_step_info).

    Statuses describing the iteration (diverged, K-solve not converged or singular) are
    returned, not raised; argument and runtime errors raise LmError.
    """
    dim, n = X.shape
    for t, nm in [(X, "X"), (Y, "Y"), (p, "p")] + ([(q1, "q1")] if q1 is not None else []):
        _check_tensor(t, params.dim, n, F64, nm)
    o = lm_match_opts(float(h), float(tol), 0, int(steps), 0, int(cg_max_iter), float(cg_rtol), None, 0, int(solver))
    info = lm_step_info()
    st = load().lm_feedback_step(ctypes.byref(params), ctypes.byref(o), n, _ptr(X), _ptr(Y), _ptr(p), _ptr(q1),
                                 ctypes.byref(info), _stream(stream))
    if st in raise_on:
        raise LmError(st, last_error())
    return st, info


def lm_velocity(params: lm_params, q, p, x, u, stream=None):
    dim, n = q.shape
    m = x.shape[1]
    for t, nm in [(q, "q"), (p, "p")]:
        _check_tensor(t, params.dim, n, params.dtype, nm)
    for t, nm in [(x, "x"), (u, "u")]:
        _check_tensor(t, params.dim, m, params.dtype, nm)
    return _check(load().lm_velocity(ctypes.byref(params), n, _ptr(q), _ptr(p), m, _ptr(x), _ptr(u),
                                     _stream(stream)))


def lm_flow_points(params: lm_params, q0, p0, x0, t1: float, steps: int, x1, q1=None, p1=None, stream=None):
    """Shoots (q0, p0) over [0, t1] and carries the points x0 (dim, m) along the velocity
    field; x(t1) to x1, and q(t1), p(t1) to q1, p1 when given."""
    dim, n = q0.shape
    m = x0.shape[1]
    for t, nm in [(q0, "q0"), (p0, "p0"), (q1, "q1"), (p1, "p1")]:
        if t is not None:
            _check_tensor(t, params.dim, n, params.dtype, nm)
    for t, nm in [(x0, "x0"), (x1, "x1")]:
        _check_tensor(t, params.dim, m, params.dtype, nm)
    return _check(load().lm_flow_points(ctypes.byref(params), n, _ptr(q0), _ptr(p0), m, _ptr(x0), float(t1),
                                        int(steps), _ptr(q1), _ptr(p1), _ptr(x1), _stream(stream)))


def lm_rhs_vjp(params: lm_params, q, p, a, b, aq, ap, stream=None):
    dim, n = q.shape
    for t, nm in [(q, "q"), (p, "p"), (a, "a"), (b, "b"), (aq, "aq"), (ap, "ap")]:
        _check_tensor(t, params.dim, n, F64, nm)
    return _check(load().lm_rhs_vjp(ctypes.byref(params), n, _ptr(q), _ptr(p), _ptr(a), _ptr(b), _ptr(aq), _ptr(ap),
                                    _stream(stream)))


def lm_shoot_adjoint(params: lm_params, q0, p0, t1: float, steps: int, ckpt_every: int, gq1, gp1, gq0, gp0,
                     q1=None, p1=None, stream=None):
    dim, n = q0.shape
    for t, nm in [(q0, "q0"), (p0, "p0"), (gq1, "gq1"), (gp1, "gp1"), (gq0, "gq0"), (gp0, "gp0")] + \
            [(t, nm) for t, nm in [(q1, "q1"), (p1, "p1")] if t is not None]:
        _check_tensor(t, params.dim, n, F64, nm)
    return _check(load().lm_shoot_adjoint(ctypes.byref(params), n, _ptr(q0), _ptr(p0), float(t1), int(steps),
                                          int(ckpt_every), _ptr(gq1), _ptr(gp1), _ptr(gq0), _ptr(gp0), _ptr(q1),
                                          _ptr(p1), _stream(stream)))


def lm_energy_grad(params: lm_params, X, Y, p0, lam: float, steps: int, grad, ckpt_every: int = 0, q1=None,
                   reg: float = 1.0, stream=None) -> float:
    """E(p0) = reg/2 p0^T K p0 + lam/2 |q(1) - Y|^2; writes its gradient to grad, returns E."""
    dim, n = X.shape
    for t, nm in [(X, "X"), (Y, "Y"), (p0, "p0"), (grad, "grad")] + ([(q1, "q1")] if q1 is not None else []):
        _check_tensor(t, params.dim, n, F64, nm)
    E = ctypes.c_double(0.0)
    _check(load().lm_energy_grad(ctypes.byref(params), n, _ptr(X), _ptr(Y), _ptr(p0), float(lam), float(reg),
                                 int(steps), int(ckpt_every), ctypes.byref(E), _ptr(grad), _ptr(q1),
                                 _stream(stream)))
    return E.value


def lm_lbfgs_match(params: lm_params, X, Y, p0, lam: float, steps: int, reg: float = 1.0, gtol: float = 1e-6,
                   match_tol: float = 0.0, max_iter: int = 200, history: int = 8, ckpt_every: int = 10,
                   stream=None, raise_on=(LM_EINVAL, LM_ENOMEM, LM_EHIP, LM_EUNSUPPORTED)):
    """Gradient-based matching by L-BFGS on the GPU, in place on p0.  Returns (status, info)."""
    dim, n = X.shape
    for t, nm in [(X, "X"), (Y, "Y"), (p0, "p0")]:
        _check_tensor(t, params.dim, n, F64, nm)
    o = lm_lbfgs_opts(float(lam), float(reg), float(gtol), float(match_tol), int(max_iter), int(history),
                      int(steps), int(ckpt_every))
    info = lm_lbfgs_info()
    st = load().lm_lbfgs_match(ctypes.byref(params), ctypes.byref(o), n, _ptr(X), _ptr(Y), _ptr(p0),
                               ctypes.byref(info), _stream(stream))
    if st in raise_on:
        raise LmError(st, last_error())
    return st, info


# ------------------------------------------------------------------ batches of problems

def _offs_array(offs):
    """offs: a sequence of B + 1 int64 offsets (host).  Returns (B, ctypes array)."""
    vals = [int(v) for v in offs]
    arr = (ctypes.c_int64 * len(vals))(*vals)
    return len(vals) - 1, arr


def _tuning_ptr(tuning):
    return None if tuning is None else ctypes.byref(tuning)


def lm_batch_default_tuning(offs) -> lm_batch_tuning:
    """Launch shape that needs no measurement (host only: no GPU call)."""
    B, arr = _offs_array(offs)
    t = lm_batch_tuning()
    _check(load().lm_batch_default_tuning(B, arr, ctypes.byref(t)))
    return t


def lm_batch_autotune(params: lm_params, offs, q, p, stream=None) -> lm_batch_tuning:
    B, arr = _offs_array(offs)
    for t, nm in [(q, "q"), (p, "p")]:
        _check_tensor(t, params.dim, arr[B], params.dtype, nm)
    t = lm_batch_tuning()
    _check(load().lm_batch_autotune(ctypes.byref(params), B, arr, _ptr(q), _ptr(p), ctypes.byref(t),
                                    _stream(stream)))
    return t


def lm_rhs_batched(params: lm_params, offs, q, p, dq, dp, tuning=None, stream=None):
    B, arr = _offs_array(offs)
    for t, nm in [(q, "q"), (p, "p"), (dq, "dq"), (dp, "dp")]:
        _check_tensor(t, params.dim, arr[B], params.dtype, nm)
    return _check(load().lm_rhs_batched(ctypes.byref(params), B, arr, _ptr(q), _ptr(p), _ptr(dq), _ptr(dp),
                                        _tuning_ptr(tuning), _stream(stream)))


def lm_shoot_batched(params: lm_params, offs, q0, p0, t1: float, steps: int, q1, p1, tuning=None, stream=None):
    B, arr = _offs_array(offs)
    for t, nm in [(q0, "q0"), (p0, "p0"), (q1, "q1"), (p1, "p1")]:
        _check_tensor(t, params.dim, arr[B], params.dtype, nm)
    return _check(load().lm_shoot_batched(ctypes.byref(params), B, arr, _ptr(q0), _ptr(p0), float(t1), int(steps),
                                          _ptr(q1), _ptr(p1), _tuning_ptr(tuning), _stream(stream)))


def lm_feedback_match_batched(params: lm_params, offs, X, Y, p0, h: float, tol: float, steps: int,
                              max_iter: int = 500, q1=None, tuning=None, f32_switch: float = 0.0, stream=None,
                              raise_on=(LM_EINVAL, LM_ENOMEM, LM_EHIP, LM_EUNSUPPORTED)):
    """Algorithm 1 for every problem of a batch, in place on p0.

    Returns (status, infos, statuses): one lm_match_info and one status per problem.
    """
    B, arr = _offs_array(offs)
    for t, nm in [(X, "X"), (Y, "Y"), (p0, "p0")] + ([(q1, "q1")] if q1 is not None else []):
        _check_tensor(t, params.dim, arr[B], F64, nm)
    o = lm_match_opts(float(h), float(tol), int(max_iter), int(steps), 0, 0, 0.0, None, 0, SOLVE_DENSE,
                      float(f32_switch))
    infos = (lm_match_info * B)()
    stats = (ctypes.c_int32 * B)()
    st = load().lm_feedback_match_batched(ctypes.byref(params), ctypes.byref(o), B, arr, _ptr(X), _ptr(Y),
                                          _ptr(p0), _ptr(q1), infos, stats, _tuning_ptr(tuning), _stream(stream))
    if st in raise_on:
        raise LmError(st, last_error())
    return st, list(infos), list(stats)


def lm_version() -> str:
    return load().lm_version().decode()
