"""Python binding of libsmsq.so (the C ABI in include/smsq.h).

Argument marshalling only: every step of the method runs in the HIP kernels
behind the C ABI.  PyTorch supplies device memory (tensors on ``cuda``) and
the current HIP stream.  There is no CPU fallback: if the library is missing
or fails to load, every call raises.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsmsq.so")

OK, ERR_INVALID, ERR_UNSUPPORTED, ERR_HIP, ERR_NONFINITE, ERR_WORKSPACE = range(6)
F32, F64 = 0, 1

SYMBOLS = [
    "smsq_model_create", "smsq_model_destroy", "smsq_workspace_size", "smsq_svgd_step",
    "smsq_viterbi_step", "smsq_backtrack", "smsq_batch_step", "smsq_run_batch",
    "smsq_run_sequence", "smsq_get_device_status", "smsq_clear_device_status",
    "smsq_status_string", "smsq_max_particles",
    "smsq_batch_plan_create", "smsq_batch_plan_tune", "smsq_batch_run", "smsq_batch_storage",
    "smsq_batch_plan_info", "smsq_batch_status", "smsq_batch_plan_destroy",
    "smsq_init_mlp_create", "smsq_init_mlp_destroy", "smsq_init_mlp_params", "smsq_init_mlp_sync",
    "smsq_init_set_create", "smsq_init_set_destroy", "smsq_init_features", "smsq_init_mlp_forward",
    "smsq_init_mlp_backward", "smsq_init_mixture_nll", "smsq_init_mlp_train_step", "smsq_init_mlp_sample",
    "smsq_batch_plan_set_init", "smsq_run_sequence_noalloc", "smsq_viterbi_lattice_batch",
    "smsq_backtrack_steps",
]


class SmsqError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        super().__init__("%s failed: %s (%d)" % (where, status_string(status), status))


class ModelDesc(C.Structure):
    _fields_ = [("kind", C.c_int), ("d", C.c_int), ("obs_dim", C.c_int), ("n_obs", C.c_int),
                ("q_var", C.c_double * 16), ("params", C.c_double * 64)]


class BatchSeq(C.Structure):
    _fields_ = [("model", C.c_int), ("n", C.c_int), ("T", C.c_int), ("use_proposal", C.c_int),
                ("seed", C.c_uint64), ("x0", C.c_void_p), ("z", C.c_void_p), ("z_mask", C.c_void_p),
                ("xmap_out", C.c_void_p), ("logpost_out", C.c_void_p)]


class BatchInfo(C.Structure):
    _fields_ = [("count", C.c_int), ("T_max", C.c_int), ("waves", C.c_int), ("grid", C.c_int),
                ("lds_bytes", C.c_size_t), ("device_bytes", C.c_size_t), ("tuned_ms", C.c_double * 2)]


class InitExample(C.Structure):
    _fields_ = [("model", C.c_int), ("t", C.c_int), ("n", C.c_int), ("n_prev", C.c_int),
                ("x_prev", C.c_void_p), ("phi_prev", C.c_void_p), ("z", C.c_void_p), ("z_mask", C.c_void_p),
                ("particles", C.c_void_p), ("seed", C.c_uint64), ("seq", C.c_int)]


class SvgdOpts(C.Structure):
    _fields_ = [("n_iter", C.c_int), ("step", C.c_double), ("bw_scale", C.c_double),
                ("bw_mode", C.c_int), ("trans_mode", C.c_int), ("kernel", C.c_int), ("weights", C.c_int),
                ("step_kernel", C.c_int)]


KERNELS = {"rbf": 0, "imq": 1, "matern32": 2}
STEP_KERNELS = {"auto": 0, "wave": 1, "valu": 2, "mfma": 3, "coop": 4}


_lib = None


def load(path: str = LIB_PATH):
    """Loads libsmsq.so; raises if it is not built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError("libsmsq.so is not built (%s); run __graft_entry__.build()" % path)
    L = C.CDLL(path)
    vp, i32, i64, u64, u32, dbl = C.c_void_p, C.c_int, C.c_long, C.c_uint64, C.c_uint32, C.c_double
    L.smsq_model_create.argtypes = [C.POINTER(ModelDesc), C.POINTER(vp)]
    L.smsq_model_destroy.argtypes = [vp]
    L.smsq_workspace_size.argtypes = [vp, i32, i32, i32, i32, C.POINTER(C.c_size_t)]
    L.smsq_svgd_step.argtypes = [vp, i32, i32, i32, vp, vp, vp, vp, i32, vp, C.POINTER(SvgdOpts),
                                 vp, vp, C.c_size_t, vp]
    L.smsq_viterbi_step.argtypes = [vp, i32, i32, i32, vp, vp, vp, vp, i32, vp, vp, vp, vp, vp, vp,
                                    dbl, vp, C.c_size_t, vp]
    L.smsq_backtrack_steps.argtypes = [i32, i32, C.POINTER(C.c_int), i32, vp, vp, vp, vp, vp, C.c_size_t, vp]
    L.smsq_backtrack.argtypes = [i32, i32, i32, i32, i32, vp, vp, vp, vp, vp, vp, vp, vp,
                                 C.c_size_t, vp]
    L.smsq_batch_step.argtypes = [vp, i32, i32, i32, i32, vp, i64, vp, vp, i64, vp, i64, i32, vp,
                                  i64, i32, u64, u32, C.POINTER(SvgdOpts), vp, vp, vp, i64, dbl, vp,
                                  C.c_size_t, vp]
    L.smsq_run_batch.argtypes = [vp, i32, i32, i32, i32, vp, vp, vp, u64, C.POINTER(SvgdOpts), vp,
                                 vp, vp, vp, C.c_size_t, vp]
    L.smsq_run_sequence.argtypes = [vp, i32, i32, i32, vp, vp, vp, u64, C.POINTER(SvgdOpts), vp,
                                    vp, vp, vp, C.c_size_t, vp]
    L.smsq_get_device_status.argtypes = [vp, C.POINTER(C.c_int)]
    L.smsq_clear_device_status.argtypes = [vp, vp]
    L.smsq_status_string.argtypes = [C.c_int]
    L.smsq_status_string.restype = C.c_char_p
    L.smsq_max_particles.argtypes = [vp, i32]
    L.smsq_batch_plan_create.argtypes = [C.POINTER(vp), C.POINTER(SvgdOpts), i32, C.POINTER(BatchSeq), i32,
                                         C.POINTER(vp)]
    L.smsq_batch_plan_tune.argtypes = [vp, i32, vp]
    L.smsq_batch_run.argtypes = [vp, i32, vp]
    L.smsq_batch_storage.argtypes = [vp, i32, C.POINTER(vp), C.POINTER(vp), C.POINTER(vp)]
    L.smsq_batch_plan_info.argtypes = [vp, C.POINTER(BatchInfo)]
    L.smsq_batch_status.argtypes = [vp, C.POINTER(C.c_int)]
    L.smsq_batch_plan_destroy.argtypes = [vp]
    L.smsq_init_mlp_create.argtypes = [u64, i32, C.POINTER(vp)]
    L.smsq_init_mlp_destroy.argtypes = [vp]
    L.smsq_init_mlp_params.argtypes = [vp, C.POINTER(vp), C.POINTER(vp), C.POINTER(C.c_size_t)]
    L.smsq_init_mlp_sync.argtypes = [vp, vp]
    L.smsq_init_set_create.argtypes = [C.POINTER(vp), i32, C.POINTER(InitExample), i32, C.POINTER(vp)]
    L.smsq_init_set_destroy.argtypes = [vp]
    L.smsq_init_features.argtypes = [vp, vp, i32, i32, vp, vp, vp, vp]
    L.smsq_init_mlp_forward.argtypes = [vp, i32, vp, vp, vp]
    L.smsq_init_mlp_backward.argtypes = [vp, i32, vp, vp]
    L.smsq_init_mixture_nll.argtypes = [vp, i32, i32, vp, vp, vp, dbl, vp, vp, vp]
    L.smsq_init_mlp_train_step.argtypes = [vp, vp, i32, i32, dbl, vp, vp]
    L.smsq_init_mlp_sample.argtypes = [vp, vp, i32, i32, vp, vp]
    L.smsq_batch_plan_set_init.argtypes = [vp, vp]
    L.smsq_viterbi_lattice_batch.argtypes = [i32, i32, i32, i32, vp, vp, vp, vp, vp, vp, dbl, vp, C.c_size_t, vp]
    L.smsq_run_sequence_noalloc.argtypes = [vp, i32, i32, i32, vp, vp, vp, u64, C.POINTER(SvgdOpts), vp, vp,
                                            vp, vp, vp]
    for name in SYMBOLS:
        fn = getattr(L, name)
        if fn.restype is None or fn.restype is C.c_int:
            fn.restype = C.c_int
    L.smsq_status_string.restype = C.c_char_p
    _lib = L
    return L


def status_string(st: int) -> str:
    return load().smsq_status_string(st).decode()


def _check(st: int, where: str):
    if st != OK:
        raise SmsqError(st, where)


def _dt(dtype) -> int:
    if dtype in (torch.float32, "f32", F32):
        return F32
    if dtype in (torch.float64, "f64", F64):
        return F64
    raise ValueError("dtype must be float32 or float64")


def torch_dtype(dtype) -> torch.dtype:
    return torch.float64 if _dt(dtype) == F64 else torch.float32


def _ptr(t: Optional[torch.Tensor], dtype: Optional[torch.dtype] = None, name: str = "") -> Optional[int]:
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("%s must be a device tensor" % name)
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    if dtype is not None and t.dtype != dtype:
        raise ValueError("%s must have dtype %s, got %s" % (name, dtype, t.dtype))
    return t.data_ptr()


def _stream(stream=None) -> int:
    s = torch.cuda.current_stream() if stream is None else stream
    return s.cuda_stream


def opts(n_iter: int, step: float, bw_scale: float = 1.0, bw_mode: int = 0,
         trans_mode: int = 0, kernel=0, weights: int = 0, step_kernel=0) -> SvgdOpts:
    """SVGD options; kernel: 0/"rbf", 1/"imq", 2/"matern32"; weights 1: mixture
    weights from the previous step's forward-recursion scores (in the drivers);
    step_kernel: 0/"auto", 1/"wave", 2/"valu", 3/"mfma", 4/"coop" (forces a
    step kernel wherever the shape fits it)."""
    k = KERNELS[kernel] if isinstance(kernel, str) else int(kernel)
    sk = STEP_KERNELS[step_kernel] if isinstance(step_kernel, str) else int(step_kernel)
    return SvgdOpts(int(n_iter), float(step), float(bw_scale), int(bw_mode), int(trans_mode), k, int(weights), sk)


def opts_from(o, step_kernel=0) -> SvgdOpts:
    return opts(o.n_iter, o.step, o.bw_scale, o.bw_mode, o.trans_mode, getattr(o, "kernel", 0),
                getattr(o, "weights", 0), step_kernel)


class Model:
    """Owns a model handle (smsq_model_create / smsq_model_destroy)."""

    def __init__(self, desc):
        L = load()
        md = ModelDesc()
        md.kind, md.d, md.obs_dim, md.n_obs = int(desc.kind), int(desc.d), int(desc.obs_dim), int(desc.n_obs)
        q = np.zeros(16)
        q[:len(desc.q_var)] = desc.q_var
        p = np.zeros(64)
        p[:len(desc.params)] = desc.params
        md.q_var[:] = list(q)
        md.params[:] = list(p)
        h = C.c_void_p()
        _check(L.smsq_model_create(C.byref(md), C.byref(h)), "smsq_model_create")
        self.handle = h
        self.d = md.d
        self.obs_dim = md.obs_dim
        self.n_obs = md.n_obs

    def close(self):
        if self.handle:
            load().smsq_model_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def max_particles(self, dtype) -> int:
        return load().smsq_max_particles(self.handle, _dt(dtype))

    def workspace_size(self, dtype, batch: int, T: int, n: int) -> int:
        b = C.c_size_t(0)
        _check(load().smsq_workspace_size(self.handle, _dt(dtype), batch, T, n, C.byref(b)),
               "smsq_workspace_size")
        return b.value


HEADER_BYTES = 256


def workspace(nbytes: int = HEADER_BYTES, device="cuda") -> torch.Tensor:
    """Zeroed device workspace of nbytes bytes."""
    return torch.zeros(max(int(nbytes), HEADER_BYTES), dtype=torch.uint8, device=device)


def device_status(ws: torch.Tensor) -> int:
    torch.cuda.synchronize()
    out = C.c_int(0)
    _check(load().smsq_get_device_status(_ptr(ws, torch.uint8, "ws"), C.byref(out)),
           "smsq_get_device_status")
    return out.value


def clear_device_status(ws: torch.Tensor, stream=None):
    _check(load().smsq_clear_device_status(_ptr(ws, torch.uint8, "ws"), _stream(stream)),
           "smsq_clear_device_status")


def svgd_step(model: Model, dtype, t: int, x_prev: torch.Tensor, log_w_prev: Optional[torch.Tensor],
              z_t: torch.Tensor, z_mask: Optional[torch.Tensor], x: torch.Tensor, o: SvgdOpts,
              h_out: Optional[torch.Tensor] = None, ws: Optional[torch.Tensor] = None, stream=None):
    """In-place SVGD step on x [n, d] (smsq_svgd_step)."""
    td = torch_dtype(dtype)
    ws = workspace() if ws is None else ws
    st = load().smsq_svgd_step(model.handle, _dt(dtype), t, x_prev.shape[0], _ptr(x_prev, td, "x_prev"),
                               _ptr(log_w_prev, td, "log_w_prev"), _ptr(z_t, td, "z_t"),
                               _ptr(z_mask, torch.uint8, "z_mask"), x.shape[0], _ptr(x, td, "x"),
                               C.byref(o), _ptr(h_out, td, "h_out"), _ptr(ws, torch.uint8, "ws"),
                               ws.numel(), _stream(stream))
    _check(st, "smsq_svgd_step")
    return x


def _out(t: torch.Tensor, dtype, n: int, name: str) -> torch.Tensor:
    if t.dtype != dtype or t.numel() != n or not t.is_contiguous():
        raise ValueError(f"{name}: expected a contiguous {dtype} tensor of {n} elements")
    return t


def viterbi_step(model: Optional[Model], dtype, t: int, phi_prev: torch.Tensor, *, x_prev=None,
                 z_t=None, z_mask=None, x=None, lattice=None, loglik=None, tie_tol: float = 0.0,
                 want_flags: bool = True, ws: Optional[torch.Tensor] = None, stream=None,
                 phi_out: Optional[torch.Tensor] = None, psi_out: Optional[torch.Tensor] = None):
    """Forward-recursion step (smsq_viterbi_step).  Returns (phi, psi, flags);
    phi_out / psi_out, when given, are contiguous [n] tensors written in place
    (e.g. a row of a [T, n] back-pointer array)."""
    td = torch_dtype(dtype)
    n_prev = phi_prev.shape[0]
    n = lattice.shape[0] if lattice is not None else x.shape[0]
    dev = phi_prev.device
    phi = torch.empty(n, dtype=td, device=dev) if phi_out is None else _out(phi_out, td, n, "phi_out")
    psi = torch.empty(n, dtype=torch.int32, device=dev) if psi_out is None else _out(psi_out, torch.int32, n, "psi_out")
    flags = torch.empty(n, dtype=torch.uint8, device=dev) if want_flags else None
    ws = workspace(device=dev) if ws is None else ws
    st = load().smsq_viterbi_step(model.handle if model is not None else None, _dt(dtype), t, n_prev,
                                  _ptr(x_prev, td, "x_prev"), _ptr(phi_prev, td, "phi_prev"),
                                  _ptr(z_t, td, "z_t"), _ptr(z_mask, torch.uint8, "z_mask"), n,
                                  _ptr(x, td, "x"), _ptr(lattice, td, "lattice"),
                                  _ptr(loglik, td, "loglik"), _ptr(phi, td), _ptr(psi), _ptr(flags),
                                  float(tie_tol), _ptr(ws, torch.uint8, "ws"), ws.numel(),
                                  _stream(stream))
    _check(st, "smsq_viterbi_step")
    return phi, psi, flags


def viterbi_lattice_batch(dtype, phi_prev: torch.Tensor, lattice: torch.Tensor, loglik: torch.Tensor,
                          tie_tol: float = 0.0, want_flags: bool = True, ws: Optional[torch.Tensor] = None,
                          stream=None):
    """Lattice-mode forward recursion of B lattices in one launch
    (smsq_viterbi_lattice_batch): phi_prev [B, n_prev], lattice [B, n, n_prev],
    loglik [B, n].  Returns (phi [B, n], psi [B, n], flags [B, n] or None)."""
    td = torch_dtype(dtype)
    B, n, n_prev = lattice.shape
    dev = lattice.device
    phi = torch.empty((B, n), dtype=td, device=dev)
    psi = torch.empty((B, n), dtype=torch.int32, device=dev)
    flags = torch.empty((B, n), dtype=torch.uint8, device=dev) if want_flags else None
    ws = workspace(device=dev) if ws is None else ws
    st = load().smsq_viterbi_lattice_batch(_dt(dtype), B, n, n_prev, _ptr(lattice, td, "lattice"),
                                           _ptr(loglik, td, "loglik"), _ptr(phi_prev, td, "phi_prev"), _ptr(phi),
                                           _ptr(psi), _ptr(flags), float(tie_tol), _ptr(ws, torch.uint8, "ws"),
                                           ws.numel(), _stream(stream))
    _check(st, "smsq_viterbi_lattice_batch")
    return phi, psi, flags


def backtrack(dtype, psi: torch.Tensor, phi_T: torch.Tensor, particles=None, x0=None,
              ws: Optional[torch.Tensor] = None, stream=None):
    """Backtracking over [batch, T, n] back-pointers.  Returns (idx, J, xmap or None)."""
    td = torch_dtype(dtype)
    if psi.dim() == 2:
        psi = psi.unsqueeze(0)
        phi_T = phi_T.unsqueeze(0)
        if particles is not None:
            particles = particles.unsqueeze(0)
            x0 = x0.unsqueeze(0)
    B, T, n = psi.shape
    d = particles.shape[-1] if particles is not None else 0
    dev = psi.device
    idx = torch.empty((B, T), dtype=torch.int32, device=dev)
    J = torch.empty(B, dtype=td, device=dev)
    xmap = torch.empty((B, T + 1, d), dtype=td, device=dev) if particles is not None else None
    ws = workspace(device=dev) if ws is None else ws
    st = load().smsq_backtrack(_dt(dtype), B, T, n, d, _ptr(psi, torch.int32, "psi"),
                               _ptr(phi_T, td, "phi_T"), _ptr(idx), _ptr(J), _ptr(particles, td, "particles"),
                               _ptr(x0, td, "x0"), _ptr(xmap), _ptr(ws, torch.uint8, "ws"), ws.numel(),
                               _stream(stream))
    _check(st, "smsq_backtrack")
    return idx, J, xmap


def backtrack_steps(dtype, psi: torch.Tensor, phi_T: torch.Tensor, n_t, ws: Optional[torch.Tensor] = None,
                    stream=None):
    """Backtracking of one sequence whose particle count changes by step:
    psi [T, n_max] int32 (row t-1: psi_t in its first n_t[t] entries), phi_T
    [n_t[T]], n_t the T + 1 counts (n_t[0] = 1).  Returns (idx [T], J [1])."""
    td = torch_dtype(dtype)
    T, n_max = psi.shape
    counts = [int(c) for c in n_t]
    if len(counts) != T + 1:
        raise ValueError("n_t needs T + 1 = %d counts, got %d" % (T + 1, len(counts)))
    dev = psi.device
    idx = torch.empty(T, dtype=torch.int32, device=dev)
    J = torch.empty(1, dtype=td, device=dev)
    ws = workspace(HEADER_BYTES + 4 * (T + 1), device=dev) if ws is None else ws
    arr = (C.c_int * (T + 1))(*counts)
    st = load().smsq_backtrack_steps(_dt(dtype), T, arr, n_max, _ptr(psi, torch.int32, "psi"),
                                     _ptr(phi_T, td, "phi_T"), _ptr(idx), _ptr(J), _ptr(ws, torch.uint8, "ws"),
                                     ws.numel(), _stream(stream))
    _check(st, "smsq_backtrack_steps")
    return idx, J


def _batched(t: Optional[torch.Tensor], dtype: Optional[torch.dtype], name: str):
    """(pointer, element stride between sequences) of a [B, ...] view whose
    per-sequence block is contiguous."""
    if t is None:
        return None, 0
    if not t.is_cuda:
        raise ValueError("%s must be a device tensor" % name)
    if dtype is not None and t.dtype != dtype:
        raise ValueError("%s must have dtype %s, got %s" % (name, dtype, t.dtype))
    inner = t[0] if t.shape[0] > 0 else t
    if not inner.is_contiguous():
        raise ValueError("%s: each sequence's block must be contiguous" % name)
    return t.data_ptr(), (t.stride(0) if t.shape[0] > 1 else inner.numel())


def batch_step(model: Model, dtype, t: int, x_prev: torch.Tensor, phi_prev: Optional[torch.Tensor],
               z_t: torch.Tensor, z_mask: Optional[torch.Tensor], x: torch.Tensor, o: SvgdOpts, *,
               init_given: bool = False, seed: int = 0, seq_offset: int = 0, phi=None, psi=None,
               flags=None, tie_tol: float = 0.0, ws: Optional[torch.Tensor] = None, stream=None):
    """One step of Algorithm 2 for a batch (smsq_batch_step).

    x_prev [B, n_prev, d], phi_prev [B, n_prev] or None (t = 1), z_t [B, obs_dim],
    z_mask [B, n_obs] or None, x [B, n, d]; phi / psi / flags [B, n].  Each may be
    a strided view (e.g. one step of a [B, T, ...] buffer) as long as every
    sequence's block is contiguous.  phi_prev, phi, psi and flags share one
    stride.
    Returns (phi, psi, flags).
    """
    td = torch_dtype(dtype)
    B, n, _ = x.shape
    dev = x.device
    phi = torch.empty((B, n), dtype=td, device=dev) if phi is None else phi
    psi = torch.empty((B, n), dtype=torch.int32, device=dev) if psi is None else psi
    ws = workspace(device=dev) if ws is None else ws
    xp_ptr, xp_s = _batched(x_prev, td, "x_prev")
    ph_ptr, ph_s = _batched(phi_prev, td, "phi_prev")
    z_ptr, z_s = _batched(z_t, td, "z_t")
    m_ptr, m_s = _batched(z_mask, torch.uint8, "z_mask")
    x_ptr, x_s = _batched(x, td, "x")
    phi_ptr, o_s = _batched(phi, td, "phi")
    psi_ptr, o_s2 = _batched(psi, torch.int32, "psi")
    fl_ptr, o_s3 = _batched(flags, torch.uint8, "flags")
    if o_s2 != o_s or (flags is not None and o_s3 != o_s) or (phi_prev is not None and B > 1 and ph_s != o_s):
        raise ValueError("phi_prev, phi, psi and flags must share one sequence stride")
    st = load().smsq_batch_step(model.handle, _dt(dtype), B, t, x_prev.shape[1], xp_ptr, xp_s, ph_ptr,
                                z_ptr, z_s, m_ptr, m_s, n, x_ptr, x_s, 1 if init_given else 0, int(seed),
                                int(seq_offset), C.byref(o), phi_ptr, psi_ptr, fl_ptr, o_s,
                                float(tie_tol), _ptr(ws, torch.uint8, "ws"), ws.numel(), _stream(stream))
    _check(st, "smsq_batch_step")
    return phi, psi, flags


def run_batch(model: Model, dtype, x0: torch.Tensor, z: torch.Tensor, z_mask: Optional[torch.Tensor],
              n: int, o: SvgdOpts, seed: int, *, particles: Optional[torch.Tensor] = None,
              ws: Optional[torch.Tensor] = None, stream=None):
    """Algorithm 2 for B sequences (smsq_run_batch).  x0 [B, d], z [B, T, obs_dim].

    Returns (xmap [B, T+1, d], J [B]).
    """
    td = torch_dtype(dtype)
    B, T, _ = z.shape
    d = x0.shape[1]
    dev = x0.device
    if ws is None:
        ws = workspace(model.workspace_size(dtype, B, T, n), device=dev)
    xmap = torch.empty((B, T + 1, d), dtype=td, device=dev)
    J = torch.empty(B, dtype=td, device=dev)
    st = load().smsq_run_batch(model.handle, _dt(dtype), B, T, n, _ptr(x0, td, "x0"), _ptr(z, td, "z"),
                               _ptr(z_mask, torch.uint8, "z_mask"), int(seed), C.byref(o), _ptr(xmap),
                               _ptr(J), _ptr(particles, td, "particles"), _ptr(ws, torch.uint8, "ws"),
                               ws.numel(), _stream(stream))
    _check(st, "smsq_run_batch")
    return xmap, J


def run_sequence(model: Model, dtype, x0: torch.Tensor, z: torch.Tensor, z_mask: Optional[torch.Tensor],
                 n: int, o: SvgdOpts, seed: int, *, particles: Optional[torch.Tensor] = None,
                 ws: Optional[torch.Tensor] = None, stream=None):
    """Algorithm 2 for one sequence (smsq_run_sequence).  x0 [d], z [T, obs_dim]."""
    td = torch_dtype(dtype)
    T = z.shape[0]
    d = x0.shape[0]
    dev = x0.device
    if ws is None:
        ws = workspace(model.workspace_size(dtype, 1, T, n), device=dev)
    xmap = torch.empty((T + 1, d), dtype=td, device=dev)
    J = torch.empty(1, dtype=td, device=dev)
    st = load().smsq_run_sequence(model.handle, _dt(dtype), T, n, _ptr(x0, td, "x0"), _ptr(z, td, "z"),
                                  _ptr(z_mask, torch.uint8, "z_mask"), int(seed), C.byref(o), _ptr(xmap),
                                  _ptr(J), _ptr(particles, td, "particles"), _ptr(ws, torch.uint8, "ws"),
                                  ws.numel(), _stream(stream))
    _check(st, "smsq_run_sequence")
    return xmap, J


def run_sequence_noalloc(model: Model, dtype, x0: torch.Tensor, z: torch.Tensor, z_mask: Optional[torch.Tensor],
                         n: int, o: SvgdOpts, seed: int, *, particles: Optional[torch.Tensor] = None,
                         stream=None):
    """Algorithm 2 for one sequence in the library's own device memory
    (smsq_run_sequence_noalloc: no workspace, nothing allocated by the call).
    Returns (xmap [T+1, d], J [1], status [1] int32)."""
    td = torch_dtype(dtype)
    T = z.shape[0]
    d = x0.shape[0]
    dev = x0.device
    xmap = torch.empty((T + 1, d), dtype=td, device=dev)
    J = torch.empty(1, dtype=td, device=dev)
    status = torch.empty(1, dtype=torch.int32, device=dev)
    st = load().smsq_run_sequence_noalloc(model.handle, _dt(dtype), T, n, _ptr(x0, td, "x0"), _ptr(z, td, "z"),
                                          _ptr(z_mask, torch.uint8, "z_mask"), int(seed), C.byref(o), _ptr(xmap),
                                          _ptr(J), _ptr(particles, td, "particles"), _ptr(status),
                                          _stream(stream))
    _check(st, "smsq_run_sequence_noalloc")
    return xmap, J, status


class BatchPlan:
    """Batched ragged plan (smsq_batch_plan_*): independent FP32 sequences of
    different model family, n and T, one persistent launch per time step.

    models: list of Model; opts: list of SvgdOpts (one per model);
    seqs: list of dicts with keys model, n, x0 [d], z [T, obs_dim], z_mask
    ([T, n_obs] uint8 or None), seed, use_proposal (optional, default 1;
    only matters once a proposal network is set).
    The plan allocates xmap [T+1, d] and J [1] per sequence (``xmap``, ``J``).
    """

    def __init__(self, models, opts_list, seqs):
        L = load()
        self.models = models
        self.opts = (SvgdOpts * len(opts_list))(*opts_list)
        self._keep = []
        self.xmap, self.J = [], []
        arr = (BatchSeq * len(seqs))()
        for i, q in enumerate(seqs):
            k = int(q["model"])
            d = models[k].d if 0 <= k < len(models) else 1  # a bad index is the C ABI's to reject
            z = q["z"]
            T = z.shape[0]
            x0 = q["x0"]
            xm = torch.empty((T + 1, d), dtype=torch.float32, device=x0.device)
            J = torch.empty(1, dtype=torch.float32, device=x0.device)
            self.xmap.append(xm)
            self.J.append(J)
            mask = q.get("z_mask")
            self._keep += [x0, z, mask]
            arr[i] = BatchSeq(k, int(q["n"]), int(T), int(q.get("use_proposal", 1)), int(q["seed"]),
                              _ptr(x0, torch.float32, "x0"), _ptr(z, torch.float32, "z"),
                              _ptr(mask, torch.uint8, "z_mask"), _ptr(xm), _ptr(J))
        handles = (C.c_void_p * len(models))(*[m.handle for m in models])
        h = C.c_void_p()
        _check(L.smsq_batch_plan_create(handles, self.opts, len(models), arr, len(seqs), C.byref(h)),
               "smsq_batch_plan_create")
        self.handle = h
        self.count = len(seqs)
        self.seqs = seqs

    def tune(self, steps: int = 3, stream=None):
        _check(load().smsq_batch_plan_tune(self.handle, int(steps), _stream(stream)), "smsq_batch_plan_tune")
        return self.info()

    def run(self, use_graph: bool = False, stream=None):
        _check(load().smsq_batch_run(self.handle, 1 if use_graph else 0, _stream(stream)), "smsq_batch_run")

    def set_init(self, mlp: Optional["InitMLP"]):
        """Initial particles of steps t >= 2 from the proposal network (None:
        the predictive initialisation)."""
        _check(load().smsq_batch_plan_set_init(self.handle, mlp.handle if mlp is not None else None),
               "smsq_batch_plan_set_init")
        self._mlp = mlp

    def info(self) -> dict:
        i = BatchInfo()
        _check(load().smsq_batch_plan_info(self.handle, C.byref(i)), "smsq_batch_plan_info")
        return {"count": i.count, "T_max": i.T_max, "waves": i.waves, "grid": i.grid,
                "lds_bytes": i.lds_bytes, "device_bytes": i.device_bytes, "tuned_ms": list(i.tuned_ms)}

    def status(self) -> int:
        out = C.c_int(0)
        _check(load().smsq_batch_status(self.handle, C.byref(out)), "smsq_batch_status")
        return out.value

    def storage(self, seq: int):
        """Views of sequence seq's particles [T, n, d], phi [T, n] and psi [T, n]."""
        pp, ph, ps = C.c_void_p(), C.c_void_p(), C.c_void_p()
        _check(load().smsq_batch_storage(self.handle, seq, C.byref(pp), C.byref(ph), C.byref(ps)),
               "smsq_batch_storage")
        q = self.seqs[seq]
        T, n, d = q["z"].shape[0], int(q["n"]), self.models[q["model"]].d
        dev = q["x0"].device
        return (_wrap(pp.value, (T, n, d), torch.float32, dev), _wrap(ph.value, (T, n), torch.float32, dev),
                _wrap(ps.value, (T, n), torch.int32, dev))

    def close(self):
        if getattr(self, "handle", None):
            load().smsq_batch_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _wrap(ptr: int, shape, dtype, device) -> torch.Tensor:
    """A tensor copy of device memory owned by the library (copied with a
    device-to-device copy so that torch owns the result)."""
    n = int(np.prod(shape))
    out = torch.empty(shape, dtype=dtype, device=device)
    nbytes = n * out.element_size()
    torch.cuda.synchronize()
    err = _hip().hipMemcpy(C.c_void_p(out.data_ptr()), C.c_void_p(ptr), C.c_size_t(nbytes), 3)
    if err != 0:
        raise RuntimeError("hipMemcpy failed (%d)" % err)
    return out


_hip_lib = None


def _hip():
    global _hip_lib
    if _hip_lib is None:
        _hip_lib = C.CDLL("libamdhip64.so")
        _hip_lib.hipMemcpy.argtypes = [C.c_void_p, C.c_void_p, C.c_size_t, C.c_int]
        _hip_lib.hipMemcpy.restype = C.c_int
    return _hip_lib


def _copy_into(ptr: int, src: torch.Tensor):
    """Device-to-device copy of a contiguous tensor into library-owned memory."""
    src = src.contiguous()
    torch.cuda.synchronize()
    err = _hip().hipMemcpy(C.c_void_p(ptr), C.c_void_p(src.data_ptr()), C.c_size_t(src.numel() * src.element_size()), 3)
    if err != 0:
        raise RuntimeError("hipMemcpy failed (%d)" % err)


N_INIT_PARAMS = 113272
INIT_FEAT, INIT_OUT = 64, 120


class InitMLP:
    """Proposal network of the learned initialisation (smsq_init_mlp_*)."""

    def __init__(self, seed: int = 0, max_batch: int = 4096):
        h = C.c_void_p()
        _check(load().smsq_init_mlp_create(int(seed), int(max_batch), C.byref(h)), "smsq_init_mlp_create")
        self.handle = h
        self.max_batch = max_batch

    def _ptrs(self):
        p, g, n = C.c_void_p(), C.c_void_p(), C.c_size_t()
        _check(load().smsq_init_mlp_params(self.handle, C.byref(p), C.byref(g), C.byref(n)), "smsq_init_mlp_params")
        return p.value, g.value, n.value

    def params(self) -> torch.Tensor:
        p, _, n = self._ptrs()
        return _wrap(p, (n,), torch.float32, "cuda")

    def grads(self) -> torch.Tensor:
        _, g, n = self._ptrs()
        return _wrap(g, (n,), torch.float32, "cuda")

    def set_params(self, P: torch.Tensor):
        p, _, n = self._ptrs()
        if P.numel() != n or P.dtype != torch.float32 or not P.is_cuda:
            raise ValueError("parameters must be a float32 device tensor of %d values" % n)
        _copy_into(p, P)
        _check(load().smsq_init_mlp_sync(self.handle, _stream(None)), "smsq_init_mlp_sync")
        torch.cuda.synchronize()

    def save(self, path: str):
        """Writes the FP32 parameters to a .npy file (no pickled objects)."""
        np.save(path, self.params().detach().cpu().numpy(), allow_pickle=False)

    def load_params(self, path: str):
        """Reads parameters written by save (plain array, allow_pickle=False)
        and refreshes the BF16 weight copies and the optimiser state."""
        P = np.load(path, allow_pickle=False)
        self.set_params(torch.as_tensor(np.ascontiguousarray(P, dtype=np.float32), device="cuda"))

    def forward(self, F: torch.Tensor) -> torch.Tensor:
        B = F.shape[0]
        out = torch.empty((B, INIT_OUT), dtype=torch.float32, device=F.device)
        _check(load().smsq_init_mlp_forward(self.handle, B, _ptr(F, torch.float32, "features"), _ptr(out),
                                            _stream(None)), "smsq_init_mlp_forward")
        return out

    def backward(self, dout: torch.Tensor):
        _check(load().smsq_init_mlp_backward(self.handle, dout.shape[0], _ptr(dout, torch.float32, "dout"),
                                             _stream(None)), "smsq_init_mlp_backward")

    def features(self, iset: "InitSet", first: int = 0, count: Optional[int] = None):
        count = iset.count - first if count is None else count
        F = torch.empty((count, INIT_FEAT), dtype=torch.float32, device="cuda")
        A = torch.empty((count, 8), dtype=torch.float32, device="cuda")
        Sc = torch.empty((count, 8), dtype=torch.float32, device="cuda")
        _check(load().smsq_init_features(self.handle, iset.handle, first, count, _ptr(F), _ptr(A), _ptr(Sc),
                                         _stream(None)), "smsq_init_features")
        return F, A, Sc

    def train_step(self, iset: "InitSet", first: int, count: int, lr: float) -> torch.Tensor:
        loss = torch.empty(1, dtype=torch.float32, device="cuda")
        _check(load().smsq_init_mlp_train_step(self.handle, iset.handle, first, count, float(lr), _ptr(loss),
                                               _stream(None)), "smsq_init_mlp_train_step")
        return loss

    def sample(self, iset: "InitSet", first: int = 0, count: Optional[int] = None) -> torch.Tensor:
        count = iset.count - first if count is None else count
        used = torch.empty(count, dtype=torch.int32, device="cuda")
        _check(load().smsq_init_mlp_sample(self.handle, iset.handle, first, count, _ptr(used), _stream(None)),
               "smsq_init_mlp_sample")
        return used

    def close(self):
        if getattr(self, "handle", None):
            load().smsq_init_mlp_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class InitSet:
    """Examples of the proposal (smsq_init_set_*): dicts with keys model, t,
    x_prev [n_prev, d], phi_prev [n_prev], z [obs_dim], z_mask or None,
    particles [n, d] (targets, or where samples go), seed, seq."""

    def __init__(self, models, examples):
        arr = (InitExample * len(examples))()
        self._keep = []
        for i, q in enumerate(examples):
            P = q["particles"]
            arr[i] = InitExample(int(q["model"]), int(q["t"]), P.shape[0], q["x_prev"].shape[0],
                                 _ptr(q["x_prev"], torch.float32, "x_prev"), _ptr(q["phi_prev"], torch.float32, "phi_prev"),
                                 _ptr(q["z"], torch.float32, "z"), _ptr(q.get("z_mask"), torch.uint8, "z_mask"),
                                 _ptr(P, torch.float32, "particles"), int(q.get("seed", 0)), int(q.get("seq", 0)))
            self._keep += [q["x_prev"], q["phi_prev"], q["z"], q.get("z_mask"), P]
        handles = (C.c_void_p * len(models))(*[m.handle for m in models])
        h = C.c_void_p()
        _check(load().smsq_init_set_create(handles, len(models), arr, len(examples), C.byref(h)),
               "smsq_init_set_create")
        self.handle = h
        self.count = len(examples)
        self.models = models

    def nll(self, out: torch.Tensor, anchors: torch.Tensor, scales: torch.Tensor, first: int = 0,
            gscale: float = 1.0):
        count = out.shape[0]
        loss = torch.empty(count, dtype=torch.float32, device="cuda")
        dout = torch.empty((count, INIT_OUT), dtype=torch.float32, device="cuda")
        _check(load().smsq_init_mixture_nll(self.handle, first, count, _ptr(out, torch.float32, "out"),
                                            _ptr(anchors, torch.float32, "anchors"),
                                            _ptr(scales, torch.float32, "scales"), float(gscale), _ptr(loss),
                                            _ptr(dout), _stream(None)), "smsq_init_mixture_nll")
        return loss, dout

    def close(self):
        if getattr(self, "handle", None):
            load().smsq_init_set_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
