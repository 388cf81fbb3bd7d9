"""Stein-MAP-Seq CPU FP64 oracle -- TEST INFRASTRUCTURE ONLY.

A numpy/ctypes front-end to ``smsq_oracle.c``: a plain scalar FP64
implementation of the method, written from the paper (arXiv 2312.08684).  Only
the tests, the smoke check and the benchmark's CPU-baseline leg may import
this package; the product library never does, and this package imports
nothing from it.

Passages followed (paper numbering): eq. SSM (models), eq. SVGD_newupdate /
SVGD_initial_newupdate (Stein step, Lemma IV.3), eq. forward_recursion,
backtracking (Sec. IV-B), Algorithm 2 (Stein-MAP-Seq), J(s) of Theorem IV.1.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "smsq_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lock = threading.Lock()
_lib = None

OK, INVALID, NONFINITE = 0, 1, 4


class OrModel(C.Structure):
    _fields_ = [("kind", C.c_int), ("d", C.c_int), ("obs_dim", C.c_int), ("n_obs", C.c_int),
                ("q_var", C.c_double * 16), ("params", C.c_double * 64)]


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (-O2, no FP contraction, no fast-math)."""
    if force or not os.path.exists(_LIB_PATH) or \
            os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fPIC",
                               "-fopenmp", "-shared", "-std=c99", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


_dp = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_ip = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
_u8 = np.ctypeslib.ndpointer(dtype=np.uint8, flags="C_CONTIGUOUS")
_u32 = np.ctypeslib.ndpointer(dtype=np.uint32, flags="C_CONTIGUOUS")
_vp = C.c_void_p


def lib():
    global _lib
    with _lock:
        if _lib is None:
            L = C.CDLL(build())
            M = C.POINTER(OrModel)
            L.or_philox4x32_10.argtypes = [_u32, _u32, _u32]
            L.or_set_threads.argtypes = [C.c_int]
            L.or_get_threads.restype = C.c_int
            L.or_normals.argtypes = [C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint32, C.c_int, _dp]
            L.or_transition_mean.argtypes = [M, C.c_int, _dp, _dp]
            L.or_log_transition.argtypes = [M, _dp, _dp]
            L.or_log_transition.restype = C.c_double
            L.or_loglik.argtypes = [M, _dp, _vp, _dp]
            L.or_loglik.restype = C.c_double
            L.or_grad_loglik.argtypes = [M, _dp, _vp, _dp, _dp]
            L.or_arm_fk.argtypes = [M, _dp, _dp]
            L.or_lower_median.argtypes = [_dp, C.c_long]
            L.or_lower_median.restype = C.c_double
            L.or_bandwidth.argtypes = [_dp, C.c_int, C.c_int, C.c_double, C.POINTER(C.c_double)]
            L.or_bandwidth.restype = C.c_double
            L.or_scores.argtypes = [M, C.c_int, _dp, _vp, _dp, _vp, C.c_int, _dp, C.c_int, _dp]
            L.or_kernel.argtypes = [C.c_int, C.c_double, C.c_double, C.POINTER(C.c_double),
                                    C.POINTER(C.c_double)]
            L.or_stein_phi.argtypes = [C.c_int, C.c_int, _dp, _dp, C.c_double, C.c_int, _dp]
            L.or_svgd_step.argtypes = [M, C.c_int, C.c_int, _dp, _vp, _dp, _vp, C.c_int, _dp,
                                       C.c_int, C.c_double, C.c_double, C.c_int, C.c_int, C.c_int,
                                       _vp]
            L.or_viterbi_lattice.argtypes = [C.c_int, C.c_int, _dp, _dp, _dp, C.c_double,
                                             _dp, _ip, _u8]
            L.or_viterbi_particle.argtypes = [M, C.c_int, C.c_int, _dp, _dp, _dp, _vp, C.c_int,
                                              _dp, C.c_double, _dp, _ip, _u8]
            L.or_particle_lattice.argtypes = [M, C.c_int, C.c_int, _dp, _dp, _vp, C.c_int, _dp,
                                              _dp, _dp]
            L.or_backtrack.argtypes = [C.c_int, C.c_int, _ip, _dp, _ip, C.POINTER(C.c_double)]
            L.or_path_score.argtypes = [M, C.c_int, _dp, _dp, _vp]
            L.or_path_score.restype = C.c_double
            L.or_predictive_init.argtypes = [M, C.c_int, C.c_int, _dp, C.c_int, C.c_uint64,
                                             C.c_uint32, _dp]
            L.or_run_sequence.argtypes = [M, C.c_int, C.c_int, _dp, _dp, _vp, C.c_uint64,
                                          C.c_uint32, C.c_int, C.c_double, C.c_double, C.c_int,
                                          C.c_int, C.c_int, C.c_int, _dp, C.POINTER(C.c_double), _vp,
                                          _vp, _vp, _vp]
            _lib = L
    return _lib


def model(desc) -> OrModel:
    """OrModel from any object with kind, d, obs_dim, n_obs, q_var, params."""
    m = OrModel()
    m.kind, m.d, m.obs_dim, m.n_obs = int(desc.kind), int(desc.d), int(desc.obs_dim), int(desc.n_obs)
    q = np.zeros(16)
    q[:len(desc.q_var)] = desc.q_var
    p = np.zeros(64)
    p[:len(desc.params)] = desc.params
    m.q_var[:] = list(q)
    m.params[:] = list(p)
    return m


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _maskptr(mask):
    if mask is None:
        return None, None
    m = np.ascontiguousarray(mask, dtype=np.uint8)
    return m, m.ctypes.data


def set_threads(n: int) -> None:
    """Threads of the oracle's particle loops and median sort (results do
    not depend on it)."""
    lib().or_set_threads(int(n))


def get_threads() -> int:
    return int(lib().or_get_threads())


# -- primitives ------------------------------------------------------------------

def philox4x32_10(ctr, key):
    out = np.zeros(4, dtype=np.uint32)
    lib().or_philox4x32_10(np.ascontiguousarray(ctr, dtype=np.uint32),
                           np.ascontiguousarray(key, dtype=np.uint32), out)
    return out


def normals(seed, seq, t, i, d):
    out = np.zeros(16)
    lib().or_normals(seed, seq, t, i, d, out)
    return out[:d].copy()


def transition_mean(desc, t, x):
    x = _f64(x)
    out = np.zeros(desc.d)
    lib().or_transition_mean(C.byref(model(desc)), t, x, out)
    return out


def log_transition(desc, x, mean):
    return lib().or_log_transition(C.byref(model(desc)), _f64(x), _f64(mean))


def loglik(desc, z, mask, x):
    mk, mp = _maskptr(mask)
    return lib().or_loglik(C.byref(model(desc)), _f64(z), mp, _f64(x))


def grad_loglik(desc, z, mask, x):
    mk, mp = _maskptr(mask)
    g = np.zeros(desc.d)
    lib().or_grad_loglik(C.byref(model(desc)), _f64(z), mp, _f64(x), g)
    return g


def arm_fk(desc, q):
    out = np.zeros(3)
    lib().or_arm_fk(C.byref(model(desc)), _f64(q), out)
    return out


def lower_median(values):
    v = _f64(values).copy()
    return lib().or_lower_median(v, v.size)


def bandwidth(x, bw_scale=1.0):
    x = _f64(x)
    med = C.c_double(0.0)
    h = lib().or_bandwidth(x, x.shape[0], x.shape[1], bw_scale, C.byref(med))
    return h, med.value


def scores(desc, t, x_prev, log_w, z, mask, x, trans_mode=0):
    """Scores at particles x given the previous particle set x_prev."""
    x_prev = _f64(x_prev)
    means = np.stack([transition_mean(desc, t, xp) for xp in x_prev])
    return scores_from_means(desc, means, log_w, z, mask, x, trans_mode)


def scores_from_means(desc, means, log_w, z, mask, x, trans_mode=0):
    means = _f64(means)
    x = _f64(x)
    lw = None if log_w is None else _f64(log_w)
    mk, mp = _maskptr(mask)
    s = np.zeros_like(x)
    lib().or_scores(C.byref(model(desc)), means.shape[0], means,
                    None if lw is None else lw.ctypes.data, _f64(z), mp,
                    x.shape[0], x, trans_mode, s)
    return s


KERNEL_RBF, KERNEL_IMQ, KERNEL_MATERN = 0, 1, 2


def kernel(kind, D, h):
    """(f, w) of a kernel at squared distance D: kappa = f, grad_{x_k} kappa = w (x_i - x_k)."""
    f, w = C.c_double(0.0), C.c_double(0.0)
    lib().or_kernel(int(kind), float(D), float(h), C.byref(f), C.byref(w))
    return f.value, w.value


def stein_phi(x, s, h, kernel=KERNEL_RBF):
    x = _f64(x)
    s = _f64(s)
    phi = np.zeros_like(x)
    lib().or_stein_phi(x.shape[0], x.shape[1], x, s, h, int(kernel), phi)
    return phi


def svgd_step(desc, t, x_prev, log_w, z, mask, x, n_iter, step, bw_scale=1.0,
              bw_mode=0, trans_mode=0, kernel=KERNEL_RBF):
    """Returns (updated particles, bandwidth per iteration, status)."""
    x_prev = _f64(x_prev).reshape(-1, desc.d)
    x = _f64(x).reshape(-1, desc.d).copy()
    lw = None if log_w is None else _f64(log_w)
    mk, mp = _maskptr(mask)
    h = np.zeros(max(n_iter, 1))
    st = lib().or_svgd_step(C.byref(model(desc)), t, x_prev.shape[0], x_prev,
                            None if lw is None else lw.ctypes.data, _f64(z), mp,
                            x.shape[0], x, n_iter, step, bw_scale, bw_mode, trans_mode,
                            int(kernel), h.ctypes.data)
    return x, h[:n_iter], st


def viterbi_lattice(A, ell, phi_prev, tie_tol=1e-9):
    A = _f64(A)
    n, n_prev = A.shape
    phi = np.zeros(n)
    psi = np.zeros(n, dtype=np.int32)
    fl = np.zeros(n, dtype=np.uint8)
    st = lib().or_viterbi_lattice(n, n_prev, A, _f64(ell), _f64(phi_prev), tie_tol, phi, psi, fl)
    return phi, psi, fl, st


def viterbi_particle(desc, t, x_prev, phi_prev, z, mask, x, tie_tol=1e-9):
    x_prev = _f64(x_prev).reshape(-1, desc.d)
    x = _f64(x).reshape(-1, desc.d)
    mk, mp = _maskptr(mask)
    n = x.shape[0]
    phi = np.zeros(n)
    psi = np.zeros(n, dtype=np.int32)
    fl = np.zeros(n, dtype=np.uint8)
    st = lib().or_viterbi_particle(C.byref(model(desc)), t, x_prev.shape[0], x_prev,
                                   _f64(phi_prev), _f64(z), mp, n, x, tie_tol, phi, psi, fl)
    return phi, psi, fl, st


def particle_lattice(desc, t, x_prev, z, mask, x):
    x_prev = _f64(x_prev).reshape(-1, desc.d)
    x = _f64(x).reshape(-1, desc.d)
    mk, mp = _maskptr(mask)
    A = np.zeros((x.shape[0], x_prev.shape[0]))
    ell = np.zeros(x.shape[0])
    lib().or_particle_lattice(C.byref(model(desc)), t, x_prev.shape[0], x_prev, _f64(z), mp,
                              x.shape[0], x, A, ell)
    return A, ell


def backtrack(psi, phi_T):
    psi = np.ascontiguousarray(psi, dtype=np.int32)
    T, n = psi.shape
    idx = np.zeros(T, dtype=np.int32)
    J = C.c_double(0.0)
    st = lib().or_backtrack(T, n, psi, _f64(phi_T), idx, C.byref(J))
    return idx, J.value, st


def path_score(desc, path, z, mask=None):
    path = _f64(path)
    mk, mp = _maskptr(mask)
    return lib().or_path_score(C.byref(model(desc)), path.shape[0] - 1, path, _f64(z), mp)


def predictive_init(desc, t, x_prev, n, seed, seq):
    x_prev = _f64(x_prev).reshape(-1, desc.d)
    x = np.zeros((n, desc.d))
    lib().or_predictive_init(C.byref(model(desc)), t, x_prev.shape[0], x_prev, n, seed, seq, x)
    return x


def run_sequence(desc, T, n, x0, z, mask, seed, seq, n_iter, step, bw_scale=1.0,
                 bw_mode=0, trans_mode=0, want_tables=False, kernel=KERNEL_RBF, weights=0):
    """Algorithm 2 for one sequence.  Returns a dict.  weights 1: the previous
    step's forward-recursion scores are the mixture log-weights of the next
    step's target (w_j proportional to exp(phi_{t-1}(j)))."""
    d = desc.d
    mk, mp = _maskptr(mask)
    xmap = np.zeros((T + 1, d))
    J = C.c_double(0.0)
    parts = np.zeros((T, n, d)) if want_tables else None
    phi = np.zeros((T, n)) if want_tables else None
    psi = np.zeros((T, n), dtype=np.int32) if want_tables else None
    idx = np.zeros(T, dtype=np.int32)
    st = lib().or_run_sequence(C.byref(model(desc)), T, n, _f64(x0), _f64(z), mp, seed, seq,
                               n_iter, step, bw_scale, bw_mode, trans_mode, int(kernel), int(weights),
                               xmap, C.byref(J),
                               None if parts is None else parts.ctypes.data,
                               None if phi is None else phi.ctypes.data,
                               None if psi is None else psi.ctypes.data, idx.ctypes.data)
    return dict(xmap=xmap, J=J.value, status=st, particles=parts, phi=phi, psi=psi, idx=idx)
