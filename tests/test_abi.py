"""The C-ABI library loads and exports every symbol include/smsq.h declares;
host-only entry points validate their arguments (no device work)."""
import ctypes as C
import os
import re

import numpy as np

from paper_2312_08684_amd import scenarios as S
from paper_2312_08684_amd import smsq

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    src = open(os.path.join(ROOT, "include", "smsq.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(smsq_[a-z_]+)\s*\(", src)))


def test_every_declared_symbol_is_exported():
    L = smsq.load()
    names = declared_symbols()
    assert len(names) >= 13
    for name in names:
        assert hasattr(L, name), name
    assert sorted(names) == sorted(smsq.SYMBOLS)


def test_status_strings():
    for st in range(6):
        assert smsq.status_string(st)
    assert smsq.status_string(99) == "unknown status"


def test_model_validation_host_only():
    for name in ("growth1d", "range2d", "cv4d", "arm7", "lingauss"):
        m = smsq.Model(S._model_for(name, 0))
        assert m.max_particles("f32") >= (1024 if name != "arm7" else 1024)
        assert m.workspace_size("f32", 2, 10, 64) > 256
        m.close()
    bad = S._model_for("arm7", 0)
    bad.q_var[2] = 0.0
    try:
        smsq.Model(bad)
        raise AssertionError("zero variance accepted")
    except smsq.SmsqError as e:
        assert e.status == smsq.ERR_INVALID
    bad = S._model_for("cv4d", 0)
    bad.obs_dim = 7
    try:
        smsq.Model(bad)
        raise AssertionError("odd detection layout accepted")
    except smsq.SmsqError as e:
        assert e.status == smsq.ERR_INVALID


def test_workspace_size_grows_with_batch():
    m = smsq.Model(S._model_for("range2d", 0))
    a = m.workspace_size("f32", 1, 50, 256)
    b = m.workspace_size("f32", 8, 50, 256)
    c = m.workspace_size("f64", 8, 50, 256)
    assert a < b < c
    assert b >= 8 * 50 * 256 * 2 * 4


def test_viterbi_step_out_tensors_validated_host_only():
    """phi_out / psi_out must be contiguous tensors of the step's dtype and n
    elements; a mismatch is rejected before anything is launched."""
    import torch
    m = smsq.Model(S._model_for("range2d", 0))
    phi_prev = torch.zeros(5)
    x = torch.zeros((7, 2))
    bad = [dict(phi_out=torch.empty(7, dtype=torch.float64)),
           dict(phi_out=torch.empty(6)),
           dict(psi_out=torch.empty(7, dtype=torch.int64)),
           dict(psi_out=torch.empty((7, 2), dtype=torch.int32)[:, 0])]
    for kw in bad:
        try:
            smsq.viterbi_step(m, "f32", 2, phi_prev, x_prev=torch.zeros((5, 2)), z_t=torch.zeros(3), x=x, **kw)
            raise AssertionError("accepted %s" % list(kw))
        except ValueError as e:
            assert "_out" in str(e)
    m.close()


def test_backtrack_steps_validates_counts_host_only():
    """smsq_backtrack_steps checks its sizes, counts (n_t[0] = 1, 1..n_max)
    and workspace size before any device work; the stand-in addresses below
    are never dereferenced."""
    L = smsq.load()
    fake = C.c_void_p(0x1000)

    def call(counts, n_max=8, T=None, ws_bytes=None):
        T = len(counts) - 1 if T is None else T
        arr = (C.c_int * max(1, len(counts)))(*counts)
        wb = smsq.HEADER_BYTES + 4 * (T + 1) if ws_bytes is None else ws_bytes
        return L.smsq_backtrack_steps(smsq.F32, T, arr, n_max, fake, fake, fake, fake, fake, wb, None)

    assert call([1, 3, 8, 2], T=0) == smsq.ERR_INVALID          # T >= 1
    assert call([2, 3, 8, 2]) == smsq.ERR_INVALID              # n_0 = 1
    assert call([1, 3, 9, 2]) == smsq.ERR_INVALID              # above n_max
    assert call([1, 3, 0, 2]) == smsq.ERR_INVALID              # at least one particle
    assert call([1, 3, 8, 2], n_max=0) == smsq.ERR_INVALID
    assert call([1, 3, 8, 2], ws_bytes=smsq.HEADER_BYTES + 15) == smsq.ERR_WORKSPACE
    assert L.smsq_backtrack_steps(smsq.F32, 3, None, 8, fake, fake, fake, fake, fake, 512, None) == smsq.ERR_INVALID
