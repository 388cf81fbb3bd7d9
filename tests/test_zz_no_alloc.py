"""smsq_run_sequence_noalloc (Algorithm 2 in the library's own device memory)
against smsq_run_sequence with a caller workspace: the same kernels, so the
MAP trajectory, J and every step's particles agree bit for bit.  Two calls in
a row, the second smaller than the first (the array keeps the first call's
contents), then a call that sees a non-finite observation (status
SMSQ_ERR_NONFINITE) followed by a clean one (the status word is cleared at
the start of each run), and the size limit (rejected on the host)."""
import numpy as np
import pytest
import torch

import oracle as O
from paper_2312_08684_amd import scenarios as S
from paper_2312_08684_amd import smsq

pytestmark = pytest.mark.gpu
DEV = "cuda"


def _inputs(name, n, T, L, seed, dt):
    wl = S.make_workload(name, B=1, seed=seed, T=T, n=n, n_iter=L)
    td = torch.float64 if dt == "f64" else torch.float32
    x0 = torch.tensor(wl.x0[0], dtype=td, device=DEV)
    z = torch.tensor(wl.z[0], dtype=td, device=DEV)
    mask = None if wl.mask is None else torch.tensor(wl.mask[0], dtype=torch.uint8, device=DEV)
    return wl, x0, z, mask, td


def _both(name, n, T, L, seed, dt, z_override=None):
    wl, x0, z, mask, td = _inputs(name, n, T, L, seed, dt)
    if z_override is not None:
        z = z_override(z)
    model = smsq.Model(wl.model)
    o = smsq.opts_from(wl.opts)
    d = wl.model.d
    pa = torch.zeros((T, n, d), dtype=td, device=DEV)
    pb = torch.zeros((T, n, d), dtype=td, device=DEV)
    print("CASE noalloc", name, n, T, L, dt, flush=True)
    xa, Ja = smsq.run_sequence(model, dt, x0, z, mask, n, o, 17, particles=pa)
    xb, Jb, st = smsq.run_sequence_noalloc(model, dt, x0, z, mask, n, o, 17, particles=pb)
    torch.cuda.synchronize()
    return wl, (xa, Ja, pa), (xb, Jb, pb), int(st.cpu()[0])


@pytest.mark.parametrize("dt", ["f32", "f64"])
def test_noalloc_matches_workspace_entry_point_twice(dt):
    cases = [("range2d", 192, 14, 12), ("range2d", 40, 9, 12)] if dt == "f32" else \
        [("growth1d", 32, 20, 40), ("growth1d", 20, 11, 40)]
    for name, n, T, L in cases:                      # the second call is smaller
        wl, (xa, Ja, pa), (xb, Jb, pb), st = _both(name, n, T, L, 1300, dt)
        assert st == smsq.OK
        assert torch.equal(xa, xb) and torch.equal(Ja, Jb) and torch.equal(pa, pb)
        # and both against the oracle at the parity bar (J within 1e-3 max(|J|, T))
        mask = None if wl.mask is None else wl.mask[0]
        res = O.run_sequence(wl.model, T, n, wl.x0[0], wl.z[0], mask, 17, 0, L, wl.opts.step)
        J = float(Jb.cpu()[0])
        dJ = abs(J - res["J"]) / max(abs(res["J"]), T)
        print("J noalloc %.8f oracle %.8f rel %.3e" % (J, res["J"], dJ))
        assert dJ <= 1e-3


def test_noalloc_status_is_per_run():
    def poison(z):
        z = z.clone()
        z[-1, 0] = float("nan")     # the last step's observation
        return z
    _, _, (_, _, _), st = _both("range2d", 64, 8, 6, 1301, "f32", z_override=poison)
    assert st == smsq.ERR_NONFINITE
    _, (xa, Ja, pa), (xb, Jb, pb), st = _both("range2d", 48, 6, 6, 1302, "f32")
    assert st == smsq.OK
    assert torch.equal(xa, xb) and torch.equal(Ja, Jb)


def test_noalloc_rejects_runs_beyond_its_memory():
    wl, x0, z, mask, td = _inputs("arm7", 1024, 4, 2, 1303, "f32")
    model = smsq.Model(wl.model)
    zbig = torch.zeros((600, 3), dtype=torch.float32, device=DEV)   # 600 x 1024 x 7 FP32 > 16 MiB
    with pytest.raises(smsq.SmsqError) as e:
        smsq.run_sequence_noalloc(model, "f32", x0, zbig, None, 1024, smsq.opts_from(wl.opts), 1)
    assert e.value.status == smsq.ERR_WORKSPACE
