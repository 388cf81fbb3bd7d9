"""Multi-workgroup Algorithm 2 steps (several workgroups per sequence that own
its target tasks and exchange particles, score rows and median data every
SVGD iteration) against the CPU FP64 oracle (Algorithm 2; eq.
SVGD_newupdate, eq. forward_recursion).

The drivers take this path by themselves for sequences of 512 particles or
more while the batch leaves most compute units idle; step_kernel = "coop"
forces it at the smaller ragged sizes here (every size whose 64-particle
tasks split evenly over the workgroups).  Tolerances as in the other parity
tests: J within 1e-3 max(|J|, T) of the oracle's, teacher-forced particles
within 1e-4 of the positions and the move bounds of parity_bounds.py."""
import numpy as np
import pytest
import torch

import oracle as O
from paper_2312_08684_amd import scenarios as S
from paper_2312_08684_amd import smsq
from parity_bounds import check_move

pytestmark = pytest.mark.gpu
DEV = "cuda"


def _run(wl, B, T, n, sk, seed, particles=None):
    model = smsq.Model(wl.model)
    x0 = torch.tensor(wl.x0[:B], dtype=torch.float32, device=DEV)
    z = torch.tensor(wl.z[:B, :T], dtype=torch.float32, device=DEV).contiguous()
    mk = None if wl.mask is None else torch.tensor(wl.mask[:B, :T], dtype=torch.uint8, device=DEV).contiguous()
    ws = smsq.workspace(model.workspace_size("f32", B, T, n))
    o = smsq.opts(wl.opts.n_iter, wl.opts.step, step_kernel=sk)
    xmap, J = smsq.run_batch(model, "f32", x0, z, mk, n, o, seed, particles=particles, ws=ws)
    torch.cuda.synchronize()
    return xmap.cpu().double().numpy(), J.cpu().double().numpy(), smsq.device_status(ws)


# (workload, n, T, L): 4, 6, 4 and 16 target tasks; ragged tails of 56, 54, 6 and 24
@pytest.mark.parametrize("name,n,T,L", [("range2d", 200, 8, 10), ("cv4d", 330, 6, 10), ("growth1d", 250, 10, 30),
                                        ("arm7", 1000, 4, 20)])
def test_coop_free_running_against_oracle(name, n, T, L):
    print("CASE coop free-running", name, n, T, L, flush=True)
    wl = S.make_workload(name, B=2, seed=1400, T=T, n=n, n_iter=L)
    xg, Jg, st = _run(wl, 2, T, n, "coop", 41)
    assert st == smsq.OK
    for b in range(2):
        mask = None if wl.mask is None else wl.mask[b]
        res = O.run_sequence(wl.model, T, n, wl.x0[b], wl.z[b], mask, 41, b, L, wl.opts.step)
        dJ = abs(Jg[b] - res["J"]) / max(abs(res["J"]), T)
        Jpath = O.path_score(wl.model, xg[b], wl.z[b], mask)
        print("seq %d: J coop %.6f oracle %.6f rel %.3e (FP32 vs FP64), path score %.6f"
              % (b, Jg[b], res["J"], dJ, Jpath), flush=True)
        assert dJ <= 1e-3
        assert abs(Jpath - Jg[b]) <= 1e-3 * max(abs(Jg[b]), T)


def test_coop_teacher_forced_step_three_sequences():
    """Three 7-DOF arm sequences of 1024 particles in one launch (16
    workgroups each): step 2 of each from its step-1 particles and the same
    Philox draws, against one oracle SVGD step."""
    print("CASE coop teacher-forced arm7 x3", flush=True)
    wl = S.make_workload("arm7", B=3, seed=1401, T=2)
    B, T, n, d, L = 3, 2, wl.n, wl.model.d, wl.opts.n_iter
    parts = torch.zeros((B, T, n, d), dtype=torch.float32, device=DEV)
    _, _, st = _run(wl, B, T, n, "auto", 43, particles=parts)
    assert st == smsq.OK
    parts = parts.cpu().double().numpy()
    for b in range(B):
        x_init = O.predictive_init(wl.model, 2, parts[b, 0], n, 43, b)
        xo, _, so = O.svgd_step(wl.model, 2, parts[b, 0], None, wl.z[b, 1], None, x_init, L, wl.opts.step)
        assert so == O.OK
        rel = np.linalg.norm(parts[b, 1] - xo) / np.linalg.norm(xo)
        print("seq %d: rel X err %.3e" % (b, rel), flush=True)
        assert rel <= 1e-4
        print("   " + check_move(parts[b, 1], xo, x_init, L, "f32"), flush=True)


def test_coop_agrees_with_one_workgroup_kernel():
    """The same runs on one workgroup per sequence and on several: FP32
    rounding apart (the sums run in another order), the same MAP paths."""
    print("CASE coop vs one workgroup", flush=True)
    wl = S.make_workload("cv4d", B=4, seed=1402, T=6, n=512, n_iter=20)
    xa, Ja, sa = _run(wl, 4, 6, 512, "mfma", 45)
    xb, Jb, sb = _run(wl, 4, 6, 512, "auto", 45)
    assert sa == smsq.OK and sb == smsq.OK
    rel = np.abs(Ja - Jb) / np.maximum(np.abs(Ja), 6)
    print("max rel dJ %.3e, max |dx| %.3e" % (rel.max(), np.abs(xa - xb).max()), flush=True)
    assert rel.max() <= 1e-5
    assert np.abs(xa - xb).max() <= 1e-3


def test_coop_nonfinite_observation_sets_status():
    print("CASE coop non-finite", flush=True)
    wl = S.make_workload("arm7", B=1, seed=1403, T=3, n=1024, n_iter=5)
    wl.z[0, -1, 0] = np.nan      # the last step's observation
    _, _, st = _run(wl, 1, 3, 1024, "auto", 47)
    assert st == smsq.ERR_NONFINITE
    wl = S.make_workload("arm7", B=1, seed=1403, T=3, n=1024, n_iter=5)
    _, _, st = _run(wl, 1, 3, 1024, "auto", 47)
    assert st == smsq.OK
