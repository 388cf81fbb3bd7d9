"""The FP32 workloads at their full sizes against the CPU FP64 oracle
(Algorithm 2; eq. SVGD_newupdate, eq. forward_recursion).

Fixtures (tests/golden/full_*.npz) hold the inputs and the oracle's results,
written by tests/golden/make_fullsize_fixtures.py (oracle and input
generator only):
  * free-running: the GPU's J within 1e-3 max(|J|, T) of the oracle's J
    (the benchmark spec's trajectory log-posterior tolerance), and J equal to the
    path score of the GPU's own MAP trajectory (evaluated in FP64 by the
    oracle); the FP32-vs-FP64 differences of J and of the trajectory are
    printed per case;
  * teacher-forced: the oracle's particles of step t_s - 1 and the
    predictive initial particles of step t_s (oracle, same Philox counters)
    go through one GPU SVGD step; the result against the oracle's step-t_s
    particles at the parity tolerances (relative to the positions, and to
    the move as parity_bounds.py states)."""
import os

import numpy as np
import pytest
import torch

import oracle as O
from paper_2312_08684_amd import scenarios as S
from paper_2312_08684_amd import smsq
from parity_bounds import check_move

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
DEV = "cuda"
TOL_J = 1e-3
TOL_X = 1e-4
CASES = ["full_range2d", "full_cv4d", "full_arm7"]


def load_fixture(name):
    f = np.load(os.path.join(GOLDEN, name + ".npz"), allow_pickle=False)
    fx = {k: f[k] for k in f.files}
    fx["workload"] = str(fx["workload"])
    fx["mask"] = fx["mask"] if int(fx["has_mask"]) else None
    return fx


def fixture_model(fx):
    return S.make_workload(fx["workload"], B=1, seed=int(fx["data_seed"]), n=int(fx["n"]), T=int(fx["T"])).model


@pytest.mark.parametrize("name", CASES)
def test_full_size_free_running_against_oracle(name):
    fx = load_fixture(name)
    desc = fixture_model(fx)
    n, T, L = int(fx["n"]), int(fx["T"]), int(fx["L"])
    print("CASE full-size free-running", name, n, T, L, flush=True)
    model = smsq.Model(desc)
    x0 = torch.tensor(fx["x0"], dtype=torch.float32, device=DEV)
    z = torch.tensor(fx["z"], dtype=torch.float32, device=DEV)
    mk = None if fx["mask"] is None else torch.tensor(fx["mask"], dtype=torch.uint8, device=DEV)
    xmap, J = smsq.run_sequence(model, "f32", x0, z, mk, n, smsq.opts(L, float(fx["step"])), int(fx["key"]))
    torch.cuda.synchronize()
    xg = xmap.cpu().double().numpy()
    Jg = float(J.cpu()[0])
    Jo = float(fx["J"])
    dJ = abs(Jg - Jo) / max(abs(Jo), T)
    Jpath = O.path_score(desc, xg, fx["z"], fx["mask"])
    same = np.mean(np.all(np.abs(xg[1:] - fx["xmap"][1:]) <= 1e-3 * (1 + np.abs(fx["xmap"][1:])), axis=1))
    print("J gpu %.6f oracle %.6f: rel %.3e (FP32 vs FP64); path score of the GPU trajectory %.6f; "
          "trajectory max |dx| %.3e, steps within 1e-3: %.3f"
          % (Jg, Jo, dJ, Jpath, np.abs(xg - fx["xmap"]).max(), same), flush=True)
    assert dJ <= TOL_J
    assert abs(Jpath - Jg) <= TOL_J * max(abs(Jg), T)


@pytest.mark.parametrize("name", CASES)
def test_full_size_teacher_forced_step_against_oracle(name):
    fx = load_fixture(name)
    desc = fixture_model(fx)
    n, L, ts = int(fx["n"]), int(fx["L"]), int(fx["t_sample"])
    print("CASE full-size teacher-forced step", name, n, L, "t =", ts, flush=True)
    xprev = fx["x_prev_sample"]
    x_init = O.predictive_init(desc, ts, xprev, n, int(fx["key"]), 0)
    mask = None if fx["mask"] is None else fx["mask"][ts - 1]
    model = smsq.Model(desc)
    xg = torch.tensor(x_init, dtype=torch.float32, device=DEV)
    smsq.svgd_step(model, "f32", ts, torch.tensor(xprev, dtype=torch.float32, device=DEV), None,
                   torch.tensor(fx["z"][ts - 1], dtype=torch.float32, device=DEV),
                   None if mask is None else torch.tensor(mask, dtype=torch.uint8, device=DEV), xg,
                   smsq.opts(L, float(fx["step"])))
    torch.cuda.synchronize()
    xg = xg.cpu().double().numpy()
    xo = fx["x_sample"]
    rel = np.linalg.norm(xg - xo) / np.linalg.norm(xo)
    print("rel X err %.3e" % rel)
    assert rel <= TOL_X
    print(check_move(xg, xo, x_init, L, "f32"))


@pytest.mark.parametrize("n", [1000, 4000])
def test_pf_map_seq_full_size_against_oracle(n):
    """The PF-MAP-Seq workload at the bench's sizes: 200 steps of the
    range-only model over bootstrap-PF sets of n particles (eq.
    forward_recursion, Sec. IV-B).  The GPU recursion (FP32, without tie
    flags, back-pointers written in place as the bench does) and backtrack
    against the oracle's FP64 J (fixture); and the oracle's FP64 score of the
    GPU's particle path against that J."""
    import sys
    if GOLDEN not in sys.path:
        sys.path.insert(0, GOLDEN)
    import make_fullsize_fixtures as MF
    print("CASE pf-map-seq full size", n, flush=True)
    f = np.load(os.path.join(GOLDEN, "pf_map_seq_%d.npz" % n), allow_pickle=False)
    J_o, idx_o = float(f["J"]), f["idx"]
    desc, x0, z, mask, parts = MF.pf_map_seq_inputs(n)
    T = parts.shape[0]
    model = smsq.Model(desc)
    ws = smsq.workspace()
    P = torch.tensor(parts, dtype=torch.float32, device=DEV)
    X0 = torch.tensor(x0, dtype=torch.float32, device=DEV)
    Z = torch.tensor(z, dtype=torch.float32, device=DEV)
    M = torch.tensor(mask, dtype=torch.uint8, device=DEV)
    psi_all = torch.empty((T, n), dtype=torch.int32, device=DEV)
    phi_buf = [torch.empty(n, dtype=torch.float32, device=DEV) for _ in range(2)]
    phi = torch.zeros(1, dtype=torch.float32, device=DEV)
    for t in range(1, T + 1):
        phi, _, _ = smsq.viterbi_step(model, "f32", t, phi, x_prev=X0 if t == 1 else P[t - 2], z_t=Z[t - 1],
                                      z_mask=M[t - 1], x=P[t - 1], want_flags=False, ws=ws,
                                      phi_out=phi_buf[t % 2], psi_out=psi_all[t - 1])
    idx, J, _ = smsq.backtrack("f32", psi_all, phi, ws=ws)
    assert smsq.device_status(ws) == smsq.OK
    J = float(J.cpu().reshape(-1)[0])
    idx = idx.cpu().numpy().reshape(-1)
    path = np.concatenate([x0, parts[np.arange(T), idx]])
    J_path = O.path_score(desc, path, z, mask)
    tol = TOL_J * max(abs(J_o), T)
    print("J gpu %.6f oracle %.6f (rel %.2e); oracle score of the gpu path %.6f; path agreement %.3f"
          % (J, J_o, abs(J - J_o) / max(abs(J_o), T), J_path, np.mean(idx == idx_o)), flush=True)
    assert abs(J - J_o) <= tol
    assert abs(J_path - J_o) <= tol
