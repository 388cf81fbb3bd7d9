"""Batched ragged form (smsq_batch_plan_*): sequences of different model
family, particle count and length advance one time step per persistent
launch.  Every sequence's result must match the single-sequence path
(smsq_run_sequence, same model, n, T, seed and options): the batched launch
runs the same step body per sequence, and neither the exact median, the
per-task sums nor the forward recursion depends on which workgroup shape
took the step.  The body is compiled into a different kernel, where the
compiler may contract a few multiply-adds differently, so particles agree to
a few FP32 ulps (measured up to 1e-7 of the particle scale after 9 steps),
not bit for bit; the bound below is a hundred times that.  hipGraph replays must reproduce the
eager run bit for bit."""
import numpy as np
import pytest
import torch

import oracle as O
from paper_2312_08684_amd import scenarios as S
from paper_2312_08684_amd import smsq

pytestmark = pytest.mark.gpu

# (family, n, T, L): ragged in every dimension; n spans one to sixteen
# 64-particle tasks, with ragged tails
MIX = [
    ("arm7", 1024, 4, 12),
    ("cv4d", 512, 6, 10),
    ("range2d", 256, 9, 10),
    ("growth1d", 32, 7, 20),
    ("arm7", 200, 5, 12),
    ("range2d", 100, 3, 10),
    ("cv4d", 96, 8, 10),
    ("growth1d", 64, 2, 20),
    ("arm7", 64, 6, 12),
]


def _build(mix, base_seed=0):
    models, opts, seqs = [], [], []
    for i, (name, n, T, L) in enumerate(mix):
        wl = S.make_workload(name, B=1, seed=base_seed + i, n=n, T=T, n_iter=L)
        models.append(smsq.Model(wl.model))
        opts.append(smsq.opts_from(wl.opts))
        seqs.append({
            "model": i, "n": n, "seed": 1000 + i,
            "x0": torch.tensor(wl.x0[0], dtype=torch.float32, device="cuda"),
            "z": torch.tensor(wl.z[0], dtype=torch.float32, device="cuda"),
            "z_mask": (torch.tensor(wl.mask[0], dtype=torch.uint8, device="cuda")
                       if wl.mask is not None else None),
        })
    return models, opts, seqs


def _single(models, opts, q):
    m = models[q["model"]]
    T = q["z"].shape[0]
    parts = torch.empty((T, q["n"], m.d), dtype=torch.float32, device="cuda")
    xmap, J = smsq.run_sequence(m, "f32", q["x0"], q["z"], q["z_mask"], q["n"], opts[q["model"]], q["seed"],
                                particles=parts)
    torch.cuda.synchronize()
    return xmap, J, parts


REL = 1e-5


def _check_equal(plan, models, opts, seqs, mix=MIX):
    for i, q in enumerate(seqs):
        xmap, J, parts = _single(models, opts, q)
        p_parts, _, _ = plan.storage(i)
        a, b = p_parts.cpu().double().numpy(), parts.cpu().double().numpy()
        scale = max(1.0, np.abs(b).max())
        err = np.abs(a - b).max() / scale
        print("sequence %d %s: particles rel err %.2e, J %.7g vs %.7g" % (i, mix[i] if i < len(mix) else "",
              err, plan.J[i].item(), J.item()), flush=True)
        assert err <= REL, "sequence %d particles differ: %.3e" % (i, err)
        xa, xb = plan.xmap[i].cpu().double().numpy(), xmap.cpu().double().numpy()
        assert np.abs(xa - xb).max() <= REL * max(1.0, np.abs(xb).max()), "sequence %d MAP path" % i
        assert abs(plan.J[i].item() - J.item()) <= REL * max(1.0, abs(J.item())), "sequence %d J" % i


def test_batch_matches_single_sequences_16_waves():
    models, opts, seqs = _build(MIX)
    plan = smsq.BatchPlan(models, opts, seqs)
    info = plan.info()
    assert info["waves"] == 16 and info["T_max"] == 9 and info["count"] == len(MIX)
    plan.run()
    torch.cuda.synchronize()
    assert plan.status() == smsq.OK
    _check_equal(plan, models, opts, seqs)
    for J in plan.J:
        assert np.isfinite(J.item())


def test_batch_with_map_conditioned_weights():
    """weights = 1 (mixture weights from the previous forward-recursion
    scores) in a plan matches the single-sequence path with the same option."""
    models, opts, seqs = _build(MIX[1:6], base_seed=70)
    opts = [smsq.opts(o.n_iter, o.step, o.bw_scale, o.bw_mode, o.trans_mode, weights=1) for o in opts]
    plan = smsq.BatchPlan(models, opts, seqs)
    plan.run()
    torch.cuda.synchronize()
    assert plan.status() == smsq.OK
    _check_equal(plan, models, opts, seqs, MIX[1:6])
    # and the weights change the result
    plain = smsq.BatchPlan(models, [smsq.opts(o.n_iter, o.step, o.bw_scale) for o in opts], seqs)
    plain.run()
    torch.cuda.synchronize()
    assert any(abs(a.item() - b.item()) > 1e-3 * max(1.0, abs(b.item())) for a, b in zip(plan.J, plain.J))


def test_batch_autotuner_and_8_wave_shape():
    models, opts, seqs = _build(MIX, base_seed=50)
    plan = smsq.BatchPlan(models, opts, seqs)
    info = plan.tune(steps=3)
    print("autotuner", info, flush=True)
    assert info["tuned_ms"][0] > 0 and info["tuned_ms"][1] > 0
    assert info["waves"] == (8 if info["tuned_ms"][1] < info["tuned_ms"][0] else 16)
    plan.run()
    torch.cuda.synchronize()
    assert plan.status() == smsq.OK
    _check_equal(plan, models, opts, seqs)


def test_batch_autotuner_remembers_plan_shapes():
    """A second plan of the same shape takes the first one's tuned shape
    and timings without running the tuner again; another shape is timed."""
    models, opts, seqs = _build(MIX[:5], base_seed=55)
    first = smsq.BatchPlan(models, opts, seqs).tune(steps=3)
    again = smsq.BatchPlan(models, opts, seqs).tune(steps=3)
    print("tuner", first, again, flush=True)
    assert again["tuned_ms"] == first["tuned_ms"] and again["waves"] == first["waves"]
    other = list(MIX[:5])
    other[1] = (other[1][0], other[1][1] - 64, other[1][2], other[1][3])
    models2, opts2, seqs2 = _build(other, base_seed=55)
    plan = smsq.BatchPlan(models2, opts2, seqs2)
    info = plan.tune(steps=3)
    assert info["tuned_ms"] != first["tuned_ms"]
    plan.run()
    torch.cuda.synchronize()
    assert plan.status() == smsq.OK


def test_batch_graph_replays_match_eager():
    models, opts, seqs = _build(MIX[:6], base_seed=80)
    plan = smsq.BatchPlan(models, opts, seqs)
    plan.run()
    torch.cuda.synchronize()
    ref = [(x.clone(), J.clone()) for x, J in zip(plan.xmap, plan.J)]
    s = torch.cuda.Stream()
    for rep in range(3):
        for x, J in zip(plan.xmap, plan.J):
            x.fill_(float("nan"))
            J.fill_(float("nan"))
        torch.cuda.synchronize()
        with torch.cuda.stream(s):
            plan.run(use_graph=True, stream=s)
        s.synchronize()
        # eager work between replays
        junk = torch.randn(1 << 16, device="cuda").sum()
        torch.cuda.synchronize()
        assert np.isfinite(junk.item())
        for i, (x, J) in enumerate(zip(plan.xmap, plan.J)):
            assert torch.equal(x, ref[i][0]), "replay %d sequence %d" % (rep, i)
            assert torch.equal(J, ref[i][1]), "replay %d sequence %d" % (rep, i)
        assert plan.status() == smsq.OK


def test_batch_plan_argument_errors():
    models, opts, seqs = _build(MIX[:2])
    bad = [dict(seqs[0], model=5)]
    with pytest.raises(smsq.SmsqError):
        smsq.BatchPlan(models, opts, bad)
    big = [dict(seqs[0], n=1025)]
    with pytest.raises(smsq.SmsqError):
        smsq.BatchPlan(models, opts, big)
    # the linear-Gaussian family runs in plans at d = 2 only
    lg3 = S.lingauss_model(np.eye(3) * 0.9, np.eye(3)[:1], [0.05, 0.05, 0.05], [0.1])
    q = {"model": 0, "n": 32, "seed": 1, "x0": torch.zeros(3, device="cuda"),
         "z": torch.zeros((3, lg3.obs_dim), device="cuda"), "z_mask": None}
    with pytest.raises(smsq.SmsqError) as e:
        smsq.BatchPlan([smsq.Model(lg3)], [smsq.opts(10, 0.01)], [q])
    assert e.value.status == smsq.ERR_UNSUPPORTED
    arm = S.make_workload("scenario_d", B=1, seed=0, T=3)     # the 14-D manipulator runs outside plans
    q3 = dict(q, x0=torch.zeros(14, device="cuda"), z=torch.zeros((3, 3), device="cuda"))
    with pytest.raises(smsq.SmsqError) as e:
        smsq.BatchPlan([smsq.Model(arm.model)], [smsq.opts_from(arm.opts)], [q3])
    assert e.value.status == smsq.ERR_UNSUPPORTED
    imq = [smsq.opts(o.n_iter, o.step, o.bw_scale, kernel="imq") for o in opts]   # plans run the RBF kernel
    with pytest.raises(smsq.SmsqError) as e:
        smsq.BatchPlan(models, imq, seqs)
    assert e.value.status == smsq.ERR_UNSUPPORTED


POSE_MIX = [
    ("scenario_b", 20, 6, 10),
    ("lingauss", 64, 7, 10),
    ("range2d", 100, 4, 10),
    ("scenario_b", 130, 5, 10),
    ("lingauss", 300, 3, 10),
    ("arm7", 64, 4, 12),
]


def test_batch_pose_and_linear_gaussian_families():
    """The pose family (Sec. V-B, d = 3, unknown association) and the
    linear-Gaussian family at d = 2 in a plan, beside other families: every
    sequence matches the single-sequence path; a proposal network cannot be
    attached to such a plan (its features cover the other four families)."""
    models, opts, seqs = _build(POSE_MIX, base_seed=300)
    plan = smsq.BatchPlan(models, opts, seqs)
    plan.run()
    torch.cuda.synchronize()
    assert plan.status() == smsq.OK
    _check_equal(plan, models, opts, seqs, POSE_MIX)
    # and the new families against the FP64 oracle (Algorithm 2, same keys)
    for i, (name, n, T, L) in enumerate(POSE_MIX):
        if name not in ("scenario_b", "lingauss"):
            continue
        wl = S.make_workload(name, B=1, seed=300 + i, n=n, T=T, n_iter=L)
        o = wl.opts
        res = O.run_sequence(wl.model, T, n, wl.x0[0], wl.z[0], None if wl.mask is None else wl.mask[0],
                             seqs[i]["seed"], 0, o.n_iter, o.step, o.bw_scale, o.bw_mode, o.trans_mode)
        assert res["status"] == O.OK
        J = plan.J[i].item()
        print("oracle %s n=%d: J plan %.6f oracle %.6f" % (name, n, J, res["J"]), flush=True)
        assert abs(J - res["J"]) <= 1e-3 * max(abs(res["J"]), T)
    with pytest.raises(smsq.SmsqError) as e:
        plan.set_init(smsq.InitMLP(seed=0, max_batch=len(seqs)))
    assert e.value.status == smsq.ERR_UNSUPPORTED


def test_full_ragged_mix_sampled_sequences():
    """The batched plan at the benchmark's full size: 4096 sequences of the
    four families (N in {32, ..., 1024}, T in [50, 200], full iteration
    counts) in one plan with graph replay.  One sequence per family (the
    largest N, then the smallest T) against the CPU FP64 oracle's results on
    the same inputs and Philox key (fixtures tests/golden/mix_*.npz, written
    by tests/golden/make_fullsize_fixtures.py):
      * the plan's J within 1e-3 max(|J|, T) of the oracle's J, and equal
        to the path score of the plan's own MAP trajectory (FP64, oracle);
      * teacher-forced through the plan: the plan's particles of step
        t_s - 1, the predictive initial particles of step t_s regenerated by
        the oracle from the plan's Philox key, one oracle SVGD step, against
        the plan's particles of step t_s (1e-4 of the positions; the move
        as parity_bounds.py states);
      * the plan's J within 1e-3 max(|J|, T) of the standalone Algorithm 2
        on the same inputs.
    FP32-vs-FP64 differences are printed per family."""
    import oracle as O
    from paper_2312_08684_amd import learned as LI
    from parity_bounds import check_move
    from test_gpu_fullsize import load_fixture
    spec = LI.mix(4096, seed=11, T_lo=50, T_hi=200)
    mx = LI.Mix(spec)
    plan, J, _, models, seqs = LI.run(mx, 1.0, warm=False)
    assert plan.status() == smsq.OK
    Jn = J.cpu().numpy() if hasattr(J, "cpu") else np.asarray(J)
    assert np.all(np.isfinite(Jn))
    _, opts, _ = LI.build(mx, 1.0)
    for fam in ("growth1d", "range2d", "cv4d", "arm7"):
        fx = load_fixture("mix_" + fam)
        i = int(fx["mix_index"])
        _, n, T, sd = spec[i]
        assert (n, T, sd + 7) == (int(fx["n"]), int(fx["T"]), int(fx["key"]))
        wl = mx.wls[i]
        assert np.array_equal(wl.z[0], fx["z"]) and np.array_equal(wl.x0[0], fx["x0"])
        mask = None if wl.mask is None else wl.mask[0]
        Jp = float(plan.J[i].item())
        Jo = float(fx["J"])
        xp = plan.xmap[i].cpu().double().numpy()
        Jpath = O.path_score(wl.model, xp, wl.z[0], mask)
        print("%s n=%d T=%d: plan J %.4f oracle J %.4f (rel %.3e, FP32 vs FP64), path score %.4f, "
              "trajectory max |dx| %.3e" % (fam, n, T, Jp, Jo, abs(Jp - Jo) / max(abs(Jo), T), Jpath,
                                            np.abs(xp - fx["xmap"]).max()), flush=True)
        assert abs(Jp - Jo) <= 1e-3 * max(abs(Jo), T)
        assert abs(Jpath - Jp) <= 1e-3 * max(abs(Jp), T)
        # teacher-forced step t_s through the plan's storage
        ts = int(fx["t_sample"])
        parts, _, _ = plan.storage(i)
        parts = parts.cpu().double().numpy()
        x_init = O.predictive_init(wl.model, ts, parts[ts - 2], n, sd + 7, 0)
        L, eps = opts[i].n_iter, opts[i].step
        xo, _, st = O.svgd_step(wl.model, ts, parts[ts - 2], None, wl.z[0][ts - 1],
                                None if mask is None else mask[ts - 1], x_init, L, eps)
        assert st == O.OK
        rel = np.linalg.norm(parts[ts - 1] - xo) / np.linalg.norm(xo)
        print("  teacher-forced plan step t=%d: rel X err %.3e" % (ts, rel), flush=True)
        assert rel <= 1e-4
        print("  " + check_move(parts[ts - 1], xo, x_init, L, "f32"), flush=True)
        # and the standalone path on the same inputs
        q = seqs[i]
        _, Js = smsq.run_sequence(models[i], "f32", q["x0"], q["z"], q["z_mask"], n, opts[i], q["seed"])
        Js = float(Js.cpu()[0])
        assert abs(Jp - Js) <= 1e-3 * max(abs(Js), T)
