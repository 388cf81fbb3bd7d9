"""Learned initial particles inside batched runs.

1. Plumbing: with zero SVGD iterations a plan's step particles are its
   initial particles (re-centred once, so equal up to one FP32 rounding);
   for sequences using the proposal they must equal the standalone sampler's
   draws on the same inputs, and the other sequences must keep the
   predictive initialisation of a plain plan (bit for bit).
2. Gain: a network trained on particle sets the plain method converged to
   must, at half the SVGD iterations, bring held-out sequences closer to the
   full-iteration plain MAP log-posterior J than the predictive
   initialisation at half the iterations does (mean J gap and the share of
   sequences within 1e-3 max(|J|, T)), while taking no longer."""
import numpy as np
import pytest
import torch

from paper_2312_08684_amd import learned as LI
from paper_2312_08684_amd import smsq

pytestmark = pytest.mark.gpu


def test_plan_draws_from_the_proposal():
    spec = [("arm7", 128, 4, 11), ("range2d", 100, 5, 12), ("cv4d", 64, 3, 13), ("growth1d", 32, 4, 14)]
    models, opts, seqs = LI.build(spec, gate={"arm7": True, "range2d": True, "cv4d": False, "growth1d": True})
    opts = [smsq.opts(0, o.step, o.bw_scale, 0, 0) for o in opts]     # no SVGD: particles stay initial
    mlp = smsq.InitMLP(seed=9, max_batch=64)
    plan = smsq.BatchPlan(models, opts, seqs)
    plan.set_init(mlp)
    plan.run()
    torch.cuda.synchronize()
    assert plan.status() == smsq.OK
    plain = smsq.BatchPlan(models, opts, [dict(q, use_proposal=0) for q in seqs])
    plain.run()
    torch.cuda.synchronize()
    for i, (fam, n, T, _) in enumerate(spec):
        parts, phi, _ = plan.storage(i)
        pparts, _, _ = plain.storage(i)
        assert torch.equal(parts[0], pparts[0]), "step 1 is always predictive"
        for t in range(2, T + 1):
            if seqs[i]["use_proposal"]:
                tgt = torch.empty_like(parts[t - 1])
                ex = {"model": i, "t": t, "x_prev": parts[t - 2], "phi_prev": phi[t - 2], "z": seqs[i]["z"][t - 1],
                      "z_mask": None if seqs[i]["z_mask"] is None else seqs[i]["z_mask"][t - 1],
                      "particles": tgt, "seed": seqs[i]["seed"], "seq": 0}
                used = mlp.sample(smsq.InitSet(models, [ex])).cpu().numpy()
                torch.cuda.synchronize()
                assert used[0] == 1
                scale = max(1.0, tgt.abs().max().item())
                assert (parts[t - 1] - tgt).abs().max().item() <= 1e-6 * scale, (fam, t)
            else:
                assert torch.equal(parts[t - 1], pparts[t - 1]), (fam, t)


def test_trained_proposal_gains_at_half_the_iterations():
    torch.manual_seed(0)
    train_spec = LI.mix(160, seed=1, T_lo=12, T_hi=24, n_choices=(32, 128, 256, 512))
    plan, _, _, models, seqs = LI.run(train_spec, 1.0)
    ex = LI.examples(plan, train_spec, seqs)
    mlp = smsq.InitMLP(seed=5, max_batch=1024)
    losses = LI.train(mlp, models, ex, steps=3000, batch=512, lr=1e-3, log_every=500)
    print("training NLL", ["%.3f" % v for v in losses], flush=True)
    assert losses[-1] < losses[0]
    val_spec = LI.mix(48, seed=3, T_lo=12, T_hi=24, n_choices=(32, 128, 256, 512))
    gain = LI.choose_gate(mlp, val_spec, 0.5)
    gate = {f: g["use"] for f, g in gain.items()}
    print("validation gain per family", gain, flush=True)
    test_spec = LI.mix(96, seed=2, T_lo=12, T_hi=24, n_choices=(32, 128, 256, 512))
    _, Jfull, t_full, _, _ = LI.run(test_spec, 1.0)
    _, Jp, t_p, _, _ = LI.run(test_spec, 0.5)
    _, Jl, t_l, _, _ = LI.run(test_spec, 0.5, mlp=mlp, gate=gate)
    gp, gl = float(np.mean(Jp - Jfull)), float(np.mean(Jl - Jfull))
    mp, ml = float(np.mean(LI.matched(Jp, Jfull, test_spec))), float(np.mean(LI.matched(Jl, Jfull, test_spec)))
    print("half iterations: plain gap %.3f match %.2f (%.3f s) | learned gap %.3f match %.2f (%.3f s) | full %.3f s"
          % (gp, mp, t_p, gl, ml, t_l, t_full), flush=True)
    assert gl > gp and ml > mp
    assert t_l < t_full
