"""The seeded input generators (CPU): the bootstrap particle filter that
supplies the PF-MAP-Seq grid, and host-side validation of the Sec. V-B and
V-D model descriptions."""
import math

import numpy as np

from paper_2312_08684_amd import scenarios as S
from paper_2312_08684_amd import smsq


def _range_loglik(model, z, x):
    p = model.params
    nb = int(p[1])
    bc = p[2:2 + 2 * nb].reshape(nb, 2)
    r = np.sqrt(((x[:, None, :] - bc[None]) ** 2).sum(-1))
    return -0.5 * ((z[None, :nb] - r) ** 2).sum(1) / p[0]


def test_bootstrap_pf_particles_propagate_weight_and_resample():
    wl = S.make_workload("range2d", B=1, seed=21, T=30)
    n = 4000
    P = S.bootstrap_pf_particles(wl.model, wl.x0[0], wl.z[0], None, n, seed=5)
    assert P.shape == (30, n, 2)
    assert np.array_equal(P, S.bootstrap_pf_particles(wl.model, wl.x0[0], wl.z[0], None, n, seed=5))
    assert not np.array_equal(P, S.bootstrap_pf_particles(wl.model, wl.x0[0], wl.z[0], None, n, seed=6))
    # step 1: x_0 plus the random-walk noise
    sd = math.sqrt(wl.model.q_var[0])
    assert np.all(np.abs(P[0].mean(0) - wl.x0[0]) < 5 * sd / math.sqrt(n))
    assert np.all(np.abs(P[0].std(0) / sd - 1) < 0.05)
    # resampling: the likelihood-weighted mean of step t is where step t+1's
    # cloud starts (up to the random-walk noise and the resampling spread)
    for t in range(0, 29, 7):
        lw = _range_loglik(wl.model, wl.z[0, t], P[t])
        w = np.exp(lw - lw.max())
        w /= w.sum()
        wmean = (w[:, None] * P[t]).sum(0)
        ess = 1.0 / (w ** 2).sum()
        spread = P[t].std(0).max() / math.sqrt(ess) + sd / math.sqrt(n)
        assert np.all(np.abs(P[t + 1].mean(0) - wmean) < 6 * spread), t


def test_pose_and_arm14_descriptions_validate_on_the_host():
    for desc in (S._model_for("scenario_b", 0), S._model_for("scenario_d", 0)):
        m = smsq.Model(desc)
        assert m.workspace_size("f32", 2, 10, 20) > 256
        m.close()
    # LDS bounds the particle count of the 14-D model's vector-ALU step
    arm = smsq.Model(S._model_for("scenario_d", 0))
    assert 256 <= arm.max_particles("f32") < 1024
    arm.close()
    for field, value in ((5, 0.0), (5, 9.0), (3, -1.0)):
        pose = S.se2_model()
        pose.params[field] = value
        try:
            smsq.Model(pose)
            raise AssertionError("bad pose description accepted")
        except smsq.SmsqError as e:
            assert e.status == smsq.ERR_INVALID
