"""Seeded synthetic workloads shaped like the paper's demonstration scenarios.

This module is the one place that both the HIP path and the CPU oracle take
their inputs from.  It builds model descriptions (plain numbers: kind, state
dimension, observation sizes, diagonal process-noise variances and model
constants) and simulates ground-truth trajectories and observations with
numpy's seeded generator.  It holds none of the estimator's arithmetic: no
SVGD, no bandwidth, no mixture score, no Viterbi.  The state-space simulation
below is the data-generating process of each scenario (paper Sec. II, eq. SSM,
and the scenario models of Sec. V), written here independently of both the
oracle's and the kernels' log-density code.

Scenario shapes (synthetic stand-ins for the paper's workloads):

* ``growth1d``  -- 1-D nonstationary growth model with a squared observation,
  the bimodal sign-ambiguity benchmark of Sec. V-A (constants of the FP64
  workload: 0.5x + 25x/(1+x^2) + 8cos(1.2t), Q=10, z=x^2/20, R=1).
* ``range2d``   -- 2-D random-walk position observed by ranges to beacons, with
  a window of steps in which only one beacon is visible (stand-in for the
  UWB range-only experiment of Sec. V-C, whose dataset is not available).
* ``cv4d``      -- 4-D constant-velocity target with M detections per step, one
  from the target and the rest uniform clutter, handled by a detection /
  clutter mixture likelihood (shape of the unknown-association scenario of
  Sec. V-B).
* ``arm7``      -- 7 revolute joints observed through the forward kinematics of
  a standard-DH serial chain (joint-space stand-in for Sec. V-D).
* ``lingauss``  -- linear-Gaussian model, used as a closed-form pin (its MAP
  trajectory is the Rauch-Tung-Striebel smoother mean).
* ``se2``       -- the SE(2) pose of Sec. V-B (heading turns by omega dt, the
  position moves v dt along the new heading) observed by one range-bearing
  measurement per step from one of four landmarks whose identity the
  estimator does not know; the simulated measurements carry heavy-tailed
  outliers that the estimator's likelihood does not model.
* ``arm14``     -- the 14-D manipulator of Sec. V-D: joint angles and
  velocities of the 7-joint DH chain under second-order dynamics driven by
  joint-wise sinusoidal accelerations, observed through the end-effector
  position.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np

# Model kinds, numbered as in include/smsq.h.
GROWTH1D = 0
RANGE2D = 1
CV4D = 2
ARM7 = 3
LINGAUSS = 4
SE2 = 5
ARM14 = 6

KIND_NAMES = {GROWTH1D: "growth1d", RANGE2D: "range2d", CV4D: "cv4d",
              ARM7: "arm7", LINGAUSS: "lingauss", SE2: "se2", ARM14: "arm14"}

N_PARAMS = 64
MAX_D = 16


@dataclasses.dataclass
class ModelDesc:
    """Plain-number description of a state-space model.

    Transition: x_t ~ N(f_t(x_{t-1}), diag(q_var)).  Observation model and the
    meaning of ``params`` depend on ``kind`` (layout documented in
    include/smsq.h next to smsq_model_desc_t).
    """
    kind: int
    d: int
    obs_dim: int
    n_obs: int
    q_var: np.ndarray          # [16] float64, first d used
    params: np.ndarray         # [64] float64

    def copy(self) -> "ModelDesc":
        return ModelDesc(self.kind, self.d, self.obs_dim, self.n_obs,
                         self.q_var.copy(), self.params.copy())


@dataclasses.dataclass
class SvgdOpts:
    n_iter: int
    step: float
    bw_scale: float = 1.0
    bw_mode: int = 0          # 0: bandwidth recomputed every iteration, 1: once per step
    trans_mode: int = 0       # 0: log-sum-exp transition mixture, 1: mean of gradients


@dataclasses.dataclass
class Workload:
    """One batch of synthetic sequences sharing a model."""
    name: str
    model: ModelDesc
    opts: SvgdOpts
    n: int                    # particles per step
    T: int                    # time steps
    x0: np.ndarray            # [B, d] known initial states
    z: np.ndarray             # [B, T, obs_dim] observations
    mask: Optional[np.ndarray]  # [B, T, n_obs] uint8 or None
    truth: np.ndarray         # [B, T+1, d] simulated states (x_0 included)
    dtype: str                # "f32" or "f64"

    @property
    def batch(self) -> int:
        return self.x0.shape[0]


def _desc(kind, d, obs_dim, n_obs, q_var, params) -> ModelDesc:
    q = np.zeros(MAX_D)
    q[:d] = q_var
    p = np.zeros(N_PARAMS)
    p[:len(params)] = params
    return ModelDesc(kind, d, obs_dim, n_obs, q, p)


# ---------------------------------------------------------------------------
# Model descriptions
# ---------------------------------------------------------------------------

def growth1d_model(a=0.5, b=25.0, c=8.0, omega=1.2, phase=0.0, q=10.0,
                   kobs=1.0 / 20.0, r=1.0) -> ModelDesc:
    """f_t(x) = a x + b x/(1+x^2) + c cos(omega t + phase); z = kobs x^2 + N(0, r)."""
    return _desc(GROWTH1D, 1, 1, 1, [q], [a, b, c, omega, phase, kobs, r])


def range2d_model(beacons: np.ndarray, sigma_q=0.3, sigma_z=0.5) -> ModelDesc:
    """Random walk, ranges to beacons.  params = [r_var, n_b, bx0, by0, bx1, ...]."""
    beacons = np.asarray(beacons, dtype=np.float64).reshape(-1, 2)
    nb = beacons.shape[0]
    assert 1 <= nb <= 16
    return _desc(RANGE2D, 2, nb, nb, [sigma_q ** 2] * 2,
                 [sigma_z ** 2, float(nb)] + list(beacons.reshape(-1)))


def cv4d_model(n_det=10, dt=0.1, sigma_q=0.5, sigma_z=0.3, p_d=0.9,
               volume=2500.0) -> ModelDesc:
    """Constant velocity; z = M detections (x,y).  params = [dt, r_var, P_D, V]."""
    assert 1 <= n_det <= 16
    return _desc(CV4D, 4, 2 * n_det, n_det, [sigma_q ** 2] * 4,
                 [dt, sigma_z ** 2, p_d, volume])


ARM7_ALPHA = np.array([math.pi / 2, -math.pi / 2, math.pi / 2, -math.pi / 2,
                       math.pi / 2, -math.pi / 2, 0.0])


def arm7_model(link_a: np.ndarray, alpha: np.ndarray = ARM7_ALPHA,
               link_d: Optional[np.ndarray] = None, sigma_q=0.02,
               sigma_z=0.01) -> ModelDesc:
    """Random-walk joints; z = end-effector position of a standard-DH chain.

    params = [r_var, a_1..a_7, alpha_1..alpha_7, d_1..d_7].
    """
    link_a = np.asarray(link_a, dtype=np.float64)
    alpha = np.asarray(alpha, dtype=np.float64)
    link_d = np.zeros(7) if link_d is None else np.asarray(link_d, dtype=np.float64)
    assert link_a.shape == (7,) and alpha.shape == (7,) and link_d.shape == (7,)
    return _desc(ARM7, 7, 3, 1, [sigma_q ** 2] * 7,
                 [sigma_z ** 2] + list(link_a) + list(alpha) + list(link_d))


def arm14_model(link_a: np.ndarray, alpha: np.ndarray = ARM7_ALPHA,
                link_d: Optional[np.ndarray] = None, dt=0.02, q_p=1.0, q_v=5e-3,
                sigma_z=0.1, amp=0.5, freq=0.2, phase_step=1.0) -> ModelDesc:
    """Sec. V-D: x = [q; qdot] in R^14, q_t = q + qdot dt, qdot_t = qdot +
    u_{t-1} dt + noise, u_{t-1,i} = amp sin(freq (t - 1) + phase_step i);
    Q = diag(q_p dt^2 I_7, q_v I_7); z = end-effector position + N(0, sigma_z^2 I).

    params = [r_var, a_1..a_7, alpha_1..alpha_7, d_1..d_7, dt, amp, freq, phase_step].
    """
    link_a = np.asarray(link_a, dtype=np.float64)
    alpha = np.asarray(alpha, dtype=np.float64)
    link_d = np.zeros(7) if link_d is None else np.asarray(link_d, dtype=np.float64)
    assert link_a.shape == (7,) and alpha.shape == (7,) and link_d.shape == (7,)
    return _desc(ARM14, 14, 3, 1, [q_p * dt * dt] * 7 + [q_v] * 7,
                 [sigma_z ** 2] + list(link_a) + list(alpha) + list(link_d) + [dt, amp, freq, phase_step])


def lingauss_model(A: np.ndarray, C: np.ndarray, q_var, r_var) -> ModelDesc:
    """x_t = A x_{t-1} + N(0, diag q); z = C x + N(0, diag r).

    params = [A (d x d row-major, 16 slots), C (obs x d row-major, 16 slots),
    r (4 slots)].  d <= 4 and obs_dim <= 4.
    """
    A = np.asarray(A, dtype=np.float64)
    C = np.asarray(C, dtype=np.float64)
    d = A.shape[0]
    o = C.shape[0]
    assert A.shape == (d, d) and C.shape == (o, d) and 1 <= d <= 4 and 1 <= o <= 4
    p = np.zeros(36)
    p[:d * d] = A.reshape(-1)
    p[16:16 + o * d] = C.reshape(-1)
    p[32:32 + o] = np.asarray(r_var, dtype=np.float64).reshape(o)
    return _desc(LINGAUSS, d, o, 1, np.asarray(q_var, dtype=np.float64).reshape(d), p)


# Sec. V-B constants: alpha_x = alpha_y = 0.3, alpha_theta = 0.105, dt = 0.1,
# range and bearing noise std 1 m and 0.44 rad, four landmarks, 630 steps.
# The paper gives neither the controls nor the landmark positions: one
# counter-clockwise loop of radius 10 m in the 630 steps (v = R omega) and
# landmarks at the corners of a 24 m square around the loop's centre.
SE2_RADIUS = 10.0
SE2_OMEGA = 2.0 * math.pi / (630 * 0.1)
SE2_LANDMARKS = np.array([[12.0, 12.0], [-12.0, 12.0], [-12.0, -12.0], [12.0, -12.0]])
SE2_SIGMA0 = np.array([0.2, 0.2, 0.035])     # std of the initial pose about the reference start


def se2_model(dt=0.1, v=SE2_RADIUS * SE2_OMEGA, omega=SE2_OMEGA, alpha=(0.3, 0.3, 0.105),
              sigma_r=1.0, sigma_b=0.44, landmarks=SE2_LANDMARKS) -> ModelDesc:
    """SE(2) pose, one range-bearing measurement from an unknown landmark.

    q_var = (alpha dt)^2 per coordinate.  params = [dt, v, omega, r_var,
    b_var, n_l, gx_1, gy_1, ..., gx_nl, gy_nl] with n_l <= 8.
    """
    lm = np.asarray(landmarks, dtype=np.float64).reshape(-1, 2)
    assert 1 <= lm.shape[0] <= 8
    q = [(a * dt) ** 2 for a in alpha]
    return _desc(SE2, 3, 2, 1, q, [dt, v, omega, sigma_r ** 2, sigma_b ** 2, float(lm.shape[0])]
                 + list(lm.reshape(-1)))


# ---------------------------------------------------------------------------
# Simulation of the data-generating process (numpy, seeded)
# ---------------------------------------------------------------------------

def _growth_f(p, t, x):
    a, b, c, om, ph = p[0], p[1], p[2], p[3], p[4]
    return a * x + b * x / (1.0 + x * x) + c * math.cos(om * t + ph)


def dh_forward_kinematics(q: np.ndarray, link_a, alpha, link_d) -> np.ndarray:
    """End-effector position of a standard-DH chain (data generation only)."""
    T = np.eye(4)
    for i in range(len(q)):
        ct, st = math.cos(q[i]), math.sin(q[i])
        ca, sa = math.cos(alpha[i]), math.sin(alpha[i])
        Ti = np.array([[ct, -st * ca, st * sa, link_a[i] * ct],
                       [st, ct * ca, -ct * sa, link_a[i] * st],
                       [0.0, sa, ca, link_d[i]],
                       [0.0, 0.0, 0.0, 1.0]])
        T = T @ Ti
    return T[:3, 3].copy()


def _se2_f(p, x):
    th = x[2] + p[2] * p[0]
    return np.array([x[0] + p[1] * p[0] * math.cos(th), x[1] + p[1] * p[0] * math.sin(th), th])


def _arm14_f(p, t, x):
    dt, amp, freq, ph = p[22], p[23], p[24], p[25]
    u = amp * np.sin(freq * (t - 1) + ph * np.arange(7))
    return np.concatenate([x[:7] + dt * x[7:], x[7:] + dt * u])


def _wrap(a):
    return (a + math.pi) % (2.0 * math.pi) - math.pi


def se2_reference(model: ModelDesc, T: int) -> np.ndarray:
    """Noise-free reference poses [T+1, 3] from the loop's start pose."""
    ref = np.zeros((T + 1, 3))
    ref[0] = [SE2_RADIUS, 0.0, math.pi / 2]
    for t in range(1, T + 1):
        ref[t] = _se2_f(model.params, ref[t - 1])
    return ref


def simulate(model: ModelDesc, T: int, B: int, seed: int, *,
             unobs_window=(80, 120), clutter_box=50.0, outlier_prob=0.1, outlier_scale=5.0):
    """Simulate B independent sequences.  Returns (x0, truth, z, mask)."""
    rng = np.random.default_rng(seed)
    d = model.d
    p = model.params
    sq = np.sqrt(model.q_var[:d])
    truth = np.zeros((B, T + 1, d))
    z = np.zeros((B, T, model.obs_dim))
    mask = None
    for b in range(B):
        if model.kind == GROWTH1D:
            x = np.array([rng.normal(0.0, math.sqrt(5.0))])
        elif model.kind == RANGE2D:
            x = rng.uniform(5.0, 15.0, size=2)
        elif model.kind == CV4D:
            x = np.concatenate([[0.0, 0.0], rng.normal(0.0, 1.0, size=2)])
        elif model.kind == ARM7:
            x = rng.uniform(-0.5, 0.5, size=7)
        elif model.kind == SE2:
            x = se2_reference(model, 0)[0] + SE2_SIGMA0 * rng.normal(size=3)
        elif model.kind == ARM14:
            # joint angles U[-0.5, 0.5] at rest, then N(0, diag(1 deg^2, 2 deg^2))
            mu0 = np.concatenate([rng.uniform(-0.5, 0.5, size=7), np.zeros(7)])
            x = mu0 + np.radians(np.repeat([1.0, 2.0], 7)) * rng.normal(size=14)
        else:
            x = rng.normal(0.0, 1.0, size=d)
        truth[b, 0] = x
        for t in range(1, T + 1):
            if model.kind == GROWTH1D:
                m = np.array([_growth_f(p, t, x[0])])
            elif model.kind == CV4D:
                dt = p[0]
                m = np.array([x[0] + dt * x[2], x[1] + dt * x[3], x[2], x[3]])
            elif model.kind == LINGAUSS:
                A = p[:d * d].reshape(d, d)
                m = A @ x
            elif model.kind == SE2:
                m = _se2_f(p, x)
            elif model.kind == ARM14:
                m = _arm14_f(p, t, x)
            else:
                m = x.copy()
            x = m + sq * rng.normal(size=d)
            truth[b, t] = x
            if model.kind == GROWTH1D:
                z[b, t - 1, 0] = p[5] * x[0] ** 2 + math.sqrt(p[6]) * rng.normal()
            elif model.kind == RANGE2D:
                nb = int(p[1])
                bc = p[2:2 + 2 * nb].reshape(nb, 2)
                r = np.sqrt(((bc - x[None, :]) ** 2).sum(1))
                z[b, t - 1, :nb] = r + math.sqrt(p[0]) * rng.normal(size=nb)
            elif model.kind == CV4D:
                M = model.n_obs
                det = np.empty((M, 2))
                det[0] = x[:2] + math.sqrt(p[1]) * rng.normal(size=2)
                det[1:] = x[None, :2] + rng.uniform(-clutter_box / 2, clutter_box / 2,
                                                     size=(M - 1, 2))
                det = det[rng.permutation(M)]
                z[b, t - 1] = det.reshape(-1)
            elif model.kind == SE2:
                # one measurement from a landmark drawn uniformly; with
                # probability outlier_prob both noises are outlier_scale
                # times wider (heavy tails the likelihood does not model)
                lm = p[6:6 + 2 * int(p[5])].reshape(-1, 2)[int(rng.integers(int(p[5])))]
                sc = outlier_scale if rng.uniform() < outlier_prob else 1.0
                dx, dy = x[0] - lm[0], x[1] - lm[1]
                z[b, t - 1, 0] = math.hypot(dx, dy) + sc * math.sqrt(p[3]) * rng.normal()
                z[b, t - 1, 1] = _wrap(math.atan2(dy, dx) + sc * math.sqrt(p[4]) * rng.normal())
            elif model.kind in (ARM7, ARM14):
                la, al, ld = p[1:8], p[8:15], p[15:22]
                z[b, t - 1] = (dh_forward_kinematics(x[:7], la, al, ld)
                               + math.sqrt(p[0]) * rng.normal(size=3))
            else:
                o = model.obs_dim
                C = p[16:16 + o * d].reshape(o, d)
                r = p[32:32 + o]
                z[b, t - 1] = C @ x + np.sqrt(r) * rng.normal(size=o)
        if model.kind == RANGE2D:
            if mask is None:
                mask = np.ones((B, T, model.n_obs), dtype=np.uint8)
            lo, hi = unobs_window
            if T >= lo:
                keep = int(rng.integers(model.n_obs))
                for t in range(lo, min(hi, T) + 1):
                    mask[b, t - 1, :] = 0
                    mask[b, t - 1, keep] = 1
    return truth[:, 0].copy(), truth, z, mask


def bootstrap_pf_particles(model: ModelDesc, x0: np.ndarray, z: np.ndarray, mask: Optional[np.ndarray],
                           n: int, seed: int) -> np.ndarray:
    """Particle sets of a bootstrap particle filter on the range-only model,
    the grid that a PF-MAP-Seq forward recursion runs on (Sec. V baselines:
    stratified resampling at every step).  The filter is input generation
    for that workload, not part of the estimator: it propagates the resampled
    particles through the random walk, weights them by the range likelihood
    and resamples.  Returns [T, n, 2], the propagated particles of each step
    (before resampling, so they are distinct)."""
    assert model.kind == RANGE2D
    rng = np.random.default_rng(seed)
    p = model.params
    nb = int(p[1])
    bc = p[2:2 + 2 * nb].reshape(nb, 2)
    sq = np.sqrt(model.q_var[:2])
    T = z.shape[0]
    parts = np.zeros((T, n, 2))
    anc = np.broadcast_to(np.asarray(x0, dtype=np.float64), (n, 2))
    for t in range(T):
        x = anc + sq * rng.normal(size=(n, 2))
        parts[t] = x
        rr = np.sqrt(((x[:, None, :] - bc[None]) ** 2).sum(-1))
        on = np.ones(nb, dtype=bool) if mask is None else mask[t].astype(bool)
        lw = -0.5 * (((z[t, :nb][None, :] - rr) ** 2) / p[0])[:, on].sum(1)
        w = np.exp(lw - lw.max())
        cdf = np.cumsum(w / w.sum())
        u = (np.arange(n) + rng.uniform(size=n)) / n
        anc = x[np.minimum(np.searchsorted(cdf, u), n - 1)]
    return parts


# ---------------------------------------------------------------------------
# The five workload shapes
# ---------------------------------------------------------------------------

def _model_for(name: str, seed: int) -> ModelDesc:
    rng = np.random.default_rng(10_000 + seed)
    if name == "growth1d":
        return growth1d_model()
    if name == "range2d":
        return range2d_model(rng.uniform(0.0, 20.0, size=(3, 2)))
    if name == "cv4d":
        return cv4d_model()
    if name == "arm7":
        return arm7_model(rng.uniform(0.1, 0.4, size=7))
    if name == "scenario_a":
        # Sec. V-A (the 1-D benchmark): x_t = 0.9 x + 10 x / (1 + x^2)
        # + 8 cos(1.2 (t - 1)) + v, v ~ N(0, 5); z = 0.05 x^2 + r, r ~ N(0, 4^2)
        return growth1d_model(a=0.9, b=10.0, c=8.0, omega=1.2, phase=-1.2, q=5.0, kobs=0.05, r=16.0)
    if name == "scenario_b":
        return se2_model()
    if name == "scenario_d":
        # Sec. V-D; the DH chain is not tabulated: the arm7 chain's links
        return arm14_model(rng.uniform(0.1, 0.4, size=7))
    if name == "lingauss":
        d = 2
        A = np.array([[1.0, 0.1], [0.0, 0.95]])
        C = np.array([[1.0, 0.0]])
        return lingauss_model(A, C, [0.05, 0.02], [0.1])
    raise ValueError(name)


# name -> (n, T, n_iter, step, dtype)
PRESETS = {
    "growth1d": (32, 50, 100, 0.05, "f64"),
    "range2d": (256, 200, 50, 0.005, "f32"),
    "cv4d": (512, 100, 50, 0.005, "f32"),
    "arm7": (1024, 100, 100, 1e-5, "f32"),
    "lingauss": (64, 20, 50, 0.01, "f64"),
    # Sec. V-A with the paper's own constants, N_s = 10, 100 steps, 100
    # iterations; eps = 0.5: at the stated 0.005 the particles hardly move
    # in this model (the scores are O(0.1)), see the design notes
    "scenario_a": (10, 100, 100, 0.5, "f64"),
    # Sec. V-B: N_s = 20, 630 steps, 100 iterations; eps = 1e-4 because the
    # heading's transition precision 1/(0.105 * 0.1)^2 ~ 9e3 makes the
    # stated 0.005 diverge (eps * curvature must stay below 2)
    "scenario_b": (20, 630, 100, 1e-4, "f32"),
    # Sec. V-D: N_s = 20 (of 10..30), 100 steps (length not stated), 100
    # iterations; eps = 2e-4 because the joint-angle transition precision
    # 1/(q_p dt^2) = 2500 makes the stated 0.005 diverge
    "scenario_d": (20, 100, 100, 2e-4, "f32"),
}


def make_workload(name: str, *, B: int = 1, seed: int = 0, n: Optional[int] = None,
                  T: Optional[int] = None, n_iter: Optional[int] = None,
                  step: Optional[float] = None, dtype: Optional[str] = None,
                  bw_scale: float = 1.0, model_seed: int = 0) -> Workload:
    pn, pT, pL, pe, pdt = PRESETS[name]
    n = pn if n is None else n
    T = pT if T is None else T
    L = pL if n_iter is None else n_iter
    eps = pe if step is None else step
    dt = pdt if dtype is None else dtype
    model = _model_for(name, model_seed)
    x0, truth, z, mask = simulate(model, T, B, seed)
    return Workload(name, model, SvgdOpts(L, eps, bw_scale), n, T, x0, z, mask,
                    truth, dt)


# The ragged mix of the batched form: families with their own preset
# iteration counts and step sizes, particle counts and lengths drawn
# uniformly per sequence.
MIX_FAMILIES = ("growth1d", "range2d", "cv4d", "arm7")
MIX_PARTICLES = (32, 128, 256, 512, 1024)


def mix(count: int, seed: int, T_lo: int, T_hi: int, n_choices=MIX_PARTICLES,
        families=MIX_FAMILIES):
    """(family, n, T, data seed) of `count` sequences drawn uniformly; the
    sequence's Philox key is its data seed + 7."""
    rng = np.random.default_rng(seed)
    return [(families[int(rng.integers(0, len(families)))], int(rng.choice(n_choices)),
             int(rng.integers(T_lo, T_hi + 1)), int(seed) * 100000 + i) for i in range(count)]


def random_particles(rng: np.random.Generator, n: int, d: int, center=None,
                     scale=1.0) -> np.ndarray:
    c = np.zeros(d) if center is None else np.asarray(center)
    return c[None, :] + scale * rng.normal(size=(n, d))
