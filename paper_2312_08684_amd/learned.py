"""Learned initial particles: data generation, training, gating, evaluation.

Host-side orchestration of the proposal network (``smsq.InitMLP``) around
batched ragged runs (``smsq.BatchPlan``); every numerical step runs in the
library's kernels.  The recipe:

1. run the plain method (predictive initialisation) on a training mix of
   sequences, with more iterations than the runs it will serve (twice each
   family's L in the benchmark, so the targets are nearer convergence);
   every step t >= 2 of every sequence gives one example: the previous
   step's particles and forward-recursion scores, the observation, and the
   particles SVGD converged to (the proposal's target);
2. train the network by Adam on the mixture NLL of those targets;
3. on a validation mix, compare the MAP log-posterior J reached with a
   reduced iteration count from the proposal against the predictive
   initialisation, per model family, and keep the proposal only where it
   gains (measured by the final J it leads to);
4. run with the reduced iteration count and the gate.
"""
from __future__ import annotations

import time
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np
import torch

from . import scenarios as S
from . import smsq

FAMILIES = S.MIX_FAMILIES
PARTICLES = S.MIX_PARTICLES
mix = S.mix


class Mix:
    """Synthetic workloads of a mix with their models and device arrays,
    built once and shared by every run of the mix."""

    def __init__(self, spec):
        self.spec = list(spec)
        self.wls, self.models, self.data = [], [], []
        for fam, n, T, sd in self.spec:
            wl = S.make_workload(fam, B=1, seed=sd, n=n, T=T)
            self.wls.append(wl)
            self.models.append(smsq.Model(wl.model))
            self.data.append({
                "x0": torch.tensor(wl.x0[0], dtype=torch.float32, device="cuda"),
                "z": torch.tensor(wl.z[0], dtype=torch.float32, device="cuda"),
                "z_mask": (torch.tensor(wl.mask[0], dtype=torch.uint8, device="cuda")
                           if wl.mask is not None else None)})

    def __len__(self):
        return len(self.spec)


def build(spec, L_scale: float = 1.0, gate: Optional[Dict[str, bool]] = None):
    """Models, options and sequence dicts of a mix (a spec list or a Mix);
    each family keeps its own iteration count L (scaled by L_scale) and step
    size."""
    mx = spec if isinstance(spec, Mix) else Mix(spec)
    opts, seqs = [], []
    for i, ((fam, n, T, sd), wl) in enumerate(zip(mx.spec, mx.wls)):
        L = max(1, int(round(wl.opts.n_iter * L_scale)))
        opts.append(smsq.opts(L, wl.opts.step, wl.opts.bw_scale, 0, 0))
        seqs.append(dict(mx.data[i], model=i, n=n, seed=sd + 7,
                         use_proposal=1 if (gate is None or gate.get(fam, False)) else 0))
    return mx.models, opts, seqs


def run(spec, L_scale: float = 1.0, mlp: Optional[smsq.InitMLP] = None, gate=None, use_graph: bool = True,
        tune: bool = False, warm: bool = True):
    """One timed run of a mix (a spec list or a Mix), after one untimed run
    that builds the graph (without `warm`, the timed run also captures it:
    host work of milliseconds against seconds of GPU work).  Returns (plan,
    J [count], seconds, models, seqs)."""
    models, opts, seqs = build(spec, L_scale, gate)
    plan = smsq.BatchPlan(models, opts, seqs)
    if tune:
        plan.tune(3)
    if mlp is not None:
        plan.set_init(mlp)
    stream = torch.cuda.Stream()
    if warm:
        with torch.cuda.stream(stream):
            plan.run(use_graph=use_graph, stream=stream)
    stream.synchronize()
    t0 = time.perf_counter()
    with torch.cuda.stream(stream):
        plan.run(use_graph=use_graph, stream=stream)
    stream.synchronize()
    dt = time.perf_counter() - t0
    if plan.status() != smsq.OK:
        raise RuntimeError("non-finite values in a batched run")
    J = np.array([j.item() for j in plan.J])
    return plan, J, dt, models, seqs


def examples(plan: smsq.BatchPlan, spec, seqs) -> List[dict]:
    """Training examples (steps t >= 2) of a finished plain run."""
    ex = []
    for i, (fam, n, T, sd) in enumerate(spec.spec if isinstance(spec, Mix) else spec):
        parts, phi, _ = plan.storage(i)
        for t in range(2, T + 1):
            ex.append({"model": i, "t": t, "x_prev": parts[t - 2], "phi_prev": phi[t - 2],
                       "z": seqs[i]["z"][t - 1],
                       "z_mask": None if seqs[i]["z_mask"] is None else seqs[i]["z_mask"][t - 1],
                       "particles": parts[t - 1], "seed": 0, "seq": 0})
    return ex


def train(mlp: smsq.InitMLP, models, ex: List[dict], steps: int, batch: int = 512, lr: float = 1e-3,
          seed: int = 0, log_every: int = 0) -> List[float]:
    """Adam on the mixture NLL over minibatches of a shuffled example set;
    the learning rate drops to lr / 3 for the last 30% of the steps."""
    rng = np.random.default_rng(seed)
    order = rng.permutation(len(ex))
    iset = smsq.InitSet(models, [ex[k] for k in order])
    E = len(ex)
    b = min(batch, E, mlp.max_batch)
    losses = []
    for step in range(steps):
        first = (step * b) % max(1, E - b + 1)
        loss = mlp.train_step(iset, first, b, lr if step < 0.7 * steps else lr / 3)
        if log_every and (step % log_every == 0 or step == steps - 1):
            losses.append(loss.item())
    if not losses:
        losses.append(loss.item())
    iset.close()
    return losses


def choose_gate(mlp: smsq.InitMLP, spec, L_scale: float) -> Dict[str, dict]:
    """Per family, on a validation mix at the reduced iteration count: the
    proposal's J against the predictive initialisation's (mean and median
    gain) and the share of sequences each brings within the match rule of
    the full-iteration plain J.  ``use`` = median gain > 0 and no loss of
    matched share; the median keeps a few far-drifted sequences from
    deciding for a family."""
    spec = spec if isinstance(spec, Mix) else Mix(spec)
    _, Jf, _, _, _ = run(spec, 1.0)
    _, Jp, _, _, _ = run(spec, L_scale)
    _, Jl, _, _, _ = run(spec, L_scale, mlp=mlp, gate={f: True for f in FAMILIES})
    out = {}
    for f in FAMILIES:
        idx = [i for i, sp in enumerate(spec.spec) if sp[0] == f]
        if not idx:
            out[f] = {"use": False}
            continue
        sub = [spec.spec[i] for i in idx]
        mp = float(np.mean(matched(Jp[idx], Jf[idx], sub)))
        ml = float(np.mean(matched(Jl[idx], Jf[idx], sub)))
        d = Jl[idx] - Jp[idx]
        out[f] = {"mean_gain": float(np.mean(d)), "median_gain": float(np.median(d)), "matched_plain": mp,
                  "matched_learned": ml, "use": bool(np.median(d) > 0.0 and ml >= mp)}
    return out


def iterations_to_match(J_by_frac: Dict[float, np.ndarray], J_ref, spec) -> np.ndarray:
    """Per sequence, the smallest fraction of the full iteration count whose
    run matches the reference J (NaN where none of the runs does)."""
    out = np.full(len(J_ref), np.nan)
    for f in sorted(J_by_frac, reverse=True):
        out[matched(J_by_frac[f], J_ref, spec)] = f
    return out


def matched(J, J_ref, spec, rel: float = 1e-3) -> np.ndarray:
    """J within rel * max(|J_ref|, T) of the reference (or above it)."""
    T = np.array([sp[2] for sp in (spec.spec if isinstance(spec, Mix) else spec)], dtype=np.float64)
    return J >= J_ref - rel * np.maximum(np.abs(J_ref), T)
