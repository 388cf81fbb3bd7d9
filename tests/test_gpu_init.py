"""Learned particle proposal on the GPU (smsq_init_*) against the CPU oracle
(oracle/init_mlp.py).

The GPU forward and backward take BF16 operands with FP32 accumulation; the
oracle applies the same BF16 roundings to the same operands and accumulates
in FP64, so the bound is the FP32 accumulation error (rel. 1e-3 as stated
for the proposal network, measured far below).  Features and the mixture NLL
are FP32 against FP64 (rel. 1e-4).  The sampler is checked against the
closed-form moments of the mixture (5 sigma)."""
import numpy as np
import pytest
import torch

from oracle import init_mlp as M
from paper_2312_08684_amd import scenarios as S
from paper_2312_08684_amd import smsq

pytestmark = pytest.mark.gpu


def _rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return np.abs(a - b).max() / max(1e-30, np.abs(b).max())


def _mlp_with(P):
    mlp = smsq.InitMLP(seed=1, max_batch=256)
    mlp.set_params(torch.tensor(P, dtype=torch.float32, device="cuda"))
    return mlp


def test_forward_matches_oracle():
    rng = np.random.default_rng(11)
    P = rng.normal(scale=0.15, size=M.N_PARAMS).astype(np.float32).astype(np.float64)
    F = rng.normal(size=(37, M.FEAT)).astype(np.float32)
    mlp = _mlp_with(P)
    out = mlp.forward(torch.tensor(F, device="cuda")).cpu().numpy()
    ref, _ = M.forward(P, F.astype(np.float64), bf16=True)
    err = _rel(out, ref)
    print("forward rel err %.3e" % err)
    assert err <= 1e-3


def test_backward_matches_oracle():
    rng = np.random.default_rng(12)
    P = rng.normal(scale=0.15, size=M.N_PARAMS).astype(np.float32).astype(np.float64)
    F = rng.normal(size=(53, M.FEAT)).astype(np.float32)
    dout = rng.normal(size=(53, M.OUT)).astype(np.float32)
    mlp = _mlp_with(P)
    mlp.forward(torch.tensor(F, device="cuda"))
    mlp.backward(torch.tensor(dout, device="cuda"))
    G = mlp.grads().cpu().numpy()
    _, cache = M.forward(P, F.astype(np.float64), bf16=True)
    R = M.backward(cache, dout.astype(np.float64), bf16=True)
    for name, lo, hi in [("W1", M.OFF_W1, M.OFF_B1), ("b1", M.OFF_B1, M.OFF_W2), ("W2", M.OFF_W2, M.OFF_B2),
                         ("b2", M.OFF_B2, M.OFF_W3), ("W3", M.OFF_W3, M.OFF_B3), ("b3", M.OFF_B3, M.N_PARAMS)]:
        err = _rel(G[lo:hi], R[lo:hi])
        print("backward %s rel err %.3e" % (name, err))
        assert err <= 1e-3, name


def _examples(name, n, seed, T=4, L=10):
    """A short plain run of one sequence; examples for steps 2..T (targets:
    the converged particles of the run)."""
    wl = S.make_workload(name, B=1, seed=seed, n=n, T=T, n_iter=L)
    model = smsq.Model(wl.model)
    x0 = torch.tensor(wl.x0[0], dtype=torch.float32, device="cuda")
    z = torch.tensor(wl.z[0], dtype=torch.float32, device="cuda")
    mask = torch.tensor(wl.mask[0], dtype=torch.uint8, device="cuda") if wl.mask is not None else None
    o = smsq.opts_from(wl.opts)
    parts = torch.empty((T, n, wl.model.d), dtype=torch.float32, device="cuda")
    ws = smsq.workspace(model.workspace_size("f32", 1, T, n))
    phis = torch.empty((1, T, n), dtype=torch.float32, device="cuda")
    psis = torch.empty((1, T, n), dtype=torch.int32, device="cuda")
    x0v = x0.view(1, 1, -1)
    for t in range(1, T + 1):
        xp = x0v if t == 1 else parts[t - 2].unsqueeze(0)
        php = None if t == 1 else phis[:, t - 2]
        smsq.batch_step(model, "f32", t, xp, php, z[t - 1].unsqueeze(0),
                        None if mask is None else mask[t - 1].unsqueeze(0), parts[t - 1].unsqueeze(0), o, seed=7,
                        phi=phis[:, t - 1], psi=psis[:, t - 1], ws=ws)
    torch.cuda.synchronize()
    ex = []
    for t in range(2, T + 1):
        ex.append({"model": 0, "t": t, "x_prev": parts[t - 2], "phi_prev": phis[0, t - 2], "z": z[t - 1],
                   "z_mask": None if mask is None else mask[t - 1], "particles": parts[t - 1], "seed": 5, "seq": 0})
    return wl, model, ex


@pytest.mark.parametrize("name,n", [("growth1d", 32), ("range2d", 100), ("cv4d", 64), ("arm7", 128)])
def test_features_match_oracle(name, n):
    wl, model, ex = _examples(name, n, seed=3)
    mlp = smsq.InitMLP(seed=0, max_batch=16)
    iset = smsq.InitSet([model], ex)
    F, A, Sc = mlp.features(iset)
    F, A, Sc = F.cpu().numpy(), A.cpu().numpy(), Sc.cpu().numpy()
    for k, q in enumerate(ex):
        Fr, Ar, Sr = M.features(wl.model, q["t"], q["x_prev"].cpu().numpy(), q["phi_prev"].cpu().numpy(),
                                q["z"].cpu().numpy(), None if q["z_mask"] is None else q["z_mask"].cpu().numpy(),
                                q["particles"].shape[0])
        assert np.abs(F[k] - Fr).max() <= 1e-4 * max(1.0, np.abs(Fr).max()), (k, np.abs(F[k] - Fr).max())
        assert np.abs(A[k] - Ar).max() <= 1e-5 * max(1.0, np.abs(Ar).max())
        assert np.abs(Sc[k] - Sr).max() <= 1e-6 * max(1.0, np.abs(Sr).max())


def test_mixture_nll_matches_oracle():
    wl, model, ex = _examples("arm7", 128, seed=4)
    iset = smsq.InitSet([model], ex)
    mlp = smsq.InitMLP(seed=0, max_batch=16)
    _, A, Sc = mlp.features(iset)
    rng = np.random.default_rng(13)
    out = rng.normal(scale=0.5, size=(len(ex), M.OUT)).astype(np.float32)
    out[:, 8::M.COMP] = rng.uniform(-1.0, 1.0, size=(len(ex), M.K))   # moderate log-scales
    loss, dout = iset.nll(torch.tensor(out, device="cuda"), A, Sc, gscale=1.0)
    loss, dout = loss.cpu().numpy(), dout.cpu().numpy()
    for k, q in enumerate(ex):
        lr, gr = M.mixture_nll(out[k].astype(np.float64), A[k].cpu().numpy(), Sc[k].cpu().numpy(),
                               q["particles"].cpu().numpy())
        assert abs(loss[k] - lr) <= 1e-4 * max(1.0, abs(lr)), (k, loss[k], lr)
        assert np.abs(dout[k] - gr).max() <= 1e-4 * max(1.0, np.abs(gr).max()), k


def test_sampler_moments():
    wl, model, ex = _examples("cv4d", 64, seed=6)
    d = wl.model.d
    rng = np.random.default_rng(17)
    # W3 = 0: the outputs are b3, a mixture chosen here
    P = rng.normal(scale=0.1, size=M.N_PARAMS)
    P[M.OFF_W3:M.OFF_B3] = 0.0
    b3 = np.zeros(M.OUT)
    for c in range(M.K):
        b3[c * M.COMP] = rng.normal()
        b3[c * M.COMP + 1: c * M.COMP + 1 + d] = rng.normal(scale=2.0, size=d)
        b3[c * M.COMP + 8: c * M.COMP + 8 + d] = rng.uniform(-0.5, 0.5, size=d)
    P[M.OFF_B3:] = b3
    mlp = _mlp_with(P)
    nbig = 16384
    targets = [torch.empty((nbig, d), dtype=torch.float32, device="cuda") for _ in ex[:2]]
    sex = [dict(q, particles=tg, seq=k) for k, (q, tg) in enumerate(zip(ex[:2], targets))]
    iset = smsq.InitSet([model], sex)
    used = mlp.sample(iset).cpu().numpy()
    torch.cuda.synchronize()
    assert list(used) == [1, 1]
    _, A, Sc = mlp.features(iset)
    for k in range(2):
        X = targets[k].cpu().numpy().astype(np.float64)
        nh = X.shape[0]
        m, v = M.mixture_moments(b3, A[k].cpu().numpy(), Sc[k].cpu().numpy(), d)
        se = np.sqrt(v / nh)
        assert np.all(np.abs(X.mean(axis=0) - m) <= 5 * se), (X.mean(axis=0), m, se)
        # variance of the sample variance ~ 2 v^2 / n for near-Gaussian tails; mixtures: use the 4th moment
        v4 = ((X - X.mean(axis=0)) ** 4).mean(axis=0)
        sev = np.sqrt(np.maximum(v4 - v ** 2, 1e-30) / nh)
        assert np.all(np.abs(X.var(axis=0) - v) <= 5 * sev), (X.var(axis=0), v, sev)


def test_sampler_falls_back_on_nonfinite_outputs():
    wl, model, ex = _examples("range2d", 100, seed=8)
    P = np.zeros(M.N_PARAMS)
    P[M.OFF_B3] = np.inf
    mlp = _mlp_with(P)
    target = torch.full((100, wl.model.d), 7.0, device="cuda")
    iset = smsq.InitSet([model], [dict(ex[0], particles=target)])
    used = mlp.sample(iset).cpu().numpy()
    torch.cuda.synchronize()
    assert list(used) == [0]
    assert torch.all(target == 7.0)


def test_training_lowers_the_loss():
    exs, models = [], []
    for i, (name, n) in enumerate([("arm7", 128), ("range2d", 100), ("cv4d", 64), ("growth1d", 32)]):
        wl, model, ex = _examples(name, n, seed=20 + i, T=6)
        models.append(model)
        exs += [dict(q, model=i) for q in ex]
    iset = smsq.InitSet(models, exs)
    mlp = smsq.InitMLP(seed=3, max_batch=len(exs))
    first = mlp.train_step(iset, 0, len(exs), 1e-3).item()
    for _ in range(200):
        last = mlp.train_step(iset, 0, len(exs), 1e-3)
    last = last.item()
    print("mixture NLL %.4f -> %.4f" % (first, last))
    assert np.isfinite(last) and last < first - 1.0


def test_parameters_save_and_load(tmp_path):
    """A trained-looking parameter set survives save / load_params bit for
    bit, and the reloaded network computes the same outputs."""
    rng = np.random.default_rng(12)
    P = rng.normal(scale=0.1, size=M.N_PARAMS).astype(np.float32)
    a = _mlp_with(P.astype(np.float64))
    path = str(tmp_path / "proposal.npy")
    a.save(path)
    b = smsq.InitMLP(seed=7, max_batch=256)
    assert not torch.equal(a.params(), b.params())
    b.load_params(path)
    assert torch.equal(a.params(), b.params())
    F = torch.tensor(rng.normal(size=(9, M.FEAT)).astype(np.float32), device="cuda")
    assert torch.equal(a.forward(F), b.forward(F))
    a.close()
    b.close()


def test_adam_update_matches_oracle():
    """Two training steps: the parameter update of each against the oracle's
    Adam step (Kingma & Ba, Algorithm 1) for the gradient the step computed
    (read back from the network's gradient buffer), with the moments carried
    from the first step into the second.  The constants are the ones the
    kernel holds in FP32 (beta1 = 0.9f, beta2 = 0.999f, eps = 1e-8f, lr as a
    float).  Bound per element: one FP32 ulp of the new parameter plus
    1e-5 of the update the absolute values of the first moment's two terms
    would give, lr c1 (|b1 m| + |(1 - b1) g|) / (sqrt(v_hat) + eps): the FP32
    moment can cancel when the gradient changes sign, and its rounding error
    is relative to the terms, not to their sum.  A dropped bias correction or
    eps inside the square root moves the update by a factor, far outside
    it."""
    exs, models = [], []
    for i, (name, n) in enumerate([("arm7", 128), ("range2d", 100), ("growth1d", 32)]):
        wl, model, ex = _examples(name, n, seed=40 + i, T=5)
        models.append(model)
        exs += [dict(q, model=i) for q in ex]
    iset = smsq.InitSet(models, exs)
    rng = np.random.default_rng(21)
    P0 = rng.normal(scale=0.05, size=M.N_PARAMS).astype(np.float32)
    mlp = _mlp_with(P0.astype(np.float64))
    f32 = lambda v: float(np.float32(v))
    lr = 3e-3
    cst = dict(lr=f32(lr), b1=f32(0.9), b2=f32(0.999), eps=f32(1e-8))
    m = v = np.zeros(M.N_PARAMS)
    P = P0.astype(np.float64)
    for step in (1, 2):
        mlp.train_step(iset, 0, len(exs), lr)
        torch.cuda.synchronize()
        Pg = mlp.params().cpu().numpy().astype(np.float64)
        G = mlp.grads().cpu().numpy().astype(np.float64)
        mag = cst["b1"] * np.abs(m) + (1 - cst["b1"]) * np.abs(G)
        Po, m, v = M.adam_step(P, G, m, v, step, **cst)
        upd = np.abs(Po - P)
        vh = v / (1 - cst["b2"] ** step)
        scale = cst["lr"] * mag / (1 - cst["b1"] ** step) / (np.sqrt(vh) + cst["eps"])
        bound = np.abs(Po) * 2.0 ** -23 + 1e-5 * scale + 1e-30
        err = np.abs(Pg - Po)
        small = np.sqrt(v / (1 - cst["b2"] ** step)) < 10 * cst["eps"]
        print("adam step %d: max err/bound %.3f, max |update| %.3e, %d of %d elements with sqrt(v_hat) < 10 eps"
              % (step, (err / bound).max(), upd.max(), int((small & (G != 0)).sum()), M.N_PARAMS))
        assert np.all(err <= bound), (step, int(np.argmax(err / bound)))
        assert upd.max() > 1e-4
        P = Pg
    mlp.close()
