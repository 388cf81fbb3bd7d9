"""Pins of the learned-proposal oracle (oracle/init_mlp.py), CPU only.

Backpropagation is checked against central finite differences of the
forward pass, the mixture NLL gradient against finite differences of the
NLL, the NLL of a mixture of identical components against scipy's normal
log-density, the bfloat16 rounding against hand-worked ties, and the
features of a set of identical particles against their closed form."""
import os

import numpy as np
import pytest
from scipy import stats

import oracle as O
from oracle import init_mlp as M
from paper_2312_08684_amd import scenarios as S


def _params(rng, scale=0.2):
    P = rng.normal(scale=scale, size=M.N_PARAMS)
    return P


def test_bf16_rounding_ties_to_even():
    x = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, -2.0 - 2 ** -8, -2.0 - 2 ** -7 - 2 ** -9, 0.0])
    r = M.bf16_round(x)
    # spacing 2^-7 on [1, 2), 2^-6 on [2, 4).  Halfway 1 + 2^-8 -> even mantissa
    # 1.0; 1 + 1.5 * 2^-7 (halfway) -> 1 + 2^-6; -2 - 2^-8 is below the halfway
    # point -2 - 2^-7 -> -2; -2 - 2^-7 - 2^-9 is above it -> -2 - 2^-6
    assert list(r) == [1.0, 1.0, 1.0 + 2 ** -6, -2.0, -2.0 - 2 ** -6, 0.0]


def test_backward_matches_finite_differences():
    rng = np.random.default_rng(3)
    P = _params(rng)
    F = rng.normal(size=(5, M.FEAT))
    dout = rng.normal(size=(5, M.OUT))
    out, cache = M.forward(P, F, bf16=False)
    G = M.backward(cache, dout, bf16=False)

    def f(Pv):
        return float((M.forward(Pv, F, bf16=False)[0] * dout).sum())

    idx = np.concatenate([rng.choice(np.arange(M.OFF_W1, M.OFF_B1), 8), rng.choice(np.arange(M.OFF_B1, M.OFF_W2), 4),
                          rng.choice(np.arange(M.OFF_W2, M.OFF_B2), 8), rng.choice(np.arange(M.OFF_B2, M.OFF_W3), 4),
                          rng.choice(np.arange(M.OFF_W3, M.OFF_B3), 8), rng.choice(np.arange(M.OFF_B3, M.N_PARAMS), 4)])
    h = 1e-6
    for i in idx:
        e = np.zeros_like(P)
        e[i] = h
        fd = (f(P + e) - f(P - e)) / (2 * h)
        assert abs(fd - G[i]) <= 1e-6 * max(1.0, abs(fd)), (i, fd, G[i])


def test_mixture_nll_gradient_matches_finite_differences():
    rng = np.random.default_rng(5)
    d = 3
    out = rng.normal(scale=0.5, size=M.OUT)
    out[8 + 1] = -9.0          # one log-scale below the clamp: zero gradient
    a = np.zeros(8)
    a[:d] = rng.normal(size=d)
    s = np.ones(8)
    s[:d] = [0.5, 1.0, 2.0]
    X = a[:d] + rng.normal(size=(20, d))
    loss, g = M.mixture_nll(out, a, s, X)
    h = 1e-6
    for i in range(M.OUT):
        c, q = divmod(i, M.COMP)
        if (1 + d <= q < 8) or q >= 8 + d:
            assert g[i] == 0.0
            continue
        e = np.zeros_like(out)
        e[i] = h
        fd = (M.mixture_nll(out + e, a, s, X)[0] - M.mixture_nll(out - e, a, s, X)[0]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(fd)), (i, fd, g[i])
    assert g[8 + 1] == 0.0


def test_identical_components_reduce_to_one_gaussian():
    rng = np.random.default_rng(7)
    mu, rho, s = 0.3, -0.4, 1.7
    out = np.zeros(M.OUT)
    for c in range(M.K):
        out[c * M.COMP + 0] = rng.normal()      # any weights: the components coincide
        out[c * M.COMP + 1] = mu
        out[c * M.COMP + 8] = rho
    a = np.zeros(8)
    a[0] = 2.0
    sv = np.ones(8)
    sv[0] = s
    X = rng.normal(size=(50, 1))
    loss, _ = M.mixture_nll(out, a, sv, X)
    ref = -stats.norm.logpdf(X[:, 0], loc=2.0 + s * mu, scale=s * np.exp(rho)).mean()
    assert abs(loss - ref) <= 1e-12 * max(1.0, abs(ref))


def test_features_of_identical_particles():
    wl = S.make_workload("arm7", B=1, seed=0, T=3)
    desc = wl.model
    d = desc.d
    x = np.tile(wl.truth[0, 1], (6, 1))
    phi = np.array([0.0, 2.0, 1.0, 2.0, -1.0, 0.5])   # first maximum at index 1
    F, a, s = M.features(desc, 2, x, phi, wl.z[0, 1], None, 128)
    a_ref = O.transition_mean(desc, 2, x[1])
    sq = np.sqrt(np.asarray(desc.q_var[:d]))
    assert F[3] == 1.0 and F[:3].sum() == 0.0
    assert F[4] == pytest.approx(np.log(128) / 7.0, abs=1e-15)
    assert np.allclose(F[5:5 + d], 0.0, atol=1e-12)
    assert np.allclose(F[12:12 + d], np.log(1e-6) / 8.0, atol=1e-9)
    g = O.grad_loglik(desc, wl.z[0, 1], None, a_ref)
    assert np.allclose(F[19:19 + d], np.arcsinh(sq * g) / 4.0, atol=0)
    ll = O.loglik(desc, wl.z[0, 1], None, a_ref)
    assert F[26] == pytest.approx(np.arcsinh(ll) / 8.0, abs=1e-15)
    assert np.allclose(a[:d], a_ref, atol=0) and np.all(a[d:] == 0)
    assert np.allclose(s[:d], sq, atol=0)
    assert np.all(F[27:] == 0.0)


def test_features_do_not_depend_on_position():
    """A rigid shift of the previous set moves the anchor but changes no
    feature: range2d's transition mean commutes with the shift, and with every
    observation masked out the likelihood summaries are zero at any anchor."""
    wl = S.make_workload("range2d", B=1, seed=0, T=3)
    desc = wl.model
    rng = np.random.default_rng(2)
    x = wl.truth[0, 1] + 0.1 * rng.normal(size=(8, desc.d))
    phi = rng.normal(size=8)
    mask = np.zeros(desc.n_obs, dtype=np.uint8)     # every observation masked out: g = 0, ll = 0
    F1, a1, _ = M.features(desc, 2, x, phi, wl.z[0, 1], mask, 64)
    F2, a2, _ = M.features(desc, 2, x + np.array([30.0, -12.0]), phi, wl.z[0, 1], mask, 64)
    assert not np.allclose(a1, a2)
    assert np.allclose(F1, F2, atol=1e-12)


# ---------------------------------------------------------------------------
# Mixture moments and the Adam update
# ---------------------------------------------------------------------------

def _two_component_out(w, mu, sd):
    """Outputs whose mixture (a = 0, s = 1, d = 1) has components with
    weights w, means mu and standard deviations sd; the other six components
    get a logit of -1e30 (weight exactly zero)."""
    out = np.zeros(M.OUT)
    for c in range(M.K):
        out[c * M.COMP] = -1e30
    for c, (wc, mc, sc) in enumerate(zip(w, mu, sd)):
        out[c * M.COMP] = np.log(wc)
        out[c * M.COMP + 1] = mc
        out[c * M.COMP + 8] = np.log(sc)
    return out


def test_mixture_moments_two_components_by_hand():
    """Weights (1/4, 3/4), means (-1, 3), standard deviations (1/2, 2):
    mean = -1/4 + 9/4 = 2; E[x^2] = 1/4 (1/4 + 1) + 3/4 (4 + 9) = 161/16, so
    the variance is 161/16 - 4 = 97/16 (law of total variance: the mean of
    the component variances 13/16 plus the variance of the means 3)."""
    out = _two_component_out([0.25, 0.75], [-1.0, 3.0], [0.5, 2.0])
    a, s = np.zeros(8), np.ones(8)
    m, v = M.mixture_moments(out, a, s, 1)
    assert m[0] == pytest.approx(2.0, abs=1e-14)
    assert v[0] == pytest.approx(97.0 / 16.0, abs=1e-13)


def test_mixture_moments_follow_anchor_and_scale():
    """Mean a + s mu and variance s^2 sigma^2 per dimension: the same two
    components placed at a = 5 with scale s = 3 (d = 2, second dimension a
    single point mass at the anchor's offset 0 with log-scale -7 clamped)."""
    out = _two_component_out([0.25, 0.75], [-1.0, 3.0], [0.5, 2.0])
    for c in range(2):
        out[c * M.COMP + 2] = 0.0
        out[c * M.COMP + 9] = -20.0       # clamped to -7
    a = np.array([5.0, -1.0, 0, 0, 0, 0, 0, 0])
    s = np.array([3.0, 0.5, 1, 1, 1, 1, 1, 1])
    m, v = M.mixture_moments(out, a, s, 2)
    assert m == pytest.approx([5.0 + 3.0 * 2.0, -1.0], abs=1e-13)
    assert v == pytest.approx([9.0 * 97.0 / 16.0, 0.25 * np.exp(-14.0)], rel=1e-12)


def _golden_adam():
    rows = []
    with open(os.path.join(os.path.dirname(__file__), "golden", "adam_two_step.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                rows.append([float(v) for v in line.split()])
    return np.array(rows)


def test_adam_two_steps_by_hand():
    g = _golden_adam()
    P0, g1, g2, P1_ref, P2_ref = g.T
    zero = np.zeros_like(P0)
    P1, m1, v1 = M.adam_step(P0, g1, zero, zero, 1, 0.1)
    P2, _, _ = M.adam_step(P1, g2, m1, v1, 2, 0.1)
    assert np.allclose(P1, P1_ref, rtol=1e-14, atol=1e-15)
    assert np.allclose(P2, P2_ref, rtol=1e-13, atol=1e-15)


def test_adam_first_step_and_constant_gradient_closed_form():
    """With m_0 = v_0 = 0 the bias correction makes the first step
    -lr g / (|g| + eps) for any beta1, beta2; a gradient that stays constant
    keeps m_hat = g and v_hat = g^2 at every step, so every step is the same."""
    rng = np.random.default_rng(4)
    P = rng.normal(size=50)
    g = rng.normal(size=50) * np.logspace(-9, 1, 50)
    m = v = np.zeros(50)
    want = -0.01 * g / (np.abs(g) + 1e-8)
    for t in range(1, 6):
        Pn, m, v = M.adam_step(P, g, m, v, t, 0.01, b1=0.8, b2=0.99)
        assert np.allclose(Pn - P, want, rtol=1e-9, atol=1e-18), t
        P = Pn
