"""GPU parity: the HIP path (through the C ABI) against the CPU FP64 oracle.

Tolerances (stated per result):
  * forward recursion fed the oracle's FP64 lattice: bit-exact phi, psi, flags;
  * backtracking: bit-exact indices and score;
  * SVGD step, teacher-forced (same previous and initial particles on both
    sides): ||X_gpu - X_oracle||_F / ||X_oracle||_F <= 1e-4 in FP32 and
    <= 1e-10 in FP64, after the full iteration count; the same difference
    against the oracle's move ||X_oracle - X_init||_F (bounds and their
    FP32 rounding floor in parity_bounds.py);
  * trajectory log-posterior J: |dJ| <= 1e-3 max(|J|, T).
The FP32-vs-FP64 errors measured here are printed with each case.
"""
import math

import numpy as np
import pytest
import torch

import oracle as O
from paper_2312_08684_amd import scenarios as S
from paper_2312_08684_amd import smsq
from parity_bounds import check_move

pytestmark = pytest.mark.gpu

DEV = "cuda"
TOL_X = {"f32": 1e-4, "f64": 1e-10}
TOL_H = {"f32": 1e-5, "f64": 1e-12}
TOL_J = 1e-3
TIE_F32 = 2.0 ** -20


def dev(a, dtype):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device=DEV)


def tdt(dt):
    return torch.float64 if dt == "f64" else torch.float32


def host(t):
    return t.detach().cpu().numpy()


def announce(*what):
    print("CASE", *what, flush=True)


# ---------------------------------------------------------------------------
# Forward recursion
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("n,n_prev", [(1, 1), (7, 1), (64, 64), (100, 37), (130, 257), (1024, 1024),
                                      (1500, 700), (50, 2050)])
def test_viterbi_lattice_f64_bit_exact(n, n_prev):
    announce("viterbi lattice f64", n, n_prev)
    rng = np.random.default_rng(n * 1000 + n_prev)
    A = rng.normal(size=(n, n_prev)) * 5
    ell = rng.normal(size=n)
    phi_prev = rng.normal(size=n_prev) * 10
    # plant exact ties and -inf rows
    if n_prev > 3:
        A[0, 2] = A[0, 1] = A[0].max() + 1.0
        phi_prev[1] = phi_prev[2]
    if n > 2:
        A[2, :] = -np.inf
    phi_o, psi_o, fl_o, st_o = O.viterbi_lattice(A, ell, phi_prev, tie_tol=1e-9)
    ws = smsq.workspace()
    phi, psi, fl = smsq.viterbi_step(None, "f64", 1, dev(phi_prev, torch.float64),
                                     lattice=dev(A, torch.float64), loglik=dev(ell, torch.float64),
                                     tie_tol=1e-9, ws=ws)
    assert np.array_equal(host(psi), psi_o)
    assert np.array_equal(host(phi), phi_o)
    assert np.array_equal(host(fl), fl_o)
    assert smsq.device_status(ws) == smsq.OK


@pytest.mark.parametrize("n_prev", [5, 8])
def test_viterbi_lattice_nan_sets_status(n_prev):
    announce("viterbi lattice nan", n_prev)
    A = np.zeros((3, n_prev))
    A[1, n_prev - 2] = np.nan
    ws = smsq.workspace()
    smsq.viterbi_step(None, "f64", 1, dev(np.zeros(n_prev), torch.float64), lattice=dev(A, torch.float64),
                      loglik=dev(np.zeros(3), torch.float64), ws=ws)
    assert smsq.device_status(ws) == smsq.ERR_NONFINITE


@pytest.mark.parametrize("n,n_prev", [(100, 37), (64, 128), (7, 1)])
def test_viterbi_lattice_batch_f64_bit_exact(n, n_prev):
    """Several lattices in one launch (smsq_viterbi_lattice_batch): each
    bit-exact against the oracle, as the single-lattice call is."""
    announce("viterbi lattice batch f64", n, n_prev)
    rng = np.random.default_rng(n + 3 * n_prev)
    B = 3
    A = rng.normal(size=(B, n, n_prev)) * 5
    ell = rng.normal(size=(B, n))
    php = rng.normal(size=(B, n_prev)) * 10
    A[1, 0, :] = -np.inf
    if n_prev > 3:
        A[2, 1, 1] = A[2, 1, 2] = A[2, 1].max() + 1.0
        php[2, 1] = php[2, 2]
    ws = smsq.workspace()
    phi, psi, fl = smsq.viterbi_lattice_batch("f64", dev(php, torch.float64), dev(A, torch.float64),
                                              dev(ell, torch.float64), tie_tol=1e-9, ws=ws)
    assert smsq.device_status(ws) == smsq.OK
    for b in range(B):
        phi_o, psi_o, fl_o, _ = O.viterbi_lattice(A[b], ell[b], php[b], tie_tol=1e-9)
        assert np.array_equal(host(psi)[b], psi_o)
        assert np.array_equal(host(phi)[b], phi_o)
        assert np.array_equal(host(fl)[b], fl_o)


@pytest.mark.parametrize("n,n_prev", [(33, 65), (512, 512), (64, 4096), (300, 1028)])
def test_viterbi_lattice_f32(n, n_prev):
    announce("viterbi lattice f32", n, n_prev)
    rng = np.random.default_rng(7 + n)
    A = (rng.normal(size=(n, n_prev)) * 5).astype(np.float32)
    ell = rng.normal(size=n).astype(np.float32)
    phi_prev = (rng.normal(size=n_prev) * 10).astype(np.float32)
    # an exact tie across two lanes' vectors in row 0: the lower index wins
    tie = n_prev > 260
    if tie:
        A[0, 3] = A[0, 260] = A[0].max() + 50.0
        phi_prev[3] = phi_prev[260] = phi_prev.max()
    phi_o, psi_o, fl_o, _ = O.viterbi_lattice(A.astype(np.float64), ell.astype(np.float64),
                                              phi_prev.astype(np.float64), tie_tol=TIE_F32)
    phi, psi, fl = smsq.viterbi_step(None, "f32", 1, dev(phi_prev, torch.float32),
                                     lattice=dev(A, torch.float32), loglik=dev(ell, torch.float32),
                                     tie_tol=TIE_F32)
    psi, phi = host(psi), host(phi).astype(np.float64)
    sure = fl_o == 0
    assert np.array_equal(psi[sure], psi_o[sure])
    c = A.astype(np.float64) + phi_prev[None, :]
    best = c.max(1)
    chosen = c[np.arange(n), psi]
    assert np.all(chosen >= best - 4 * TIE_F32 * np.maximum(1, np.abs(best)))
    assert np.allclose(phi, phi_o, rtol=1e-6, atol=1e-5)
    if tie:
        assert psi[0] == 3


def _particle_case(name, n, n_prev, seed):
    wl = S.make_workload(name, B=1, seed=seed, T=3)
    desc = wl.model
    rng = np.random.default_rng(seed + 17)
    sd = np.sqrt(desc.q_var[:desc.d])
    xp = wl.truth[0, 1][None, :] + 2 * sd * rng.normal(size=(n_prev, desc.d))
    means = np.stack([O.transition_mean(desc, 2, v) for v in xp])
    x = means[rng.integers(n_prev, size=n)] + sd * rng.normal(size=(n, desc.d))
    return wl, desc, xp, x


@pytest.mark.parametrize("name", ["growth1d", "range2d", "cv4d", "arm7", "lingauss", "scenario_b", "scenario_d"])
@pytest.mark.parametrize("dt", ["f32", "f64"])
@pytest.mark.parametrize("flags", [True, False])
def test_viterbi_particle_mode(name, dt, flags):
    """Particle mode per model, with and without tie flags (rows in blocks
    of 4..16 per workgroup pass for the states that fit it, two waves per row
    for the others)."""
    announce("viterbi particle", name, dt, flags)
    n, n_prev = 150, 77
    wl, desc, xp, x = _particle_case(name, n, n_prev, 3)
    z = wl.z[0, 1]
    mask = None if wl.mask is None else wl.mask[0, 1]
    rng = np.random.default_rng(5)
    phi_prev = rng.normal(size=n_prev) * 3
    td = tdt(dt)
    if dt == "f32":
        xp = xp.astype(np.float32).astype(np.float64)
        x = x.astype(np.float32).astype(np.float64)
        phi_prev = phi_prev.astype(np.float32).astype(np.float64)
        z = z.astype(np.float32).astype(np.float64)
    tol = 1e-5 if dt == "f32" else 1e-9
    phi_o, psi_o, fl_o, st = O.viterbi_particle(desc, 2, xp, phi_prev, z, mask, x, tie_tol=tol)
    assert st == O.OK
    model = smsq.Model(desc)
    phi, psi, fl = smsq.viterbi_step(model, dt, 2, dev(phi_prev, td), x_prev=dev(xp, td), z_t=dev(z, td),
                                     z_mask=None if mask is None else dev(mask, torch.uint8),
                                     x=dev(x, td), tie_tol=tol, want_flags=flags)
    psi, phi = host(psi), host(phi).astype(np.float64)
    sure = fl_o == 0
    assert sure.mean() > 0.5
    assert np.array_equal(psi[sure], psi_o[sure])
    A, ell = O.particle_lattice(desc, 2, xp, z, mask, x)
    c = A + phi_prev[None, :]
    best = c.max(1)
    assert np.all(c[np.arange(n), psi] >= best - 4 * tol * np.maximum(1, np.abs(best)))
    if flags:
        # tie flags wherever the runner-up gap is clearly on one side of
        # tie_tol max(1, |best|)
        c2 = c.copy()
        c2[np.arange(n), c.argmax(1)] = -np.inf
        gap = best - c2.max(1)
        thr = tol * np.maximum(1.0, np.abs(best))
        clear0, clear1 = gap > 1.5 * thr, gap < 0.5 * thr
        fl = host(fl)
        print("tie flags: %d clear 0, %d clear 1" % (clear0.sum(), clear1.sum()))
        assert clear0.sum() > 0
        assert np.all(fl[clear0] == 0) and np.all(fl[clear1] == 1)
        assert np.array_equal(fl[clear0 | clear1], fl_o[clear0 | clear1])
    err = np.abs(phi - phi_o) / np.maximum(1, np.abs(phi_o))
    print("phi rel err", err.max())
    # FP32 evaluation of the log-densities (e.g. the arm's forward kinematics,
    # d ell / d p ~ |z - p| / r ~ 500 times a ~1e-7 position rounding) bounds
    # the FP32 error near 1e-4 relative
    assert err.max() <= (1e-4 if dt == "f32" else 1e-12)


@pytest.mark.parametrize("name", ["range2d", "cv4d", "arm7"])
@pytest.mark.parametrize("dt", ["f32", "f64"])
def test_viterbi_particle_tie_flags(name, dt):
    """Tie flags of particle mode (eq. forward_recursion; runner-up within
    tie_tol max(1, |best|)) against the oracle's, on every row whose gap is
    clearly on one side of the threshold.  Exact duplicates of the previous
    particles with the highest scores (as resampling makes) give exact ties;
    the others give clear gaps."""
    announce("viterbi particle tie flags", name, dt)
    n, n_prev = 400, 300
    wl, desc, xp, x = _particle_case(name, n, n_prev, 21)
    z = wl.z[0, 1]
    mask = None if wl.mask is None else wl.mask[0, 1]
    phi_prev = np.random.default_rng(22).normal(size=n_prev) * 3
    top = np.argsort(phi_prev[:n_prev - 4])[-4:]
    xp[n_prev - 4:] = xp[top]
    phi_prev[n_prev - 4:] = phi_prev[top]
    td = tdt(dt)
    if dt == "f32":
        xp, x, phi_prev, z = (v.astype(np.float32).astype(np.float64) for v in (xp, x, phi_prev, z))
    tol = 1e-5 if dt == "f32" else 1e-9
    phi_o, psi_o, fl_o, st = O.viterbi_particle(desc, 2, xp, phi_prev, z, mask, x, tie_tol=tol)
    assert st == O.OK
    ws = smsq.workspace()
    _, _, fl = smsq.viterbi_step(smsq.Model(desc), dt, 2, dev(phi_prev, td), x_prev=dev(xp, td), z_t=dev(z, td),
                                 z_mask=None if mask is None else dev(mask, torch.uint8), x=dev(x, td),
                                 tie_tol=tol, ws=ws)
    assert smsq.device_status(ws) == smsq.OK
    A, _ = O.particle_lattice(desc, 2, xp, z, mask, x)
    c = A + phi_prev[None, :]
    best = c.max(1)
    c[np.arange(n), c.argmax(1)] = -np.inf
    gap = best - c.max(1)
    thr = tol * np.maximum(1.0, np.abs(best))
    clear0, clear1 = gap > 1.5 * thr, gap < 0.5 * thr
    fl = host(fl)
    print("tie flags: %d clear 0, %d clear 1, %d between" % (clear0.sum(), clear1.sum(), n - clear0.sum() - clear1.sum()))
    assert clear0.sum() > 0 and clear1.sum() > 0
    assert np.array_equal(fl_o[clear0 | clear1], clear1[clear0 | clear1].astype(np.uint8))
    assert np.all(fl[clear0] == 0) and np.all(fl[clear1] == 1)


@pytest.mark.parametrize("dt", ["f32", "f64"])
def test_backtrack_bit_exact(dt):
    announce("backtrack", dt)
    rng = np.random.default_rng(11)
    B, T, n = 5, 40, 70
    psi = rng.integers(0, n, size=(B, T, n)).astype(np.int32)
    phi_T = rng.normal(size=(B, n))
    phi_T[0, 3] = phi_T[0, 9] = phi_T[0].max() + 1   # tie -> lowest index
    if dt == "f32":
        phi_T = phi_T.astype(np.float32).astype(np.float64)
    parts = rng.normal(size=(B, T, n, 3))
    x0 = rng.normal(size=(B, 3))
    td = tdt(dt)
    idx, J, xmap = smsq.backtrack(dt, dev(psi, torch.int32), dev(phi_T, td), dev(parts, td), dev(x0, td))
    idx, J, xmap = host(idx), host(J), host(xmap)
    for b in range(B):
        ii, jj, st = O.backtrack(psi[b], phi_T[b])
        assert np.array_equal(idx[b], ii)
        assert J[b] == (np.float32(jj) if dt == "f32" else jj)
        assert np.array_equal(xmap[b, 0], x0[b].astype(np.float32) if dt == "f32" else x0[b])
        want = parts[b, np.arange(T), ii]
        assert np.array_equal(xmap[b, 1:], want.astype(np.float32) if dt == "f32" else want)


@pytest.mark.parametrize("dt", ["f32", "f64"])
@pytest.mark.parametrize("case", ["ragged", "ties", "all_neg_inf", "one_step", "uniform"])
def test_backtrack_steps_bit_exact(dt, case):
    """Backtracking with a particle count per step (n_t[0] = 1).  The walk
    reads only entries i < n_t[t] of row t-1, so the oracle's uniform
    backtrack over rows padded to n_max (padding phi_T with -inf, psi with 0)
    gives the same path; padding entries of the device psi hold indices out
    of range, which a walk that strayed into them would flag."""
    announce("backtrack_steps", dt, case)
    rng = np.random.default_rng({"ragged": 21, "ties": 22, "all_neg_inf": 23, "one_step": 24, "uniform": 25}[case])
    T = 1 if case == "one_step" else 37
    n_max = 300
    if case == "uniform":
        counts = [1] + [n_max] * T
    else:
        counts = [1] + [int(c) for c in rng.integers(1, n_max + 1, size=T)]
        counts[-1] = max(counts[-1], 5)
    psi = np.full((T, n_max), n_max + 7, dtype=np.int32)        # padding: out of range
    for t in range(1, T + 1):
        psi[t - 1, :counts[t]] = rng.integers(0, counts[t - 1], size=counts[t])
    nT = counts[T]
    phi_T = rng.normal(size=nT)
    if case == "ties":
        phi_T[[1, 4]] = phi_T.max() + 1.0
    if case == "all_neg_inf":
        phi_T[:] = -np.inf
    if dt == "f32":
        phi_T = phi_T.astype(np.float32).astype(np.float64)
    td = tdt(dt)
    ws = smsq.workspace(smsq.HEADER_BYTES + 4 * (T + 1))
    idx, J = smsq.backtrack_steps(dt, dev(psi, torch.int32), dev(phi_T, td), counts, ws=ws)
    idx, J = host(idx), host(J)
    pad_psi = np.where(psi >= n_max, 0, psi).astype(np.int32)
    pad_phi = np.concatenate([phi_T, np.full(n_max - nT, -np.inf)])
    ii, jj, st = O.backtrack(pad_psi, pad_phi)
    assert np.array_equal(idx, ii), case
    assert J[0] == (np.float32(jj) if dt == "f32" else jj)
    for t in range(1, T + 1):
        assert 0 <= idx[t - 1] < counts[t]
    want = smsq.ERR_NONFINITE if case == "all_neg_inf" else smsq.OK
    assert smsq.device_status(ws) == want
    if case == "uniform":   # equal counts: the same path as the uniform entry point
        i2, J2, _ = smsq.backtrack(dt, dev(psi, torch.int32), dev(phi_T, td))
        assert np.array_equal(host(i2)[0], idx) and host(J2)[0] == J[0]


def test_backtrack_steps_flags_out_of_range_pointer():
    """A back-pointer at or beyond the previous step's count (but inside the
    row) is reported through the workspace status; the walk goes on from 0."""
    announce("backtrack_steps", "f64", "bad pointer")
    T, n_max = 4, 16
    counts = [1, 3, 8, 5, 6]
    psi = np.zeros((T, n_max), dtype=np.int32)
    psi[3, :6] = 7            # step 4 points at index 7 of step 3, which holds 5 particles
    phi_T = np.arange(6, dtype=np.float64)
    ws = smsq.workspace(smsq.HEADER_BYTES + 4 * (T + 1))
    idx, J = smsq.backtrack_steps("f64", dev(psi, torch.int32), dev(phi_T, torch.float64), counts, ws=ws)
    assert smsq.device_status(ws) == smsq.ERR_NONFINITE
    assert host(idx).tolist() == [0, 0, 0, 5] and host(J)[0] == 5.0


@pytest.mark.parametrize("n,n_prev", [(4000, 4000), (2000, 1999), (1, 3000), (2500, 1), (777, 1025),
                                      (8200, 600), (33, 5000)])
@pytest.mark.parametrize("dt", ["f32", "f64"])
@pytest.mark.parametrize("flags", [True, False])
def test_viterbi_particle_mode_large(n, n_prev, dt, flags):
    """Particle mode at PF-MAP-Seq sizes (up to 4000 x 4000 edges of the
    range-only model), with one row, one previous particle, ragged tails,
    more rows than one pass of the rows kernel's grid covers and a table
    of several load chunks."""
    announce("viterbi particle large", n, n_prev, dt, flags)
    wl, desc, xp, x = _particle_case("range2d", n, n_prev, 4)
    z = wl.z[0, 1]
    rng = np.random.default_rng(6)
    phi_prev = rng.normal(size=n_prev) * 3
    td = tdt(dt)
    if dt == "f32":
        xp, x, phi_prev, z = (v.astype(np.float32).astype(np.float64) for v in (xp, x, phi_prev, z))
    tol = 1e-5 if dt == "f32" else 1e-9
    phi_o, psi_o, fl_o, st = O.viterbi_particle(desc, 2, xp, phi_prev, z, None, x, tie_tol=tol)
    assert st == O.OK
    ws = smsq.workspace()
    phi, psi, fl = smsq.viterbi_step(smsq.Model(desc), dt, 2, dev(phi_prev, td), x_prev=dev(xp, td),
                                     z_t=dev(z, td), x=dev(x, td), tie_tol=tol, ws=ws, want_flags=flags)
    assert smsq.device_status(ws) == smsq.OK
    psi, phi = host(psi), host(phi).astype(np.float64)
    sure = fl_o == 0
    assert np.array_equal(psi[sure], psi_o[sure])
    if n_prev == 1:
        assert np.all(psi == 0)
        if flags:
            assert np.all(host(fl) == 0)
    err = np.abs(phi - phi_o) / np.maximum(1, np.abs(phi_o))
    print("phi rel err %.3e, sure rows %.3f" % (err.max(), sure.mean()))
    # FP32: the range log-likelihood dominates (d ell / d r = e / r_var, up to
    # ~8 per beacon, times the ~3e-6 rounding of ranges near 20), as in the
    # per-model test above
    assert err.max() <= (1e-4 if dt == "f32" else 1e-12)


@pytest.mark.parametrize("name,n,n_prev", [("cv4d", 2000, 1999), ("cv4d", 777, 1025), ("scenario_b", 1000, 1000),
                                           ("cv4d", 33, 2040)])
@pytest.mark.parametrize("flags", [True, False])
def test_viterbi_particle_f64_rows_wider_states(name, n, n_prev, flags):
    """FP64 states of 3 and 4 dimensions on the rows kernel at sizes that
    span several row passes, table chunks and a ragged last tile: psi equal
    on every row the oracle does not flag as a near tie, phi to 1e-12."""
    announce("viterbi particle f64 rows", name, n, n_prev, flags)
    wl, desc, xp, x = _particle_case(name, n, n_prev, 8)
    assert desc.d in (3, 4)
    z = wl.z[0, 1]
    mask = None if wl.mask is None else wl.mask[0, 1]
    phi_prev = np.random.default_rng(9).normal(size=n_prev) * 3
    tol = 1e-9
    phi_o, psi_o, fl_o, st = O.viterbi_particle(desc, 2, xp, phi_prev, z, mask, x, tie_tol=tol)
    assert st == O.OK
    ws = smsq.workspace()
    phi, psi, fl = smsq.viterbi_step(smsq.Model(desc), "f64", 2, dev(phi_prev, torch.float64),
                                     x_prev=dev(xp, torch.float64), z_t=dev(z, torch.float64),
                                     z_mask=None if mask is None else dev(mask, torch.uint8),
                                     x=dev(x, torch.float64), tie_tol=tol, ws=ws, want_flags=flags)
    assert smsq.device_status(ws) == smsq.OK
    psi, phi = host(psi), host(phi)
    sure = fl_o == 0
    assert np.array_equal(psi[sure], psi_o[sure])
    err = np.abs(phi - phi_o) / np.maximum(1, np.abs(phi_o))
    print("d %d phi rel err %.3e, sure rows %.3f" % (desc.d, err.max(), sure.mean()))
    assert err.max() <= 1e-12
    if flags:
        clear = np.abs(host(fl).astype(int) - fl_o.astype(int)) == 0
        assert clear.mean() > 0.99


@pytest.mark.parametrize("dt", ["f32", "f64"])
def test_viterbi_step_out_tensors(dt):
    """phi_out / psi_out (a row of a [T, n] back-pointer array) receive the
    same values the step returns when it allocates its outputs."""
    announce("viterbi out tensors", dt)
    n, n_prev = 1200, 900
    wl, desc, xp, x = _particle_case("range2d", n, n_prev, 12)
    td = tdt(dt)
    model = smsq.Model(desc)
    ws = smsq.workspace()
    phi_prev = dev(np.random.default_rng(3).normal(size=n_prev), td)
    args = dict(x_prev=dev(xp, td), z_t=dev(wl.z[0, 1], td), x=dev(x, td), want_flags=False, ws=ws)
    phi_a, psi_a, _ = smsq.viterbi_step(model, dt, 2, phi_prev, **args)
    psi_all = torch.full((3, n), -7, dtype=torch.int32, device=DEV)
    phi_o = torch.full((n,), 5.0, dtype=td, device=DEV)
    phi_b, psi_b, _ = smsq.viterbi_step(model, dt, 2, phi_prev, phi_out=phi_o, psi_out=psi_all[1], **args)
    assert phi_b.data_ptr() == phi_o.data_ptr() and psi_b.data_ptr() == psi_all[1].data_ptr()
    assert torch.equal(phi_a, phi_o) and torch.equal(psi_a, psi_all[1])
    assert torch.all(psi_all[0] == -7) and torch.all(psi_all[2] == -7)
    assert smsq.device_status(ws) == smsq.OK


@pytest.mark.parametrize("dt", ["f32", "f64"])
@pytest.mark.parametrize("flags", [True, False])
@pytest.mark.parametrize("case", ["nan_score", "inf_row", "dead_block"])
def test_viterbi_particle_nonfinite(case, dt, flags):
    """Non-finite inputs in particle mode: a NaN previous score (every row
    sees a NaN edge: status non-finite, NaN never the argmax), a row at
    infinity (its scores are all -inf: index 0) and previous scores that are
    -inf on a whole block of the table; each against the oracle."""
    announce("viterbi particle nonfinite", case, dt, flags)
    n, n_prev = 300, 700
    wl, desc, xp, x = _particle_case("range2d", n, n_prev, 8)
    z = wl.z[0, 1]
    rng = np.random.default_rng(9)
    phi_prev = rng.normal(size=n_prev) * 3
    if case == "nan_score":
        phi_prev[5] = np.nan
    elif case == "inf_row":
        x[17, 0] = np.inf
    else:
        phi_prev[:600] = -np.inf
    td = tdt(dt)
    if dt == "f32":
        xp, x, phi_prev, z = (v.astype(np.float32).astype(np.float64) for v in (xp, x, phi_prev, z))
    tol = 1e-5 if dt == "f32" else 1e-9
    phi_o, psi_o, fl_o, st = O.viterbi_particle(desc, 2, xp, phi_prev, z, None, x, tie_tol=tol)
    ws = smsq.workspace()
    phi, psi, _ = smsq.viterbi_step(smsq.Model(desc), dt, 2, dev(phi_prev, td), x_prev=dev(xp, td),
                                    z_t=dev(z, td), x=dev(x, td), tie_tol=tol, ws=ws, want_flags=flags)
    status = smsq.device_status(ws)
    assert (status == smsq.ERR_NONFINITE) == (st == O.NONFINITE), (status, st)
    psi, phi = host(psi), host(phi).astype(np.float64)
    sure = fl_o == 0
    if case == "inf_row":
        assert psi[17] == 0 and psi_o[17] == 0 and phi[17] == phi_o[17]
    assert np.array_equal(psi[sure], psi_o[sure])
    fin = np.isfinite(phi_o)
    assert np.array_equal(np.isfinite(phi), fin)
    err = np.abs(phi[fin] - phi_o[fin]) / np.maximum(1, np.abs(phi_o[fin]))
    assert err.max() <= (1e-5 if dt == "f32" else 1e-12)


@pytest.mark.parametrize("dt", ["f32", "f64"])
@pytest.mark.parametrize("flags", [True, False])
def test_pf_map_seq_forward_recursion(dt, flags):
    """The PF-MAP-Seq workload: forward recursion and backtrack over the
    particle sets of a bootstrap particle filter (1500 particles per step,
    12 steps of the range-only model), step by step against the oracle fed
    the same scores, then free-running to the MAP log-posterior."""
    announce("pf-map-seq", dt, flags)
    T, n = 12, 1500
    wl = S.make_workload("range2d", B=1, seed=1008, T=T)
    desc = wl.model
    parts = S.bootstrap_pf_particles(desc, wl.x0[0], wl.z[0], None, n, seed=9)
    td = tdt(dt)
    rnd = (lambda v: v.astype(np.float32).astype(np.float64)) if dt == "f32" else (lambda v: v)
    parts, x0, z = rnd(parts), rnd(wl.x0[0][None, :]), rnd(wl.z[0])
    tol = 1e-5 if dt == "f32" else 1e-9
    model = smsq.Model(desc)
    ws = smsq.workspace()
    phi_o = np.zeros(1)
    phi_g = torch.zeros(1, dtype=td, device=DEV)
    psi_all = torch.zeros((T, n), dtype=torch.int32, device=DEV)
    psi_o_all = np.zeros((T, n), dtype=np.int32)
    flag_counts = [0, 0]
    for t in range(1, T + 1):
        xp = x0 if t == 1 else parts[t - 2]
        ph_o, ps_o, fl_o, st = O.viterbi_particle(desc, t, xp, phi_o, z[t - 1], None, parts[t - 1], tie_tol=tol)
        assert st == O.OK
        # same scores on both sides for this step's comparison
        ph_t, ps_t, fl_t = smsq.viterbi_step(model, dt, t, dev(rnd(phi_o), td), x_prev=dev(xp, td),
                                             z_t=dev(z[t - 1], td), x=dev(parts[t - 1], td), tie_tol=tol, ws=ws,
                                             want_flags=flags)
        sure = fl_o == 0
        assert np.array_equal(host(ps_t)[sure], ps_o[sure]), t
        if flags:
            # tie flags against the oracle's scores wherever the runner-up gap
            # is clearly on one side of tie_tol max(1, |best|)
            A, _ = O.particle_lattice(desc, t, xp, z[t - 1], None, parts[t - 1])
            c = A + rnd(phi_o)[None, :]
            top = c.argmax(1)
            best = c[np.arange(n), top]
            c[np.arange(n), top] = -np.inf
            gap = best - c.max(1)
            thr = tol * np.maximum(1.0, np.abs(best))
            clear0, clear1 = gap > 1.5 * thr, gap < 0.5 * thr
            fl_t = host(fl_t)
            assert np.all(fl_t[clear0] == 0) and np.all(fl_t[clear1] == 1), t
            assert np.array_equal(fl_o[clear0 | clear1], fl_t[clear0 | clear1]), t
            flag_counts[0] += int(clear0.sum())
            flag_counts[1] += int(clear1.sum())
        err = np.abs(host(ph_t).astype(np.float64) - ph_o) / np.maximum(1, np.abs(ph_o))
        assert err.max() <= (1e-5 if dt == "f32" else 1e-12), (t, err.max())
        # free-running chain on the GPU's own scores
        phi_g, psi_g, _ = smsq.viterbi_step(model, dt, t, phi_g, x_prev=dev(xp, td), z_t=dev(z[t - 1], td),
                                            x=dev(parts[t - 1], td), tie_tol=tol, ws=ws, want_flags=flags)
        psi_all[t - 1] = psi_g
        psi_o_all[t - 1] = ps_o
        phi_o = ph_o
    assert smsq.device_status(ws) == smsq.OK
    idx, J, _ = smsq.backtrack(dt, psi_all, phi_g, ws=ws)
    idx_o, J_o, st = O.backtrack(psi_o_all, phi_o)
    J = float(host(J).reshape(-1)[0])
    dJ = abs(J - J_o) / max(abs(J_o), T)
    print("J gpu %.8f oracle %.8f rel %.3e; path agreement %.3f" % (J, J_o, dJ,
          np.mean(host(idx).reshape(-1) == idx_o)))
    assert dJ <= (1e-5 if dt == "f32" else 1e-12)
    if dt == "f64":
        assert np.array_equal(host(idx).reshape(-1), idx_o)
    if flags:
        print("tie flags compared: %d clear 0, %d clear 1" % tuple(flag_counts))
        assert flag_counts[0] > 0


# ---------------------------------------------------------------------------
# SVGD step, teacher-forced
# ---------------------------------------------------------------------------

def _svgd_case(name, n, n_prev, seed, dt):
    wl, desc, xp, x = _particle_case(name, n, n_prev, seed)
    z = wl.z[0, 1]
    mask = None if wl.mask is None else wl.mask[0, 1]
    if dt == "f32":
        xp = xp.astype(np.float32).astype(np.float64)
        x = x.astype(np.float32).astype(np.float64)
        z = z.astype(np.float32).astype(np.float64)
    return wl, desc, xp, x, z, mask


def _compare_svgd(desc, dt, xp, log_w, z, mask, x, L, step, bw_scale=1.0, bw_mode=0, trans_mode=0, kernel=0,
                  step_kernel="auto"):
    td = tdt(dt)
    xo, ho, st = O.svgd_step(desc, 2, xp, log_w, z, mask, x, L, step, bw_scale, bw_mode, trans_mode, kernel)
    assert st == O.OK
    model = smsq.Model(desc)
    xg = dev(x, td)
    hg = torch.zeros(max(L, 1), dtype=td, device=DEV)
    ws = smsq.workspace()
    smsq.svgd_step(model, dt, 2, dev(xp, td), None if log_w is None else dev(log_w, td), dev(z, td),
                   None if mask is None else dev(mask, torch.uint8), xg,
                   smsq.opts(L, step, bw_scale, bw_mode, trans_mode, kernel, step_kernel=step_kernel), h_out=hg,
                   ws=ws)
    assert smsq.device_status(ws) == smsq.OK
    xg, hg = host(xg).astype(np.float64), host(hg).astype(np.float64)[:L]
    rel = np.linalg.norm(xg - xo) / np.linalg.norm(xo)
    herr = np.abs(hg - ho).max() / np.abs(ho).max() if L else 0.0
    print("rel X err %.3e  rel h err %.3e" % (rel, herr))
    assert rel <= TOL_X[dt]
    print(check_move(xg, xo, x, L, dt))
    assert herr <= TOL_H[dt]
    return xo, xg


SVGD_CASES = [
    ("growth1d", 32, 32, 100, 0.05),
    ("growth1d", 100, 33, 40, 0.05),
    ("range2d", 257, 200, 20, 0.005),
    ("cv4d", 130, 64, 20, 0.005),
    ("arm7", 200, 129, 20, 1e-5),
    ("lingauss", 70, 70, 30, 0.01),
    ("scenario_b", 20, 20, 100, 1e-4),
    ("scenario_b", 300, 130, 30, 1e-4),
    ("scenario_d", 20, 20, 100, 2e-4),
    ("scenario_d", 150, 70, 30, 2e-4),
    # the range-only and clutter workloads at their full particle counts and
    # iteration counts (one teacher-forced step)
    ("range2d", 256, 256, 50, 0.005),
    ("cv4d", 512, 512, 50, 0.005),
    # d <= 3 with sixteen 64-particle tasks (one MFMA per tile, no source
    # splits) and a ragged tail
    ("range2d", 1000, 600, 10, 0.005),
]


@pytest.mark.parametrize("name,n,n_prev,L,step", SVGD_CASES)
@pytest.mark.parametrize("dt", ["f32", "f64"])
def test_svgd_step_teacher_forced(name, n, n_prev, L, step, dt):
    announce("svgd step", name, n, n_prev, L, dt)
    wl, desc, xp, x, z, mask = _svgd_case(name, n, n_prev, 21, dt)
    _compare_svgd(desc, dt, xp, None, z, mask, x, L, step)


@pytest.mark.parametrize("name,n,n_prev,L,step", SVGD_CASES)
def test_svgd_step_vector_alu_kernel(name, n, n_prev, L, step):
    """The FP32 vector-ALU step kernel (selected instead of the matrix-core one)."""
    announce("svgd step valu", name, n, n_prev, L)
    sk = "valu"
    wl, desc, xp, x, z, mask = _svgd_case(name, n, n_prev, 22, "f32")
    _compare_svgd(desc, "f32", xp, None, z, mask, x, L, step, step_kernel=sk)


@pytest.mark.parametrize("variant", ["weights", "mean_reading", "per_step_bw", "bw3", "one_particle",
                                     "two_particles", "ragged_1025", "ties_16x16", "ties_4x64"])
def test_svgd_step_variants(variant):
    """Option and shape variants.  ties_GxC: C copies of each of G distinct
    particles (identical particles stay identical under the update), so the
    median distance has hundreds (16x16) or thousands (4x64) of exact copies:
    the window selection meets a candidate bin over its limit or an
    overflowing window buffer and takes its fallbacks."""
    announce("svgd variant", variant)
    name, n, n_prev, L, step = "range2d", 96, 50, 15, 0.005
    log_w, bw_scale, bw_mode, trans_mode = None, 1.0, 0, 0
    if variant == "one_particle":
        n = 1
    if variant == "two_particles":
        n = 2
    if variant == "ragged_1025":
        name, n, n_prev, L, step = "cv4d", 1025, 300, 3, 0.005
    if variant.startswith("ties_"):
        n, L = 256, 6
    wl, desc, xp, x, z, mask = _svgd_case(name, n, n_prev, 4, "f32")
    if variant.startswith("ties_"):
        groups, copies = (int(v) for v in variant[5:].split("x"))
        x = np.repeat(x[:groups], copies, axis=0)
    if variant == "weights":
        rng = np.random.default_rng(3)
        log_w = np.log(rng.dirichlet(np.ones(n_prev))).astype(np.float32).astype(np.float64)
    if variant == "mean_reading":
        trans_mode = 1
    if variant == "per_step_bw":
        bw_mode = 1
    if variant == "bw3":
        bw_scale = 3.0
    _compare_svgd(desc, "f32", xp, log_w, z, mask, x, L, step, bw_scale, bw_mode, trans_mode)


WAVE_CASES = [
    ("growth1d", 1, 1, 30, 0.05, "f64"),
    ("growth1d", 2, 64, 30, 0.05, "f64"),
    ("growth1d", 10, 10, 100, 0.05, "f64"),
    ("range2d", 16, 16, 50, 0.005, "f32"),
    ("scenario_b", 10, 10, 100, 1e-4, "f32"),
    ("growth1d", 20, 20, 100, 0.05, "f64"),
    ("growth1d", 64, 64, 50, 0.05, "f64"),
    ("range2d", 33, 17, 20, 0.005, "f32"),
    ("cv4d", 40, 64, 20, 0.005, "f32"),
    ("arm7", 64, 50, 20, 1e-5, "f32"),
    ("lingauss", 30, 30, 30, 0.01, "f64"),
    ("scenario_b", 20, 20, 100, 1e-4, "f32"),
    ("scenario_d", 20, 20, 100, 2e-4, "f64"),
    ("scenario_d", 30, 11, 40, 2e-4, "f32"),
]


@pytest.mark.parametrize("name,n,n_prev,L,step,dt", WAVE_CASES)
def test_svgd_step_one_wave_kernel(name, n, n_prev, L, step, dt):
    """The one-wave kernel (particles in lane registers, readlane broadcasts)
    on every family, from one particle to 64, against the oracle; the pair
    counts span every register blocking of the median's selection (1, 2, 4,
    8, 16 and 32 distances per lane)."""
    announce("svgd step wave", name, n, n_prev, L, dt)
    sk = "wave"
    wl, desc, xp, x, z, mask = _svgd_case(name, n, n_prev, 24, dt)
    _compare_svgd(desc, dt, xp, None, z, mask, x, L, step, step_kernel=sk)


@pytest.mark.parametrize("variant", ["weights", "mean_reading", "per_step_bw", "bw3", "imq", "matern32",
                                     "ties_2x5", "ties_4x4", "ties_2x10", "ties_8x8"])
@pytest.mark.parametrize("dt", ["f32", "f64"])
def test_svgd_step_one_wave_variants(variant, dt):
    """Options and exact ties on the one-wave kernel (range-only model)."""
    announce("svgd wave variant", variant, dt)
    sk = "wave"
    n, n_prev = 48, 40
    if variant.startswith("ties_"):
        groups, copies = (int(v) for v in variant[5:].split("x"))
        n = groups * copies
    wl, desc, xp, x, z, mask = _svgd_case("range2d", n, n_prev, 25, dt)
    if variant.startswith("ties_"):
        x = np.repeat(x[:groups], copies, axis=0)
    log_w, bw_scale, bw_mode, trans_mode, kernel = None, 1.0, 0, 0, 0
    if variant == "weights":
        rng = np.random.default_rng(3)
        log_w = np.log(rng.dirichlet(np.ones(n_prev)))
        if dt == "f32":
            log_w = log_w.astype(np.float32).astype(np.float64)
    if variant == "mean_reading":
        trans_mode = 1
    if variant == "per_step_bw":
        bw_mode = 1
    if variant == "bw3":
        bw_scale = 3.0
    if variant in ("imq", "matern32"):
        kernel = smsq.KERNELS[variant]
    _compare_svgd(desc, dt, xp, log_w, z, mask, x, 15, 0.005, bw_scale, bw_mode, trans_mode, kernel,
                  step_kernel=sk)


@pytest.mark.parametrize("variant", ["ties_16x16", "ties_4x64", "ties_2x10"])
@pytest.mark.parametrize("dt", ["f32", "f64"])
def test_svgd_step_ties_vector_alu(variant, dt):
    """The vector-ALU kernel's median under exact ties: copies of a few
    distinct particles put hundreds or thousands of equal distances at the
    median, so the window gathers them all or overflows (radix fallback);
    ties_2x10 (20 particles) takes the all-pairs path with 90 zero
    distances below the median's rank."""
    announce("svgd ties valu", variant, dt)
    sk = "valu"
    groups, copies = (int(v) for v in variant[5:].split("x"))
    wl, desc, xp, x, z, mask = _svgd_case("range2d", groups * copies, 50, 5, dt)
    x = np.repeat(x[:groups], copies, axis=0)
    _compare_svgd(desc, dt, xp, None, z, mask, x, 6, 0.005, step_kernel=sk)


@pytest.mark.parametrize("n,n_prev", [(1, 50), (2, 50), (20, 20), (31, 7), (32, 32)])
def test_svgd_step_small_n_matrix_core(n, n_prev):
    """Up to 32 particles single steps take the one-wave kernel (or the
    vector-ALU kernel); batched plans still run the matrix-core kernel
    there, forced here."""
    announce("svgd step small n mfma", n, n_prev)
    sk = "mfma"
    wl, desc, xp, x, z, mask = _svgd_case("range2d", n, n_prev, 23, "f32")
    _compare_svgd(desc, "f32", xp, None, z, mask, x, 40, 0.005, step_kernel=sk)


KERNEL_CASES = [
    ("growth1d", 32, 32, 100, 0.05, "f64"),
    ("growth1d", 10, 10, 100, 0.05, "f64"),
    ("growth1d", 40, 40, 100, 0.05, "f32"),
    ("range2d", 257, 200, 20, 0.005, "f32"),
    ("cv4d", 130, 64, 20, 0.005, "f64"),
    ("arm7", 200, 129, 20, 1e-5, "f32"),
]


@pytest.mark.parametrize("kernel", ["imq", "matern32"])
@pytest.mark.parametrize("name,n,n_prev,L,step,dt", KERNEL_CASES)
def test_svgd_step_kernel_ablation(kernel, name, n, n_prev, L, step, dt):
    """The IMQ and Matern-3/2 kernels of the kernel ablation (vector-ALU step
    kernel) against the oracle, at the ablation's particle counts and larger."""
    announce("svgd step kernel", kernel, name, n, n_prev, L, dt)
    wl, desc, xp, x, z, mask = _svgd_case(name, n, n_prev, 23, dt)
    k = smsq.KERNELS[kernel]
    for bw_scale in (0.5, 3.0) if name == "growth1d" else (1.0,):
        _compare_svgd(desc, dt, xp, None, z, mask, x, L, step, bw_scale=bw_scale, kernel=k)


def test_svgd_step_full_arm7_shape():
    """N = 1024, d = 7, 100 iterations: the arm workload's step at full size."""
    announce("svgd step full arm7 1024x7 L=100")
    wl, desc, xp, x, z, mask = _svgd_case("arm7", 1024, 1024, 8, "f32")
    _compare_svgd(desc, "f32", xp, None, z, mask, x, 100, 1e-5)


def test_svgd_nonfinite_observation_sets_status():
    announce("svgd nan observation")
    wl, desc, xp, x, z, mask = _svgd_case("range2d", 64, 64, 5, "f32")
    z = z.copy()
    z[0] = np.nan
    model = smsq.Model(desc)
    ws = smsq.workspace()
    smsq.svgd_step(model, "f32", 2, dev(xp, torch.float32), None, dev(z, torch.float32), None,
                   dev(x, torch.float32), smsq.opts(3, 0.005), ws=ws)
    assert smsq.device_status(ws) == smsq.ERR_NONFINITE


# ---------------------------------------------------------------------------
# Algorithm 2 end to end
# ---------------------------------------------------------------------------

def test_run_sequence_growth1d_full_f64():
    """The 1-D growth workload at full size (N=32, T=50, L=100, eps=0.05), FP64."""
    announce("run_sequence growth1d full f64")
    wl = S.make_workload("growth1d", B=1, seed=1000)
    desc = wl.model
    o = wl.opts
    res = O.run_sequence(desc, wl.T, wl.n, wl.x0[0], wl.z[0], None, 77, 0, o.n_iter, o.step)
    model = smsq.Model(desc)
    xmap, J = smsq.run_sequence(model, "f64", dev(wl.x0[0], torch.float64), dev(wl.z[0], torch.float64),
                                None, wl.n, smsq.opts_from(o), 77)
    xmap, J = host(xmap), float(host(J)[0])
    dJ = abs(J - res["J"]) / max(abs(res["J"]), wl.T)
    print("J gpu %.10f oracle %.10f rel %.3e  max|dx| %.3e" % (J, res["J"], dJ, np.abs(xmap - res["xmap"]).max()))
    assert dJ <= TOL_J
    assert np.allclose(xmap, res["xmap"], rtol=1e-6, atol=1e-6)


@pytest.mark.parametrize("kernel", ["rbf", "imq", "matern32"])
def test_run_sequence_scenario_a_f64(kernel):
    """The paper's Scenario A model (Sec. V-A constants), N = 10, T = 100,
    L = 100: Algorithm 2 against the oracle for each kernel."""
    announce("run_sequence scenario_a f64", kernel)
    wl = S.make_workload("scenario_a", B=1, seed=1005)
    desc, o, k = wl.model, wl.opts, smsq.KERNELS[kernel]
    res = O.run_sequence(desc, wl.T, wl.n, wl.x0[0], wl.z[0], None, 79, 0, o.n_iter, o.step, kernel=k)
    model = smsq.Model(desc)
    xmap, J = smsq.run_sequence(model, "f64", dev(wl.x0[0], torch.float64), dev(wl.z[0], torch.float64),
                                None, wl.n, smsq.opts(o.n_iter, o.step, kernel=k), 79)
    xmap, J = host(xmap), float(host(J)[0])
    dJ = abs(J - res["J"]) / max(abs(res["J"]), wl.T)
    print("J gpu %.10f oracle %.10f rel %.3e" % (J, res["J"], dJ))
    assert dJ <= TOL_J
    assert np.allclose(xmap, res["xmap"], rtol=1e-6, atol=1e-6)


def test_run_sequence_scenario_b_f64():
    """The Sec. V-B pose scenario at its full length: N = 20, T = 630, L = 100,
    one range-bearing measurement per step from an unknown landmark, with
    outliers in the simulated data.  Algorithm 2 against the oracle."""
    announce("run_sequence scenario_b f64")
    wl = S.make_workload("scenario_b", B=1, seed=1006)
    desc, o = wl.model, wl.opts
    res = O.run_sequence(desc, wl.T, wl.n, wl.x0[0], wl.z[0], None, 81, 0, o.n_iter, o.step)
    model = smsq.Model(desc)
    xmap, J = smsq.run_sequence(model, "f64", dev(wl.x0[0], torch.float64), dev(wl.z[0], torch.float64),
                                None, wl.n, smsq.opts_from(o), 81)
    xmap, J = host(xmap), float(host(J)[0])
    dJ = abs(J - res["J"]) / max(abs(res["J"]), wl.T)
    print("J gpu %.10f oracle %.10f rel %.3e" % (J, res["J"], dJ))
    assert dJ <= TOL_J
    assert np.allclose(xmap, res["xmap"], rtol=1e-6, atol=1e-6)


def test_run_sequence_scenario_d_f64():
    """The Sec. V-D 14-D manipulator (joint angles and velocities, end-effector
    observations): N = 20, T = 100, L = 100, Algorithm 2 against the oracle."""
    announce("run_sequence scenario_d f64")
    wl = S.make_workload("scenario_d", B=1, seed=1007)
    desc, o = wl.model, wl.opts
    res = O.run_sequence(desc, wl.T, wl.n, wl.x0[0], wl.z[0], None, 83, 0, o.n_iter, o.step)
    model = smsq.Model(desc)
    xmap, J = smsq.run_sequence(model, "f64", dev(wl.x0[0], torch.float64), dev(wl.z[0], torch.float64),
                                None, wl.n, smsq.opts_from(o), 83)
    xmap, J = host(xmap), float(host(J)[0])
    dJ = abs(J - res["J"]) / max(abs(res["J"]), wl.T)
    print("J gpu %.10f oracle %.10f rel %.3e" % (J, res["J"], dJ))
    assert dJ <= TOL_J
    assert np.allclose(xmap, res["xmap"], rtol=1e-6, atol=1e-6)


@pytest.mark.parametrize("kernel", ["imq", "matern32"])
def test_run_sequence_growth1d_kernels_f64(kernel):
    """Algorithm 2 with the ablation's kernels, 1-D growth model at N = 10."""
    announce("run_sequence growth1d f64", kernel)
    wl = S.make_workload("growth1d", B=1, seed=1003, n=10, T=30)
    desc = wl.model
    o = wl.opts
    k = smsq.KERNELS[kernel]
    res = O.run_sequence(desc, wl.T, wl.n, wl.x0[0], wl.z[0], None, 78, 0, o.n_iter, o.step, kernel=k)
    model = smsq.Model(desc)
    xmap, J = smsq.run_sequence(model, "f64", dev(wl.x0[0], torch.float64), dev(wl.z[0], torch.float64),
                                None, wl.n, smsq.opts(o.n_iter, o.step, kernel=k), 78)
    xmap, J = host(xmap), float(host(J)[0])
    dJ = abs(J - res["J"]) / max(abs(res["J"]), wl.T)
    print("J gpu %.10f oracle %.10f rel %.3e" % (J, res["J"], dJ))
    assert dJ <= TOL_J
    assert np.allclose(xmap, res["xmap"], rtol=1e-6, atol=1e-6)


@pytest.mark.parametrize("name,n,T,L,dt", [("growth1d", 32, 30, 100, "f64"), ("range2d", 64, 12, 10, "f32"),
                                           ("cv4d", 80, 8, 10, "f32")])
def test_run_sequence_map_conditioned_weights(name, n, T, L, dt):
    """Mixture weights w_j proportional to exp(phi_{t-1}(j)) (weights = 1)."""
    announce("run_sequence weights from scores", name, n, T, L, dt)
    wl = S.make_workload(name, B=1, seed=1004, T=T, n=n, n_iter=L)
    desc = wl.model
    o = wl.opts
    mask = None if wl.mask is None else wl.mask[0]
    res = O.run_sequence(desc, T, n, wl.x0[0], wl.z[0], mask, 6, 0, o.n_iter, o.step, weights=1)
    base = O.run_sequence(desc, T, n, wl.x0[0], wl.z[0], mask, 6, 0, o.n_iter, o.step)
    model = smsq.Model(desc)
    td = tdt(dt)
    xmap, J = smsq.run_sequence(model, dt, dev(wl.x0[0], td), dev(wl.z[0], td),
                                None if mask is None else dev(mask, torch.uint8), n,
                                smsq.opts(o.n_iter, o.step, weights=1), 6)
    xmap, J = host(xmap).astype(np.float64), float(host(J)[0])
    dJ = abs(J - res["J"]) / max(abs(res["J"]), T)
    print("J gpu %.8f oracle %.8f (uniform weights %.8f) rel %.3e" % (J, res["J"], base["J"], dJ))
    assert dJ <= TOL_J
    if dt == "f64":
        assert np.allclose(xmap, res["xmap"], rtol=1e-6, atol=1e-6)


@pytest.mark.parametrize("name,n,T,L", [("range2d", 64, 12, 10), ("cv4d", 80, 8, 10), ("arm7", 96, 6, 10),
                                        ("lingauss", 48, 10, 20), ("scenario_b", 20, 120, 100),
                                        ("scenario_d", 20, 40, 100)])
def test_run_sequence_f32_free_running(name, n, T, L):
    announce("run_sequence f32", name, n, T, L)
    wl = S.make_workload(name, B=1, seed=1001, T=T, n=n, n_iter=L)
    desc = wl.model
    o = wl.opts
    mask = None if wl.mask is None else wl.mask[0]
    res = O.run_sequence(desc, T, n, wl.x0[0], wl.z[0], mask, 5, 0, o.n_iter, o.step)
    model = smsq.Model(desc)
    parts = torch.zeros((T, n, desc.d), dtype=torch.float32, device=DEV)
    xmap, J = smsq.run_sequence(model, "f32", dev(wl.x0[0], torch.float32), dev(wl.z[0], torch.float32),
                                None if mask is None else dev(mask, torch.uint8), n, smsq.opts_from(o), 5,
                                particles=parts)
    xmap, J = host(xmap).astype(np.float64), float(host(J)[0])
    dJ = abs(J - res["J"]) / max(abs(res["J"]), T)
    print("J gpu %.6f oracle %.6f rel %.3e" % (J, res["J"], dJ))
    assert dJ <= TOL_J
    # J is the path score of the returned trajectory (evaluated by the oracle in FP64)
    Jpath = O.path_score(desc, xmap, wl.z[0], mask)
    assert abs(Jpath - J) <= TOL_J * max(abs(J), T)


@pytest.mark.parametrize("case", ["one_particle", "one_step", "all_masked", "one_particle_f64"])
def test_run_sequence_edge_cases(case):
    """Algorithm 2 at its edges against the oracle: a single particle per step
    (SVGD is gradient ascent, the lattice a chain), a single time step, and
    observations masked out everywhere (the estimate follows the dynamics)."""
    announce("run_sequence edge", case)
    name, n, T, L, dt = "range2d", 40, 6, 10, "f32"
    if case.startswith("one_particle"):
        n = 1
    if case == "one_particle_f64":
        name, dt, T, L = "growth1d", "f64", 12, 30
    if case == "one_step":
        T = 1
    wl = S.make_workload(name, B=1, seed=1009, T=T, n=n, n_iter=L)
    desc, o = wl.model, wl.opts
    mask = None if wl.mask is None else wl.mask[0].copy()
    if case == "all_masked":
        mask[:] = 0
    res = O.run_sequence(desc, T, n, wl.x0[0], wl.z[0], mask, 13, 0, o.n_iter, o.step)
    td = tdt(dt)
    model = smsq.Model(desc)
    xmap, J = smsq.run_sequence(model, dt, dev(wl.x0[0], td), dev(wl.z[0], td),
                                None if mask is None else dev(mask, torch.uint8), n, smsq.opts_from(o), 13)
    xmap, J = host(xmap).astype(np.float64), float(host(J)[0])
    dJ = abs(J - res["J"]) / max(abs(res["J"]), T)
    print("J gpu %.8f oracle %.8f rel %.3e" % (J, res["J"], dJ))
    assert dJ <= TOL_J
    if dt == "f64":
        assert np.allclose(xmap, res["xmap"], rtol=1e-6, atol=1e-6)
    else:   # FP32 may pick another near-tied particle: J of its own path instead
        Jpath = O.path_score(desc, xmap, wl.z[0], mask)
        assert abs(Jpath - J) <= TOL_J * max(abs(J), T)


def test_run_batch_matches_single_runs_and_is_deterministic():
    announce("run_batch determinism")
    wl = S.make_workload("range2d", B=3, seed=1002, T=10, n=48, n_iter=8)
    desc = wl.model
    model = smsq.Model(desc)
    o = smsq.opts_from(wl.opts)
    x0 = dev(wl.x0, torch.float32)
    z = dev(wl.z, torch.float32)
    mk = dev(wl.mask, torch.uint8)
    xm1, J1 = smsq.run_batch(model, "f32", x0, z, mk, wl.n, o, 9)
    xm2, J2 = smsq.run_batch(model, "f32", x0, z, mk, wl.n, o, 9)
    assert torch.equal(xm1, xm2) and torch.equal(J1, J2)
    # sequence b of a batch uses Philox counter word 2 = b; a single run uses 0
    xs, Js = smsq.run_sequence(model, "f32", x0[0].contiguous(), z[0].contiguous(), mk[0].contiguous(),
                               wl.n, o, 9)
    assert torch.equal(xs, xm1[0]) and torch.equal(Js, J1[:1])


def test_run_batch_full_arm7_sampled_step():
    """Full arm workload (N=1024, d=7, L=100, T=100) in the benchmark's launch
    configuration; the oracle recomputes a sampled step from the GPU's previous
    particles (predictive initial particles from the same Philox counters) and
    the score J along the returned path."""
    announce("run_batch full arm7 sampled step")
    wl = S.make_workload("arm7", B=2, seed=1003)
    desc = wl.model
    o = wl.opts
    model = smsq.Model(desc)
    B, T, n, d = wl.batch, wl.T, wl.n, desc.d
    parts = torch.zeros((B, T, n, d), dtype=torch.float32, device=DEV)
    xmap, J = smsq.run_batch(model, "f32", dev(wl.x0, torch.float32), dev(wl.z, torch.float32), None, n,
                             smsq.opts_from(o), 31, particles=parts)
    parts, xmap, J = host(parts).astype(np.float64), host(xmap).astype(np.float64), host(J).astype(np.float64)
    assert np.all(np.isfinite(parts))
    for b in range(B):
        Jpath = O.path_score(desc, xmap[b], wl.z[b])
        print("seq %d J %.4f path score %.4f" % (b, J[b], Jpath))
        assert abs(Jpath - J[b]) <= TOL_J * max(abs(J[b]), T)
    t = 57
    b = 1
    xprev = parts[b, t - 2]
    x_init = O.predictive_init(desc, t, xprev, n, 31, b)
    xo, _, st = O.svgd_step(desc, t, xprev, None, wl.z[b, t - 1], None, x_init, o.n_iter, o.step)
    rel = np.linalg.norm(parts[b, t - 1] - xo) / np.linalg.norm(xo)
    print("sampled step t=%d rel X err %.3e" % (t, rel))
    assert rel <= TOL_X["f32"]
    print(check_move(parts[b, t - 1], xo, x_init, o.n_iter, "f32"))


# ---------------------------------------------------------------------------
# Argument errors (no device work is enqueued)
# ---------------------------------------------------------------------------

def test_argument_errors():
    announce("argument errors")
    desc = S._model_for("range2d", 0)
    model = smsq.Model(desc)
    x = torch.zeros((4, 2), device=DEV)
    z = torch.zeros(3, device=DEV)
    with pytest.raises(smsq.SmsqError) as e:
        smsq.svgd_step(model, "f32", 1, torch.zeros((1, 2), device=DEV), None, z, None, x,
                       smsq.opts(-1, 0.1))
    assert e.value.status == smsq.ERR_INVALID
    with pytest.raises(smsq.SmsqError) as e:
        smsq.svgd_step(model, "f32", 1, torch.zeros((1, 2), device=DEV), None, z, None, x,
                       smsq.opts(2, 0.1), ws=torch.zeros(16, dtype=torch.uint8, device=DEV))
    assert e.value.status == smsq.ERR_WORKSPACE
    big = model.max_particles("f32") + 1
    with pytest.raises(smsq.SmsqError) as e:
        smsq.svgd_step(model, "f32", 1, torch.zeros((1, 2), device=DEV), None, z, None,
                       torch.zeros((big, 2), device=DEV), smsq.opts(2, 0.1))
    assert e.value.status == smsq.ERR_UNSUPPORTED
    bad = desc.copy()
    bad.d = 3
    with pytest.raises(smsq.SmsqError):
        smsq.Model(bad)
    for field, value in ((5, 0.0), (5, 9.0), (5, 2.5), (3, 0.0), (4, -1.0), (6, float("nan"))):
        pose = S.se2_model()          # landmark count 1..8, positive variances, finite constants
        pose.params[field] = value
        with pytest.raises(smsq.SmsqError) as e:
            smsq.Model(pose)
        assert e.value.status == smsq.ERR_INVALID
    for field, value in (("d", 7), ("d", 17), ("obs_dim", 2)):
        arm = S._model_for("scenario_d", 0)   # d = 14 exactly; at most 16 anywhere
        setattr(arm, field, value)
        with pytest.raises(smsq.SmsqError):
            smsq.Model(arm)
    arm = S._model_for("scenario_d", 0)
    arm.params[24] = float("inf")
    with pytest.raises(smsq.SmsqError):
        smsq.Model(arm)
    # particle-mode forward recursion: the n_prev means table must fit LDS
    # (FP64 at d = 14: 17 slots of 8 bytes per previous particle)
    arm = smsq.Model(S._model_for("scenario_d", 0))
    with pytest.raises(smsq.SmsqError) as e:
        smsq.viterbi_step(arm, "f64", 2, torch.zeros(1300, dtype=torch.float64, device=DEV),
                          x_prev=torch.zeros((1300, 14), dtype=torch.float64, device=DEV),
                          z_t=torch.zeros(3, dtype=torch.float64, device=DEV),
                          x=torch.zeros((8, 14), dtype=torch.float64, device=DEV))
    assert e.value.status == smsq.ERR_UNSUPPORTED
    with pytest.raises(smsq.SmsqError) as e:   # no such kernel
        smsq.svgd_step(model, "f32", 1, torch.zeros((1, 2), device=DEV), None, z, None, x,
                       smsq.opts(2, 0.1, kernel=3))
    assert e.value.status == smsq.ERR_INVALID
