"""Bounds of the SVGD parity checks shared by the GPU tests.

Besides the position-relative error ||X_gpu - X_ora||_F / ||X_ora||_F, a
teacher-forced step is judged on the move: ||X_gpu - X_ora||_F against the
oracle's displacement ||X_ora - X_init||_F.  In FP32 the positions carry a
rounding floor of about 2^-24 ||X|| per operation, which a random walk over
L iterations grows to sqrt(L) 2^-24 ||X||; where the particles move little
against their distance from the origin (the clutter model's large cloud) that
floor, not the kernel, sets the displacement-relative error, so the FP32
bound is 1e-3 of the displacement plus ten times that floor.  A dropped
iteration moves every particle by about 1/L of its displacement, far above
either term.  Per particle (those moving at least a tenth of the RMS move)
the bound catches errors confined to a few particles (a wrong tile or split
of the sources), which are of the order of the particle's own move: 0.1 of
it in FP32 (rounding, amplified by sharp likelihoods over the iterations,
reaches a few 1e-2 there), 1e-8 in FP64."""
import numpy as np

TOL_DISP = {"f32": 1e-3, "f64": 1e-9}
TOL_DISP_PARTICLE = {"f32": 1e-1, "f64": 1e-8}
EPS_F32 = 2.0 ** -24


def move_errors(xg, xo, x0):
    """(error over the displacement, worst per-particle ratio over the
    moving particles, absolute error, displacement norm)."""
    dg = np.linalg.norm(xg - xo, axis=1)
    dm = np.linalg.norm(xo - x0, axis=1)
    err, disp = np.linalg.norm(dg), np.linalg.norm(dm)
    rms = np.sqrt(np.mean(dm ** 2))
    moving = dm >= 0.1 * rms
    pp = float((dg[moving] / dm[moving]).max()) if rms > 0 and moving.any() else 0.0
    return err / max(disp, 1e-300), pp, err, disp


def check_move(xg, xo, x0, L, dt):
    """Asserts the move bounds; returns the printed summary."""
    rel_disp, pp, err, disp = move_errors(xg, xo, x0)
    floor = 10.0 * np.sqrt(max(L, 1)) * EPS_F32 * np.linalg.norm(xo) if dt == "f32" else 0.0
    msg = ("rel displacement err %.3e (FP32 rounding floor %.3e of the displacement), worst moving particle %.3e"
           % (rel_disp, floor / max(disp, 1e-300), pp))
    if L:
        assert err <= TOL_DISP[dt] * disp + floor, msg
        assert pp <= TOL_DISP_PARTICLE[dt], msg
    return msg
