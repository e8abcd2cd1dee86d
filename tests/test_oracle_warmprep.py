"""Pins of the numpy reference of the warm start's data preparation
(oracle/warmprep.py): the symmetrisation against a brute-force average over
the eight symmetry matrices, and the projection against its defining
properties (mass, momentum, clamping, non-finite fallback)."""
import numpy as np

from oracle import warmprep

MATS = [np.array(m) for m in ([[1, 0], [0, 1]], [[-1, 0], [0, 1]], [[1, 0], [0, -1]], [[-1, 0], [0, -1]],
                              [[0, 1], [1, 0]], [[0, -1], [1, 0]], [[0, 1], [-1, 0]], [[0, -1], [-1, 0]])]


def _brute(rho, u):
    n, ny, nx = rho.shape
    c = np.array([nx // 2, ny // 2])
    r = np.zeros_like(rho)
    v = np.zeros_like(u)
    for k in range(n):
        for y in range(ny):
            for x in range(nx):
                p = np.array([x, y]) - c
                for M in MATS:
                    qx, qy = (c + M @ p) % np.array([nx, ny])
                    r[k, y, x] += rho[k, qy, qx] / 8
                    v[k, :, y, x] += M.T @ u[k, :, qy, qx] / 8
    return r, v


def test_symmetrize_equals_group_average():
    rng = np.random.default_rng(0)
    for side in (6, 7):
        rho = rng.normal(size=(2, side, side))
        u = rng.normal(size=(2, 2, side, side))
        r, v = warmprep.d4_symmetrize(rho, u)
        rb, vb = _brute(rho, u)
        assert np.allclose(r, rb, atol=1e-14) and np.allclose(v, vb, atol=1e-14)


def test_symmetrized_field_is_invariant():
    rng = np.random.default_rng(1)
    rho = rng.normal(size=(1, 8, 8))
    u = rng.normal(size=(1, 2, 8, 8))
    r, v = warmprep.d4_symmetrize(rho, u)
    r2, v2 = warmprep.d4_symmetrize(r, v)
    assert np.allclose(r2, r, atol=1e-15) and np.allclose(v2, v, atol=1e-15)
    # a radially symmetric field and a (periodic) radial vector field pass
    # unchanged
    y, x = np.mgrid[0:8, 0:8] - 4
    rad = np.exp(-(x ** 2 + y ** 2) / 5.0)[None]
    vec = np.stack([np.sin(np.pi * x / 4) * rad[0], np.sin(np.pi * y / 4) * rad[0]])[None]
    r3, v3 = warmprep.d4_symmetrize(rad, vec)
    assert np.allclose(r3, rad, atol=1e-15) and np.allclose(v3, vec, atol=1e-15)


def test_projection_keeps_mass_and_removes_momentum():
    rng = np.random.default_rng(2)
    rho0 = 2.5 + rng.random((3, 9, 9))
    pred = rng.normal(size=(3, 9, 9, 16))
    for sym in (False, True):
        rho, u = warmprep.project(pred, rho0, 0.2, 1e-3, True, sym, 1e-3, 10.0)
        assert np.allclose(rho.sum(axis=(1, 2)), rho0.sum(axis=(1, 2)), rtol=1e-14)
        mom = (rho[:, None] * u).sum(axis=(2, 3))
        assert np.abs(mom).max() < 1e-15 * rho.sum()
    rho, u = warmprep.project(pred, rho0, 0.2, 1e-3, False, True, 1e-3, 10.0)
    assert np.all(u == 0.0)


def test_projection_clamps_and_falls_back_on_nonfinite():
    rho0 = np.full((2, 4, 4), 3.0)
    pred = np.zeros((2, 4, 4, 16))
    pred[0, 0, 0, 0] = 100.0          # rho = 23 before the clamp
    pred[1, 1, 2, 1] = np.nan
    rho, u = warmprep.project(pred, rho0, 0.2, 1e-3, True, False, 1e-3, 10.0)
    assert rho[0].max() == 10.0
    assert np.array_equal(rho[1], rho0[1]) and np.all(u[1] == 0.0)


def test_features_and_targets_layout():
    rho0 = np.arange(2 * 3 * 3, dtype=float).reshape(2, 3, 3)
    x = warmprep.features([[1, 2, 3, 4, 5], [6, 7, 8, 9, 10]], rho0, 1.0, 2.0)
    assert x.shape == (2, 3, 3, 16) and x[1, 2, 1, 4] == 10 and x[1, 2, 1, 5] == (rho0[1, 2, 1] - 1) / 2
    assert np.all(x[..., 6:] == 0)
    vel = np.ones((2, 2, 3, 3))
    y = warmprep.targets(rho0 + 0.4, rho0, vel, 0.2, 0.5)
    assert np.allclose(y[..., 0], 2.0) and np.allclose(y[..., 1:3], 2.0) and np.all(y[..., 3:] == 0)
