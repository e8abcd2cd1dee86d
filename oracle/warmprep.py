"""TEST INFRASTRUCTURE ONLY: numpy reference of the warm start's data
preparation (network features and targets, and the projection of a
prediction onto an admissible initial field).

Fields are [n, Y, X] (x fastest), velocities [n, 2, Y, X]; the drop of every
problem is centred on the node (Y/2, X/2).
"""
import numpy as np


def features(consts, rho0, rho_mean, rho_scale):
    """consts [n, 5], rho0 [n, Y, X] -> [n, Y, X, 16] (float32 values)."""
    n, ny, nx = rho0.shape
    x = np.zeros((n, ny, nx, 16))
    x[..., :5] = np.asarray(consts, dtype=np.float64)[:, None, None, :]
    x[..., 5] = (rho0 - rho_mean) / rho_scale
    return x.astype(np.float32)


def targets(rho, rho0, vel, s_rho, s_u):
    """rho, rho0 [n, Y, X], vel [n, 2, Y, X] -> [n, Y, X, 16]."""
    y = np.zeros(rho.shape + (16,))
    y[..., 0] = (rho - rho0) / s_rho
    y[..., 1] = vel[:, 0] / s_u
    y[..., 2] = vel[:, 1] / s_u
    return y.astype(np.float32)


def d4_symmetrize(rho, u):
    """Average over the eight symmetries of the square about the centre
    node: reflections x -> -x, y -> -y and the transposition x <-> y (and
    their products), a scalar as rho(g p), a vector as M_g^T u(g p)."""
    ny, nx = rho.shape[-2:]
    assert nx == ny, "square lattices only"
    mirror = (2 * (nx // 2) - np.arange(nx)) % nx          # x -> 2c - x (periodic)
    fx = lambda a: np.take(a, mirror, axis=-1)            # a(-X, Y)
    fy = lambda a: np.take(a, mirror, axis=-2)            # a(X, -Y)
    tr = lambda a: np.swapaxes(a, -1, -2)                  # a(Y, X)
    ux, uy = u[:, 0], u[:, 1]
    imgs = [(rho, ux, uy), (fx(rho), -fx(ux), fx(uy)), (fy(rho), fy(ux), -fy(uy)),
            (fx(fy(rho)), -fx(fy(ux)), -fx(fy(uy)))]
    imgs += [(tr(r), tr(b), tr(a)) for r, a, b in imgs]
    r = sum(i[0] for i in imgs) / 8.0
    vx = sum(i[1] for i in imgs) / 8.0
    vy = sum(i[2] for i in imgs) / 8.0
    return r, np.stack([vx, vy], axis=1)


def project(pred, rho0, s_rho, s_u, with_velocity, symmetrize, rho_lo, rho_hi):
    """pred [n, Y, X, c] -> (rho [n, Y, X], u [n, 2, Y, X]): decode,
    symmetrize, restore the cold start's mass by a uniform shift, clamp,
    remove the mass-weighted mean velocity.  Problems with a non-finite
    prediction get (rho0, 0)."""
    pred = np.asarray(pred, dtype=np.float64)
    rho = rho0 + s_rho * pred[..., 0]
    u = np.zeros((rho.shape[0], 2) + rho.shape[1:])
    if with_velocity:
        u[:, 0] = s_u * pred[..., 1]
        u[:, 1] = s_u * pred[..., 2]
    bad = ~(np.isfinite(rho).all(axis=(1, 2)) & np.isfinite(u).all(axis=(1, 2, 3)))
    if symmetrize:
        rho, u = d4_symmetrize(rho, u)
    npt = rho.shape[1] * rho.shape[2]
    rho = rho + ((rho0.sum(axis=(1, 2)) - rho.sum(axis=(1, 2))) / npt)[:, None, None]
    rho = np.clip(rho, rho_lo, rho_hi)
    rho[bad] = rho0[bad]
    u[bad] = 0.0
    m = rho.sum(axis=(1, 2))
    for a in range(2):
        u[:, a] -= ((rho * u[:, a]).sum(axis=(1, 2)) / m)[:, None, None]
    return rho, u
