"""Exact-arithmetic pins of the oracle's whole time step.

The step is evaluated in exact rational arithmetic (Python ``fractions``) on
tiny periodic lattices, straight from the paper's definitions:

- moments, Eq. (rho);
- the printed 2D stencils of Eq. (best) as 3x3 matrices, and the 3D stencils
  as sums over the D3Q19 velocities with A = 1/6, B = 1/12, C = 1/3,
  D = 1/6 and the centre E = -6C - 12D (Eq. (laplacian3d));
- the van der Waals pressure, Eq. (p0), c_s^2 = dp0/drho and the lambda of
  Eq. (viscous);
- the equilibrium of Eq. (equilibrium) written as its tensor sums, with the
  optimum weights of the summary (2D) and of Eq. (3dres) (3D, with the two
  readings w_1-6 = 1/6 and axial w^aa = 5/12), and Eq. (feq0);
- for the forcing scheme the 2D body force exactly as printed in section
  "Using a forcing method" (g_x from the E/F stencils of (M_xx - M_yy)/2 and
  M_xy, g_y by exchanging the labels), and in 3D the divergence of the kappa
  part of the pressure tensor, Eq. (pt);
- the BGK collision and streaming of Eq. (latbolt).

The exact state after a few steps then pins the FP64 oracle to round-off
(brute force on tiny inputs).  Its totals pin ``oracle.totals``; a boosted
fluid, whose total momentum is fixed by the input alone, pins the sign and
the component order of the momentum.
"""
from fractions import Fraction as Fr

import numpy as np
import pytest

import oracle

A_F, B_F, T_F = 9.0 / 49.0, 2.0 / 21.0, 0.56


class Exact:
    """One periodic lattice in exact rational arithmetic."""

    def __init__(self, q, shape, scheme, tau, kappa, golden):
        self.q, self.scheme = q, scheme
        self.dim = 2 if q == 9 else 3
        self.nx, self.ny = shape[0], shape[1]
        self.nz = shape[2] if len(shape) > 2 else 1
        self.a, self.b, self.T = Fr(9, 49), Fr(2, 21), Fr(14, 25)
        self.kappa, self.tau = Fr(kappa).limit_denominator(1000), Fr(tau).limit_denominator(1000)
        key = "d2q9_velocities" if q == 9 else "d3q19_velocities"
        self.e = [tuple(v) + (0,) * (3 - len(v)) for v in golden[key]["e"]]
        self._weights()

    # -- weights ---------------------------------------------------------------
    def _weights(self):
        q, e = self.q, self.e
        self.w, self.wp, self.wt = [Fr(0)] * q, [Fr(0)] * q, [Fr(0)] * q
        # wm[(a, b)][i]: weight of kappa d_a rho d_b rho (a <= b)
        self.wm = {}
        for a in range(3):
            for b in range(a, 3):
                self.wm[(a, b)] = [Fr(0)] * q
        for i in range(1, q):
            ax = sum(1 for c in e[i] if c) == 1
            if self.q == 9:
                # summary: w = w^p = w^t = 1/3 (axis), 1/12 (diagonal);
                # w^xx_1-2 = w^yy_3-4 = 1/3, w^xx_3-4 = w^yy_1-2 = -1/6,
                # w^xx_5-8 = w^yy_5-8 = -1/24, w^xy = e_x e_y / 4
                self.w[i] = self.wp[i] = self.wt[i] = Fr(1, 3) if ax else Fr(1, 12)
                for a in range(2):
                    if ax:
                        self.wm[(a, a)][i] = Fr(1, 3) if e[i][a] else Fr(-1, 6)
                    else:
                        self.wm[(a, a)][i] = Fr(-1, 24)
                self.wm[(0, 1)][i] = Fr(e[i][0] * e[i][1], 4)
            else:
                # Eq. (3dres) with w_1-6 = 1/6 and axial w^aa = 5/12
                self.w[i] = self.wp[i] = self.wt[i] = Fr(1, 6) if ax else Fr(1, 12)
                for a in range(3):
                    if ax:
                        self.wm[(a, a)][i] = Fr(5, 12) if e[i][a] else Fr(-1, 3)
                    else:
                        self.wm[(a, a)][i] = Fr(-1, 24) if e[i][a] else Fr(1, 12)
                for a, b in ((0, 1), (1, 2), (0, 2)):
                    self.wm[(a, b)][i] = Fr(e[i][a] * e[i][b], 4)

    # -- lattice ---------------------------------------------------------------
    def idx(self, x, y, z=0):
        return ((z % self.nz) * self.ny + (y % self.ny)) * self.nx + (x % self.nx)

    def sites(self):
        for z in range(self.nz):
            for y in range(self.ny):
                for x in range(self.nx):
                    yield x, y, z

    # -- stencils --------------------------------------------------------------
    def grad(self, fld, x, y, z):
        if self.dim == 2:
            # Eq. (best): (1/12) [[-1 0 1], [-4 0 4], [-1 0 1]], rows y = +1, 0, -1
            K = [[-1, 0, 1], [-4, 0, 4], [-1, 0, 1]]
            gx = sum(Fr(K[r][c], 12) * fld[self.idx(x + c - 1, y + 1 - r)]
                     for r in range(3) for c in range(3))
            # the y stencil is the transpose: row y = +1 is (1 4 1) / 12
            gy = sum(Fr(K[c][2 - r], 12) * fld[self.idx(x + c - 1, y + 1 - r)]
                     for r in range(3) for c in range(3))
            return [gx, gy, Fr(0)]
        out = [Fr(0)] * 3
        for i in range(1, self.q):
            ei = self.e[i]
            k = Fr(1, 6) if sum(map(abs, ei)) == 1 else Fr(1, 12)
            v = fld[self.idx(x + ei[0], y + ei[1], z + ei[2])]
            for a in range(3):
                out[a] += k * ei[a] * v
        return out

    def lap(self, fld, x, y, z):
        if self.dim == 2:
            # Eq. (best): (1/6) [[1 4 1], [4 -20 4], [1 4 1]]
            K = [[1, 4, 1], [4, -20, 4], [1, 4, 1]]
            return sum(Fr(K[r][c], 6) * fld[self.idx(x + c - 1, y + 1 - r)]
                       for r in range(3) for c in range(3))
        C, D = Fr(1, 3), Fr(1, 6)
        acc = (-6 * C - 12 * D) * fld[self.idx(x, y, z)]
        for i in range(1, self.q):
            ei = self.e[i]
            acc += (C if sum(map(abs, ei)) == 1 else D) * fld[self.idx(x + ei[0], y + ei[1], z + ei[2])]
        return acc

    # -- thermodynamics --------------------------------------------------------
    def p0(self, r):
        return r * self.T / (1 - self.b * r) - self.a * r * r

    def cs2(self, r):
        return self.T / (1 - self.b * r) ** 2 - 2 * self.a * r

    # -- one site --------------------------------------------------------------
    def feq(self, rho, j, d, lap, with_m):
        dim = self.dim
        u = [j[a] / rho for a in range(3)]
        lam = (self.tau - Fr(1, 2)) / 3 * (1 - 3 * self.cs2(rho))
        ud = sum(u[g] * d[g] for g in range(dim))
        X = [[rho * u[al] * u[be] + lam * (u[al] * d[be] + u[be] * d[al] + (ud if al == be else 0))
              for be in range(3)] for al in range(3)]
        p0 = self.p0(rho)
        out = [Fr(0)] * self.q
        for i in range(1, self.q):
            ei = self.e[i]
            v = sum(ei[al] * j[al] for al in range(dim))
            v += Fr(3, 2) * sum((ei[al] * ei[be] - (Fr(1, 3) if al == be else 0)) * X[al][be]
                                for al in range(dim) for be in range(dim))
            v = self.w[i] * v + self.wp[i] * p0 - self.wt[i] * self.kappa * rho * lap
            if with_m:
                for (a, b), wab in self.wm.items():
                    if a < dim and b < dim:
                        v += wab[i] * self.kappa * d[a] * d[b]
            out[i] = v
        out[0] = rho - sum(out[1:])
        return out

    def forcing(self, u, g):
        dim = self.dim
        F = [Fr(0)] * self.q
        for i in range(1, self.q):
            ei = self.e[i]
            v = sum(ei[al] * g[al] for al in range(dim))
            v += Fr(3, 2) * sum((ei[al] * ei[be] - (Fr(1, 3) if al == be else 0))
                                * (u[al] * g[be] + u[be] * g[al])
                                for al in range(dim) for be in range(dim))
            F[i] = self.w[i] * v
        F[0] = -sum(F[1:])
        return F

    def body_force(self, d):
        """g at every site from the gradient field d[s] = (dx, dy, dz)."""
        n = self.nx * self.ny * self.nz
        M = {(a, b): [self.kappa * d[s][a] * d[s][b] for s in range(n)]
             for a in range(3) for b in range(3)}
        g = []
        if self.dim == 2:
            # section "Using a forcing method", E = 1/3 and F = 1/12:
            # g_x = -[E/F x-stencil] (M_xx - M_yy)/2 - [E/F y-stencil] M_xy
            E, F = Fr(1, 3), Fr(1, 12)
            SX = [[-F, 0, F], [-E, 0, E], [-F, 0, F]]   # rows y = +1, 0, -1
            SY = [[F, E, F], [0, 0, 0], [-F, -E, -F]]
            half = [(M[(0, 0)][s] - M[(1, 1)][s]) / 2 for s in range(n)]
            mhalf = [-h for h in half]

            def app(S, fld, x, y):
                return sum(S[r][c] * fld[self.idx(x + c - 1, y + 1 - r)]
                           for r in range(3) for c in range(3))
            for x, y, z in self.sites():
                gx = -app(SX, half, x, y) - app(SY, M[(0, 1)], x, y)
                # exchange x and y: the derivative stencils swap, and
                # (M_yy - M_xx)/2 replaces (M_xx - M_yy)/2
                gy = -app(SY, mhalf, x, y) - app(SX, M[(0, 1)], x, y)
                g.append([gx, gy, Fr(0)])
            return g
        # 3D: g_a = -d_b (M_ab - delta_ab M_cc / 2), gradient stencil A, B
        tr = [M[(0, 0)][s] + M[(1, 1)][s] + M[(2, 2)][s] for s in range(n)]
        Tab = {(a, b): [M[(a, b)][s] - (tr[s] / 2 if a == b else 0) for s in range(n)]
               for a in range(3) for b in range(3)}
        for x, y, z in self.sites():
            ga = [Fr(0)] * 3
            for a in range(3):
                for b in range(3):
                    ga[a] -= self.grad(Tab[(a, b)], x, y, z)[b]
            g.append(ga)
        return g

    # -- whole lattice ---------------------------------------------------------
    def moments(self, f):
        n = self.nx * self.ny * self.nz
        rho = [sum(f[i][s] for i in range(self.q)) for s in range(n)]
        j = [[sum(f[i][s] * self.e[i][a] for i in range(self.q)) for a in range(3)]
             for s in range(n)]
        return rho, j

    def init(self, rho0, u0):
        n = len(rho0)
        f = [[None] * n for _ in range(self.q)]
        for x, y, z in self.sites():
            s = self.idx(x, y, z)
            d = self.grad(rho0, x, y, z)
            lp = self.lap(rho0, x, y, z)
            j = [rho0[s] * u0[a][s] for a in range(3)]
            fe = self.feq(rho0[s], j, d, lp, self.scheme == 0)
            for i in range(self.q):
                f[i][s] = fe[i]
        return f

    def step(self, f):
        n = len(f[0])
        rho, j = self.moments(f)
        grads = [None] * n
        laps = [None] * n
        for x, y, z in self.sites():
            s = self.idx(x, y, z)
            grads[s] = self.grad(rho, x, y, z)
            laps[s] = self.lap(rho, x, y, z)
        g = self.body_force(grads) if self.scheme == 1 else None
        out = [[None] * n for _ in range(self.q)]
        for x, y, z in self.sites():
            s = self.idx(x, y, z)
            fe = self.feq(rho[s], j[s], grads[s], laps[s], self.scheme == 0)
            F = self.forcing([j[s][a] / rho[s] for a in range(3)], g[s]) if g else [0] * self.q
            for i in range(self.q):
                ei = self.e[i]
                out[i][self.idx(x + ei[0], y + ei[1], z + ei[2])] = (
                    f[i][s] - (f[i][s] - fe[i]) / self.tau + F[i])
        return out


def _inputs(shape, seed):
    """Random densities k/8 in [2.625, 4.25] and velocities k/512 in
    [-1/64, 1/64]: exact in both number systems, and with small denominators
    so that the exact fractions stay tractable for a few steps."""
    rng = np.random.default_rng(seed)
    n = int(np.prod(shape))
    rho0 = [Fr(int(k), 8) for k in rng.integers(21, 35, n)]
    dim = len(shape)
    u0 = [[Fr(int(k), 512) for k in rng.integers(-8, 9, n)] if a < dim else [Fr(0)] * n
          for a in range(3)]
    return rho0, u0


def _to_np(f):
    return np.array([[float(v) for v in row] for row in f])


# (exact denominators grow about 30-fold in bits per step: three D2Q9 steps
# take about a second, a third D3Q19 step about a minute, so D3Q19 runs two)
CASES = [(9, 0, (5, 4), 3), (9, 1, (5, 4), 3), (19, 0, (3, 4, 3), 2), (19, 1, (3, 4, 3), 2)]


@pytest.mark.parametrize("q,scheme,shape,steps", CASES)
def test_oracle_step_equals_exact_arithmetic(q, scheme, shape, steps, golden):
    """The FP64 oracle equals the exact rational evaluation of the paper's
    step (random densities and velocities, non-unit tau) to round-off after
    every step, for both lattices and both schemes."""
    tau, kappa = 0.8, 0.025
    ex = Exact(q, shape, scheme, tau, kappa, golden)
    rho0, u0 = _inputs(shape, 31 + q + scheme)
    fe = ex.init(rho0, u0)
    p = oracle.params(q=q, scheme=scheme, shape=shape, a=A_F, b=B_F, T=T_F, kappa=kappa, tau=tau)
    fo = oracle.init(p, np.array([float(v) for v in rho0]),
                     np.array([[float(v) for v in row] for row in u0]))
    scale = np.max(np.abs(_to_np(fe)))
    assert np.max(np.abs(fo - _to_np(fe))) / scale < 1e-15
    for _ in range(steps):
        fe = ex.step(fe)
        fo = oracle.run(p, fo, 1)
        err = np.max(np.abs(fo - _to_np(fe))) / scale
        assert err < 1e-13, err
    # totals of the exact state pin oracle.totals (mass, momentum components)
    rho, j = ex.moments(fe)
    m_ex = float(sum(rho))
    P_ex = np.array([float(sum(js[a] for js in j)) for a in range(3)])
    m_o, P_o = oracle.totals(p, fo)
    assert abs(m_o - m_ex) / m_ex < 1e-14
    assert np.max(np.abs(P_o - P_ex)) / m_ex < 1e-14


@pytest.mark.parametrize("q,scheme,shape", [(9, 0, (12, 10)), (9, 1, (12, 10)),
                                            (19, 0, (8, 7, 6)), (19, 1, (8, 7, 6))])
def test_totals_of_a_boosted_and_a_moving_blob(q, scheme, shape):
    """Momentum of known sign and components: a uniform boost U of a
    non-uniform density has total momentum U * sum(rho0), and a blob moving
    with velocity V inside a fluid at rest has sum over the blob of rho0 V
    (the moment identity sum_i f_i^eq e_i = rho u of Appendix A, Eq. (pcons)'s
    first-order companion).  Both schemes conserve it exactly under the
    step (Appendix A; the forcing moments sum to zero net force)."""
    n = int(np.prod(shape))
    rng = np.random.default_rng(5)
    rho0 = rng.uniform(2.6, 4.4, n)
    dim = 2 if q == 9 else 3
    U = np.array([0.013, -0.007, 0.004])[:dim]
    p = oracle.params(q=q, scheme=scheme, shape=shape, a=A_F, b=B_F, T=T_F, kappa=0.025, tau=0.9)
    u0 = np.zeros((3, n))
    u0[:dim] = U[:, None]
    m, P = oracle.totals(p, oracle.init(p, rho0, u0))
    assert abs(m - rho0.sum()) / m < 1e-14
    assert np.max(np.abs(P[:dim] - U * rho0.sum())) < 1e-13 * m
    if dim == 2:
        assert P[2] == 0.0
    # a blob: the first quarter of the sites moves with V, the rest is at rest
    V = np.array([-0.011, 0.017, -0.005])[:dim]
    u0 = np.zeros((3, n))
    blob = np.arange(n) < n // 4
    u0[:dim, blob] = V[:, None]
    f = oracle.init(p, rho0, u0)
    m, P = oracle.totals(p, f)
    want = V * rho0[blob].sum()
    assert np.max(np.abs(P[:dim] - want)) < 1e-13 * m
    # the step keeps both totals (FP64 round-off)
    m1, P1 = oracle.totals(p, oracle.run(p, f, 20))
    assert abs(m1 - m) / m < 1e-13
    assert np.max(np.abs(P1[:dim] - want)) < 1e-12 * m
    # mass equals the sum of the observed density field
    rho, vel = oracle.observe(p, f)
    assert abs(rho.sum() - m) / m < 1e-14
