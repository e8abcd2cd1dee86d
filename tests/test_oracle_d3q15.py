"""D3Q15 against D3Q19: section "Extension to 3D" states that 19 lattice
vectors are necessary for the reduction in spurious velocities, without the
3D analysis or any D3Q15 tables.  The oracle builds D3Q15 as the paper
builds D3Q19: weights with the second moments of Appendix A and, where a
choice remains, an isotropic leading error (the scalar terms on faces 1/3,
corners 1/24; stencil corner coefficients B = 1/24, D = 1/12); the w^xx
corner weight c and the w^p, w^t corner weights stay free.

Pinned here: the tables meet the moment identities for every choice of the
free weights; the stencils are exact to the orders the paper's Taylor
expansions require, with an isotropic leading error at the stated B, D.
Measured (the comparison): with the isotropic choice the tuned equilibrium
is linearly unstable at the paper's 3D kappa = 0.02 (stable at 0.005); it is
stable when w^t sits on the corners; and the best stable D3Q15 choice found
leaves a steady drop's spurious velocity several times above D3Q19's.
"""
import itertools

import numpy as np
import pytest

import oracle as O

A, B_ = 9.0 / 49.0, 2.0 / 21.0


def _p0(rho, T):
    return rho * T / (1.0 - B_ * rho) - A * rho * rho


def _cs2(rho, T, h=1e-5):
    f = lambda r: _p0(r, T)
    return (-f(rho + 2 * h) + 8 * f(rho + h) - 8 * f(rho - h) + f(rho - 2 * h)) / (12 * h)


@pytest.mark.parametrize("over", [{}, dict(wt_d=1 / 8, wp_d=1 / 8, wxx_d=-1 / 32, B=1 / 12),
                                  dict(wt_d=0.01, wp_d=0.07, wxx_d=0.05, D=0.1)])
@pytest.mark.parametrize("lambda_on", [1, 0])
def test_d3q15_equilibrium_moments(over, lambda_on):
    """Eqs. (ncons), (pcons), (focons) for any choice of the free weights."""
    rng = np.random.default_rng(77)
    T, kappa, tau = 0.53, 0.023, 0.83
    p = O.params(q=15, shape=(4, 4, 4), T=T, kappa=kappa, tau=tau, lambda_on=lambda_on, **over)
    e = O.tables(p)["e"].astype(float)
    assert len(e) == 15
    for _ in range(20):
        rho = rng.uniform(1.2, 6.5)
        j, d = rng.normal(0, 0.05, 3), rng.normal(0, 0.7, 3)
        lap = rng.normal(0, 0.8)
        feq = O.feq_site(p, rho, j, d, lap)
        u = j / rho
        assert feq.sum() == pytest.approx(rho, rel=1e-14)
        np.testing.assert_allclose(feq @ e, j, atol=1e-14)
        lam = (tau - 0.5) / 3.0 * (1.0 - 3.0 * _cs2(rho, T)) if lambda_on else 0.0
        for a, b in itertools.product(range(3), repeat=2):
            dab = float(a == b)
            P = (_p0(rho, T) - kappa * rho * lap - 0.5 * kappa * d @ d) * dab + kappa * d[a] * d[b]
            want = P + rho * u[a] * u[b] + lam * (u[a] * d[b] + u[b] * d[a] + dab * u @ d)
            assert feq @ (e[:, a] * e[:, b]) == pytest.approx(want, abs=1e-9)
        for a, b, c in itertools.product(range(3), repeat=3):
            I = np.eye(3)
            want = rho / 3.0 * (I[a, b] * u[c] + I[a, c] * u[b] + I[b, c] * u[a])
            assert feq @ (e[:, a] * e[:, b] * e[:, c]) == pytest.approx(want, abs=1e-14)


def _apply(st, fn):
    """sum over the 3x3x3 stencil (paper layout) of coefficient * fn(dx, dy, dz)"""
    acc = 0.0
    for sl, r, c in itertools.product(range(3), repeat=3):
        if st[sl, r, c] != 0.0:
            acc += st[sl, r, c] * fn(c - 1, 1 - r, 1 - sl)
    return acc


def test_d3q15_stencils_reach_faces_and_corners_with_isotropic_leading_error():
    p = O.params(q=15, shape=(4, 4, 4))
    st = O.stencils(p)
    for name in ("gx", "lap"):
        for sl, r, c in itertools.product(range(3), repeat=3):
            nnz = (c != 1) + (r != 1) + (sl != 1)
            if nnz == 2:
                assert st[name][sl, r, c] == 0.0  # no edges on D3Q15
    # gradient: exact on linear fields; its cubic error is (1/6) lambda d_x lap
    # with the same coefficient for x^3 and for x y^2 (isotropy)
    assert _apply(st["gx"], lambda x, y, z: x) == pytest.approx(1.0, abs=1e-15)
    assert _apply(st["gx"], lambda x, y, z: y) == pytest.approx(0.0, abs=1e-15)
    e3 = _apply(st["gx"], lambda x, y, z: x ** 3)
    exy = _apply(st["gx"], lambda x, y, z: x * y * y)
    assert e3 == pytest.approx(3 * exy, abs=1e-15)
    # Laplacian: zero on constants, exact on quadratics; isotropic
    # fourth-order error
    assert _apply(st["gx"], lambda x, y, z: 1.0) == pytest.approx(0.0, abs=1e-15)
    assert _apply(st["lap"], lambda x, y, z: 1.0) == pytest.approx(0.0, abs=1e-14)
    assert _apply(st["lap"], lambda x, y, z: x * x) == pytest.approx(2.0, abs=1e-15)
    assert _apply(st["lap"], lambda x, y, z: x * y) == pytest.approx(0.0, abs=1e-15)
    x4 = _apply(st["lap"], lambda x, y, z: x ** 4)
    x2y2 = _apply(st["lap"], lambda x, y, z: x * x * y * y)
    assert x4 == pytest.approx(3 * x2y2, abs=1e-14)


def _uniform_stable(q, rho_b, kappa, **over):
    from paper_0710_5470_amd import inputs
    n = 12
    p = O.params(q=q, shape=(n, n, n), a=A, b=B_, T=0.56, kappa=kappa, tau=1.0, **over)
    f = O.run(p, O.init(p, rho_b + inputs.uniform_noise((n, n, n), 1e-6, 3)), 300)
    r = O.observe(p, f)[0]
    spread = r.max() - r.min()
    return bool(np.isfinite(spread) and spread < 1e-5)


def test_d3q15_stability_of_the_uniform_fluid():
    from oracle import thermo
    g, l, _ = thermo.coexistence(A, B_, 0.56)
    for rho_b in (g, l):
        assert _uniform_stable(19, rho_b, 0.02)
        assert not _uniform_stable(15, rho_b, 0.02)         # isotropic weights
        assert _uniform_stable(15, rho_b, 0.005)
        assert _uniform_stable(15, rho_b, 0.02, wt_d=1 / 8)  # w^t on the corners


@pytest.mark.slow
def test_d3q15_best_choice_leaves_larger_spurious_velocities_than_d3q19():
    """A steady drop (R = 11 on 32^3, T = 0.56, kappa = 0.02, tau = 1, 1000
    steps): D3Q19 at the paper's weights against the best stable D3Q15
    choice of a scan over the free corner weights (w^t = w^p = 1/8 on the
    corners, w^xx corner c = -1/32, B = 1/12): measured 1.27e-5 against
    1.03e-4."""
    from oracle import thermo
    from paper_0710_5470_amd import inputs
    g, l, _ = thermo.coexistence(A, B_, 0.56)
    n = 32
    rho0 = inputs.tanh_drop((n, n, n), 11.0, l, g, 2.0)

    def umax(q, **over):
        p = O.params(q=q, shape=(n, n, n), a=A, b=B_, T=0.56, kappa=0.02, tau=1.0, **over)
        v = O.observe(p, O.run(p, O.init(p, rho0), 1000))[1]
        return np.sqrt((v ** 2).sum(0)).max()

    u19 = umax(19)
    u15 = umax(15, wt_d=1 / 8, wp_d=1 / 8, wxx_d=-1 / 32, B=1 / 12)
    assert np.isfinite(u15)
    assert u15 > 5 * u19
