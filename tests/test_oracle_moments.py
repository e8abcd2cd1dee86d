"""Moment identities of the oracle's equilibrium and forcing term (Appendix A).

For random site inputs the equilibrium must satisfy
  sum f_eq = rho, sum f_eq e_a = rho u_a                         (Eq. (ncons))
  sum f_eq e_a e_b = P_ab + rho u_a u_b + lambda(u_a d_b rho + u_b d_a rho
                     + delta_ab u.grad rho)                        (Eq. (pcons))
  sum f_eq e_a e_b e_c = (rho/3)(d_ab u_c + d_ac u_b + d_bc u_a)   (Eq. (focons))
with P_ab from Eq. (pt) built from the discrete gradient and Laplacian, and
the forcing term must satisfy the three forcing moment conditions.
In the forcing scheme the kappa d_a rho d_b rho part of P_ab moves into the
body force, so the equilibrium's second moment lacks it.
"""
import itertools

import numpy as np
import pytest

import oracle

A, B_ = 9.0 / 49.0, 2.0 / 21.0


def p0_eq_p0(rho, T):
    """Eq. (p0), typed from the paper."""
    return rho * T / (1.0 - B_ * rho) - A * rho * rho


def cs2_numeric(rho, T, h=1e-5):
    """c_s^2 = dp0/drho by a fourth-order central difference."""
    f = lambda r: p0_eq_p0(r, T)
    return (-f(rho + 2 * h) + 8 * f(rho + h) - 8 * f(rho - h) + f(rho - 2 * h)) / (12 * h)


@pytest.mark.parametrize("q", [9, 19])
@pytest.mark.parametrize("scheme", [0, 1])
@pytest.mark.parametrize("lambda_on", [1, 0])
def test_equilibrium_moments(q, scheme, lambda_on):
    rng = np.random.default_rng(1234 + q + 10 * scheme + 100 * lambda_on)
    dim = 2 if q == 9 else 3
    T, kappa, tau = 0.53, 0.023, 0.83
    shape = (4, 4) if q == 9 else (4, 4, 4)
    p = oracle.params(q=q, scheme=scheme, shape=shape, T=T, kappa=kappa, tau=tau,
                      lambda_on=lambda_on)
    e = oracle.tables(p)["e"].astype(float)
    for _ in range(20):
        rho = rng.uniform(1.2, 6.5)
        j = np.zeros(3)
        j[:dim] = rng.normal(0, 0.05, dim)
        d = np.zeros(3)
        d[:dim] = rng.normal(0, 0.7, dim)
        lap = rng.normal(0, 0.8)
        feq = oracle.feq_site(p, rho, j, d, lap)
        u = j / rho
        assert feq.sum() == pytest.approx(rho, rel=1e-14)
        for a in range(dim):
            assert np.dot(feq, e[:, a]) == pytest.approx(j[a], abs=1e-14)
        pb = p0_eq_p0(rho, T)
        nu = (tau - 0.5) / 3.0
        lam = nu * (1.0 - 3.0 * cs2_numeric(rho, T)) if lambda_on else 0.0
        udg = np.dot(u[:dim], d[:dim])
        for a, b in itertools.product(range(dim), repeat=2):
            dab = 1.0 if a == b else 0.0
            P = (pb - kappa * rho * lap) * dab
            if scheme == 0:
                P += -0.5 * kappa * np.dot(d[:dim], d[:dim]) * dab + kappa * d[a] * d[b]
            want = P + rho * u[a] * u[b] + lam * (u[a] * d[b] + u[b] * d[a] + dab * udg)
            got = np.dot(feq, e[:, a] * e[:, b])
            assert got == pytest.approx(want, abs=1e-9), (a, b)
        for a, b, c in itertools.product(range(dim), repeat=3):
            d_ = np.eye(3)
            want = (rho / 3.0) * (d_[a, b] * u[c] + d_[a, c] * u[b] + d_[b, c] * u[a])
            assert np.dot(feq, e[:, a] * e[:, b] * e[:, c]) == pytest.approx(want, abs=1e-14)


@pytest.mark.parametrize("q", [9, 19])
def test_forcing_moments(q):
    rng = np.random.default_rng(99 + q)
    dim = 2 if q == 9 else 3
    p = oracle.params(q=q, scheme=1, shape=(4, 4) if q == 9 else (4, 4, 4))
    e = oracle.tables(p)["e"].astype(float)
    for _ in range(20):
        u = np.zeros(3)
        g = np.zeros(3)
        u[:dim] = rng.normal(0, 0.05, dim)
        g[:dim] = rng.normal(0, 1e-3, dim)
        F = oracle.force_site(p, u, g)
        assert abs(F.sum()) < 1e-18
        for a in range(dim):
            assert np.dot(F, e[:, a]) == pytest.approx(g[a], abs=1e-18)
        for a, b in itertools.product(range(dim), repeat=2):
            want = u[a] * g[b] + u[b] * g[a]
            assert np.dot(F, e[:, a] * e[:, b]) == pytest.approx(want, abs=1e-18)


def test_rest_forcing_closed_form():
    """F_0 = -sum_{i>=1} F_i equals -(4/3) u.g in 2D and -u.g in 3D."""
    u, g = np.array([0.01, -0.02, 0.03]), np.array([1e-3, 2e-3, -5e-4])
    F2 = oracle.force_site(oracle.params(q=9, shape=(4, 4)), u, g)
    assert F2[0] == pytest.approx(-(4.0 / 3.0) * np.dot(u[:2], g[:2]), rel=1e-13)
    F3 = oracle.force_site(oracle.params(q=19, shape=(4, 4, 4)), u, g)
    assert F3[0] == pytest.approx(-np.dot(u, g), rel=1e-13)
