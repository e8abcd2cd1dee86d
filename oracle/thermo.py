"""TEST INFRASTRUCTURE ONLY: continuum thermodynamics of the van der Waals fluid.

Used by the oracle's tests to compute the coexistence densities, the flat
interface tension and the Laplace pressure jump the lattice model should
reproduce.  Written independently of the GPU library's host solver.

Bulk pressure: Eq. (p0), p0 = rho T / (1 - b rho) - a rho^2.
Free-energy density consistent with it (p0 = rho psi' - psi):
    psi(rho) = rho T ln(rho / (1 - b rho)) - a rho^2,
chemical potential mu = psi'(rho) = T ln(rho/(1-b rho)) + T/(1-b rho) - 2 a rho.
Square-gradient term (kappa/2)|grad rho|^2 gives the kappa terms of Eq. (pt).
"""
import math

from scipy import integrate, optimize


def p0(a, b, T, rho):
    return rho * T / (1.0 - b * rho) - a * rho * rho


def psi(a, b, T, rho):
    return rho * T * math.log(rho / (1.0 - b * rho)) - a * rho * rho


def mu(a, b, T, rho):
    return T * math.log(rho / (1.0 - b * rho)) + T / (1.0 - b * rho) - 2.0 * a * rho


def critical_point(a, b):
    """T_c = 8a/(27b), rho_c = 1/(3b) (inflection of p0 with zero slope)."""
    return 8.0 * a / (27.0 * b), 1.0 / (3.0 * b)


def _spinodals(a, b, T):
    """Densities where dp0/drho = 0 (below T_c), found by bracketing."""
    _, rc = critical_point(a, b)
    dp = lambda r: T / (1.0 - b * r) ** 2 - 2.0 * a * r
    lo = optimize.brentq(dp, 1e-9, rc)
    hi = optimize.brentq(dp, rc, (1.0 - 1e-12) / b)
    return lo, hi


def coexistence(a, b, T):
    """Maxwell construction: equal pressure and equal chemical potential.

    For a trial pressure P between the spinodal pressures, take the outermost
    roots of p0(rho) = P on the gas and liquid branches; adjust P until the
    chemical potentials match.  Returns (rho_gas, rho_liquid, P).  The
    pressure bracket starts at 1e-14, so temperatures whose coexistence
    pressure is below that (T <= 0.05 for a = 9/49, b = 2/21) are not
    handled."""
    s_lo, s_hi = _spinodals(a, b, T)
    p_min, p_max = p0(a, b, T, s_hi), p0(a, b, T, s_lo)
    p_lo = max(p_min, 1e-14)

    def roots(P):
        g = optimize.brentq(lambda r: p0(a, b, T, r) - P, P / (10.0 * T), s_lo, xtol=1e-15)
        l = optimize.brentq(lambda r: p0(a, b, T, r) - P, s_hi, (1.0 - 1e-13) / b, xtol=1e-15)
        return g, l

    def dmu(P):
        g, l = roots(P)
        return mu(a, b, T, l) - mu(a, b, T, g)

    eps = 1e-12 * (p_max - p_lo)
    P = optimize.brentq(dmu, p_lo + eps, p_max - eps, xtol=1e-15, rtol=1e-15)
    g, l = roots(P)
    return g, l, P


def grand_potential_excess(a, b, T, rho, mu_c, p_c):
    """Omega(rho) = psi - mu_c rho + p_c, zero in both coexisting bulks."""
    return psi(a, b, T, rho) - mu_c * rho + p_c


def surface_tension(a, b, T, kappa):
    """Flat-interface tension sigma = integral of sqrt(2 kappa Omega) d rho
    between the coexisting densities (first integral of the equilibrium
    profile of the square-gradient free energy)."""
    g, l, P = coexistence(a, b, T)
    mu_c = mu(a, b, T, g)

    def integrand(r):
        om = grand_potential_excess(a, b, T, r, mu_c, P)
        return math.sqrt(max(2.0 * kappa * om, 0.0))

    val, _ = integrate.quad(integrand, g, l, limit=200, epsabs=1e-13, epsrel=1e-12)
    return val


def interface_width(a, b, T, kappa):
    """(rho_l - rho_g) / max |d rho / dx| of the continuum flat profile."""
    g, l, P = coexistence(a, b, T)
    mu_c = mu(a, b, T, g)
    res = optimize.minimize_scalar(
        lambda r: -grand_potential_excess(a, b, T, r, mu_c, P), bounds=(g, l),
        method="bounded")
    om_max = -res.fun
    return (l - g) / math.sqrt(2.0 * om_max / kappa)
