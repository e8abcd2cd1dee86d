"""Pins of the oracle's lattice tables and stencils against the paper.

Velocity sets and printed weights come from tests/golden/paper_values.json.
Moment conditions come from Appendix A (Eqs. (ncons), (pcons), (focons)) with
the pressure tensor of Eq. (pt); Taylor identities of the stencils come from
Eqs. (xderiv), (laplace) and (laplacian3d).
"""
import itertools

import numpy as np
import pytest

import oracle


def _p(q, **kw):
    shape = (7, 5) if q == 9 else (7, 5, 3)
    return oracle.params(q=q, shape=shape, **kw)


@pytest.mark.parametrize("q,key", [(9, "d2q9_velocities"), (19, "d3q19_velocities")])
def test_velocity_sets_as_printed(golden, q, key):
    e = oracle.tables(_p(q))["e"]
    want = np.array(golden[key]["e"])
    assert np.array_equal(e[:, :want.shape[1]], want)
    if q == 9:
        assert np.all(e[:, 2] == 0)


def _dim(q):
    return 2 if q == 9 else 3


def _mom2(wts, e, dim):
    return np.array([[np.sum(wts * e[:, a] * e[:, b]) for b in range(dim)] for a in range(dim)])


@pytest.mark.parametrize("q", [9, 19])
def test_velocity_weight_moments(q):
    """sum w e_a e_b = delta (first moment of f_eq is rho u) and the fourth
    moment is isotropic, (1/3)(d_ab d_cd + d_ac d_bd + d_ad d_bc), which makes
    the second moment of the velocity terms equal rho u u + lambda(...)."""
    t = oracle.tables(_p(q))
    e, w, dim = t["e"].astype(float), t["w"], _dim(q)
    assert np.allclose(_mom2(w, e, dim), np.eye(dim), atol=1e-15)
    d = np.eye(dim)
    for a, b, c, dd in itertools.product(range(dim), repeat=4):
        m4 = np.sum(w * e[:, a] * e[:, b] * e[:, c] * e[:, dd])
        want = (d[a, b] * d[c, dd] + d[a, c] * d[b, dd] + d[a, dd] * d[b, c]) / 3.0
        assert m4 == pytest.approx(want, abs=1e-15)
    # odd moments vanish: weights are symmetric under e -> -e
    for i in range(1, q):
        j = [k for k in range(q) if np.array_equal(e[k], -e[i])][0]
        for name in ("w", "wp", "wt"):
            assert t[name][i] == t[name][j]
        assert np.all(t["wm"][:, i] == t["wm"][:, j])


@pytest.mark.parametrize("q", [9, 19])
def test_pressure_weight_moments(q):
    """Second moments of the pressure-tensor weights reproduce Eq. (pt):
    p0 and kappa rho lap rho are isotropic; M_aa enters P_bb with +1/2 if
    a == b and -1/2 otherwise; M_ab (a != b) enters P_ab with 1."""
    t = oracle.tables(_p(q))
    e, dim = t["e"].astype(float), _dim(q)
    assert np.allclose(_mom2(t["wp"], e, dim), np.eye(dim), atol=1e-15)
    assert np.allclose(_mom2(t["wt"], e, dim), np.eye(dim), atol=1e-15)
    pairs = [(0, 0), (1, 1), (2, 2), (0, 1), (1, 2), (2, 0)]
    for m, (a, b) in enumerate(pairs):
        if a >= dim or b >= dim:
            assert np.all(t["wm"][m] == 0.0)
            continue
        want = np.zeros((dim, dim))
        if a == b:
            want[:] = 0.0
            for c in range(dim):
                want[c, c] = 0.5 if c == a else -0.5
        else:
            want[a, b] = want[b, a] = 1.0
        got = _mom2(t["wm"][m], e, dim)
        # M_ab with a != b appears once in Eq. (equilibrium); the tensor entry
        # P_ab = P_ba = M_ab is produced by the symmetric second moment
        assert np.allclose(got, want, atol=1e-15), (m, got)


def test_optimum_2d_weights_as_printed(golden):
    g = golden["optimum_2d_weights"]
    t = oracle.tables(_p(9))
    w, wp, wt, wm = t["w"], t["wp"], t["wt"], t["wm"]
    for i in range(1, 5):
        assert w[i] == pytest.approx(g["w_1_4"]) and wp[i] == pytest.approx(g["wp_1_4"])
        assert wt[i] == pytest.approx(g["wt_1_4"]) and wm[3, i] == g["wxy_1_4"]
    for i in range(5, 9):
        assert w[i] == pytest.approx(g["w_5_8"]) and wp[i] == pytest.approx(g["wp_5_8"])
        assert wt[i] == pytest.approx(g["wt_5_8"])
        assert wm[0, i] == pytest.approx(g["wxx_5_8"]) and wm[1, i] == pytest.approx(g["wyy_5_8"])
    assert wm[3, 5] == wm[3, 6] == g["wxy_5_6"] and wm[3, 7] == wm[3, 8] == g["wxy_7_8"]
    assert wm[0, 1] == pytest.approx(g["wxx_1_2"]) and wm[1, 3] == pytest.approx(g["wyy_3_4"])
    assert wm[0, 3] == pytest.approx(g["wxx_3_4"]) and wm[1, 1] == pytest.approx(g["wyy_1_2"])


def test_3d_weights_as_printed_except_readings(golden):
    """Every entry of Eq. (3dres) is used as printed except w_1-6 and the
    axial w^aa, whose printed 1/3 fails the moment conditions above."""
    g, rd = golden["d3q19_weights_as_printed"], golden["readings"]
    t = oracle.tables(_p(19))
    w, wm = t["w"], t["wm"]
    assert np.allclose(w[7:19], g["w_7_18"])
    assert np.allclose(w[1:7], rd["d3q19_w_1_6"]) and g["w_1_6"] != rd["d3q19_w_1_6"]
    assert np.allclose(wm[0, 1:3], rd["d3q19_wxx_axial"])
    assert np.allclose(wm[1, 3:5], rd["d3q19_wxx_axial"])
    assert np.allclose(wm[2, 5:7], rd["d3q19_wxx_axial"])
    assert np.allclose(wm[0, 3:7], g["wxx_3_6"])
    assert np.allclose(wm[0, 7:11], g["wxx_7_10"]) and np.allclose(wm[0, 15:19], g["wxx_15_18"])
    assert np.allclose(wm[0, 11:15], g["wxx_11_14"])
    assert wm[3, 7] == wm[3, 10] == g["wxy_7_10"] and wm[3, 8] == wm[3, 9] == g["wxy_8_9"]
    # the printed values really do fail the conditions: with w_1-6 = 1/3 the
    # xx second moment would be 2/3 + 8/12 = 4/3, and with w^xx_1,2 = 1/3 the
    # M_xx moment would be 1/3 instead of 1/2
    assert 2 * g["w_1_6"] + 8 * g["w_7_18"] == pytest.approx(4.0 / 3.0)
    assert 2 * g["wxx_12_axial"] + 8 * g["wxx_7_10"] == pytest.approx(1.0 / 3.0)
    # the printed stencil coefficients are the lattice weights (A = w_face)
    s = oracle.stencils(_p(19))
    assert s["gx"][1, 1, 2] == pytest.approx(g["A"]) and s["gx"][1, 0, 2] == pytest.approx(g["B"])
    assert s["lap"][1, 1, 2] == pytest.approx(g["C"]) and s["lap"][1, 0, 2] == pytest.approx(g["D"])


def test_best_2d_stencils_as_printed(golden):
    g = golden["best_stencils_2d"]
    s = oracle.stencils(_p(9))
    assert np.allclose(12 * s["gx"][1], g["dx_times_12"], atol=1e-14)
    assert np.allclose(6 * s["lap"][1], g["lap_times_6"], atol=1e-14)
    # the y derivative is the x stencil with x and y interchanged
    assert np.allclose(12 * s["gy"][1], np.array(g["dx_times_12"]).T[::-1, ::-1], atol=1e-14)
    # the optimum force stencil (F = 1/12) is the same as the gradient
    assert np.allclose(s["fx"], s["gx"]) and np.allclose(s["fy"], s["gy"])


def _poly_field(shape, fn):
    nx, ny = shape[0], shape[1]
    nz = shape[2] if len(shape) > 2 else 1
    cx, cy, cz = nx // 2, ny // 2, nz // 2
    z, y, x = np.meshgrid(np.arange(nz) - cz, np.arange(ny) - cy, np.arange(nx) - cx,
                          indexing="ij")
    return fn(x.astype(float), y.astype(float), z.astype(float)), (cz * ny + cy) * nx + cx


@pytest.mark.parametrize("q", [9, 19])
@pytest.mark.parametrize("B,D", [(1 / 12, 1 / 6), (0.0, 0.25), (0.05, 0.1)])
def test_stencil_taylor_identities(q, B, D):
    """Exact results of the stencils on polynomials at the centre site:
    d_x(x) = 1, d_x(x^3) = 1 (the (1/6) dx^2 d_x^3 term), d_x(x y^2) = 4B
    (the 2B dx^2 d_y^2 d_x term), lap(x^2) = 2, lap(x^4) = 2 (the dx^2/12
    d_x^4 term), lap(x^2 y^2) = 4D (the D dx^2 d_x^2 d_y^2 term)."""
    shape = (9, 9) if q == 9 else (9, 9, 9)
    p = oracle.params(q=q, shape=shape, B=B, D=D)
    cases = [
        (lambda x, y, z: x, 0, 1.0), (lambda x, y, z: x ** 3, 0, 1.0),
        (lambda x, y, z: x * y * y, 0, 4 * B), (lambda x, y, z: y, 1, 1.0),
        (lambda x, y, z: y ** 3, 1, 1.0), (lambda x, y, z: y * x * x, 1, 4 * B),
        (lambda x, y, z: x * x + 0 * y, 0, 0.0), (lambda x, y, z: 1.0 + 0 * x, 1, 0.0),
    ]
    if q == 19:
        cases += [(lambda x, y, z: z, 2, 1.0), (lambda x, y, z: z ** 3, 2, 1.0),
                  (lambda x, y, z: x * z * z, 0, 4 * B), (lambda x, y, z: z * y * y, 2, 4 * B)]
    for fn, comp, want in cases:
        fld, c = _poly_field(shape, fn)
        grad, lap = oracle.derivatives(p, fld)
        assert grad[comp, c] == pytest.approx(want, abs=1e-13)
    lcases = [(lambda x, y, z: x * x, 2.0), (lambda x, y, z: y * y, 2.0),
              (lambda x, y, z: x ** 4, 2.0), (lambda x, y, z: x * x * y * y, 4 * D),
              (lambda x, y, z: 3.0 + x + y + 0 * z, 0.0)]
    if q == 19:
        lcases += [(lambda x, y, z: z * z, 2.0), (lambda x, y, z: z ** 4, 2.0),
                   (lambda x, y, z: x * x * z * z, 4 * D), (lambda x, y, z: y * y * z * z, 4 * D)]
    for fn, want in lcases:
        fld, c = _poly_field(shape, fn)
        _, lap = oracle.derivatives(p, fld)
        assert lap[c] == pytest.approx(want, abs=1e-12)


def test_simple_stencil_is_B0():
    """Eq. (simple): the central difference (rho(r+e1) - rho(r+e2)) / 2."""
    s = oracle.stencils(_p(9, B=0.0))
    want = np.array([[0, 0, 0], [-0.5, 0, 0.5], [0, 0, 0]])
    assert np.array_equal(s["gx"][1], want)
