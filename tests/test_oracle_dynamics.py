"""Pins of the oracle's time step (Eq. (latbolt)) against structure the paper
fixes: the BGK form, the streaming direction, mass and momentum
conservation (Appendix A), the divergence form of the body force, the
reduction of D3Q19 to D2Q9 for a one-site-thick system (end of Section
"Extension to 3D"), lattice symmetry and the viscosity of Eq. (viscous)."""
import numpy as np
import pytest

import oracle
from oracle import thermo
from paper_0710_5470_amd import inputs

A, B_ = 9.0 / 49.0, 2.0 / 21.0
T56, K25 = 0.56, 0.025


def _drop_state(q, scheme, shape, tau=1.0, noise=0.0, seed=5, **kw):
    g, l, _ = thermo.coexistence(A, B_, T56)
    rho0 = inputs.tanh_drop(shape, min(shape[:2]) / 4.0, l, g, 2.0)
    if noise:
        rho0 = rho0 + inputs.uniform_noise(shape, noise, seed)
    p = oracle.params(q=q, scheme=scheme, shape=shape, T=T56, kappa=K25, tau=tau, **kw)
    return p, oracle.init(p, rho0)


def _stream(p, fstar):
    """f(r + e_i) = f*(r) with periodic wrap, by index rolling."""
    e = oracle.tables(p)["e"]
    out = np.empty_like(fstar)
    for i in range(p.q):
        a = fstar[i].reshape(p.nz, p.ny, p.nx)
        a = np.roll(a, shift=(e[i][2], e[i][1], e[i][0]), axis=(0, 1, 2))
        out[i] = a.reshape(-1)
    return out


def _null_perturbation(p, rng, eps):
    """Per-site vectors orthogonal to 1, e_x, e_y (, e_z): they change no
    mass or momentum, hence neither f_eq nor F."""
    e = oracle.tables(p)["e"].astype(float)
    dim = 2 if p.q == 9 else 3
    Mt = np.vstack([np.ones(p.q)] + [e[:, a] for a in range(dim)])  # (1+dim) x q
    proj = np.eye(p.q) - Mt.T @ np.linalg.solve(Mt @ Mt.T, Mt)
    h = rng.normal(0, eps, (p.q, p.nx * p.ny * p.nz))
    return proj @ h


@pytest.mark.parametrize("q", [9, 19])
@pytest.mark.parametrize("scheme", [0, 1])
def test_bgk_relaxation_structure(q, scheme):
    """A perturbation that leaves rho and j unchanged is relaxed by exactly
    (1 - 1/tau) and streamed; at tau = 1 it disappears in one step."""
    shape = (12, 10) if q == 9 else (8, 7, 6)
    rng = np.random.default_rng(7)
    for tau in (1.0, 0.8, 1.3):
        p, f = _drop_state(q, scheme, shape, tau=tau, noise=0.01)
        d = _null_perturbation(p, rng, 1e-3)
        out0 = oracle.run(p, f, 1)
        out1 = oracle.run(p, f + d, 1)
        want = _stream(p, (1.0 - 1.0 / tau) * d)
        assert np.max(np.abs((out1 - out0) - want)) < 1e-14


@pytest.mark.parametrize("q", [9, 19])
def test_streaming_direction_moves_mass_with_momentum(q):
    """Population i travels from r to r + e_i, so the first moment of the
    mass grows by the total momentum in one step (ideal gas a = b = 0,
    kappa = 0, a moving blob in a gas at rest)."""
    shape = (24, 20) if q == 9 else (20, 18, 16)
    nx, ny = shape[0], shape[1]
    nz = shape[2] if q == 19 else 1
    blob = inputs.tanh_drop(shape, 3.0, 1.0, 0.0, 1.0)
    blob = np.where(blob > 1e-3, blob, 0.0)  # compact: the boundary rows stay at rest
    rho0 = 1.0 + 0.3 * blob
    u0 = np.zeros((3,) + rho0.shape)
    u0[0] = 0.02 * blob
    u0[1] = -0.01 * blob
    p = oracle.params(q=q, scheme=0, shape=shape, a=0.0, b=0.0, T=1.0 / 3.0, kappa=0.0)
    f = oracle.init(p, rho0, u0)
    f1 = oracle.run(p, f, 1)
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    x, y = x.reshape(-1), y.reshape(-1)
    r0, v0 = oracle.observe(p, f)
    r1, _ = oracle.observe(p, f1)
    jx, jy = (r0 * v0[0]).sum(), (r0 * v0[1]).sum()
    assert (x * r1).sum() - (x * r0).sum() == pytest.approx(jx, rel=1e-10)
    assert (y * r1).sum() - (y * r0).sum() == pytest.approx(jy, rel=1e-10)
    assert jx > 0 and jy < 0


@pytest.mark.parametrize("q", [9, 19])
@pytest.mark.parametrize("scheme", [0, 1])
def test_mass_and_momentum_conservation(q, scheme):
    shape = (32, 28) if q == 9 else (14, 12, 10)
    p, f = _drop_state(q, scheme, shape, tau=0.9, noise=0.02)
    m0, P0 = oracle.totals(p, f)
    f = oracle.run(p, f, 300)
    m1, P1 = oracle.totals(p, f)
    assert abs(m1 - m0) / m0 < 1e-12
    assert np.max(np.abs(P1 - P0)) / m0 < 1e-14


@pytest.mark.parametrize("q", [9, 19])
def test_body_force_sums_to_zero_and_matches_continuum(q):
    """g = -div(M - I tr M / 2) sums to zero over a periodic lattice and,
    for a smooth field, agrees with the analytic divergence to O(k^2)."""
    N = 64 if q == 9 else 32
    shape = (N, N) if q == 9 else (N, N, N)
    nz = N if q == 19 else 1
    kappa = 0.03
    p = oracle.params(q=q, scheme=1, shape=shape, kappa=kappa)
    z, y, x = np.meshgrid(np.arange(nz), np.arange(N), np.arange(N), indexing="ij")
    k = 2 * np.pi / N
    amp = 0.4
    if q == 9:
        rho = 3.0 + amp * np.sin(k * x) * np.cos(k * y)
        d = [amp * k * np.cos(k * x) * np.cos(k * y), -amp * k * np.sin(k * x) * np.sin(k * y),
             0 * x]
    else:
        rho = 3.0 + amp * np.sin(k * x) * np.cos(k * y) * np.cos(k * z)
        d = [amp * k * np.cos(k * x) * np.cos(k * y) * np.cos(k * z),
             -amp * k * np.sin(k * x) * np.sin(k * y) * np.cos(k * z),
             -amp * k * np.sin(k * x) * np.cos(k * y) * np.sin(k * z)]
    g = oracle.body_force(p, rho)
    scale = np.abs(g).max()
    assert np.abs(g.sum(axis=1)).max() < 1e-13 * scale * g.shape[1]
    # analytic: -d_b (kappa d_a rho d_b rho - delta_ab kappa |grad rho|^2 / 2)
    #         = -kappa (lap rho) d_a rho   (the identity d_b(d_a d_b) - d_a|d|^2/2)
    dim = 2 if q == 9 else 3
    lap = -dim * k * k * (rho - 3.0) if q == 19 else -2 * k * k * (rho - 3.0)
    for a in range(dim):
        want = (-kappa * lap * d[a]).reshape(-1)
        err = np.abs(g[a] - want).max() / np.abs(want).max()
        assert err < 3 * (k * k), (a, err)


@pytest.mark.parametrize("scheme", [0, 1])
def test_d3q19_one_site_thick_equals_d2q9(scheme):
    """With no z extent the D3Q19 populations summed over e_z evolve as the
    D2Q9 ones (lambda terms off: the D3Q19 lambda term keeps an X_zz part)."""
    shape2, shape3 = (24, 20), (24, 20, 1)
    g, l, _ = thermo.coexistence(A, B_, T56)
    rho0 = inputs.tanh_drop(shape2, 6.0, l, g, 2.0) + inputs.uniform_noise(shape2, 0.01, 3)
    p2 = oracle.params(q=9, scheme=scheme, shape=shape2, T=T56, kappa=K25, tau=0.9, lambda_on=0)
    p3 = oracle.params(q=19, scheme=scheme, shape=shape3, T=T56, kappa=K25, tau=0.9, lambda_on=0)
    f2 = oracle.run(p2, oracle.init(p2, rho0), 60)
    f3 = oracle.run(p3, oracle.init(p3, rho0), 60)
    e2, e3 = oracle.tables(p2)["e"], oracle.tables(p3)["e"]
    agg = np.zeros_like(f2)
    for i in range(19):
        k = [m for m in range(9) if e2[m][0] == e3[i][0] and e2[m][1] == e3[i][1]][0]
        agg[k] += f3[i]
    assert np.max(np.abs(agg - f2)) < 1e-12
    r2, v2 = oracle.observe(p2, f2)
    r3, v3 = oracle.observe(p3, f3)
    assert np.max(np.abs(r2 - r3)) < 1e-12 and np.max(np.abs(v2[:2] - v3[:2])) < 1e-13


@pytest.mark.parametrize("q", [9, 19])
@pytest.mark.parametrize("scheme", [0, 1])
def test_site_local_collision_matches_field_step(q, scheme):
    shape = (10, 9) if q == 9 else (7, 6, 5)
    p, f = _drop_state(q, scheme, shape, tau=0.85, noise=0.03)
    f1 = oracle.run(p, f, 1)
    e = oracle.tables(p)["e"]
    xyz = np.array([(x, y, z) for z in range(p.nz) for y in range(p.ny) for x in range(p.nx)])
    fs = oracle.collide_sites(p, f, xyz)
    for k, (x, y, z) in enumerate(xyz):
        for i in range(p.q):
            d = (((z + e[i][2]) % p.nz) * p.ny + (y + e[i][1]) % p.ny) * p.nx + (x + e[i][0]) % p.nx
            assert fs[k, i] == pytest.approx(f1[i, d], abs=1e-14)


@pytest.mark.parametrize("scheme", [0, 1])
def test_centred_drop_keeps_square_symmetry(scheme):
    N = 32
    p, f = _drop_state(9, scheme, (N, N), tau=1.0)
    f = oracle.run(p, f, 200)
    rho, v = oracle.observe(p, f)
    rho, vx, vy = rho.reshape(N, N), v[0].reshape(N, N), v[1].reshape(N, N)
    refl = lambda a: np.roll(a[:, ::-1], 1, axis=1)  # x -> -x about the centre
    assert np.max(np.abs(rho - refl(rho))) < 1e-12
    assert np.max(np.abs(vx + refl(vx))) < 1e-15 + 1e-8 * np.abs(vx).max()
    assert np.max(np.abs(rho - rho.T)) < 1e-12
    assert np.max(np.abs(vx - vy.T)) < 1e-15 + 1e-8 * np.abs(vx).max()


@pytest.mark.parametrize("q,tau", [(9, 0.8), (9, 1.2), (19, 0.9)])
def test_shear_wave_decays_with_paper_viscosity(q, tau):
    """Uniform density, kappa irrelevant: u_x = U sin(k y) decays as
    exp(-nu k^2 t) with nu = (tau - 1/2)/3 (Eq. (viscous), dx = dt = 1)."""
    N = 96 if q == 9 else 48
    shape = (4, N) if q == 9 else (2, N, 2)
    nz = 2 if q == 19 else 1
    rho_l = 4.5
    rho0 = np.full((nz, N, shape[0]) if q == 19 else (N, shape[0]), rho_l)
    k = 2 * np.pi / N
    y = np.arange(N)
    u0 = np.zeros((3,) + rho0.shape)
    prof = 1e-4 * np.sin(k * y)
    if q == 9:
        u0[0] = prof[:, None]
    else:
        u0[0] = prof[None, :, None]
    p = oracle.params(q=q, scheme=0, shape=shape, T=T56, kappa=K25, tau=tau)
    f = oracle.run(p, oracle.init(p, rho0, u0), 100)
    amp = lambda f: np.abs(oracle.observe(p, f)[1][0]).max()
    a0 = amp(f)
    f = oracle.run(p, f, 400)
    a1 = amp(f)
    nu_meas = -np.log(a1 / a0) / (400 * k * k)
    assert nu_meas == pytest.approx((tau - 0.5) / 3.0, rel=0.01)
