"""Parity at the benchmark's full sizes, in the launch configuration bench.py
times (autotuned), on sampled sites the oracle computes one by one.

For each workload of bench.py the GPU runs a few steps from its initial
state; the state before the last step (FP64 export, the paper's post-stream
f_i(r, t)) goes to the oracle's site-local collision (oracle.collide_sites),
and the oracle's post-collision f*_i(r) must equal the GPU's post-stream
f_i(r + e_i, t + 1) at every sampled site and direction.  The sample holds
every combination of tile, chunk and periodic-wrap boundary coordinates of
the launch plus seeded random sites.

Tolerances (absolute, on populations of magnitude <= 1):
  FP64 storage: 1e-13 (the oracle and the GPU evaluate the same formulas in
    FP64 from the same inputs; FMA contraction and summation order differ).
  FP32 storage, FP32 arithmetic: 1e-6, derived: the pressure and the static
    part of the equilibrium are evaluated in FP64, so the FP32 intermediates
    of a population are bounded by the rest deviation and omega times the
    density deviation (|delta_0| < 2, omega rho_dev < 2.5); the rest
    population, the largest, passes through about five FP32 roundings at
    that scale (the density sum, omega rho_dev, the class sums, the fused
    keep * delta_0 and the final add, half an ulp of 2.5 each = 1.2e-7) and
    one rounding when stored: 6 x 1.2e-7 = 7.2e-7 < 1e-6.  The moving
    populations (|delta_i| ~ 1e-2) are far below that.
"""
import os
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

ROOT = os.path.join(os.path.dirname(__file__), "..")
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

CASES = [("d3q19_256_fp32_force", 1e-6), ("d3q19_256_fp64_force", 1e-13),
         ("d2q9_1024_fp64_eq", 1e-13), ("d2q9_1024_fp64_force", 1e-13),
         ("d2q9_1024_fp32_eq", 1e-6), ("d2q9_1024_fp32_force", 1e-6)]


def _sites(shape, tile, planes, seed, nrand=1500):
    nx, ny = shape[0], shape[1]
    nz = shape[2] if len(shape) > 2 else 1
    tx, ty = tile

    def edges(n, t):
        v = {0, n - 1}
        for b in range(t, n, t):
            v |= {b - 1, b}
        return sorted(v)

    if nz > 1:
        xs, ys, zs = edges(nx, tx), edges(ny, ty), edges(nz, planes)
    else:  # D2Q9: rows of tx sites, planes along y
        xs, ys, zs = edges(nx, tx), edges(ny, planes), [0]
    rng = np.random.default_rng(seed)
    pick = lambda v, k: list(rng.choice(v, size=min(k, len(v)), replace=False))
    fixed = [(x, y, z) for x in pick(xs, 6) for y in pick(ys, 6) for z in pick(zs, 4)]
    rand = np.stack([rng.integers(0, nx, nrand), rng.integers(0, ny, nrand),
                     rng.integers(0, nz, nrand)], axis=1)
    return np.concatenate([np.array(fixed), rand]).astype(np.int32)


@pytest.mark.parametrize("wl,tol", CASES)
def test_full_size_step_matches_oracle_on_sampled_sites(wl, tol):
    import bench
    import oracle
    from paper_0710_5470_amd import autotune, lbm
    print("[gpu-case] full-size sampled parity", wl, flush=True)
    q, scheme, storage, compute, shape, T, kappa, tau, R, noise = bench.WORKLOADS[wl]
    p, rho0 = bench.make_workload(wl)
    sim = lbm.Simulation(p, rho0)
    autotune.autotune(sim, use_cache=False)
    tile_i, planes, _ = sim.launch()
    tile = lbm.lbm_tile_shape(q, tile_i)
    print("[gpu-case] launch tile", tile, "planes", planes, flush=True)
    sim.step(5)
    f0 = sim.get_state().cpu().numpy()
    sim.step(1)
    f1 = sim.get_state().cpu().numpy()
    sim.close()
    op = oracle.params(q=q, scheme=scheme, shape=shape, T=T, kappa=kappa, tau=tau)
    xyz = _sites(shape, tile, planes, seed=17)
    fs = oracle.collide_sites(op, f0, xyz)
    e = oracle.tables(op)["e"]
    nx, ny = shape[0], shape[1]
    nz = shape[2] if len(shape) > 2 else 1
    worst = 0.0
    for i in range(q):
        d = (((xyz[:, 2] + e[i][2]) % nz) * ny + (xyz[:, 1] + e[i][1]) % ny) * nx + \
            (xyz[:, 0] + e[i][0]) % nx
        worst = max(worst, float(np.max(np.abs(f1[i, d] - fs[:, i]))))
    print("[gpu-case] %s: %d sites, max |f_gpu - f_oracle| = %.3e (tol %.0e), max |f| %.3f"
          % (wl, len(xyz), worst, tol, float(np.abs(f1).max())), flush=True)
    assert np.isfinite(f1).all()
    assert worst < tol


EPS32 = 2.0 ** -24  # FP32 unit roundoff


def test_benchmark_workload_keeps_its_invariants_over_5000_steps():
    """The benchmarked workload (D3Q19 256^3, FP32 storage and arithmetic,
    forcing scheme, tau = 0.8) for 5000 steps in the autotuned launch: the
    state stays finite, the spurious velocity stays small, and the mass and
    momentum totals (reduced in FP64 from the stored deviations) move by no
    more than FP32 rounding allows.  In exact arithmetic the collision keeps
    each site's mass and, for the forcing scheme, the total momentum (the
    body force of Appendix A sums to zero over a periodic lattice), and the
    drop starts at rest, so the initial momentum is zero.  Bound, as in the
    reduction tests: every step rounds each stored deviation once and the
    collision adds a few roundings of the same size, so a total can move by
    at most 4 * steps * EPS32 * sum_r sum_i |delta_i| (taken at the start and
    at the end, whichever is larger)."""
    import bench
    from paper_0710_5470_amd import autotune, lbm
    wl = "d3q19_256_fp32_force"
    print("[gpu-case] 5000-step invariants", wl, flush=True)
    p, rho0 = bench.make_workload(wl)
    sim = lbm.Simulation(p, rho0)
    autotune.autotune(sim, use_cache=False)
    print("[gpu-case] launch", sim.launch(), flush=True)
    shift = torch.tensor(sim.shift(), dtype=torch.float64, device="cuda")

    def abs_dev():
        f = sim.get_state()
        return float((f - shift[:, None]).abs().sum())

    m0, j0 = sim.invariants()
    d0 = abs_dev()
    v0 = sim.max_spurious_u()
    steps = 5000
    for k in range(10):
        sim.step(steps // 10)
        vmax = sim.max_spurious_u()  # raises LBMError on a non-finite state
        print("[gpu-case]   step %d max|v| %.3e" % ((k + 1) * steps // 10, vmax), flush=True)
        assert vmax < 0.05
    m1, j1 = sim.invariants()
    d1 = abs_dev()
    sim.close()
    bound = 4.0 * steps * EPS32 * max(d0, d1)
    dm = abs(m1 - m0)
    dj = float(np.max(np.abs(np.array(j1) - np.array(j0))))
    print("[gpu-case] mass %.10e -> %.10e (drift %.3e, relative %.2e), |momentum| %.3e -> %.3e, "
          "bound %.3e, max|v| %.3e -> %.3e"
          % (m0, m1, dm, dm / m0, float(np.max(np.abs(j0))), float(np.max(np.abs(j1))), bound,
             v0, vmax), flush=True)
    assert np.max(np.abs(j0)) <= 1e-9 * m0
    assert dm <= bound and dj <= bound


@pytest.mark.parametrize("wl", ["d2q9_1024_fp64_eq", "d2q9_1024_fp64_force", "d2q9_1024_fp32_eq",
                                "d2q9_1024_fp32_force"])
def test_multi_drop_workloads_keep_their_invariants_over_10000_steps(wl):
    """The 1024^2 D2Q9 workloads (64 drops, both schemes, FP64 and FP32
    storage) for 10,000 steps in their autotuned launch: the state stays
    finite, max|v| stays small, and mass and momentum keep their values to
    rounding: FP64 storage within 1e-12 of the mass (every step conserves
    both exactly in exact arithmetic), FP32 storage within the rounding bound
    of the 5000-step test above, 4 * steps * EPS32 * sum_r sum_i |delta_i|."""
    import bench
    from paper_0710_5470_amd import autotune, lbm
    print("[gpu-case] 10000-step invariants", wl, flush=True)
    q, scheme, storage, compute, shape, T, kappa, tau, R, noise = bench.WORKLOADS[wl]
    p, rho0 = bench.make_workload(wl)
    sim = lbm.Simulation(p, rho0)
    autotune.autotune(sim, use_cache=False)
    print("[gpu-case] launch", sim.launch(), flush=True)
    shift = torch.tensor(sim.shift(), dtype=torch.float64, device="cuda")

    def abs_dev():
        f = sim.get_state()
        return float((f - shift[:, None]).abs().sum())

    m0, j0 = sim.invariants()
    d0 = abs_dev()
    steps = 10000
    for k in range(4):
        sim.step(steps // 4)
        vmax = sim.max_spurious_u()  # raises LBMError on a non-finite state
        assert vmax < 0.05
    m1, j1 = sim.invariants()
    d1 = abs_dev()
    sim.close()
    dm = abs(m1 - m0)
    dj = float(np.max(np.abs(np.array(j1) - np.array(j0))))
    bound = 1e-12 * m0 if storage == 0 else 4.0 * steps * EPS32 * max(d0, d1)
    print("[gpu-case] %s: mass drift %.3e (relative %.2e), momentum drift %.3e, bound %.3e, "
          "max|v| %.3e" % (wl, dm, dm / m0, dj, bound, vmax), flush=True)
    assert dm <= bound and dj <= bound
