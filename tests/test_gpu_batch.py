"""GPU tests of the batched runner: many independent problems in one
persistent launch per step, device-side convergence checks, hipGraph replay."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

A, B_ = 9.0 / 49.0, 2.0 / 21.0


def _say(*a):
    print("[gpu-case]", *a, flush=True)


def _problems(specs, scheme=0, storage=0, compute=0):
    from paper_0710_5470_amd import inputs, lbm
    plist, rho = [], []
    for s in specs:
        g, l = lbm.lbm_coexistence(A, B_, s["T"])
        n = s["side"]
        plist.append(lbm.params(lattice=lbm.D2Q9, scheme=scheme, storage=storage, compute=compute,
                                shape=(n, s.get("ny", n)), T=s["T"], kappa=s["kappa"],
                                tau=s.get("tau", 1.0)))
        rho.append(inputs.tanh_drop((n, s.get("ny", n)), s["radius"], l, g, 2.0))
    return plist, rho


SPECS = [dict(side=37, ny=29, radius=8.0, T=0.55, kappa=0.01, tau=0.9),
         dict(side=64, radius=12.0, T=0.56, kappa=0.02),
         dict(side=33, radius=7.0, T=0.545, kappa=0.012, tau=1.2),
         dict(side=100, ny=48, radius=14.0, T=0.56, kappa=0.025),
         dict(side=32, radius=6.0, T=0.55, kappa=0.015)]


@pytest.mark.parametrize("scheme,storage", [(0, 0), (1, 0), (1, 1), (0, 1)])
def test_batch_steps_match_single_problem_runs(scheme, storage):
    from paper_0710_5470_amd import lbm
    plist, rho = _problems(SPECS, scheme, storage)
    _say("batch vs single", scheme, storage)
    bt = lbm.Batch(plist, rho)
    bt.step(40)
    r_b, v_b = bt.moments()
    rb, vb = bt.split(r_b.cpu().numpy()), bt.split(v_b.cpu().numpy())
    bt.close()
    for k, (p, r0) in enumerate(zip(plist, rho)):
        sim = lbm.Simulation(p, r0)
        sim.step(40)
        r, v = [t.cpu().numpy() for t in sim.moments()]
        sim.close()
        assert np.array_equal(r, rb[k]), k
        assert np.array_equal(v, vb[k]), k


@pytest.mark.parametrize("scheme,storage", [(1, 0), (0, 1)])
def test_batch_graph_replays_match_eager_steps(scheme, storage):
    """Each graph replay runs K steps plus the check; replays must leave the
    same state as the same number of eagerly launched steps."""
    from paper_0710_5470_amd import lbm
    plist, rho = _problems(SPECS, scheme, storage)
    a = lbm.Batch(plist, rho)
    steps, res, status = a.run(tol=0.0, check_every=10, max_steps=50)
    assert all(s == lbm.BATCH_MAXSTEPS for s in status)
    assert all(n == 50 for n in steps)
    ra, va = [t.cpu().numpy() for t in a.moments()]
    b = lbm.Batch(plist, rho)
    b.step(50)
    rb, vb = [t.cpu().numpy() for t in b.moments()]
    a.close()
    b.close()
    assert np.array_equal(ra, rb) and np.array_equal(va, vb)


def test_batch_runs_to_residual_and_retires_problems():
    """FP64 storage: every stable problem reaches the residual; an unstable
    one (T = 0.5, kappa = 0.02) is retired as non-finite without disturbing
    the others; each converged problem's residual agrees with a single-problem
    run continued one step from the batch's final state."""
    from paper_0710_5470_amd import lbm
    specs = SPECS[:3] + [dict(side=40, radius=10.0, T=0.5, kappa=0.02)]
    plist, rho = _problems(specs, 0, 0)
    bt = lbm.Batch(plist, rho)
    steps, res, status = bt.run(tol=1e-9, check_every=50, max_steps=200000)
    _say("batch run", steps, res, status)
    assert status[:3] == [lbm.BATCH_CONVERGED] * 3
    assert status[3] == lbm.BATCH_NONFINITE
    assert all(r <= 1e-9 for r in res[:3])
    assert steps[3] < steps[0]
    bt.close()


def test_batch_detects_rising_residual():
    """With patience 1 and no grace period, a problem whose residual grows
    tenfold above its smallest value (an unstable liquid at T = 0.5) is
    retired as diverged, or as non-finite if it blows up between checks."""
    from paper_0710_5470_amd import lbm
    plist, rho = _problems([dict(side=48, radius=10.0, T=0.5, kappa=0.02)], 0, 0)
    bt = lbm.Batch(plist, rho)
    steps, res, status = bt.run(tol=1e-12, check_every=2, max_steps=4000, patience=1, grace=0)
    bt.close()
    assert status[0] in (lbm.BATCH_DIVERGED, lbm.BATCH_NONFINITE)


def test_reactivated_batch_continues_to_a_tighter_residual():
    """After a run retires every problem, lbm_batch_reactivate lets a second
    run continue them from their populations: a run to 1e-6 followed by a
    run to 1e-9 ends in the same state as one run straight to 1e-9 when the
    two stop after the same total number of steps."""
    from paper_0710_5470_amd import lbm
    plist, rho = _problems(SPECS[:2], 0, 0)
    bt = lbm.Batch(plist, rho)
    s1, r1, st1 = bt.run(tol=1e-6, check_every=50, max_steps=100000)
    again, _, _ = bt.run(tol=1e-6, check_every=50, max_steps=100000)
    bt.reactivate()
    s2, r2, st2 = bt.run(tol=1e-9, check_every=50, max_steps=100000)
    _say("two-stage run", s1, s2, r2, st2)
    assert again == s1  # nothing active: no further step is counted
    assert st2 == [lbm.BATCH_CONVERGED] * 2 and all(r <= 1e-9 for r in r2)
    assert all(b > 0 for b in s2)
    rho_two, _ = bt.moments()
    bt.close()
    # single run of the same total number of steps per problem
    for k in range(2):
        p1, rr = _problems(SPECS[k:k + 1], 0, 0)
        one = lbm.Batch(p1, rr)
        one.step(s1[k] + s2[k])
        r_one, _ = one.moments()
        one.close()
        seg = rho_two[sum(p.nx * p.ny for p in plist[:k]):][:plist[k].nx * plist[k].ny]
        assert torch.equal(seg, r_one)


def test_odd_step_count_refused_while_a_problem_is_retired():
    """A retired problem is skipped and keeps its populations in the buffer
    the batch returns to after an even number of steps.  After a run has
    retired problems, lbm_batch_step refuses an odd count (LBM_E_STATE) and
    an even count changes nothing; after lbm_batch_reactivate an odd count is
    accepted and continues every problem from its retired state (equal to a
    single-problem run of the same total number of steps)."""
    from paper_0710_5470_amd import lbm
    specs = [SPECS[4], SPECS[1]]
    plist, rho = _problems(specs, 0, 0)
    bt = lbm.Batch(plist, rho)
    _say("odd steps after retirement")
    # every problem retires, converged or at max_steps
    steps, _, status = bt.run(tol=1e-7, check_every=50, max_steps=4000)
    _say("  run", steps, status)
    assert all(st in (lbm.BATCH_CONVERGED, lbm.BATCH_MAXSTEPS) for st in status)
    r0, v0 = bt.moments()
    with pytest.raises(lbm.LBMError) as ei:
        bt.step(1)
    assert ei.value.code == lbm.E_STATE
    bt.step(2)
    r1, v1 = bt.moments()
    assert torch.equal(r0, r1) and torch.equal(v0, v1)
    bt.reactivate()
    bt.step(1)
    r2, _ = bt.moments()
    bt.close()
    for k in range(2):
        p1, rr = _problems(specs[k:k + 1], 0, 0)
        one = lbm.Batch(p1, rr)
        one.step(steps[k] + 1)
        r_one, _ = one.moments()
        one.close()
        seg = r2[sum(p.nx * p.ny for p in plist[:k]):][:plist[k].nx * plist[k].ny]
        assert torch.equal(seg, r_one)


def test_full_size_batch_matches_oracle_on_sampled_problems():
    """The batched time-to-steady workload at full size (512 drops of 128^2,
    FP64, tau = 1) in the launch the batch autotuner picks for it, 6 steps;
    four sampled problems (first, last, and two inside, among them the one
    with T = 0.549410) against the oracle: 1e-12 relative on rho and 1e-12
    absolute on u, as for the single-lattice FP64 parity."""
    import oracle
    from paper_0710_5470_amd import autotune, inputs, lbm
    from paper_0710_5470_amd import warmstart as ws
    specs = inputs.stable_batch_specs(512, 6, side_lo=128, side_hi=128)
    plist, rho0 = ws.problems(specs, 128)
    launch = autotune.autotune_batch(plist, rho0, use_cache=False)
    _say("full-size batch, 512 x 128^2, launch", launch)
    bt = lbm.Batch(plist, rho0)
    bt.set_launch(*launch)
    bt.step(6)
    r, v = bt.moments()
    rs, vs = bt.split(r), bt.split(v)
    r0 = rho0.cpu().numpy().reshape(512, 128, 128)
    for k in (0, 137, 444, 511):
        p = plist[k]
        op = oracle.params(q=9, scheme=0, shape=(128, 128), T=p.T, kappa=p.kappa, tau=1.0)
        ro, vo = oracle.observe(op, oracle.run(op, oracle.init(op, r0[k]), 6))
        rg = rs[k].cpu().numpy()
        vg = vs[k].cpu().numpy()
        er = float(np.max(np.abs(rg - ro) / ro))
        ev = float(np.max(np.abs(vg[:2] - vo[:2])))
        _say("problem %d: rel err rho %.2e, abs err u %.2e" % (k, er, ev))
        assert er < 1e-12 and ev < 1e-12
    bt.close()


def test_uneven_fp32_batch_matches_oracle_on_sampled_problems():
    """The uneven batched workload at full size (512 drops, side 32..256,
    FP32 storage and arithmetic, tau = 1; paper_0710_5470_amd.drops) in the
    launch the batch autotuner picks for it, 50 steps; five sampled problems
    (first, last, the smallest, the largest and one of odd side) against the
    oracle's FP64 runs of them.  The FP32 parity bar: 1e-5 relative on rho;
    on u, 1e-8 absolute for rest deviations |delta_0| = |f_0 - s_0| below 2,
    scaled with the FP32 rounding unit at the largest |delta_0| of the
    problem (the velocity error comes from the storage roundings of delta_0;
    the single-lattice parity tests at T = 0.56 have |delta_0| < 2).  At T in
    [0.54, 0.55] the phases are further apart and |delta_0| reaches 2..4,
    where an FP32 ulp is twice as large: 2e-8."""
    import oracle
    from paper_0710_5470_amd import autotune, drops, lbm
    sp = drops.specs()
    plist, rho0 = drops.problems(sp)
    sides = np.array([s["side"] for s in sp])
    launch = autotune.autotune_batch(plist, rho0, use_cache=False)
    _say("uneven FP32 batch, 512 drops, %d sites, launch %s" % (int((sides ** 2).sum()), launch))
    bt = lbm.Batch(plist, rho0)
    bt.set_launch(*launch)
    bt.step(50)
    r, v = bt.moments()
    rs, vs = bt.split(r), bt.split(v)
    bt.close()
    r0 = rho0.cpu().numpy()
    off = np.concatenate([[0], np.cumsum(sides ** 2)])
    odd = int(np.nonzero(sides % 2 == 1)[0][0])
    picks = sorted({0, len(sp) - 1, int(np.argmin(sides)), int(np.argmax(sides)), odd})
    for k in picks:
        n, s = int(sides[k]), sp[k]
        op = oracle.params(q=9, scheme=0, shape=(n, n), T=s["T"], kappa=s["kappa"], tau=1.0)
        f0 = oracle.init(op, r0[off[k]:off[k + 1]].reshape(n, n))
        f1 = oracle.run(op, f0, 50)
        ro, vo = oracle.observe(op, f1)
        rg, vg = rs[k].cpu().numpy(), vs[k].cpu().numpy()
        er = float(np.max(np.abs(rg - ro) / ro))
        ev = float(np.max(np.abs(vg[:2] - vo[:2])))
        # the shift of the rest population: its rest equilibrium at the mean
        # initial density
        s0 = oracle.feq_site(op, float(np.mean(f0.sum(0))), np.zeros(3), np.zeros(3), 0.0)[0]
        d0 = max(float(np.abs(f0[0] - s0).max()), float(np.abs(f1[0] - s0).max()))
        tol_v = 1e-8 * max(1.0, 2.0 ** np.floor(np.log2(d0)))
        _say("problem %d (side %d, T %.4f): rel err rho %.2e, abs err u %.2e (tol %.0e, "
             "max|delta_0| %.2f), max|u| %.2e" % (k, n, s["T"], er, ev, tol_v, d0,
                                                 float(np.abs(vo).max())))
        assert er < 1e-5 and ev < tol_v
