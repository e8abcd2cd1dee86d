"""Batched drop relaxation: many independent periodic D2Q9 drops of uneven
size run to their steady state in one batch.

Each problem is a square periodic lattice holding one circular drop (a tanh
profile of width 2 between the coexisting densities of the van der Waals
fluid, Eq. (p0)), relaxed by the equilibrium scheme at tau = 1 until its
steady-state residual max_r |u(r, t+1) - u(r, t)| (FP64, from the stored
populations) falls to a tolerance.  What the paper measures on such a drop
is the spurious velocity of the steady state (section "Numerical results"):
the maximum velocity magnitude in the system, reported here per problem.

The parameter ranges: side uniform in {32..256}, radius uniform in
[0.15, 0.35] x side, T uniform in [0.54, 0.55] and kappa uniform in
[0.005, min(0.02, (T - 0.5) / 3)].  Below T ~ 0.49 + 3 kappa the uniform
liquid at the Maxwell density is linearly unstable at tau = 1, so the
temperatures are the stable part of [0.45, 0.55] and kappa is capped.
"""
import time

import numpy as np
import torch

from . import autotune, inputs, lbm

A_VDW, B_VDW = 9.0 / 49.0, 2.0 / 21.0


def specs(nprob=512, seed=4, side_lo=32, side_hi=256):
    """Per-problem parameters (side, radius, T, kappa) of the uneven batch."""
    return inputs.batch_specs(nprob, seed, side_lo=side_lo, side_hi=side_hi, T_lo=0.54, T_hi=0.55,
                              kappa_cap=lambda T: (T - 0.5) / 3.0)


def problems(specs_, storage=lbm.STORE_F32_SHIFTED, compute=lbm.COMPUTE_NATIVE, tau=1.0,
             device="cuda"):
    """lbm_params of every problem and the cold initial densities,
    concatenated on the device as one [sum side^2] FP64 tensor."""
    plist, rho0 = [], []
    for s in specs_:
        g, l = lbm.lbm_coexistence(A_VDW, B_VDW, s["T"])
        n = s["side"]
        plist.append(lbm.params(lattice=lbm.D2Q9, scheme=lbm.SCHEME_EQ, storage=storage,
                                compute=compute, shape=(n, n), T=s["T"], kappa=s["kappa"], tau=tau))
        rho0.append(inputs.tanh_drop((n, n), s["radius"], l, g, 2.0).reshape(-1))
    return plist, torch.tensor(np.concatenate(rho0), dtype=torch.float64, device=device)


def _spread(v):
    v = np.asarray(v)
    return dict(min=int(v.min()), p10=int(np.percentile(v, 10)), median=int(np.median(v)),
                p90=int(np.percentile(v, 90)), max=int(v.max()))


def time_to_steady(specs_, storage=lbm.STORE_F32_SHIFTED, compute=lbm.COMPUTE_NATIVE, tol=5e-8,
                   check_every=100, max_steps=400000, tune=True):
    """Run the batch cold to the residual `tol`.  The clock starts with the
    batch's creation (initial equilibrium on the device) and stops after the
    last check; the launch shape is picked beforehand by the batch autotuner
    on a throwaway copy.  Returns the wall seconds, the per-problem step
    spread, statuses and the spurious velocities of the final states."""
    plist, rho0 = problems(specs_, storage, compute)
    launch = autotune.autotune_batch(plist, rho0) if tune else None
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    bt = lbm.Batch(plist, rho0)
    if launch is not None:
        bt.set_launch(*launch)
    steps, res, status = bt.run(tol, check_every, max_steps)
    secs = time.perf_counter() - t0
    vmax = np.array(bt.max_spurious_u())
    bt.close()
    steps, status = np.array(steps), np.array(status)
    sides = np.array([s["side"] for s in specs_])
    sites = int((sides ** 2).sum())
    return dict(problems=len(specs_), sites=sites, storage="fp32" if storage else "fp64",
                arithmetic="fp64" if (storage == lbm.STORE_F64 or compute == lbm.COMPUTE_F64)
                else "fp32", tol=tol, check_every=check_every, seconds=round(secs, 4),
                converged=int((status == lbm.BATCH_CONVERGED).sum()),
                steps=_spread(steps), site_steps=int((steps * sides ** 2).sum()),
                mlups=round(float((steps * sides ** 2).sum()) / secs / 1e6, 1),
                launch=list(launch) if launch is not None else None,
                max_spurious_u=dict(median=float(np.median(vmax)), max=float(vmax.max())))
