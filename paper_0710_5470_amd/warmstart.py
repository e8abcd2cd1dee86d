"""Learned warm start for batched drop problems.

A small periodic convolutional network (6 layers, 3x3 kernels, 32 channels,
relu) maps the drop parameters (a, b, T, kappa, R as constant planes) and the
initial density to a near-steady (rho, u_x, u_y) field.  The prediction is
averaged over the square's eight symmetries (the centred drop's steady state
has them) and given the cold start's mass and zero momentum.  The batched
lattice Boltzmann runner then starts from the equilibrium of that field,
decides convergence by its own residual and falls back to a cold start for
any problem whose residual rises tenfold above its best.

Every arithmetic step of the network runs in this library's HIP kernels
(bf16 matrix cores, FP32 accumulation; see the lbm_net_* entry points);
torch only provides device memory and streams.  Training data are steady
states that the batched runner itself produces.
"""
import math
import os
import time

import numpy as np
import torch

from . import autotune, inputs, lbm

A_VDW, B_VDW = 9.0 / 49.0, 2.0 / 21.0
# (padded cin, padded cout, real cout) per layer; 6 real input channels
LAYERS = [(16, 32, 32), (32, 32, 32), (32, 32, 32), (32, 32, 32), (32, 32, 32), (32, 16, 3)]
IN_REAL, OUT_REAL = 6, 3
CP_IN, CP_OUT = 16, 16

# feature / target scales (fixed, so a trained net can be reused)
SCALE = dict(T=(0.55, 0.01), kappa=(0.0125, 0.005), R=(0.25, 0.06), rho=(3.5, 1.0),
             drho=0.2, u=1e-3)


RHO_LO = 1e-3            # clamp of the projected density (the vdW bound is 1/b)


def _consts(specs, side):
    """Per-problem normalised constants [n, 5]: a, b (the same for every
    problem, so zero after centring), T, kappa, R / side."""
    c = np.zeros((len(specs), 5))
    for k, s in enumerate(specs):
        c[k, 2] = (s["T"] - SCALE["T"][0]) / SCALE["T"][1]
        c[k, 3] = (s["kappa"] - SCALE["kappa"][0]) / SCALE["kappa"][1]
        c[k, 4] = (s["radius"] / side - SCALE["R"][0]) / SCALE["R"][1]
    return c


def features(specs, side, rho0, device="cuda"):
    """[n, side, side, 16] FP32 network input on the device (channels:
    the constants of `_consts`, then the normalised initial density)."""
    n = len(specs)
    consts = torch.tensor(_consts(specs, side), dtype=torch.float64, device=device)
    x = torch.empty(n, side, side, CP_IN, dtype=torch.float32, device=device)
    lbm.lbm_warm_features(n, side, consts, rho0, SCALE["rho"][0], SCALE["rho"][1], x)
    return x


def targets(rho, rho0, vel, side):
    """[n, side, side, 16]: (rho - rho0) / s_rho, u_x / s_u, u_y / s_u."""
    n = rho.numel() // (side * side)
    y = torch.empty(n, side, side, CP_OUT, dtype=torch.float32, device=rho.device)
    lbm.lbm_warm_targets(rho, rho0, vel, SCALE["drho"], SCALE["u"], y)
    return y


class WarmNet:
    def __init__(self, seed=7, device="cuda"):
        self.dev = torch.device(device)
        self.params = []
        st = inputs.Stream(seed)
        for cin, cout, creal in LAYERS:
            real_in = IN_REAL if cin == CP_IN else cin
            fan_in = 9 * real_in
            W = np.zeros((9, cout, cin), dtype=np.float32)
            # He-uniform init on the real channels
            lim = math.sqrt(6.0 / fan_in)
            w = (2.0 * st.uniform(9 * creal * real_in) - 1.0) * lim
            W[:, :creal, :real_in] = w.reshape(9, creal, real_in)
            if creal == OUT_REAL:
                W *= 0.1
            b = np.zeros(cout, dtype=np.float32)
            self.params.append([torch.tensor(W, device=self.dev), torch.tensor(b, device=self.dev)])
        self.adam = [[torch.zeros_like(W), torch.zeros_like(W), torch.zeros_like(b), torch.zeros_like(b)]
                     for W, b in self.params]
        self.t = 0
        self._ws = None

    def numpy_params(self):
        return [(W.double().cpu().numpy(), b.double().cpu().numpy()) for W, b in self.params]

    def load_numpy(self, params):
        for (W, b), (Wn, bn) in zip(self.params, params):
            W.copy_(torch.as_tensor(np.asarray(Wn, dtype=np.float32)))
            b.copy_(torch.as_tensor(np.asarray(bn, dtype=np.float32)))

    def _shape(self, n, h, w, l):
        cin, cout, creal = LAYERS[l]
        return lbm._shape(n, h, w, cin, cout, creal)

    def forward(self, x):
        """x: [n, h, w, 16] FP32 device tensor -> list of pre-activations."""
        n, h, w = x.shape[0], x.shape[1], x.shape[2]
        zs = [x]
        for l, (W, b) in enumerate(self.params):
            out = torch.empty(n, h, w, LAYERS[l][1], dtype=torch.float32, device=self.dev)
            lbm.lbm_net_conv3x3_fwd(self._shape(n, h, w, l), zs[-1], l > 0, W, b, out)
            zs.append(out)
        return zs

    def backward(self, zs, dout):
        n, h, w = zs[0].shape[0], zs[0].shape[1], zs[0].shape[2]
        grads = [None] * len(self.params)
        d = dout
        for l in range(len(self.params) - 1, -1, -1):
            W, b = self.params[l]
            s = self._shape(n, h, w, l)
            need = lbm.lbm_net_conv3x3_bwd_weight_workspace(s)
            if self._ws is None or self._ws.numel() < need:
                self._ws = torch.empty(need, dtype=torch.uint8, device=self.dev)
            dW = torch.empty_like(W)
            db = torch.empty_like(b)
            lbm.lbm_net_conv3x3_bwd_weight(s, d, zs[l], l > 0, dW, db, self._ws)
            grads[l] = (dW, db)
            if l > 0:
                din = torch.empty_like(zs[l])
                lbm.lbm_net_conv3x3_bwd_data(s, d, W, zs[l], din)
                d = din
        return grads

    def loss_and_grad(self, x, y):
        zs = self.forward(x)
        pred = zs[-1]
        n = pred.shape[0] * pred.shape[1] * pred.shape[2]
        g = torch.empty_like(pred)
        part = torch.empty(1024, dtype=torch.float64, device=self.dev)
        loss = lbm.lbm_net_mse(n, CP_OUT, OUT_REAL, pred, y, g, part)
        return loss, self.backward(zs, g)

    def train_step(self, x, y, lr):
        loss, grads = self.loss_and_grad(x, y)
        self.t += 1
        for (W, b), (dW, db), (mW, vW, mb, vb) in zip(self.params, grads, self.adam):
            lbm.lbm_net_adam(W, dW, mW, vW, lr, self.t)
            lbm.lbm_net_adam(b, db, mb, vb, lr, self.t)
        return loss

    def predict(self, x, batch=32):
        out = []
        for i in range(0, x.shape[0], batch):
            out.append(self.forward(x[i:i + batch])[-1])
        return torch.cat(out)


# ---- data from the lattice Boltzmann runner --------------------------------

def problems(specs, side, storage=lbm.STORE_F64, tau=1.0, device="cuda"):
    """Lattice parameters and the cold initial densities (tanh drop between
    the Maxwell densities), concatenated on the device as [n side^2]."""
    plist, rho0 = [], []
    for s in specs:
        g, l = lbm.lbm_coexistence(A_VDW, B_VDW, s["T"])
        plist.append(lbm.params(lattice=lbm.D2Q9, scheme=lbm.SCHEME_EQ, storage=storage,
                                shape=(side, side), T=s["T"], kappa=s["kappa"], tau=tau))
        rho0.append(inputs.tanh_drop((side, side), s["radius"], l, g, 2.0).reshape(-1))
    return plist, torch.tensor(np.concatenate(rho0), dtype=torch.float64, device=device)


def steady_states(specs, side, tol=1e-10, check_every=100, max_steps=60000, rho_init=None,
                  u_init=None, patience=0, grace=0, tune=True, settle_tol=None, settle_steps=120000):
    """Run a batch (cold, or from rho_init [n side^2] / u_init [3, n side^2]
    device fields) to its residual.  Returns a dict with device fields rho
    [n side^2], vel [3, n side^2], host arrays steps, residual, status and the
    wall seconds from batch creation to the last check.  With settle_tol, the
    same batch then continues (untimed) to that tighter residual and
    rho_settled holds the density it reaches."""
    plist, rho0 = problems(specs, side)
    launch = autotune.autotune_batch(plist, rho0) if tune else None
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    bt = lbm.Batch(plist, rho0 if rho_init is None else rho_init, u_init)
    if launch is not None:
        bt.set_launch(*launch)
    steps, res, status = bt.run(tol, check_every, max_steps, patience, grace)
    secs = time.perf_counter() - t0
    rho, vel = bt.moments()
    out = dict(rho=rho, vel=vel, rho0=rho0, steps=np.array(steps), residual=np.array(res),
               status=np.array(status), seconds=secs)
    if settle_tol is not None:
        bt.reactivate()
        bt.run(settle_tol, check_every, settle_steps)
        out["rho_settled"] = bt.moments()[0]
    bt.close()
    return out


def warm_start(net, specs, side, tol=1e-10, check_every=100, max_steps=60000, patience=3,
               grace=500, symmetrize=True, with_velocity=False, settle_tol=None):
    """Predict, project (lbm_warm_project), run with the rising-residual
    check; problems that diverge or go non-finite are rerun from the cold
    start.  Returns the
    steady_states dict with per-problem total steps, final statuses, the
    fallback mask and wall seconds including inference (features, network,
    projection).  The problems themselves (parameters and cold initial
    densities) are built before the clock starts, as in steady_states."""
    n = len(specs)
    _, rho0 = problems(specs, side)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    pred = net.predict(features(specs, side, rho0))
    rho_p = torch.empty(n * side * side, dtype=torch.float64, device=net.dev)
    u_p = torch.empty(3, n * side * side, dtype=torch.float64, device=net.dev)
    lbm.lbm_warm_project(n, side, CP_OUT, pred, rho0, SCALE["drho"], SCALE["u"], with_velocity,
                         symmetrize, RHO_LO, 0.99 / B_VDW, rho_p, u_p)
    torch.cuda.synchronize()
    t_inf = time.perf_counter() - t0
    run = steady_states(specs, side, tol, check_every, max_steps, rho_init=rho_p, u_init=u_p,
                        patience=patience, grace=grace, settle_tol=settle_tol)
    # rising residual, or a state that went non-finite: rerun from the cold start
    fallback = (run["status"] == lbm.BATCH_DIVERGED) | (run["status"] == lbm.BATCH_NONFINITE)
    total = run["steps"].copy()
    status = run["status"].copy()
    secs_fb = 0.0
    if fallback.any():
        idx = np.nonzero(fallback)[0]
        sub = steady_states([specs[i] for i in idx], side, tol, check_every, max_steps)
        total[idx] += sub["steps"]
        status[idx] = sub["status"]
        secs_fb = sub["seconds"]
    run.update(steps=total, status=status, fallback=fallback, inference_seconds=t_inf,
               seconds=t_inf + run["seconds"] + secs_fb)
    return run


# ---- end-to-end experiment: generate, train, compare warm vs cold ----------

def _log(*a):
    print("[warmstart]", *a, flush=True)


def generate(nprob, side, seed, batch=512, tol=1e-10, max_steps=60000):
    """Steady states of `nprob` drops from the stable batched workload
    (side fixed), by the batched runner.  Returns (specs, x, y, steps) with
    x, y device tensors of the converged problems only."""
    specs = inputs.stable_batch_specs(nprob, seed, side_lo=side, side_hi=side)
    xs, ys, steps, kept = [], [], [], []
    for i in range(0, nprob, batch):
        sub = specs[i:i + batch]
        run = steady_states(sub, side, tol, 100, max_steps)
        ok = np.nonzero(run["status"] == lbm.BATCH_CONVERGED)[0]
        idx = torch.tensor(ok, device=run["rho"].device)
        xs.append(features(sub, side, run["rho0"]).index_select(0, idx))
        ys.append(targets(run["rho"], run["rho0"], run["vel"], side).index_select(0, idx))
        steps.append(run["steps"][ok])
        kept += [sub[k] for k in ok]
        _log("generated %d/%d steady states (%.1f s, median steps %d, status counts %s)"
             % (i + len(sub), nprob, run["seconds"], int(np.median(run["steps"])),
                np.bincount(run["status"], minlength=5).tolist()))
    return kept, torch.cat(xs), torch.cat(ys), np.concatenate(steps)


def train(net, x, y, epochs, batch=16, lr=1e-3, seed=1):
    """Plain minibatch Adam; x, y device tensors.  Returns per-epoch losses."""
    n = x.shape[0]
    st = inputs.Stream(seed)
    losses = []
    for ep in range(epochs):
        lr_ep = lr * 0.5 * (1.0 + math.cos(math.pi * ep / epochs))  # cosine decay
        order = np.argsort(st.uniform(n))
        tot = 0.0
        for i in range(0, n - batch + 1, batch):
            idx = torch.tensor(order[i:i + batch], device=net.dev)
            tot += net.train_step(x.index_select(0, idx).contiguous(),
                                  y.index_select(0, idx).contiguous(), lr_ep) * batch
        losses.append(tot / (n - n % batch))
        _log("epoch %d loss %.5f lr %.1e" % (ep, losses[-1], lr_ep))
    return losses


def _field_error(rho, ref, n):
    """Per-problem max relative density difference."""
    a = rho.reshape(n, -1)
    b = ref.reshape(n, -1)
    return ((a - b).abs() / b).amax(dim=1).cpu().numpy()


# rho: the default (symmetrised density, u = 0); rho_u: with the predicted
# velocity; raw: no symmetrisation
VARIANTS = (("rho", dict()), ("rho_u", dict(with_velocity=True)),
            ("raw", dict(symmetrize=False, with_velocity=True)))


def evaluate(net, n_eval=512, side=128, seed=6, tol=1e-10, ref_tol=1e-13, ref_steps=120000,
             variants=VARIANTS):
    """Cold start versus the warm-start variants on held-out drops, each at
    the residual `tol`; every final field is compared with a reference run
    to `ref_tol` (the same cold start, run further)."""
    specs = inputs.stable_batch_specs(n_eval, seed, side_lo=side, side_hi=side)
    cold = steady_states(specs, side, tol, settle_tol=ref_tol, settle_steps=ref_steps)
    ref = dict(rho=cold["rho_settled"])
    out = dict(n_eval=n_eval, side=side, tol=tol, ref_tol=ref_tol)

    def liquid_fraction(rho):
        r = rho.reshape(n_eval, -1)
        mid = 0.5 * (r.amax(dim=1) + r.amin(dim=1))
        return (r > mid[:, None]).double().mean(dim=1).cpu().numpy()

    lf_ref = liquid_fraction(ref["rho"])

    def summary(run, secs):
        # err: against the cold start's settled state; err_self: against the
        # state this run itself settles into (how far from steady it stopped)
        err = _field_error(run["rho"], ref["rho"], n_eval)
        err_self = _field_error(run["rho"], run["rho_settled"], n_eval)
        err_settled = _field_error(run["rho_settled"], ref["rho"], n_eval)
        conv = run["status"] == lbm.BATCH_CONVERGED
        lf = liquid_fraction(run["rho_settled"])
        other = [dict(problem=int(i), err=float(err[i]), err_self=float(err_self[i]),
                      err_settled=float(err_settled[i]), liquid_fraction=float(lf[i]),
                      ref_liquid_fraction=float(lf_ref[i]), **specs[i])
                 for i in np.nonzero(err_settled > 1e-3)[0]]
        # statistics over the problems whose cold reference is finite
        fin = np.isfinite(err_settled)
        return dict(seconds=secs, steps_total=int(run["steps"].sum()),
                    steps_median=float(np.median(run["steps"])), steps_max=int(run["steps"].max()),
                    converged=int(conv.sum()), compared=int(fin.sum()),
                    err_median=float(np.median(err[fin])), err_p90=float(np.percentile(err[fin], 90)),
                    err_max=float(err[fin].max()), err_self_median=float(np.median(err_self[fin])),
                    err_self_max=float(err_self[fin].max()),
                    unsettled=int((err_self[fin] > 1e-3).sum()), other_steady_state=other)

    out["cold"] = summary(cold, cold["seconds"])
    _log("cold: %.2f s, %s" % (cold["seconds"], out["cold"]))
    for name, kw in variants:
        w = warm_start(net, specs, side, tol, settle_tol=ref_tol, **kw)
        out[name] = summary(w, w["seconds"])
        out[name].update(fallbacks=int(w["fallback"].sum()), inference_seconds=w["inference_seconds"])
        ratio = w["steps"] / np.maximum(cold["steps"], 1)
        out[name].update(step_ratio_median=float(np.median(ratio)),
                         step_ratio_p10=float(np.percentile(ratio, 10)),
                         step_ratio_p90=float(np.percentile(ratio, 90)))
        _log("warm[%s]: %.2f s, %s" % (name, w["seconds"], out[name]))
    return out


WEIGHTS = os.path.join(os.path.dirname(os.path.abspath(__file__)), "warm_net_d2q9_128.npz")


def time_to_steady(net=None, n=512, side=128, seed=6, tol=1e-10):
    """Batched time-to-steady on held-out drops: the cold start, then the
    default warm start (inference included), each to the residual `tol`.
    Uses the shipped network when net is None."""
    if net is None:
        net = load_weights(WEIGHTS)
    specs = inputs.stable_batch_specs(n, seed, side_lo=side, side_hi=side)
    cold = steady_states(specs, side, tol)
    warm = warm_start(net, specs, side, tol)
    ok = lambda r: int((r["status"] == lbm.BATCH_CONVERGED).sum())
    return dict(problems=n, side=side, tol=tol, seed=seed,
                cold_seconds=round(cold["seconds"], 4), warm_seconds=round(warm["seconds"], 4),
                warm_inference_seconds=round(warm["inference_seconds"], 4),
                cold_steps=int(cold["steps"].sum()), warm_steps=int(warm["steps"].sum()),
                cold_converged=ok(cold), warm_converged=ok(warm),
                fallbacks=int(warm["fallback"].sum()),
                speedup=round(cold["seconds"] / warm["seconds"], 4))


def run_experiment(n_train=2048, n_eval=512, side=128, epochs=20, seed_train=5, seed_eval=6,
                   tol=1e-10, out_json=None, weights=None):
    t0 = time.perf_counter()
    _, xt, yt, _ = generate(n_train, side, seed_train, tol=tol)
    t_gen = time.perf_counter() - t0
    zero_loss = float((yt[..., :OUT_REAL].double() ** 2).mean())
    net = WarmNet(seed=7)
    t1 = time.perf_counter()
    losses = train(net, xt, yt, epochs)
    t_train = time.perf_counter() - t1
    del xt, yt
    res = dict(n_train=n_train, epochs=epochs, seconds_generate=t_gen, seconds_train=t_train,
               final_loss=losses[-1], zero_prediction_loss=zero_loss, losses=losses)
    if weights:
        np.savez(weights, *[a for W, b in net.numpy_params() for a in (W, b)])
    res.update(evaluate(net, n_eval, side, seed_eval, tol))
    if out_json:
        import json
        with open(out_json, "w") as fh:
            json.dump(res, fh, indent=1)
    return res, net


def load_weights(path, device="cuda"):
    """A WarmNet with the parameters saved by run_experiment."""
    net = WarmNet(device=device)
    with np.load(path) as d:
        arrs = [d["arr_%d" % i] for i in range(len(d.files))]
    net.load_numpy([(arrs[2 * l], arrs[2 * l + 1]) for l in range(len(arrs) // 2)])
    return net


if __name__ == "__main__":
    import argparse
    import json
    ap = argparse.ArgumentParser(description="learned warm start: generate, train, compare")
    ap.add_argument("--train", type=int, default=2048)
    ap.add_argument("--eval", type=int, default=512)
    ap.add_argument("--side", type=int, default=128)
    ap.add_argument("--epochs", type=int, default=20)
    ap.add_argument("--tol", type=float, default=1e-10)
    ap.add_argument("--out", default=None)
    ap.add_argument("--weights", default=None, help="where to save the trained parameters")
    ap.add_argument("--evaluate", default=None, metavar="WEIGHTS",
                    help="only evaluate saved parameters on the held-out drops")
    a = ap.parse_args()
    if a.evaluate:
        r = evaluate(load_weights(a.evaluate), a.eval, a.side, tol=a.tol)
        if a.out:
            with open(a.out, "w") as fh:
                json.dump(r, fh, indent=1)
    else:
        r, _ = run_experiment(a.train, a.eval, a.side, a.epochs, tol=a.tol, out_json=a.out,
                              weights=a.weights)
    print(json.dumps({k: v for k, v in r.items() if k != "losses"}))
