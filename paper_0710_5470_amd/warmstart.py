"""Learned warm start for batched drop problems.

A small periodic convolutional network (6 layers, 3x3 kernels, 32 channels,
relu) maps the drop parameters (a, b, T, kappa, R as constant planes) and the
initial density to a near-steady (rho, u_x, u_y) field.  The prediction is
averaged over the square's eight symmetries (the centred drop's steady state
has them) and given the cold start's mass and zero momentum.  The batched
lattice Boltzmann runner then starts from the equilibrium of that field,
judges convergence by its own residual and falls back to a cold start for
any problem whose residual rises tenfold above its best.

Every arithmetic step of the network runs in this library's HIP kernels
(bf16 matrix cores, FP32 accumulation; see the lbm_net_* entry points);
torch only provides device memory and streams.  Training data are steady
states that the batched runner itself produces.
"""
import math
import time

import numpy as np
import torch

from . import inputs, lbm

A_VDW, B_VDW = 9.0 / 49.0, 2.0 / 21.0
# (padded cin, padded cout, real cout) per layer; 6 real input channels
LAYERS = [(16, 32, 32), (32, 32, 32), (32, 32, 32), (32, 32, 32), (32, 32, 32), (32, 16, 3)]
IN_REAL, OUT_REAL = 6, 3
CP_IN, CP_OUT = 16, 16

# feature / target scales (fixed, so a trained net can be reused)
SCALE = dict(T=(0.55, 0.01), kappa=(0.0125, 0.005), R=(0.25, 0.06), rho=(3.5, 1.0),
             drho=0.2, u=1e-3)


def features(specs, side, rho0):
    """[n, side, side, 16] FP32 network input: a, b (constant, so zero after
    centring), T, kappa, R / side as normalised constant planes, and the
    normalised initial density."""
    n = len(specs)
    x = np.zeros((n, side, side, CP_IN), dtype=np.float32)
    for k, s in enumerate(specs):
        x[k, :, :, 2] = (s["T"] - SCALE["T"][0]) / SCALE["T"][1]
        x[k, :, :, 3] = (s["kappa"] - SCALE["kappa"][0]) / SCALE["kappa"][1]
        x[k, :, :, 4] = (s["radius"] / side - SCALE["R"][0]) / SCALE["R"][1]
        x[k, :, :, 5] = (rho0[k] - SCALE["rho"][0]) / SCALE["rho"][1]
    return x


def targets(rho0, rho, vel):
    """[n, side, side, 16]: (rho - rho0) / s_rho, u_x / s_u, u_y / s_u."""
    n, side = rho.shape[0], rho.shape[1]
    y = np.zeros((n, side, side, CP_OUT), dtype=np.float32)
    y[..., 0] = (rho - rho0) / SCALE["drho"]
    y[..., 1] = vel[:, 0] / SCALE["u"]
    y[..., 2] = vel[:, 1] / SCALE["u"]
    return y


def decode(pred, rho0):
    """Network output -> (rho, u) fields, numpy FP64."""
    rho = rho0 + SCALE["drho"] * pred[..., 0].astype(np.float64)
    u = np.stack([SCALE["u"] * pred[..., 1], SCALE["u"] * pred[..., 2]], axis=1).astype(np.float64)
    return rho, u


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

def problems(specs, side, storage=lbm.STORE_F64, tau=1.0):
    plist, rho0 = [], []
    for s in specs:
        g, l = lbm.lbm_coexistence(A_VDW, B_VDW, s["T"])
        plist.append(lbm.params(lattice=lbm.D2Q9, scheme=lbm.SCHEME_EQ, storage=storage,
                                shape=(side, side), T=s["T"], kappa=s["kappa"], tau=tau))
        rho0.append(inputs.tanh_drop((side, side), s["radius"], l, g, 2.0))
    return plist, np.stack(rho0)


def steady_states(specs, side, tol=1e-10, check_every=100, max_steps=60000, rho_init=None,
                  u_init=None, patience=0, grace=0):
    """Run a batch to its residual; returns (rho, vel [n,2,side,side], steps,
    residual, status, seconds)."""
    plist, rho0 = problems(specs, side)
    r_in = rho0 if rho_init is None else rho_init
    u_in = None
    if u_init is not None:
        u_in = np.zeros((3,) + (len(specs) * side * side,))
        u_in[0] = np.concatenate([u_init[k, 0].reshape(-1) for k in range(len(specs))])
        u_in[1] = np.concatenate([u_init[k, 1].reshape(-1) for k in range(len(specs))])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    bt = lbm.Batch(plist, list(r_in), u_in)
    steps, res, status = bt.run(tol, check_every, max_steps, patience, grace)
    secs = time.perf_counter() - t0
    rho, vel = bt.moments()
    bt.close()
    rho = rho.cpu().numpy().reshape(len(specs), side, side)
    vel = vel.cpu().numpy()[:2].reshape(2, len(specs), side, side).transpose(1, 0, 2, 3)
    return rho, vel, np.array(steps), np.array(res), np.array(status), secs


def mass_momentum_projection(rho_pred, u_pred, rho0):
    """Give each predicted field the exact mass of its cold start (uniform
    density shift) and zero total momentum (subtract the mass-weighted mean
    velocity), keeping the density inside (0, 1/b)."""
    rho = rho_pred + (rho0.sum(axis=(1, 2)) - rho_pred.sum(axis=(1, 2)))[:, None, None] / \
        (rho0.shape[1] * rho0.shape[2])
    rho = np.clip(rho, 1e-3, 0.99 / B_VDW)
    m = rho.sum(axis=(1, 2))
    u = u_pred.copy()
    for a in range(2):
        mean = (rho * u[:, a]).sum(axis=(1, 2)) / m
        u[:, a] -= mean[:, None, None]
    return rho, u


def d4_symmetrize(rho, u):
    """Average (rho [n, Y, X], u [n, 2, Y, X]) over the 8 symmetries of a
    square about the node (Y/2, X/2): the centred drop and its steady state
    are invariant under them, so this removes prediction errors that would
    seed the slow, symmetry-breaking shear modes of the periodic box."""
    fx = lambda a: np.roll(a[..., :, ::-1], 1, axis=-1)
    fy = lambda a: np.roll(a[..., ::-1, :], 1, axis=-2)
    tr = lambda a: np.swapaxes(a, -1, -2)
    ux, uy = u[:, 0], u[:, 1]
    imgs = [(rho, ux, uy), (fx(rho), -fx(ux), fx(uy)), (fy(rho), fy(ux), -fy(uy)),
            (fx(fy(rho)), -fx(fy(ux)), -fx(fy(uy)))]
    imgs += [(tr(r), tr(b), tr(a)) for r, a, b in imgs]
    r = sum(i[0] for i in imgs) / 8.0
    vx = sum(i[1] for i in imgs) / 8.0
    vy = sum(i[2] for i in imgs) / 8.0
    return r, np.stack([vx, vy], axis=1)


def warm_start(net, specs, side, tol=1e-10, check_every=100, max_steps=60000, patience=3,
               grace=500, symmetrize=True, with_velocity=True):
    """Predict, project, run with the rising-residual check; problems that
    diverge are rerun from the cold start.  Returns per-problem total steps,
    statuses, the fallback mask and wall seconds (inference included)."""
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, rho0 = problems(specs, side)
    x = torch.tensor(features(specs, side, rho0), device=net.dev)
    pred = net.predict(x).cpu().numpy()
    rho_p, u_p = decode(pred, rho0)
    # a non-finite prediction falls back to the cold initial field at once
    bad = ~(np.isfinite(rho_p).all(axis=(1, 2)) & np.isfinite(u_p).all(axis=(1, 2, 3)))
    rho_p[bad] = rho0[bad]
    u_p[bad] = 0.0
    if not with_velocity:
        u_p[:] = 0.0
    if symmetrize:
        rho_p, u_p = d4_symmetrize(rho_p, u_p)
    rho_p, u_p = mass_momentum_projection(rho_p, u_p, rho0)
    t_inf = time.perf_counter() - t0
    rho, vel, steps, res, status, secs = steady_states(specs, side, tol, check_every, max_steps,
                                                       rho_init=rho_p, u_init=u_p,
                                                       patience=patience, grace=grace)
    fallback = status == lbm.BATCH_DIVERGED
    total = steps.copy()
    secs_fb = 0.0
    if fallback.any():
        idx = np.nonzero(fallback)[0]
        sub = [specs[i] for i in idx]
        _, _, s2, r2, st2, secs_fb = steady_states(sub, side, tol, check_every, max_steps)
        total[idx] += s2
        status = status.copy()
        status[idx] = st2
    return dict(steps=total, status=status, fallback=fallback, seconds=t_inf + secs + secs_fb,
                inference_seconds=t_inf, rho=rho, vel=vel)


# ---- end-to-end experiment: generate, train, compare warm vs cold ----------

def _log(*a):
    print("[warmstart]", *a, flush=True)


def generate(nprob, side, seed, batch=512, tol=1e-10, max_steps=60000):
    """Steady states of `nprob` drops from the stable batched workload
    (side fixed), by the batched runner.  Returns (specs, x, y, steps)."""
    specs = inputs.stable_batch_specs(nprob, seed, side_lo=side, side_hi=side)
    xs, ys, steps, kept = [], [], [], []
    for i in range(0, nprob, batch):
        sub = specs[i:i + batch]
        rho, vel, st, res, status, secs = steady_states(sub, side, tol, 100, max_steps)
        _, rho0 = problems(sub, side)
        ok = status == lbm.BATCH_CONVERGED
        xs.append(features(sub, side, rho0)[ok])
        ys.append(targets(rho0, rho, vel)[ok])
        steps.append(st[ok])
        kept += [s for s, o in zip(sub, ok) if o]
        _log("generated %d/%d steady states (%.1f s, median steps %d, status counts %s)"
             % (i + len(sub), nprob, secs, int(np.median(st)), np.bincount(status, minlength=5).tolist()))
    return kept, np.concatenate(xs), np.concatenate(ys), np.concatenate(steps)


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


def run_experiment(n_train=2048, n_eval=512, side=128, epochs=20, seed_train=5, seed_eval=6,
                   tol=1e-10, out_json=None, weights=None):
    t0 = time.perf_counter()
    _, xtr, ytr, _ = generate(n_train, side, seed_train, tol=tol)
    t_gen = time.perf_counter() - t0
    net = WarmNet(seed=7)
    dev = net.dev
    xt, yt = torch.tensor(xtr, device=dev), torch.tensor(ytr, device=dev)
    t1 = time.perf_counter()
    losses = train(net, xt, yt, epochs)
    t_train = time.perf_counter() - t1
    del xt, yt
    specs = inputs.stable_batch_specs(n_eval, seed_eval, side_lo=side, side_hi=side)
    cold_rho, _, cold_steps, cold_res, cold_status, cold_secs = steady_states(specs, side, tol)
    _log("cold: %.2f s, median steps %d" % (cold_secs, int(np.median(cold_steps))))
    variants = {}
    for name, kw in (("raw", dict(symmetrize=False)), ("sym_rho_only", dict(with_velocity=False)),
                     ("sym", dict())):
        w = warm_start(net, specs, side, tol, **kw)
        _log("warm[%s]: %.2f s, median steps %d, fallbacks %d"
             % (name, w["seconds"], int(np.median(w["steps"])), int(w["fallback"].sum())))
        ok = (w["status"] == lbm.BATCH_CONVERGED) & (cold_status == lbm.BATCH_CONVERGED) & ~w["fallback"]
        diff = float(np.max(np.abs(w["rho"][ok] - cold_rho[ok]) / cold_rho[ok])) if ok.any() else None
        variants[name] = dict(seconds=w["seconds"], steps_median=float(np.median(w["steps"])),
                              steps_total=int(w["steps"].sum()), fallbacks=int(w["fallback"].sum()),
                              rho_rel_diff_vs_cold=diff)
    warm = w
    ratio = warm["steps"] / np.maximum(cold_steps, 1)
    res = dict(n_train=n_train, n_eval=n_eval, side=side, epochs=epochs, tol=tol,
               seconds_generate=t_gen, seconds_train=t_train, final_loss=losses[-1], losses=losses,
               cold_seconds=cold_secs, warm_seconds=warm["seconds"],
               warm_inference_seconds=warm["inference_seconds"],
               cold_steps_median=float(np.median(cold_steps)), warm_steps_median=float(np.median(warm["steps"])),
               cold_steps_total=int(cold_steps.sum()), warm_steps_total=int(warm["steps"].sum()),
               step_ratio_median=float(np.median(ratio)), step_ratio_p10=float(np.percentile(ratio, 10)),
               step_ratio_p90=float(np.percentile(ratio, 90)),
               cold_converged=int((cold_status == lbm.BATCH_CONVERGED).sum()),
               warm_converged=int((warm["status"] == lbm.BATCH_CONVERGED).sum()),
               fallbacks=int(warm["fallback"].sum()), variants=variants,
               zero_prediction_loss=float((ytr[..., :OUT_REAL].astype(np.float64) ** 2).mean()))
    if out_json:
        import json
        with open(out_json, "w") as fh:
            json.dump(res, fh, indent=1)
    if weights:
        np.savez(weights, *[a for W, b in net.numpy_params() for a in (W, b)])
    return res, net


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
    ap.add_argument("--weights", default=None)
    a = ap.parse_args()
    r, _ = run_experiment(a.train, a.eval, a.side, a.epochs, tol=a.tol, out_json=a.out, weights=a.weights)
    print(json.dumps({k: v for k, v in r.items() if k != "losses"}))
