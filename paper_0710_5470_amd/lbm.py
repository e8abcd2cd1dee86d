"""Thin Python binding of the C ABI in include/lbm.h (argument marshalling only).

Every function here has the name of the C entry point it calls.  Device
buffers are torch CUDA (HIP) tensors; the library computes everything in its
own HIP kernels and never falls back to the CPU: if the shared library is
missing, importing this module raises.

`Simulation` is a small convenience owner of one context and its workspace.
"""
import ctypes
import math
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("LBM_LIBRARY", os.path.join(_HERE, "_lib", "liblbm.so"))

D2Q9, D3Q19 = 9, 19
D3Q15 = 15  # binary stepper only (lattice comparison)
SCHEME_EQ, SCHEME_FORCE = 0, 1
STORE_F64, STORE_F32_SHIFTED = 0, 1
SHIFT_REST_EQ, SHIFT_WEIGHTS = 0, 1
COMPUTE_NATIVE, COMPUTE_F64 = 0, 1
OK, E_INVAL, E_NOMEM, E_DEVICE, E_NONFINITE, E_STATE, E_LIMIT = 0, -1, -2, -3, -4, -5, -6


class lbm_params(ctypes.Structure):
    _fields_ = [
        ("a", ctypes.c_double), ("b", ctypes.c_double), ("T", ctypes.c_double),
        ("kappa", ctypes.c_double), ("tau", ctypes.c_double),
        ("lattice", ctypes.c_int), ("scheme", ctypes.c_int), ("storage", ctypes.c_int),
        ("nx", ctypes.c_int), ("ny", ctypes.c_int), ("nz", ctypes.c_int),
        ("B", ctypes.c_double), ("D", ctypes.c_double), ("F", ctypes.c_double),
        ("wp_diag", ctypes.c_double), ("wt_diag", ctypes.c_double), ("wxx_diag", ctypes.c_double),
        ("galilean_lambda", ctypes.c_int), ("shift_mode", ctypes.c_int),
        ("rho_shift", ctypes.c_double),
        ("tile", ctypes.c_int), ("planes_per_block", ctypes.c_int),
        ("compute", ctypes.c_int),
    ]


class LBMError(RuntimeError):
    def __init__(self, code, where):
        self.code = code
        super().__init__("%s failed: %s (%d)" % (where, lbm_strerror(code), code))


if not os.path.exists(LIB_PATH):
    raise ImportError(
        "liblbm.so is not built (%s); run __graft_entry__.build() or "
        "python paper_0710_5470_amd/build.py" % LIB_PATH)

_L = ctypes.CDLL(LIB_PATH)
_vp, _dp, _ip = ctypes.c_void_p, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int)
_pp = ctypes.POINTER(lbm_params)
_sig = {
    "lbm_params_default": (None, [_pp]),
    "lbm_workspace_bytes": (ctypes.c_size_t, [_pp]),
    "lbm_init": (ctypes.c_int, [ctypes.POINTER(_vp), _pp, _vp, ctypes.c_size_t, _vp, _vp, _vp]),
    "lbm_step": (ctypes.c_int, [_vp, ctypes.c_longlong]),
    "lbm_moments": (ctypes.c_int, [_vp, _vp, _vp]),
    "lbm_max_spurious_u": (ctypes.c_int, [_vp, _dp]),
    "lbm_invariants": (ctypes.c_int, [_vp, _dp, _dp]),
    "lbm_step_observed": (ctypes.c_int, [_vp, ctypes.c_longlong, _dp, _dp]),
    "lbm_get_state": (ctypes.c_int, [_vp, _vp]),
    "lbm_set_state": (ctypes.c_int, [_vp, _vp]),
    "lbm_steps_done": (ctypes.c_longlong, [_vp]),
    "lbm_shift": (ctypes.c_int, [_vp, _dp]),
    "lbm_tile_count": (ctypes.c_int, [ctypes.c_int]),
    "lbm_tile_shape": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, _ip, _ip]),
    "lbm_set_launch": (ctypes.c_int, [_vp, ctypes.c_int, ctypes.c_int]),
    "lbm_get_launch": (ctypes.c_int, [_vp, _ip, _ip, _ip]),
    "lbm_destroy": (ctypes.c_int, [_vp]),
    "lbm_coexistence": (ctypes.c_int, [ctypes.c_double] * 3 + [_dp, _dp]),
    "lbm_strerror": (ctypes.c_char_p, [ctypes.c_int]),
    "lbm_batch_workspace_bytes": (ctypes.c_size_t, [ctypes.c_int, _pp]),
    "lbm_batch_init": (ctypes.c_int, [ctypes.POINTER(_vp), ctypes.c_int, _pp, _vp, ctypes.c_size_t,
                                      _vp, _vp, _vp]),
    "lbm_batch_step": (ctypes.c_int, [_vp, ctypes.c_longlong]),
    "lbm_batch_run": (ctypes.c_int, [_vp, ctypes.c_double, ctypes.c_int, ctypes.c_longlong,
                                     ctypes.c_int, ctypes.c_longlong,
                                     ctypes.POINTER(ctypes.c_longlong), _dp, _ip]),
    "lbm_batch_reactivate": (ctypes.c_int, [_vp]),
    "lbm_batch_max_spurious_u": (ctypes.c_int, [_vp, _dp]),
    "lbm_batch_moments": (ctypes.c_int, [_vp, _vp, _vp]),
    "lbm_batch_offset": (ctypes.c_longlong, [_vp, ctypes.c_int]),
    "lbm_batch_set_launch": (ctypes.c_int, [_vp, ctypes.c_int, ctypes.c_int]),
    "lbm_batch_get_launch": (ctypes.c_int, [_vp, _ip, _ip, _ip]),
    "lbm_batch_destroy": (ctypes.c_int, [_vp]),
    "lbm_stream_copy": (ctypes.c_int, [_vp, _vp, ctypes.c_size_t, _vp]),
}


class lbm_conv_shape(ctypes.Structure):
    _fields_ = [("nb", ctypes.c_int), ("h", ctypes.c_int), ("w", ctypes.c_int),
                ("cin", ctypes.c_int), ("cout", ctypes.c_int), ("cout_real", ctypes.c_int)]


_cs = ctypes.POINTER(lbm_conv_shape)
_sig.update({
    "lbm_net_conv3x3_fwd": (ctypes.c_int, [_cs, _vp, ctypes.c_int, _vp, _vp, _vp, _vp]),
    "lbm_net_conv3x3_bwd_data": (ctypes.c_int, [_cs, _vp, _vp, _vp, _vp, _vp]),
    "lbm_net_conv3x3_bwd_weight_workspace": (ctypes.c_size_t, [_cs]),
    "lbm_net_conv3x3_bwd_weight": (ctypes.c_int, [_cs, _vp, _vp, ctypes.c_int, _vp, _vp, _vp,
                                                  ctypes.c_size_t, _vp]),
    "lbm_net_conv3x3_bwd_weight_noalloc": (ctypes.c_int, [_cs, _vp, _vp, ctypes.c_int, _vp, _vp,
                                                          _vp]),
    "lbm_net_mse": (ctypes.c_int, [ctypes.c_longlong, ctypes.c_int, ctypes.c_int, _vp, _vp, _vp,
                                   _vp, _dp, _vp]),
    "lbm_net_adam": (ctypes.c_int, [ctypes.c_int, _vp, _vp, _vp, _vp, ctypes.c_double,
                                    ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                    ctypes.c_longlong, _vp]),
    "lbm_warm_features": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, _vp, _vp, ctypes.c_double,
                                         ctypes.c_double, _vp, _vp]),
    "lbm_warm_targets": (ctypes.c_int, [ctypes.c_longlong, _vp, _vp, _vp, ctypes.c_double,
                                        ctypes.c_double, _vp, _vp]),
    "lbm_warm_project": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, ctypes.c_int, _vp, _vp,
                                        ctypes.c_double, ctypes.c_double, ctypes.c_int, ctypes.c_int,
                                        ctypes.c_double, ctypes.c_double, _vp, _vp, _vp]),
})
class lbm_bin_params(ctypes.Structure):
    _fields_ = [
        ("phi_a", ctypes.c_double), ("phi_b", ctypes.c_double), ("kappa", ctypes.c_double),
        ("gamma", ctypes.c_double), ("tau", ctypes.c_double), ("tau_phi", ctypes.c_double),
        ("lattice", ctypes.c_int), ("nx", ctypes.c_int), ("ny", ctypes.c_int), ("nz", ctypes.c_int),
        ("wall", ctypes.c_int), ("scheme", ctypes.c_int),
        ("B", ctypes.c_double), ("D", ctypes.c_double),
        ("wp_diag", ctypes.c_double), ("wt_diag", ctypes.c_double), ("wxx_diag", ctypes.c_double),
        ("tile", ctypes.c_int), ("planes_per_block", ctypes.c_int),
    ]


_bp = ctypes.POINTER(lbm_bin_params)
_sig.update({
    "lbm_bin_params_default": (None, [_bp]),
    "lbm_bin_workspace_bytes": (ctypes.c_size_t, [_bp]),
    "lbm_bin_init": (ctypes.c_int, [ctypes.POINTER(_vp), _bp, _vp, ctypes.c_size_t, _vp, _vp, _vp,
                                    _vp]),
    "lbm_bin_step": (ctypes.c_int, [_vp, ctypes.c_longlong]),
    "lbm_bin_moments": (ctypes.c_int, [_vp, _vp, _vp, _vp, _vp]),
    "lbm_bin_max_spurious_u": (ctypes.c_int, [_vp, _dp]),
    "lbm_bin_invariants": (ctypes.c_int, [_vp, _dp, _dp, _dp]),
    "lbm_bin_get_state": (ctypes.c_int, [_vp, _vp, _vp]),
    "lbm_bin_set_state": (ctypes.c_int, [_vp, _vp, _vp]),
    "lbm_bin_steps_done": (ctypes.c_longlong, [_vp]),
    "lbm_bin_tile_count": (ctypes.c_int, [ctypes.c_int]),
    "lbm_bin_tile_shape": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, _ip, _ip]),
    "lbm_bin_set_launch": (ctypes.c_int, [_vp, ctypes.c_int, ctypes.c_int]),
    "lbm_bin_get_launch": (ctypes.c_int, [_vp, _ip, _ip, _ip]),
    "lbm_bin_destroy": (ctypes.c_int, [_vp]),
})
BATCH_RUNNING, BATCH_CONVERGED, BATCH_MAXSTEPS, BATCH_DIVERGED, BATCH_NONFINITE = 0, 1, 2, 3, 4
for _name, (_res, _args) in _sig.items():
    _f = getattr(_L, _name)
    _f.restype = _res
    _f.argtypes = _args

EXPORTED = tuple(_sig)


def _check(rc, where):
    if rc != OK:
        raise LBMError(rc, where)


def _ptr(t):
    if t is None:
        return None
    if not isinstance(t, torch.Tensor):
        return ctypes.c_void_p(int(t))
    if not t.is_cuda:
        raise ValueError("device tensor expected")
    if not t.is_contiguous():
        raise ValueError("contiguous tensor expected")
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


# ---- one function per C entry point -----------------------------------------

def lbm_strerror(code):
    return _L.lbm_strerror(int(code)).decode()


def lbm_params_default(**over):
    p = lbm_params()
    _L.lbm_params_default(ctypes.byref(p))
    for k, v in over.items():
        setattr(p, k, v)
    return p


def lbm_workspace_bytes(p):
    return int(_L.lbm_workspace_bytes(ctypes.byref(p)))


def lbm_init(p, workspace, rho0, u0=None, stream=None):
    ctx = ctypes.c_void_p()
    rc = _L.lbm_init(ctypes.byref(ctx), ctypes.byref(p), _ptr(workspace), workspace.numel() *
                     workspace.element_size(), _stream(stream), _ptr(rho0), _ptr(u0))
    _check(rc, "lbm_init")
    return ctx


def lbm_step(ctx, nsteps):
    _check(_L.lbm_step(ctx, int(nsteps)), "lbm_step")


def lbm_moments(ctx, rho=None, vel=None):
    _check(_L.lbm_moments(ctx, _ptr(rho), _ptr(vel)), "lbm_moments")


def lbm_max_spurious_u(ctx):
    out = ctypes.c_double()
    _check(_L.lbm_max_spurious_u(ctx, ctypes.byref(out)), "lbm_max_spurious_u")
    return out.value


def lbm_invariants(ctx):
    m = ctypes.c_double()
    mom = (ctypes.c_double * 3)()
    _check(_L.lbm_invariants(ctx, ctypes.byref(m), mom), "lbm_invariants")
    return m.value, [mom[0], mom[1], mom[2]]


def lbm_step_observed(ctx, nsteps):
    res, vmax = ctypes.c_double(), ctypes.c_double()
    rc = _L.lbm_step_observed(ctx, int(nsteps), ctypes.byref(res), ctypes.byref(vmax))
    if rc not in (OK, E_NONFINITE):
        _check(rc, "lbm_step_observed")
    return res.value, vmax.value, rc == OK


def lbm_get_state(ctx, f):
    _check(_L.lbm_get_state(ctx, _ptr(f)), "lbm_get_state")


def lbm_set_state(ctx, f):
    _check(_L.lbm_set_state(ctx, _ptr(f)), "lbm_set_state")


def lbm_steps_done(ctx):
    return int(_L.lbm_steps_done(ctx))


def lbm_shift(ctx, q):
    out = (ctypes.c_double * q)()
    _check(_L.lbm_shift(ctx, out), "lbm_shift")
    return list(out)


def lbm_tile_count(lattice):
    return int(_L.lbm_tile_count(int(lattice)))


def lbm_tile_shape(lattice, k):
    tx, ty = ctypes.c_int(), ctypes.c_int()
    _check(_L.lbm_tile_shape(int(lattice), int(k), ctypes.byref(tx), ctypes.byref(ty)),
           "lbm_tile_shape")
    return tx.value, ty.value


def lbm_set_launch(ctx, tile=-1, planes=0):
    _check(_L.lbm_set_launch(ctx, int(tile), int(planes)), "lbm_set_launch")


def lbm_get_launch(ctx):
    t, p, w = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
    _check(_L.lbm_get_launch(ctx, ctypes.byref(t), ctypes.byref(p), ctypes.byref(w)),
           "lbm_get_launch")
    return t.value, p.value, w.value


def lbm_destroy(ctx):
    _check(_L.lbm_destroy(ctx), "lbm_destroy")


def lbm_coexistence(a, b, T):
    g, l = ctypes.c_double(), ctypes.c_double()
    _check(_L.lbm_coexistence(float(a), float(b), float(T), ctypes.byref(g), ctypes.byref(l)),
           "lbm_coexistence")
    return g.value, l.value


def lbm_stream_copy(src, dst, nbytes, stream=None):
    """Streaming device copy of nbytes (measurement of the HBM ceiling)."""
    _check(_L.lbm_stream_copy(_ptr(src), _ptr(dst), int(nbytes), _stream(stream)), "lbm_stream_copy")


def _params_array(plist):
    arr = (lbm_params * len(plist))()
    for k, p in enumerate(plist):
        arr[k] = p
    return arr


def lbm_batch_workspace_bytes(plist):
    return int(_L.lbm_batch_workspace_bytes(len(plist), _params_array(plist)))


def lbm_batch_init(plist, workspace, rho0, u0=None, stream=None):
    if stream is None:
        raise ValueError("a batch needs a non-default stream (graph capture)")
    bt = ctypes.c_void_p()
    rc = _L.lbm_batch_init(ctypes.byref(bt), len(plist), _params_array(plist), _ptr(workspace),
                           workspace.numel() * workspace.element_size(), _stream(stream),
                           _ptr(rho0), _ptr(u0))
    _check(rc, "lbm_batch_init")
    return bt


def lbm_batch_step(bt, nsteps):
    _check(_L.lbm_batch_step(bt, int(nsteps)), "lbm_batch_step")


def lbm_batch_run(bt, nprob, tol, check_every, max_steps, patience=0, grace=0):
    steps = (ctypes.c_longlong * nprob)()
    res = (ctypes.c_double * nprob)()
    status = (ctypes.c_int * nprob)()
    _check(_L.lbm_batch_run(bt, float(tol), int(check_every), int(max_steps), int(patience),
                            int(grace), steps, res, status), "lbm_batch_run")
    return list(steps), list(res), list(status)


def lbm_batch_moments(bt, rho, vel):
    _check(_L.lbm_batch_moments(bt, _ptr(rho), _ptr(vel)), "lbm_batch_moments")


def lbm_batch_offset(bt, k):
    return int(_L.lbm_batch_offset(bt, int(k)))


def lbm_batch_set_launch(bt, tile=-1, planes=0):
    _check(_L.lbm_batch_set_launch(bt, int(tile), int(planes)), "lbm_batch_set_launch")


def lbm_batch_get_launch(bt):
    t, p, w = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
    _check(_L.lbm_batch_get_launch(bt, ctypes.byref(t), ctypes.byref(p), ctypes.byref(w)),
           "lbm_batch_get_launch")
    return t.value, p.value, w.value


def lbm_batch_max_spurious_u(bt, nprob):
    """Per-problem max |u| (or |v|); inf for a problem whose state is not
    finite."""
    out = (ctypes.c_double * nprob)()
    rc = _L.lbm_batch_max_spurious_u(bt, out)
    if rc not in (OK, E_NONFINITE):
        _check(rc, "lbm_batch_max_spurious_u")
    return list(out)


def lbm_batch_reactivate(bt):
    _check(_L.lbm_batch_reactivate(bt), "lbm_batch_reactivate")


def lbm_batch_destroy(bt):
    _check(_L.lbm_batch_destroy(bt), "lbm_batch_destroy")


def _shape(nb, h, w, cin, cout, cout_real=None):
    return lbm_conv_shape(nb, h, w, cin, cout, cout if cout_real is None else cout_real)


def lbm_net_conv3x3_fwd(shape, x, relu_in, w, b, out, stream=None):
    _check(_L.lbm_net_conv3x3_fwd(ctypes.byref(shape), _ptr(x), int(relu_in), _ptr(w), _ptr(b),
                                  _ptr(out), _stream(stream)), "lbm_net_conv3x3_fwd")


def lbm_net_conv3x3_bwd_data(shape, dout, w, zin, din, stream=None):
    _check(_L.lbm_net_conv3x3_bwd_data(ctypes.byref(shape), _ptr(dout), _ptr(w), _ptr(zin),
                                       _ptr(din), _stream(stream)), "lbm_net_conv3x3_bwd_data")


def lbm_net_conv3x3_bwd_weight_workspace(shape):
    return int(_L.lbm_net_conv3x3_bwd_weight_workspace(ctypes.byref(shape)))


def lbm_net_conv3x3_bwd_weight(shape, dout, x, relu_in, dw, db, ws, stream=None):
    _check(_L.lbm_net_conv3x3_bwd_weight(ctypes.byref(shape), _ptr(dout), _ptr(x), int(relu_in),
                                         _ptr(dw), _ptr(db), _ptr(ws),
                                         ws.numel() * ws.element_size(), _stream(stream)),
           "lbm_net_conv3x3_bwd_weight")


def lbm_net_conv3x3_bwd_weight_noalloc(shape, dout, x, relu_in, dw, db, stream=None):
    """The weight gradient with the partials in the library's fixed device
    scratch (no workspace argument, nothing allocated)."""
    _check(_L.lbm_net_conv3x3_bwd_weight_noalloc(ctypes.byref(shape), _ptr(dout), _ptr(x),
                                                 int(relu_in), _ptr(dw), _ptr(db), _stream(stream)),
           "lbm_net_conv3x3_bwd_weight_noalloc")


def lbm_net_mse(npix, c, creal, pred, target, grad, part, want_loss=True, stream=None):
    loss = ctypes.c_double()
    _check(_L.lbm_net_mse(int(npix), int(c), int(creal), _ptr(pred), _ptr(target), _ptr(grad),
                          _ptr(part), ctypes.byref(loss) if want_loss else None, _stream(stream)),
           "lbm_net_mse")
    return loss.value if want_loss else None


def lbm_net_adam(p, g, m, v, lr, t, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
    _check(_L.lbm_net_adam(p.numel(), _ptr(p), _ptr(g), _ptr(m), _ptr(v), float(lr), float(beta1),
                           float(beta2), float(eps), int(t), _stream(stream)), "lbm_net_adam")


def lbm_warm_features(nprob, side, consts, rho0, rho_mean, rho_scale, x, stream=None):
    _check(_L.lbm_warm_features(int(nprob), int(side), _ptr(consts), _ptr(rho0), float(rho_mean),
                                float(rho_scale), _ptr(x), _stream(stream)), "lbm_warm_features")


def lbm_warm_targets(rho, rho0, vel, s_rho, s_u, y, stream=None):
    _check(_L.lbm_warm_targets(int(rho.numel()), _ptr(rho), _ptr(rho0), _ptr(vel), float(s_rho),
                               float(s_u), _ptr(y), _stream(stream)), "lbm_warm_targets")


def lbm_warm_project(nprob, side, cpad, pred, rho0, s_rho, s_u, with_velocity, symmetrize, rho_lo,
                     rho_hi, rho, u, stream=None):
    _check(_L.lbm_warm_project(int(nprob), int(side), int(cpad), _ptr(pred), _ptr(rho0), float(s_rho),
                               float(s_u), int(bool(with_velocity)), int(bool(symmetrize)),
                               float(rho_lo), float(rho_hi), _ptr(rho), _ptr(u), _stream(stream)),
           "lbm_warm_project")


# ---- convenience owners -----------------------------------------------------

class Batch:
    """Owns one batch, its workspace and a non-default stream.  rho0 / u0:
    lists of per-problem arrays (or one concatenated array / tensor)."""

    def __init__(self, plist, rho0, u0=None, device="cuda"):
        self.plist = list(plist)
        self.nprob = len(self.plist)
        self.device = torch.device(device)
        self.stream = torch.cuda.Stream(device=self.device)
        nbytes = lbm_batch_workspace_bytes(self.plist)
        if nbytes == 0:
            raise LBMError(E_INVAL, "lbm_batch_workspace_bytes")
        self.sizes = [p.nx * p.ny * p.nz for p in self.plist]
        self.ntot = sum(self.sizes)
        r = self._concat(rho0, 1)
        u = self._concat(u0, 3) if u0 is not None else None
        with torch.cuda.stream(self.stream):
            self.ws = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self.stream.wait_stream(torch.cuda.current_stream())
        self.bt = lbm_batch_init(self.plist, self.ws, r, u, self.stream)
        self.offsets = [lbm_batch_offset(self.bt, k) for k in range(self.nprob + 1)]

    def _concat(self, a, ncomp):
        if isinstance(a, (list, tuple)):
            parts = [torch.as_tensor(x, dtype=torch.float64).reshape(ncomp, -1) for x in a]
            t = torch.cat(parts, dim=1)
        else:
            t = torch.as_tensor(a, dtype=torch.float64).reshape(ncomp, -1)
        assert t.shape[1] == self.ntot
        return t.reshape(-1).to(self.device).contiguous() if ncomp == 1 else \
            t.to(self.device).contiguous()

    def run(self, tol, check_every=100, max_steps=10 ** 6, patience=0, grace=0):
        return lbm_batch_run(self.bt, self.nprob, tol, check_every, max_steps, patience, grace)

    def step(self, n):
        lbm_batch_step(self.bt, n)

    def reactivate(self):
        lbm_batch_reactivate(self.bt)

    def max_spurious_u(self):
        return lbm_batch_max_spurious_u(self.bt, self.nprob)

    def moments(self):
        with torch.cuda.stream(self.stream):
            rho = torch.empty(self.ntot, dtype=torch.float64, device=self.device)
            vel = torch.empty(3, self.ntot, dtype=torch.float64, device=self.device)
        lbm_batch_moments(self.bt, rho, vel)
        self.stream.synchronize()
        return rho, vel

    def split(self, field):
        """Per-problem views of a concatenated field ([n] or [3][n])."""
        return [field[..., self.offsets[k]:self.offsets[k + 1]] for k in range(self.nprob)]

    def set_launch(self, tile=-1, planes=0):
        lbm_batch_set_launch(self.bt, tile, planes)

    def launch(self):
        return lbm_batch_get_launch(self.bt)

    def close(self):
        if self.bt is not None:
            self.stream.synchronize()
            lbm_batch_destroy(self.bt)
            self.bt = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

class Simulation:
    """Owns one context and its workspace.  rho0 / u0 may be numpy arrays or
    torch tensors ([nz][ny][nx] or [ny][nx], and [3][...] for u0)."""

    def __init__(self, params, rho0, u0=None, device="cuda", stream=None):
        self.p = params
        self.q = params.lattice
        self.n = params.nx * params.ny * params.nz
        self.device = torch.device(device)
        nbytes = lbm_workspace_bytes(params)
        if nbytes == 0:
            raise LBMError(E_INVAL, "lbm_workspace_bytes")
        self.ws = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        r = torch.as_tensor(rho0, dtype=torch.float64).reshape(-1).to(self.device).contiguous()
        u = None
        if u0 is not None:
            u = torch.as_tensor(u0, dtype=torch.float64).reshape(3, -1).to(self.device).contiguous()
        self.stream = stream
        self.ctx = lbm_init(params, self.ws, r, u, stream)

    def step(self, n):
        lbm_step(self.ctx, n)

    def moments(self):
        rho = torch.empty(self.n, dtype=torch.float64, device=self.device)
        vel = torch.empty(3, self.n, dtype=torch.float64, device=self.device)
        lbm_moments(self.ctx, rho, vel)
        return rho, vel

    def max_spurious_u(self):
        return lbm_max_spurious_u(self.ctx)

    def invariants(self):
        return lbm_invariants(self.ctx)

    def step_observed(self, n):
        return lbm_step_observed(self.ctx, n)

    def get_state(self):
        f = torch.empty(self.q, self.n, dtype=torch.float64, device=self.device)
        lbm_get_state(self.ctx, f)
        return f

    def set_state(self, f):
        f = torch.as_tensor(f, dtype=torch.float64).reshape(self.q, self.n).to(self.device)
        lbm_set_state(self.ctx, f.contiguous())

    def shift(self):
        return lbm_shift(self.ctx, self.q)

    def set_launch(self, tile=-1, planes=0):
        lbm_set_launch(self.ctx, tile, planes)

    def launch(self):
        return lbm_get_launch(self.ctx)

    @property
    def steps_done(self):
        return lbm_steps_done(self.ctx)

    def close(self):
        if self.ctx is not None:
            lbm_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def params(lattice=D2Q9, scheme=SCHEME_EQ, storage=STORE_F64, shape=(64, 64), a=9 / 49,
           b=2 / 21, T=0.56, kappa=0.025, tau=1.0, **over):
    """lbm_params from keyword arguments; shape = (nx, ny[, nz])."""
    nz = shape[2] if len(shape) > 2 else 1
    p = lbm_params_default(a=a, b=b, T=T, kappa=kappa, tau=tau, lattice=lattice, scheme=scheme,
                           storage=storage, nx=shape[0], ny=shape[1], nz=nz)
    for k, v in over.items():
        setattr(p, k, v)
    return p


NAN = math.nan


# ---- binary fluid -------------------------------------------------------------

def lbm_bin_params_default(**over):
    p = lbm_bin_params()
    _L.lbm_bin_params_default(ctypes.byref(p))
    for k, v in over.items():
        setattr(p, k, v)
    return p


def lbm_bin_workspace_bytes(p):
    return int(_L.lbm_bin_workspace_bytes(ctypes.byref(p)))


def lbm_bin_init(p, workspace, rho0, phi0, u0=None, stream=None):
    ctx = ctypes.c_void_p()
    rc = _L.lbm_bin_init(ctypes.byref(ctx), ctypes.byref(p), _ptr(workspace),
                         workspace.numel() * workspace.element_size(), _stream(stream), _ptr(rho0),
                         _ptr(phi0), _ptr(u0))
    _check(rc, "lbm_bin_init")
    return ctx


def lbm_bin_step(ctx, nsteps):
    _check(_L.lbm_bin_step(ctx, int(nsteps)), "lbm_bin_step")


def lbm_bin_moments(ctx, rho=None, phi=None, vel=None, mu=None):
    _check(_L.lbm_bin_moments(ctx, _ptr(rho), _ptr(phi), _ptr(vel), _ptr(mu)), "lbm_bin_moments")


def lbm_bin_max_spurious_u(ctx):
    out = ctypes.c_double()
    _check(_L.lbm_bin_max_spurious_u(ctx, ctypes.byref(out)), "lbm_bin_max_spurious_u")
    return out.value


def lbm_bin_invariants(ctx):
    m, ph = ctypes.c_double(), ctypes.c_double()
    mom = (ctypes.c_double * 3)()
    _check(_L.lbm_bin_invariants(ctx, ctypes.byref(m), ctypes.byref(ph), mom), "lbm_bin_invariants")
    return m.value, ph.value, list(mom)


def lbm_bin_get_state(ctx, f, g):
    _check(_L.lbm_bin_get_state(ctx, _ptr(f), _ptr(g)), "lbm_bin_get_state")


def lbm_bin_set_state(ctx, f, g):
    _check(_L.lbm_bin_set_state(ctx, _ptr(f), _ptr(g)), "lbm_bin_set_state")


def lbm_bin_steps_done(ctx):
    return int(_L.lbm_bin_steps_done(ctx))


def lbm_bin_tile_count(lattice):
    return int(_L.lbm_bin_tile_count(int(lattice)))


def lbm_bin_tile_shape(lattice, k):
    tx, ty = ctypes.c_int(), ctypes.c_int()
    _check(_L.lbm_bin_tile_shape(int(lattice), int(k), ctypes.byref(tx), ctypes.byref(ty)),
           "lbm_bin_tile_shape")
    return tx.value, ty.value


def lbm_bin_set_launch(ctx, tile=-1, planes=0):
    _check(_L.lbm_bin_set_launch(ctx, int(tile), int(planes)), "lbm_bin_set_launch")


def lbm_bin_get_launch(ctx):
    t, c, w = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
    _check(_L.lbm_bin_get_launch(ctx, ctypes.byref(t), ctypes.byref(c), ctypes.byref(w)),
           "lbm_bin_get_launch")
    return t.value, c.value, w.value


def lbm_bin_destroy(ctx):
    _check(_L.lbm_bin_destroy(ctx), "lbm_bin_destroy")


def bin_params(lattice=D2Q9, shape=(64, 64), phi_a=-0.02, phi_b=0.02, kappa=0.04, gamma=1.0,
               tau=1.0, tau_phi=1.0, **over):
    """lbm_bin_params from keyword arguments; shape = (nx, ny[, nz])."""
    nz = shape[2] if len(shape) > 2 else 1
    return lbm_bin_params_default(phi_a=phi_a, phi_b=phi_b, kappa=kappa, gamma=gamma, tau=tau,
                                  tau_phi=tau_phi, lattice=lattice, nx=shape[0], ny=shape[1],
                                  nz=nz, **over)


class BinarySimulation:
    """Owns one binary-fluid context and its workspace (fields as numpy
    arrays or torch tensors, x fastest)."""

    def __init__(self, params, rho0, phi0, u0=None, device="cuda", stream=None):
        self.p = params
        self.q = params.lattice
        self.n = params.nx * params.ny * params.nz
        self.device = torch.device(device)
        nbytes = lbm_bin_workspace_bytes(params)
        if nbytes == 0:
            raise LBMError(E_INVAL, "lbm_bin_workspace_bytes")
        self.ws = torch.empty(nbytes, dtype=torch.uint8, device=self.device)

        def dev(a, ncomp=None):
            t = torch.as_tensor(a, dtype=torch.float64)
            t = t.reshape(-1) if ncomp is None else t.reshape(ncomp, -1)
            return t.to(self.device).contiguous()

        self.ctx = lbm_bin_init(params, self.ws, dev(rho0), dev(phi0),
                                None if u0 is None else dev(u0, 3), stream)

    def step(self, n):
        lbm_bin_step(self.ctx, n)

    def moments(self):
        """(rho[n], phi[n], u[3][n], mu[n])."""
        t = [torch.empty(s, dtype=torch.float64, device=self.device)
             for s in (self.n, self.n, (3, self.n), self.n)]
        lbm_bin_moments(self.ctx, *t)
        return tuple(t)

    def max_spurious_u(self):
        return lbm_bin_max_spurious_u(self.ctx)

    def invariants(self):
        return lbm_bin_invariants(self.ctx)

    def get_state(self):
        f = torch.empty(self.q, self.n, dtype=torch.float64, device=self.device)
        g = torch.empty_like(f)
        lbm_bin_get_state(self.ctx, f, g)
        return f, g

    def set_state(self, f, g):
        f = torch.as_tensor(f, dtype=torch.float64).reshape(self.q, self.n).to(self.device)
        g = torch.as_tensor(g, dtype=torch.float64).reshape(self.q, self.n).to(self.device)
        lbm_bin_set_state(self.ctx, f.contiguous(), g.contiguous())

    def set_launch(self, tile=-1, planes=0):
        lbm_bin_set_launch(self.ctx, tile, planes)

    def launch(self):
        return lbm_bin_get_launch(self.ctx)

    @property
    def steps_done(self):
        return lbm_bin_steps_done(self.ctx)

    def close(self):
        if self.ctx is not None:
            lbm_bin_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
