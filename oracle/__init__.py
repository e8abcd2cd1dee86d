"""TEST INFRASTRUCTURE ONLY: the FP64 CPU oracle for the free-energy LBM step.

Only tests, the smoke check and the benchmark's CPU-baseline leg may import
this package.  It shares no code with the GPU library.  Python-side helpers
(thermodynamics, observables) live in ``oracle.thermo``; the stepper itself
is plain C in ``oracle.c`` (see its header for the paper passages it follows).
"""
import ctypes
import os

import numpy as np

from . import build as _build

_lib = None


class OrcParams(ctypes.Structure):
    _fields_ = [
        ("q", ctypes.c_int), ("scheme", ctypes.c_int),
        ("nx", ctypes.c_int), ("ny", ctypes.c_int), ("nz", ctypes.c_int),
        ("lambda_on", ctypes.c_int),
        ("a", ctypes.c_double), ("b", ctypes.c_double), ("T", ctypes.c_double),
        ("kappa", ctypes.c_double), ("tau", ctypes.c_double),
        ("B", ctypes.c_double), ("D", ctypes.c_double), ("F", ctypes.c_double),
        ("wp_d", ctypes.c_double), ("wt_d", ctypes.c_double), ("wxx_d", ctypes.c_double),
    ]


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_build.LIB):
            _build.build()
        L = ctypes.CDLL(_build.LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int)
        pp = ctypes.POINTER(OrcParams)
        L.orc_run.argtypes = [pp, dp, ctypes.c_int]
        L.orc_run.restype = ctypes.c_int
        L.orc_init.argtypes = [pp, dp, dp, dp]
        L.orc_observe.argtypes = [pp, dp, dp, dp]
        L.orc_feq_site.argtypes = [pp, ctypes.c_double, dp, dp, ctypes.c_double, dp]
        L.orc_force_site.argtypes = [pp, dp, dp, dp]
        L.orc_derivatives.argtypes = [pp, dp, dp, dp]
        L.orc_body_force.argtypes = [pp, dp, dp]
        L.orc_collide_sites.argtypes = [pp, dp, ctypes.c_int, ip, dp]
        L.orc_totals.argtypes = [pp, dp, dp, dp]
        L.orc_tables.argtypes = [pp, ip, dp, dp, dp, dp]
        L.orc_stencils.argtypes = [pp] + [dp] * 7
        L.orc_p0.argtypes = [ctypes.c_double] * 4
        L.orc_p0.restype = ctypes.c_double
        L.orc_cs2.argtypes = [ctypes.c_double] * 4
        L.orc_cs2.restype = ctypes.c_double
        L.orc_set_threads.argtypes = [ctypes.c_int]
        L.orc_max_threads.restype = ctypes.c_int
        _lib = L
    return _lib


# Paper optimum parameters: B = 1/12, D = 1/6, F = 1/12 (Eq. (best) and the
# forcing section); w^p_5-8 = w^t_5-8 = 1/12, w^xx_5-8 = -1/24 (summary).
OPTIMUM = dict(B=1.0 / 12.0, D=1.0 / 6.0, F=1.0 / 12.0,
               wp_d=1.0 / 12.0, wt_d=1.0 / 12.0, wxx_d=-1.0 / 24.0)


# D3Q15 (lattice comparison only): corner stencil coefficients with an
# isotropic leading error (B = 1/24, D = 1/12), corner w^p and w^t weights
# 1/24 (the same isotropy), and the corner w^xx weight c (wxx_d); the
# second-moment conditions fix the face weights from the corner ones.
D3Q15_DEFAULT = dict(B=1.0 / 24.0, D=1.0 / 12.0, wp_d=1.0 / 24.0, wt_d=1.0 / 24.0, wxx_d=0.0)


def params(q=9, scheme=0, shape=(64, 64), a=9 / 49, b=2 / 21, T=0.5, kappa=0.01,
           tau=1.0, lambda_on=1, **over):
    """shape is (nx, ny) for D2Q9 or (nx, ny, nz) for D3Q19."""
    nx, ny = shape[0], shape[1]
    nz = shape[2] if len(shape) > 2 else 1
    kw = dict(OPTIMUM)
    if q == 15:
        kw.update(D3Q15_DEFAULT)
    kw.update(over)
    return OrcParams(q, scheme, nx, ny, nz, lambda_on, a, b, T, kappa, tau,
                     kw["B"], kw["D"], kw["F"], kw["wp_d"], kw["wt_d"], kw["wxx_d"])


def _p(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _n(p):
    return p.nx * p.ny * p.nz


def _fld(a, p):
    """Flatten a field given as [nz][ny][nx] or [ny][nx] (x fastest)."""
    a = np.ascontiguousarray(a, dtype=np.float64).reshape(-1)
    assert a.size == _n(p)
    return a


def init(p, rho0, u0=None):
    """f_i = f_i^eq(rho0, rho0 u0) of the active scheme; returns f[q][n]."""
    rho0 = _fld(rho0, p)
    f = np.empty((p.q, _n(p)))
    if u0 is not None:
        u0 = np.ascontiguousarray(u0, dtype=np.float64).reshape(3, -1)
        lib().orc_init(ctypes.byref(p), _p(rho0), _p(u0), _p(f))
    else:
        lib().orc_init(ctypes.byref(p), _p(rho0), None, _p(f))
    return f


def run(p, f, nsteps):
    """Advance f[q][n] (copy) by nsteps; returns the new array."""
    f = np.ascontiguousarray(f, dtype=np.float64).copy()
    rc = lib().orc_run(ctypes.byref(p), _p(f), int(nsteps))
    if rc != 0:
        raise ValueError("oracle rejected the parameters")
    return f


def observe(p, f):
    """(rho[n], vel[3][n]): u for the equilibrium scheme, v for the force scheme."""
    f = np.ascontiguousarray(f, dtype=np.float64)
    rho = np.empty(_n(p))
    vel = np.empty((3, _n(p)))
    lib().orc_observe(ctypes.byref(p), _p(f), _p(rho), _p(vel))
    return rho, vel


def feq_site(p, rho, j, grad, lap):
    out = np.empty(p.q)
    j = np.ascontiguousarray(j, dtype=np.float64)
    grad = np.ascontiguousarray(grad, dtype=np.float64)
    lib().orc_feq_site(ctypes.byref(p), float(rho), _p(j), _p(grad), float(lap), _p(out))
    return out


def force_site(p, u, g):
    out = np.empty(p.q)
    u = np.ascontiguousarray(u, dtype=np.float64)
    g = np.ascontiguousarray(g, dtype=np.float64)
    lib().orc_force_site(ctypes.byref(p), _p(u), _p(g), _p(out))
    return out


def derivatives(p, rho):
    rho = _fld(rho, p)
    grad = np.empty((3, _n(p)))
    lap = np.empty(_n(p))
    lib().orc_derivatives(ctypes.byref(p), _p(rho), _p(grad), _p(lap))
    return grad, lap


def body_force(p, rho):
    rho = _fld(rho, p)
    g = np.empty((3, _n(p)))
    lib().orc_body_force(ctypes.byref(p), _p(rho), _p(g))
    return g


def collide_sites(p, f, xyz):
    """Post-collision populations f*_i(r) at sites xyz[k] = (x, y, z)."""
    f = np.ascontiguousarray(f, dtype=np.float64)
    xyz = np.ascontiguousarray(xyz, dtype=np.int32).reshape(-1, 3)
    out = np.empty((xyz.shape[0], p.q))
    lib().orc_collide_sites(ctypes.byref(p), _p(f), xyz.shape[0],
                            xyz.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), _p(out))
    return out


def totals(p, f):
    f = np.ascontiguousarray(f, dtype=np.float64)
    m = ctypes.c_double()
    mom = np.empty(3)
    lib().orc_totals(ctypes.byref(p), _p(f), ctypes.byref(m), _p(mom))
    return m.value, mom


def tables(p):
    q = p.q
    e = np.empty(q * 3, dtype=np.int32)
    w, wp, wt = np.empty(q), np.empty(q), np.empty(q)
    wm = np.empty(6 * q)
    lib().orc_tables(ctypes.byref(p), e.ctypes.data_as(ctypes.POINTER(ctypes.c_int)),
                     _p(w), _p(wp), _p(wt), _p(wm))
    return dict(e=e.reshape(q, 3), w=w, wp=wp, wt=wt, wm=wm.reshape(6, q))


def stencils(p):
    arrs = [np.empty((3, 3, 3)) for _ in range(7)]
    lib().orc_stencils(ctypes.byref(p), *[_p(a) for a in arrs])
    return dict(zip(["gx", "gy", "gz", "lap", "fx", "fy", "fz"], arrs))


def p0(a, b, T, rho):
    return lib().orc_p0(a, b, T, rho)


def cs2(a, b, T, rho):
    return lib().orc_cs2(a, b, T, rho)


def set_threads(n):
    """Threads of the oracle's OpenMP loops (no effect on results)."""
    lib().orc_set_threads(int(n))


def max_threads():
    return int(lib().orc_max_threads())


# ---- binary fluid ------------------------------------------------------------

class OrcBinParams(ctypes.Structure):
    _fields_ = [("base", OrcParams), ("phi_a", ctypes.c_double), ("phi_b", ctypes.c_double),
                ("gamma", ctypes.c_double), ("tau_phi", ctypes.c_double), ("wall", ctypes.c_int)]


def bin_params(q=9, shape=(64, 64), phi_a=-0.02, phi_b=0.02, kappa=0.04, tau=1.0,
               tau_phi=1.0, gamma=1.0, wall=0, scheme=0, **over):
    """Symmetric binary fluid: bulk free energy phi_a phi^2/2 + phi_b phi^4/4
    plus kappa |grad phi|^2 / 2, ideal-gas carrier rho/3.  wall = 1 bounds
    the last axis (z in 3D, y in 2D) by two halfway bounce-back walls;
    scheme = 1 is the forcing scheme (with or without walls; not on D3Q15)."""
    base = params(q=q, scheme=scheme, shape=shape, a=0.0, b=0.0, T=0.0, kappa=kappa, tau=tau,
                  lambda_on=0, **over)
    return OrcBinParams(base, phi_a, phi_b, gamma, tau_phi, int(wall))


def _bin_lib():
    L = lib()
    if not getattr(L, "_bin_ready", False):
        dp = ctypes.POINTER(ctypes.c_double)
        bp = ctypes.POINTER(OrcBinParams)
        L.orc_bin_init.argtypes = [bp, dp, dp, dp, dp, dp]
        L.orc_bin_init.restype = ctypes.c_int
        L.orc_bin_run.argtypes = [bp, dp, dp, ctypes.c_int]
        L.orc_bin_run.restype = ctypes.c_int
        L.orc_bin_observe.argtypes = [bp, dp, dp, dp, dp, dp, dp]
        L.orc_bin_observe.restype = ctypes.c_int
        L.orc_bin_totals.argtypes = [bp, dp, dp, dp, dp, dp]
        L.orc_bin_totals.restype = ctypes.c_int
        L.orc_bin_feq_site.argtypes = [bp, ctypes.c_double, dp, ctypes.c_double, dp,
                                       ctypes.c_double, dp]
        L.orc_bin_geq_site.argtypes = [bp, ctypes.c_double, dp, ctypes.c_double, dp]
        L.orc_bin_collide_sites.argtypes = [bp, dp, dp, ctypes.c_int,
                                            ctypes.POINTER(ctypes.c_int), dp, dp]
        L.orc_bin_collide_sites.restype = ctypes.c_int
        L._bin_ready = True
    return L


def _bn(bp):
    return bp.base.nx * bp.base.ny * bp.base.nz


def bin_init(bp, rho0, phi0, u0=None):
    """(f, g) [q][n] at the binary equilibria of rho0, phi0, u0."""
    n = _bn(bp)
    rho0 = np.ascontiguousarray(rho0, dtype=np.float64).reshape(-1)
    phi0 = np.ascontiguousarray(phi0, dtype=np.float64).reshape(-1)
    assert rho0.size == n and phi0.size == n
    f = np.empty((bp.base.q, n))
    g = np.empty((bp.base.q, n))
    u = None if u0 is None else np.ascontiguousarray(u0, dtype=np.float64).reshape(3, n)
    rc = _bin_lib().orc_bin_init(ctypes.byref(bp), _p(rho0), _p(phi0),
                                 None if u is None else _p(u), _p(f), _p(g))
    if rc != 0:
        raise ValueError("oracle rejected the parameters")
    return f, g


def bin_run(bp, f, g, nsteps):
    """Advance copies of (f, g) by nsteps."""
    f = np.ascontiguousarray(f, dtype=np.float64).copy()
    g = np.ascontiguousarray(g, dtype=np.float64).copy()
    if _bin_lib().orc_bin_run(ctypes.byref(bp), _p(f), _p(g), int(nsteps)) != 0:
        raise ValueError("oracle rejected the parameters")
    return f, g


def bin_observe(bp, f, g):
    """(rho[n], phi[n], u[3][n], mu[n])."""
    n = _bn(bp)
    f = np.ascontiguousarray(f, dtype=np.float64)
    g = np.ascontiguousarray(g, dtype=np.float64)
    rho, phi, vel, mu = np.empty(n), np.empty(n), np.empty((3, n)), np.empty(n)
    _bin_lib().orc_bin_observe(ctypes.byref(bp), _p(f), _p(g), _p(rho), _p(phi), _p(vel), _p(mu))
    return rho, phi, vel, mu


def bin_totals(bp, f, g):
    """(mass, sum phi, momentum[3])."""
    f = np.ascontiguousarray(f, dtype=np.float64)
    g = np.ascontiguousarray(g, dtype=np.float64)
    m, ph = ctypes.c_double(), ctypes.c_double()
    mom = np.empty(3)
    _bin_lib().orc_bin_totals(ctypes.byref(bp), _p(f), _p(g), ctypes.byref(m), ctypes.byref(ph),
                              _p(mom))
    return m.value, ph.value, mom


def bin_feq_site(bp, rho, j, phi, grad, lap):
    out = np.empty(bp.base.q)
    j = np.ascontiguousarray(j, dtype=np.float64)
    grad = np.ascontiguousarray(grad, dtype=np.float64)
    _bin_lib().orc_bin_feq_site(ctypes.byref(bp), float(rho), _p(j), float(phi), _p(grad),
                                float(lap), _p(out))
    return out


def bin_geq_site(bp, phi, u, lap):
    out = np.empty(bp.base.q)
    u = np.ascontiguousarray(u, dtype=np.float64)
    _bin_lib().orc_bin_geq_site(ctypes.byref(bp), float(phi), _p(u), float(lap), _p(out))
    return out


def bin_collide_sites(bp, f, g, xyz):
    """Post-collision (f*, g*) [nsite][q] at sites xyz[k] = (x, y, z)."""
    f = np.ascontiguousarray(f, dtype=np.float64)
    g = np.ascontiguousarray(g, dtype=np.float64)
    xyz = np.ascontiguousarray(xyz, dtype=np.int32).reshape(-1, 3)
    fo = np.empty((xyz.shape[0], bp.base.q))
    go = np.empty_like(fo)
    _bin_lib().orc_bin_collide_sites(ctypes.byref(bp), _p(f), _p(g), xyz.shape[0],
                                     xyz.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), _p(fo),
                                     _p(go))
    return fo, go
