"""Seeded synthetic inputs shared by the GPU path, its tests and the oracle.

This module holds none of the lattice Boltzmann arithmetic: it only draws
random numbers and lays out initial density fields (drops in a gas).  The
coexistence densities are arguments; whoever calls this module computes them.

Random numbers come from SplitMix64 (Steele, Lea & Flood, "Fast splittable
pseudorandom number generators", OOPSLA 2014) used as a counter-based
generator: draw k of stream `seed` is mix(mix(seed + G) + (k + 1) G) with the
golden-ratio increment G, so any draw can be recomputed from (seed, k).

All fields are FP64 numpy arrays laid out x fastest: [ny][nx] or [nz][ny][nx].
"""
import math

import numpy as np

_G = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def _mix(z):
    z = np.asarray(z, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
    return z ^ (z >> np.uint64(31))


def splitmix64(seed, counters):
    """64-bit draws number `counters` (array of ints) of stream `seed`."""
    c = np.asarray(counters, dtype=np.uint64)
    with np.errstate(over="ignore"):
        base = _mix(np.array([seed], dtype=np.uint64) + _G)[0]
        return _mix(base + (c + np.uint64(1)) * _G)


def uniform(seed, n, offset=0):
    """n doubles in [0, 1) with 53 random bits each."""
    z = splitmix64(seed, np.arange(offset, offset + n, dtype=np.uint64))
    return (z >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)


class Stream:
    """Sequential reader over one counter-based stream."""

    def __init__(self, seed):
        self.seed = int(seed)
        self.k = 0

    def uniform(self, n=None):
        m = 1 if n is None else int(n)
        out = uniform(self.seed, m, self.k)
        self.k += m
        return float(out[0]) if n is None else out

    def integers(self, lo, hi):
        """Uniform integer in [lo, hi] inclusive."""
        return lo + min(int(self.uniform() * (hi - lo + 1)), hi - lo)


def _min_image(d, n):
    d = np.abs(d)
    return np.minimum(d, n - d)


def _dist(shape, centre):
    """Minimum-image distance of every site to `centre` (x, y[, z])."""
    axes = []
    for ax, (n, c) in enumerate(zip(shape, centre)):
        axes.append(_min_image(np.arange(n, dtype=np.float64) - c, n))
    grids = np.meshgrid(*axes, indexing="ij")  # index order x, y[, z]
    d2 = sum(g * g for g in grids)
    return np.sqrt(d2).transpose()  # -> [z][y][x] / [y][x]


def tanh_drop(shape, radius, rho_in, rho_out, width=2.0, centre=None):
    """A drop (disc or sphere) centred on a node:
    rho = (rho_in + rho_out)/2 + (rho_in - rho_out)/2 * tanh((R - d)/width),
    d the minimum-image distance to the centre; shape = (nx, ny[, nz])."""
    if centre is None:
        centre = tuple(n // 2 for n in shape)
    d = _dist(shape, centre)
    return 0.5 * (rho_in + rho_out) + 0.5 * (rho_in - rho_out) * np.tanh((radius - d) / width)


def flat_slab(nx, ny, rho_in, rho_out, half_width, width=2.0):
    """A liquid slab |x - nx/2| < half_width, two flat interfaces (x only)."""
    x = np.arange(nx, dtype=np.float64)
    d = np.abs(x - nx // 2)
    prof = 0.5 * (rho_in + rho_out) + 0.5 * (rho_in - rho_out) * np.tanh((half_width - d) / width)
    return np.tile(prof, (ny, 1))


def multi_drop(shape, ndrops, rmin, rmax, rho_gas, rho_liq, seed, width=2.0, gap=None,
               max_tries=200000):
    """`ndrops` non-overlapping drops with radii uniform in [rmin, rmax] at
    seeded centres (rejection sampling, largest first, minimum-image
    separation >= R_k + R_l + gap with gap = 4 width by default).
    rho = rho_gas + (rho_liq - rho_gas) max_k (1 + tanh((R_k - d_k)/width))/2.
    Returns (rho, centres, radii)."""
    if gap is None:
        gap = 4.0 * width
    st = Stream(seed)
    radii = sorted((rmin + (rmax - rmin) * st.uniform() for _ in range(ndrops)), reverse=True)
    centres = []
    tries = 0
    for r in radii:
        while True:
            tries += 1
            if tries > max_tries:
                raise RuntimeError("could not place the drops without overlap")
            c = tuple(st.uniform() * n for n in shape)
            ok = True
            for c2, r2 in zip(centres, radii):
                d2 = sum(_min_image(np.array(a - b), n) ** 2 for a, b, n in zip(c, c2, shape))
                if math.sqrt(d2) < r + r2 + gap:
                    ok = False
                    break
            if ok:
                centres.append(c)
                break
    s = np.zeros(tuple(reversed(shape)))
    for c, r in zip(centres, radii):
        d = _dist(shape, c)
        s = np.maximum(s, 0.5 * (1.0 + np.tanh((r - d) / width)))
    rho = rho_gas + (rho_liq - rho_gas) * s
    return rho, centres, radii


def uniform_noise(shape, amplitude, seed):
    """i.i.d. additive noise uniform in [-amplitude, amplitude), keyed by
    (seed, site index) so any site can be regenerated alone."""
    n = int(np.prod(shape))
    u = uniform(seed, n)
    return ((2.0 * u - 1.0) * amplitude).reshape(tuple(reversed(shape)))


def sphere_with_noise(n, radius, rho_gas, rho_liq, amplitude, seed, width=2.0):
    """Cubic periodic n^3 box, one centred drop plus uniform density noise."""
    rho = tanh_drop((n, n, n), radius, rho_liq, rho_gas, width)
    return rho + uniform_noise((n, n, n), amplitude, seed)


def batch_specs(nprob, seed, side_lo=32, side_hi=256, frac_lo=0.15, frac_hi=0.35,
                T_lo=0.45, T_hi=0.55, kappa_lo=0.005, kappa_hi=0.02, kappa_cap=None):
    """Parameters of a batch of independent square D2Q9 problems: side
    uniform in {side_lo..side_hi}, radius uniform in [frac_lo, frac_hi] x side,
    T uniform in [T_lo, T_hi], kappa uniform in [kappa_lo, kappa_hi] or, with
    kappa_cap (a function of T), in [kappa_lo, min(kappa_hi, kappa_cap(T))]."""
    st = Stream(seed)
    out = []
    for _ in range(nprob):
        side = st.integers(side_lo, side_hi)
        frac = frac_lo + (frac_hi - frac_lo) * st.uniform()
        T = T_lo + (T_hi - T_lo) * st.uniform()
        hi = kappa_hi if kappa_cap is None else min(kappa_hi, kappa_cap(T))
        kappa = kappa_lo + (hi - kappa_lo) * st.uniform()
        out.append(dict(side=side, radius=frac * side, T=T, kappa=kappa))
    return out


def stable_batch_specs(nprob, seed, side_lo=32, side_hi=256):
    """The batched drop workload with temperatures and interface
    coefficients moved into the range where the coexisting liquid is linearly
    stable at tau = 1: T uniform in [0.54, 0.56] and kappa uniform in
    [0.005, min(0.02, (T - 0.5) / 3)] (the uniform liquid at the Maxwell
    density needs roughly T > 0.49 + 3 kappa)."""
    return batch_specs(nprob, seed, side_lo=side_lo, side_hi=side_hi, T_lo=0.54, T_hi=0.56,
                       kappa_cap=lambda T: (T - 0.5) / 3.0)
