"""Launch-shape autotuner for the fused step kernel.

Times every (tile shape, planes per workgroup) candidate on the live
context with HIP events on the context's stream and keeps the fastest.
Results never depend on the launch shape (every shape runs the same
per-site arithmetic), so tuning only changes speed.  The best choice per
(lattice, scheme, storage, compute, extent, device) is cached in a JSON file.
"""
import hashlib
import json
import sys
import os

import torch

from . import lbm

CACHE = os.environ.get("LBM_TUNE_CACHE",
                       os.path.join(os.path.expanduser("~"), ".cache", "lbm_mi355x_tune.json"))


def _key(p):
    dev = torch.cuda.get_device_name() if torch.cuda.is_available() else "none"
    return "%s|q%d|s%d|st%d|c%d|%dx%dx%d" % (dev, p.lattice, p.scheme, p.storage, p.compute,
                                            p.nx, p.ny, p.nz)


def candidates(p):
    np_ = p.nz if p.lattice == lbm.D3Q19 else p.ny
    short = (4,) if p.lattice == lbm.D2Q9 else ()  # D2Q9: rows are short, 4-row marches pay
    planes = sorted(set(min(c, np_) for c in short + (8, 16, 32, 64, 128, 256)))
    return [(t, c) for t in range(lbm.lbm_tile_count(p.lattice)) for c in planes]


def time_launch(sim, tile, planes, steps=10, reps=2):
    """Average milliseconds per step for one launch shape."""
    sim.set_launch(tile, planes)
    stream = torch.cuda.current_stream()
    sim.step(2)
    best = float("inf")
    for _ in range(reps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        sim.step(steps)
        e1.record(stream)
        e1.synchronize()
        best = min(best, e0.elapsed_time(e1) / steps)
    return best


def autotune(sim, steps=10, use_cache=True, verbose=False):
    """Pick the fastest launch shape for `sim` and apply it.  The state
    advances by the timing steps; callers that need a fixed state should
    save it first (Simulation.get_state / set_state)."""
    key = _key(sim.p)
    cache = {}
    if use_cache and os.path.exists(CACHE):
        try:
            with open(CACHE) as fh:
                cache = json.load(fh)
        except (OSError, ValueError):
            cache = {}
    if use_cache and key in cache:
        t, c = cache[key]["tile"], cache[key]["planes"]
        sim.set_launch(t, c)
        return dict(cache[key], cached=True)
    results = []
    for t, c in candidates(sim.p):
        ms = time_launch(sim, t, c, steps)
        results.append((ms, t, c))
        if verbose:
            print("autotune tile %d planes %d: %.4f ms/step" % (t, c, ms), file=sys.stderr,
                  flush=True)
    ms, t, c = min(results)
    sim.set_launch(t, c)
    best = dict(tile=t, planes=c, ms=ms, tile_shape=lbm.lbm_tile_shape(sim.p.lattice, t))
    if use_cache:
        cache[key] = best
        try:
            os.makedirs(os.path.dirname(CACHE), exist_ok=True)
            with open(CACHE, "w") as fh:
                json.dump(cache, fh, indent=1)
        except OSError:
            pass
    return dict(best, cached=False, table=[(t_, c_, m_) for m_, t_, c_ in results])


def _batch_key(plist):
    p = plist[0]
    dev = torch.cuda.get_device_name() if torch.cuda.is_available() else "none"
    sizes = sorted((q.nx, q.ny, q.nz) for q in plist)
    sig = "%d:%s" % (len(sizes), hashlib.sha1(repr(sizes).encode()).hexdigest()[:12])
    return "%s|batch|q%d|s%d|st%d|c%d|%s" % (dev, p.lattice, p.scheme, p.storage, p.compute, sig)


def batch_candidates(plist):
    """(tile, planes per work item) pairs: powers of two, and the plane counts
    that cut the longest marching axis into 1..8 equal chunks (so that the
    number of work items can match the workgroups the chip holds at once,
    e.g. 3 chunks of 43 planes for 128^2 problems)."""
    p = plist[0]
    np_max = max(q.nz if q.lattice == lbm.D3Q19 else q.ny for q in plist)
    short = (4,) if p.lattice == lbm.D2Q9 else ()
    planes = set(min(c, np_max) for c in short + (8, 16, 32, 64))
    planes |= set(-(-np_max // k) for k in range(1, 9) if -(-np_max // k) >= 8)
    return [(t, c) for t in range(lbm.lbm_tile_count(p.lattice)) for c in sorted(planes)]


def autotune_batch(plist, rho0, steps=8, use_cache=True, verbose=False):
    """Pick the fastest (tile, planes per work item) for a batch of
    problems by timing a throwaway copy of the batch (the caller's batch
    keeps its state and step counts).  Returns (tile, planes)."""
    key = _batch_key(plist)
    cache = {}
    if use_cache and os.path.exists(CACHE):
        try:
            with open(CACHE) as fh:
                cache = json.load(fh)
        except (OSError, ValueError):
            cache = {}
    if use_cache and key in cache:
        return cache[key]["tile"], cache[key]["planes"]
    bt = lbm.Batch(plist, rho0)
    results = []
    try:
        for t, c in batch_candidates(plist):
            bt.set_launch(t, c)
            bt.step(2)
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(bt.stream)
            bt.step(steps)
            e1.record(bt.stream)
            e1.synchronize()
            ms = e0.elapsed_time(e1) / steps
            results.append((ms, t, c))
            if verbose:
                print("autotune batch tile %d planes %d: %.4f ms/step" % (t, c, ms), file=sys.stderr,
                      flush=True)
    finally:
        bt.close()
    ms, t, c = min(results)
    if use_cache:
        cache[key] = dict(tile=t, planes=c, ms=ms)
        try:
            os.makedirs(os.path.dirname(CACHE), exist_ok=True)
            with open(CACHE, "w") as fh:
                json.dump(cache, fh, indent=1)
        except OSError:
            pass
    return t, c


def binary_candidates(lattice, np_):
    """(tile, planes per workgroup) pairs of the binary-fluid step."""
    planes = sorted(set(min(c, np_) for c in (8, 16, 32, 64)))
    return [(t, c) for t in range(lbm.lbm_bin_tile_count(lattice)) for c in planes]


def autotune_binary(sim, steps=10, reps=2, verbose=False):
    """Time every launch shape of a BinarySimulation (its state advances by
    the timing steps) and apply the fastest.  Returns (tile, planes, ms)."""
    p = sim.p
    np_ = p.ny if p.lattice == lbm.D2Q9 else p.nz
    stream = torch.cuda.current_stream()
    results = []
    for t, c in binary_candidates(p.lattice, np_):
        sim.set_launch(t, c)
        sim.step(2)
        best = float("inf")
        for _ in range(reps):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            sim.step(steps)
            e1.record(stream)
            e1.synchronize()
            best = min(best, e0.elapsed_time(e1) / steps)
        results.append((best, t, c))
        if verbose:
            print("autotune binary tile %d planes %d: %.4f ms/step" % (t, c, best), file=sys.stderr,
                  flush=True)
    ms, t, c = min(results)
    sim.set_launch(t, c)
    return t, c, ms
