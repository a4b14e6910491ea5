"""Schedule search: trials per cell and domain pairing chosen by independent samples/s.

The library's launch-shape autotuner (``crmc_autotune``) tunes knobs that leave
the chain unchanged, so it can compare candidates by time alone.  The trial
schedule changes the chain itself: more trials per cell per phase amortise a
phase's staging but lengthen every domain's serial chain, and single-cell
domains halve that chain but mix more slowly (the domain acceptance and the
shifted grid of the cell schedule; the paper's own global moves are the
one-domain case).  So the schedule is chosen by what the chain delivers.  For
every candidate a handle is built on the same systems, its launch shape tuned,
the chain equilibrated, and a fixed window of sweeps timed; the score is

    sum over replicas of (sweeps/s) / (2 tau_int),

with tau_int of n_A- + n_B+ in sweeps (Sokal windowing, c = 5).  A window
shorter than 50 tau_int of some replica is flagged: its score is an estimate.
Everything runs through the library; this module only orchestrates it.
"""
from __future__ import annotations

import time

import numpy as np

from . import crmc
from .stats import tau_int


def _sync():
    import torch
    if torch.cuda.is_available():
        torch.cuda.synchronize()


def measure_schedule(systems, conds, model, trials, pairing, window, equilibrate, precision=32, seed=2024,
                     shape_sweeps=0, learned=None):
    """Score one schedule: a fresh handle on ``systems`` (one per replica),
    ``equilibrate`` sweeps, then ``window`` timed sweeps.  ``learned`` (optional)
    is a callable that switches the learned proposal on for the handle after
    equilibration (training or loading weights).  Returns a dict with the
    score and what it is made of."""
    R = len(conds)
    S = crmc.System(n_replicas=R, lB=model["lB"], rc=model["rc"], precision=precision, trials_per_cell=trials,
                    pairing=pairing, seed=seed)
    try:
        for r in range(R):
            S.build_cells(r, systems[r])
        shape = None
        if shape_sweeps:
            t = S.autotune(conds, shape_sweeps)
            shape = {"light_neighbours": t["light_neighbours"], "lds_records": t["lds_records"]}
        S.sweep_ex(conds, equilibrate)
        if learned is not None:
            learned(S)
        first = S.observe(0)["sweeps"]
        _sync()
        t0 = time.perf_counter()
        S.sweep_ex(conds, window)
        _sync()
        dt = time.perf_counter() - t0
        taus = []
        for r in range(R):
            o = S.observe(r)
            if o["status"] != 0:
                raise RuntimeError("device error during the schedule search: %s" % o)
            ser = S.series(r, first, window).astype(np.float64)
            taus.append(tau_int(ser[:, 0] + ser[:, 1]))
        sweeps_per_s = window / dt
        score = float(sum(sweeps_per_s / (2.0 * t) for t in taus))
        return {"trials_per_cell": trials, "pairing": bool(pairing), "sweeps_per_s": round(sweeps_per_s, 3),
                "ms_per_sweep": round(1e3 * dt / window, 4), "tau_int_sweeps": [round(t, 2) for t in taus],
                "independent_samples_per_s": round(score, 2),
                "window_over_50_tau": bool(window >= 50.0 * max(taus)), "launch_shape": shape}
    finally:
        S.close()


def search_schedule(systems, conds, model, trials=(4, 8, 16), pairing=(True, False), window=2000, equilibrate=300,
                    precision=32, seed=2024, shape_sweeps=0, learned=None):
    """Measure every (trials per cell, pairing) candidate and return
    ``{"best": candidate, "candidates": [...]}``, best by independent
    samples/s."""
    out = []
    for p in pairing:
        for t in trials:
            out.append(measure_schedule(systems, conds, model, t, p, window, equilibrate, precision=precision,
                                        seed=seed, shape_sweeps=shape_sweeps, learned=learned))
    best = max(out, key=lambda c: c["independent_samples_per_s"])
    return {"best": best, "candidates": out}
