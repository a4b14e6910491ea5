"""Launch-shape cache and the schedule search (needs an MI355X).

The library's autotuner keeps the shapes it chose for the rest of the process:
a handle rebuilt on the same inputs takes the cached shape without timing and
without advancing its chain.  The schedule search (trials per cell, domain
pairing) scores every candidate by independent samples/s from a chain of its
own.
"""
import numpy as np
import pytest

from workloads import nanoparticle_pair

pytestmark = pytest.mark.gpu


def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2109_07527_amd import crmc
    return crmc


def _system(crmc, s, seed):
    S = crmc.System(n_replicas=2, lB=2.0, rc=6.0, precision=32, trials_per_cell=4, seed=seed)
    for r in range(2):
        S.build_cells(r, L=s["L"], xyz=s["xyz"], kind=s["kind"], core_xyz=s["core_xyz"], core_R=s["core_R"])
    return S


def test_autotune_cache_within_the_process():
    crmc = _gpu()
    s = nanoparticle_pair(seed=9, L=48.0, R=5.0, sites=200, separation=13.0)
    conds = [dict(pH=pH, pKa=5.0, pKb=5.0, pIX_pos=0.8, pIX_neg=0.8, kappa=0.5) for pH in (5.0, 9.0)]
    S1 = _system(crmc, s, 9191)
    t1 = S1.autotune(conds, 2)
    assert not t1["cached"] and len(t1["candidates"]) > 1 and t1["sweeps_used"] > 0
    S2 = _system(crmc, s, 9191)
    t2 = S2.autotune(conds, 2)
    assert t2["cached"] and t2["sweeps_used"] == 0 and not t2["candidates"]
    assert (t2["light_neighbours"], t2["lds_records"]) == (t1["light_neighbours"], t1["lds_records"])
    assert S2.observe(0)["sweeps"] == 0  # the chain did not advance
    # another seed is another key: tuned afresh
    S3 = _system(crmc, s, 9192)
    assert not S3.autotune(conds, 2)["cached"]
    for S in (S1, S2, S3):
        S.close()


def test_schedule_search_scores_every_candidate():
    _gpu()
    from paper_2109_07527_amd.tune import search_schedule
    s = nanoparticle_pair(seed=9, L=48.0, R=5.0, sites=200, separation=13.0)
    conds = [dict(pH=pH, pKa=5.0, pKb=5.0, pIX_pos=0.8, pIX_neg=0.8, kappa=0.5) for pH in (5.0, 9.0)]
    res = search_schedule([s, s], conds, dict(lB=2.0, rc=6.0), trials=(2, 8), pairing=(True, False), window=600,
                          equilibrate=200)
    cands = res["candidates"]
    assert len(cands) == 4
    assert {(c["trials_per_cell"], c["pairing"]) for c in cands} == {(2, True), (8, True), (2, False), (8, False)}
    for c in cands:
        assert c["sweeps_per_s"] > 0 and all(t >= 0.5 for t in c["tau_int_sweeps"])
        assert c["independent_samples_per_s"] == pytest.approx(
            sum(c["sweeps_per_s"] / (2.0 * t) for t in c["tau_int_sweeps"]), rel=0.01)
    assert res["best"]["independent_samples_per_s"] == max(c["independent_samples_per_s"] for c in cands)
    # more trials per sweep mix more per sweep (single-cell or paired)
    for p in (True, False):
        by = {c["trials_per_cell"]: c for c in cands if c["pairing"] == p}
        assert np.mean(by[8]["tau_int_sweeps"]) < np.mean(by[2]["tau_int_sweeps"])
