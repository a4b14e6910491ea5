"""Recovery from cell-capacity overflow (needs an MI355X).

A replica built with a capacity far too small for its salt overflows within
a few sweeps; crmc_sweep_recover rolls back to the last good state, enlarges
the capacity and replays, and ends in exactly the state (particles in order,
per-sweep series, move statistics) of the same chain run with ample capacity.
"""
import numpy as np
import pytest

from workloads import nanoparticle_pair

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("precision", [64, 32])
def test_overflow_recovery_equals_an_ample_run(precision):
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2109_07527_amd import crmc
    s = nanoparticle_pair(seed=4, L=40.0, R=4.0, sites=120, separation=11.0)
    cond = dict(pH=7.0, pKa=5.0, pKb=5.0, pIX_pos=-0.2, pIX_neg=-0.2, kappa=0.5)  # dense salt
    kw = dict(L=s["L"], xyz=s["xyz"], kind=s["kind"], core_xyz=s["core_xyz"], core_R=s["core_R"])
    nsw = 24
    ample = crmc.System(n_replicas=2, lB=2.0, rc=6.0, precision=precision, trials_per_cell=4, seed=19)
    for r in range(2):
        ample.build_cells(r, **kw)
    ample.sweep_ex([cond, cond], nsw)
    ref = [ample.observe(r) for r in range(2)]
    assert all(o["status"] == 0 for o in ref)
    top = max(o["max_cell_count"] for o in ref)
    tiny = crmc.System(n_replicas=2, lB=2.0, rc=6.0, precision=precision, trials_per_cell=4, seed=19)
    for r in range(2):
        tiny.build_cells(r, cell_capacity=48, **kw)
    assert top > 48  # the tiny capacity must overflow
    n_rec = tiny.sweep_recover([cond, cond], nsw, chunk=5)
    assert n_rec >= 1
    for r in range(2):
        o = tiny.observe(r)
        assert o["status"] == 0 and o["sweeps"] == nsw and o["cell_capacity"] > 48
        assert o["attempts"] == ref[r]["attempts"] and o["accepts"] == ref[r]["accepts"]
        assert np.array_equal(tiny.series(r, 0, nsw), ample.series(r, 0, nsw))
        for a, b in zip(tiny.particles(r), ample.particles(r)):
            assert np.array_equal(a, b)
    tiny.close()
    ample.close()
