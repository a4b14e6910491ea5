"""Per-kernel timing and the per-workgroup trace of the phase kernel through
the C ABI (needs an MI355X): launch counts, and one record per domain and
phase with consistent contents."""
import numpy as np
import pytest

from workloads import random_sites

pytestmark = pytest.mark.gpu


def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2109_07527_amd import crmc
    return crmc


def _system(crmc, trials):
    s = random_sites(30, 20, 36.0, 7, min_dist=1.0)
    S = crmc.System(n_replicas=2, lB=2.0, rc=6.0, eps=1.0, precision=32, trials_per_cell=trials, seed=3)
    for r in range(2):
        S.build_cells(r, L=s["L"], xyz=s["xyz"], kind=s["kind"])
    cond = dict(pH=6.0, pKa=5.0, pKb=5.0, pIX_pos=1.0, pIX_neg=1.0, kappa=0.5)
    return S, [cond, dict(cond, pH=8.0)]


def test_timing_counts_every_launch():
    crmc = _gpu()
    S, conds = _system(crmc, 2)
    S.sweep_ex(conds, 2)
    crmc.crmc_set_timing(S.h, True)
    S.sweep_ex(conds, 5)
    ms, n = crmc.crmc_get_timing(S.h)
    crmc.crmc_set_timing(S.h, False)
    assert list(n) == [5, 40, 5]
    assert (ms > 0).all()


def test_trace_has_one_record_per_domain_and_phase():
    crmc = _gpu()
    trials = 3
    S, conds = _system(crmc, trials)
    S.sweep_ex(conds, 2)
    s0 = S.observe(0)["sweeps"]
    crmc.crmc_enable_trace(S.h, 100000)
    S.sweep_ex(conds, 2)
    tr, n = crmc.crmc_read_trace(S.h, 100000)
    assert n == len(tr) and n > 0
    assert set(np.unique(tr["sweep"])) == {s0, s0 + 1}
    assert set(np.unique(tr["colour"])) == set(range(8))
    # every phase of every sweep holds the same number of domains
    per = [((tr["sweep"] == sw) & (tr["colour"] == c)).sum() for sw in (s0, s0 + 1) for c in range(8)]
    assert len(set(per)) == 1
    # a domain of one cell runs `trials` trials, a reflection pair twice that
    assert set(np.unique(tr["trials"])) <= {trials, 2 * trials}
    assert (tr["t1"] >= tr["t0"]).all()
    assert (tr["own"] >= 0).all() and (tr["neighbours"] >= 0).all()
    # each domain index appears once per phase
    for sw in (s0, s0 + 1):
        for c in range(8):
            d = tr["domain"][(tr["sweep"] == sw) & (tr["colour"] == c)]
            assert len(np.unique(d)) == len(d)
