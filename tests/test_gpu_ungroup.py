"""Ungrouping on the GPU against the oracle (needs an MI355X): the same state,
the same draw index, the same labels for every particle and the same counts
(the per-particle uniforms come from one Philox counter definition)."""
import numpy as np
import pytest

import oracle
from oracle import closed_forms as cf
from workloads import nanoparticle_pair

pytestmark = pytest.mark.gpu


def test_ungrouping_labels_equal_the_oracle():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2109_07527_amd import crmc
    s = nanoparticle_pair(seed=4, L=40.0, R=4.0, sites=120, separation=11.0)
    pH, pIS = 7.5, 1.0
    pIX = cf.pIX_from_salt(pIS, pH)
    cond = dict(pH=pH, pKa=5.0, pKb=5.0, pIX_pos=pIX, pIX_neg=pIX, kappa=0.5)
    S = crmc.System(n_replicas=2, lB=2.0, rc=6.0, precision=32, trials_per_cell=4, seed=123)
    for r in range(2):
        S.build_cells(r, L=s["L"], xyz=s["xyz"], kind=s["kind"], core_xyz=s["core_xyz"], core_R=s["core_R"])
    S.sweep_ex([cond, cond], 40)
    frac = crmc.crmc_ungroup_fractions(pH, pIS, pIS, pIX, pIX)
    frac = [frac["S_pos"], frac["H"], frac["S_neg"], frac["OH"]]
    X, k, ch, sid = S.particles(1)
    nion = int(((k == 3) | (k == 4)).sum())
    assert nion > 50
    o = oracle.Oracle(s["L"], S.observe(1)["n_cells"], 2.0, 0.5, 6.0, seed=123, replica=1)
    o.load_state(X, k, ch, sid, S.observe(1)["sweeps"], energy=False)
    for draw in (0, 12345678901):
        lab, cnt = crmc.crmc_ungroup(S.h, 1, frac, draw)
        olab, ocnt = o.ungroup(frac, draw)
        assert np.array_equal(lab.astype(np.int32), olab)
        assert np.array_equal(cnt, ocnt)
        assert cnt[:3].sum() == (k == 3).sum() and cnt[3:].sum() == (k == 4).sum()
    with pytest.raises(crmc.CrmcError):
        crmc.crmc_ungroup(S.h, 1, [0.7, 0.7, 0.1, 0.1], 0)
    S.close()
