"""State invariants of FP32 chains after many sweeps (needs an MI355X):
electroneutrality, counts that match the particle list, and no free ion
closer than 1/2 to another particle or than Delta + 1/2 to a core centre
(up to FP32 rounding of the squared distance), checked by brute force on the
host from the fixed-point positions."""
import numpy as np
import pytest

import oracle
from workloads import config1, nanoparticle_pair

pytestmark = pytest.mark.gpu
ACID, BASE, XPOS, XNEG = 1, 2, 3, 4


def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2109_07527_amd import crmc
    return crmc


@pytest.mark.parametrize("case", ["np_pair", "chain40"])
def test_invariants_after_many_sweeps_fp32(case):
    crmc = _gpu()
    if case == "np_pair":
        s = nanoparticle_pair(seed=4, L=40.0, R=4.0, sites=120, separation=11.0)
        cond = dict(pH=7.0, pKa=5.0, pKb=5.0, pIX_pos=0.3, pIX_neg=0.3, kappa=0.5)
    else:
        s = config1()
        cond = dict(pH=5.0, pKa=4.5, pKb=5.0, pIX_pos=0.5, pIX_neg=0.5, kappa=0.5)
    S = crmc.System(n_replicas=2, lB=2.0, rc=6.0, eps=1.0, precision=32, trials_per_cell=4, seed=5, ion_trials=1)
    for r in range(2):
        kw = dict(L=s["L"], xyz=s["xyz"], kind=s["kind"])
        if len(s.get("core_R", [])):
            kw.update(core_xyz=s["core_xyz"], core_R=s["core_R"])
        S.build_cells(r, **kw)
    S.sweep_ex([cond, dict(cond, pH=cond["pH"] + 2.0)], 300)
    L = s["L"]
    scale = L / 2.0 ** 32
    for r in range(2):
        obs = S.observe(r)
        assert obs["status"] == 0
        X, kind, charged, sid = S.particles(r)
        kind = np.asarray(kind)
        charged = np.asarray(charged)
        q = np.where(kind == ACID, -charged, 0) + np.where(kind == BASE, charged, 0) \
            + (kind == XPOS).astype(int) - (kind == XNEG).astype(int)
        assert q.sum() == 0
        assert obs["n_acid_charged"] == int(((kind == ACID) & (charged == 1)).sum())
        assert obs["n_base_charged"] == int(((kind == BASE) & (charged == 1)).sum())
        assert obs["n_xpos"] == int((kind == XPOS).sum()) and obs["n_xneg"] == int((kind == XNEG).sum())
        assert obs["n_xpos"] + obs["n_xneg"] > 0
        # minimum-image distances on the 32-bit lattice
        Xi = np.asarray(X, dtype=np.uint32)
        ions = np.flatnonzero((kind == XPOS) | (kind == XNEG))
        for i in ions:
            d = (Xi - Xi[i]).view(np.int32).astype(np.float64) * scale
            r2 = (d * d).sum(axis=1)
            r2[i] = np.inf
            assert r2.min() >= 0.25 * (1.0 - 1e-5), (i, r2.min())
        if len(s.get("core_R", [])):
            cx = oracle.to_fixed(s["core_xyz"], L)
            for c, R in zip(cx, s["core_R"]):
                d = (Xi[ions] - c).view(np.int32).astype(np.float64) * scale
                rr = np.sqrt((d * d).sum(axis=1))
                assert rr.min() >= R * (1.0 - 1e-5), rr.min()  # Delta + 1/2 with Delta = R - 1/2
