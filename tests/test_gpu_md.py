"""Hybrid MD / CR-MC on the GPU (needs an MI355X).

A block of Langevin molecular dynamics of the free ions against the oracle's
block on the same state (FP64; positions agree to within a few lattice
units, the sums differ only in rounding order), the MC sweeps after it
bit-exact; an FP32 handle's block (FP32 pair forces) close to the oracle's;
and the hybrid protocol reaching the one-site quadrature at dilute salt on
the cell schedule (FP32).
"""
import numpy as np
import pytest

import oracle
from oracle import closed_forms as cf
from workloads import nanoparticle_pair

pytestmark = pytest.mark.gpu
RHO = 0.0269424


def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2109_07527_amd import crmc
    return crmc


def test_md_block_matches_the_oracle_then_mc_continues_bit_exact():
    crmc = _gpu()
    s = nanoparticle_pair(seed=4, L=40.0, R=4.0, sites=120, separation=11.0)
    cond = dict(pH=7.0, pKa=5.0, pKb=5.0, pIX_pos=0.3, pIX_neg=0.3, kappa=0.5)
    S = crmc.System(n_replicas=1, lB=2.0, rc=6.0, precision=64, trials_per_cell=2, seed=61)
    S.build_cells(0, L=s["L"], xyz=s["xyz"], kind=s["kind"], core_xyz=s["core_xyz"], core_R=s["core_R"])
    o = oracle.Oracle(s["L"], 6, 2.0, 0.5, 6.0, seed=61)
    o.set_conditions(cond["pH"], cond["pKa"], cond["pKb"], cond["pIX_pos"], cond["pIX_neg"])
    o.set_particles(s["xyz"], s["kind"])
    o.set_cores(s["core_xyz"], s["core_R"])
    o.set_schedule(2)
    S.sweep_ex([cond], 6)
    o.sweeps(6)
    assert S.observe(0)["n_cells"] == 6
    X0 = S.particles(0)[0]
    nion = int(((S.particles(0)[1] == 3) | (S.particles(0)[1] == 4)).sum())
    assert nion > 20
    S.md(80, 0.005, 1.0)
    o.md(80, 0.005, 1.0)
    g, r = S.particles(0), o.particles()
    for a, b in zip(g[1:], r[1:]):  # kinds, charges, site ids in the same order
        assert np.array_equal(np.asarray(a), np.asarray(b))
    d = (g[0].astype(np.int64) - r[0].astype(np.int64) + 2 ** 31) % 2 ** 32 - 2 ** 31
    assert np.abs(d).max() <= 64, np.abs(d).max()
    moved = (g[0].astype(np.int64) - X0.astype(np.int64) + 2 ** 31) % 2 ** 32 - 2 ** 31
    assert np.abs(moved).max() > 2 ** 32 / 40.0 * 0.05  # ions moved by more than 0.05 sigma
    obs = S.observe(0)
    assert obs["energy"] == pytest.approx(S.energy(0), rel=1e-12, abs=1e-12)
    assert obs["energy"] == pytest.approx(o.energy(), rel=1e-9, abs=1e-9)
    if np.abs(d).max() == 0:
        # identical positions: the MC chain goes on bit for bit
        ser = o.sweeps(4)
        S.sweep_ex([cond], 4)
        assert np.array_equal(S.series(0, 6, 4), ser)
        for a, b in zip(S.particles(0), o.particles()):
            assert np.array_equal(np.asarray(a).astype(np.int64), np.asarray(b).astype(np.int64))


def test_fp32_md_block_against_the_oracle():
    """An FP32 handle integrates with FP32 pair forces (summed in FP64): its
    state after FP32 sweeps goes to the oracle in its own particle order, and
    after 10 MD steps every coordinate is within 256 lattice units (2.4e-6
    sigma) of the oracle's FP64 block; the retained energy restarts at the
    from-scratch energy."""
    crmc = _gpu()
    s = nanoparticle_pair(seed=4, L=40.0, R=4.0, sites=120, separation=11.0)
    cond = dict(pH=7.0, pKa=5.0, pKb=5.0, pIX_pos=0.3, pIX_neg=0.3, kappa=0.5)
    S = crmc.System(n_replicas=1, lB=2.0, rc=6.0, precision=32, trials_per_cell=2, seed=62)
    S.build_cells(0, L=s["L"], xyz=s["xyz"], kind=s["kind"], core_xyz=s["core_xyz"], core_R=s["core_R"])
    S.sweep_ex([cond], 6)
    X, k, ch, sid = S.particles(0)
    assert int(((k == 3) | (k == 4)).sum()) > 20
    o = oracle.Oracle(s["L"], S.observe(0)["n_cells"], 2.0, 0.5, 6.0, seed=62)
    o.set_conditions(cond["pH"], cond["pKa"], cond["pKb"], cond["pIX_pos"], cond["pIX_neg"])
    o.set_cores(s["core_xyz"], s["core_R"])
    o.set_schedule(2)
    o.load_state(X, k, ch, sid, S.observe(0)["sweeps"])
    S.md(10, 0.005, 1.0)
    o.md(10, 0.005, 1.0)
    g, r = S.particles(0), o.particles()
    for a, b in zip(g[1:], r[1:]):
        assert np.array_equal(np.asarray(a), np.asarray(b))
    d = (g[0].astype(np.int64) - r[0].astype(np.int64) + 2 ** 31) % 2 ** 32 - 2 ** 31
    assert 0 < np.abs(d).max() <= 256, np.abs(d).max()  # FP32 forces: close, not identical
    obs = S.observe(0)
    assert obs["energy"] == pytest.approx(S.energy(0), rel=1e-12, abs=1e-12)
    assert obs["energy"] == pytest.approx(o.energy(), rel=1e-5, abs=1e-5)


def test_hybrid_md_mc_reaches_the_one_site_quadrature():
    """One acid site at dilute salt (pI_S = 6), strong coupling (lB = 8): 64
    independent replicas in one handle alternate one FP32 sweep (8 trials per
    cell, no relocation trials) with 400 MD steps; their mean P(ionized)
    matches the quadrature within 3.5 standard errors of the replica scatter."""
    crmc = _gpu()
    pIX = cf.pIX_from_salt(6.0, 7.5)
    ex = cf.one_site_ion_probability(24.0, 8.0, 0.5, 6.0, 7.5, 4.5, pIX, RHO)
    R = 64
    S = crmc.System(n_replicas=R, lB=8.0, rc=6.0, precision=32, trials_per_cell=8, seed=8080)
    for r in range(R):
        S.build_cells(r, L=24.0, xyz=np.array([[12.0, 12.0, 12.0]]), kind=np.array([1]))
    cond = dict(pH=7.5, pKa=4.5, pKb=5.0, pIX_pos=pIX, pIX_neg=pIX, kappa=0.5)
    ncyc = 1200
    for _ in range(ncyc):
        S.sweep_ex([cond] * R, 1)
        S.md(400, 0.005, 1.0)
    vals = np.array([S.series(r, 100, ncyc - 100)[:, 0].mean() for r in range(R)])
    m, se = vals.mean(), vals.std(ddof=1) / np.sqrt(R)
    assert abs(m - ex) < 3.5 * se, (m, ex, se)
    assert se < 0.02
