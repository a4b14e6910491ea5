"""The energy entry point that allocates nothing, against crmc_energy (needs
an MI355X): two calls in a row, the second on a smaller replica, each equal
to crmc_energy of the same state bit for bit (same kernel, same order)."""
import numpy as np
import pytest

from workloads import nanoparticle_pair, random_sites

pytestmark = pytest.mark.gpu


def test_energy_noalloc_matches_energy():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2109_07527_amd import crmc
    big = nanoparticle_pair(seed=4, L=40.0, R=4.0, sites=120, separation=11.0)
    small = random_sites(12, 10, 24.0, 3, min_dist=1.0)
    S = crmc.System(n_replicas=2, lB=2.0, rc=6.0, precision=32, trials_per_cell=2, seed=5)
    S.build_cells(0, L=big["L"], xyz=big["xyz"], kind=big["kind"], core_xyz=big["core_xyz"], core_R=big["core_R"])
    S.build_cells(1, L=small["L"], xyz=small["xyz"], kind=small["kind"])
    with pytest.raises(crmc.CrmcError) as ei:
        crmc.crmc_energy_noalloc(S.h, 0)  # no device state yet: it would have to allocate
    assert ei.value.code == crmc.CRMC_E_STATE
    cond = dict(pH=7.0, pKa=5.0, pKb=5.0, pIX_pos=0.8, pIX_neg=0.8, kappa=0.5)
    S.sweep_ex([cond, cond], 20)
    assert S.observe(0)["n_cells"] > S.observe(1)["n_cells"]
    e0 = crmc.crmc_energy_noalloc(S.h, 0)
    e1 = crmc.crmc_energy_noalloc(S.h, 1)  # the smaller replica right after
    assert np.isfinite(e0) and np.isfinite(e1) and e0 != 0.0 and e1 != 0.0
    assert e0 == S.energy(0)
    assert e1 == S.energy(1)
    # and once more after further sweeps, the larger replica after the smaller
    S.sweep_ex([cond, cond], 5)
    e1b = crmc.crmc_energy_noalloc(S.h, 1)
    e0b = crmc.crmc_energy_noalloc(S.h, 0)
    assert e1b == S.energy(1) and e0b == S.energy(0)
    S.close()
