"""Chains inside a caller-owned workspace (needs an MI355X).

The handle's whole device state lives in a torch uint8 tensor of
crmc_workspace_size bytes: the FP64 chain is still the oracle's bit for bit,
the library holds no device memory of its own, and a workspace that is too
small is reported as CRMC_E_NOMEM instead of being overrun.
"""
import numpy as np
import pytest

import oracle
from workloads import nanoparticle_pair

pytestmark = pytest.mark.gpu


def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2109_07527_amd import crmc
    return crmc, torch


def _system():
    s = nanoparticle_pair(seed=4, L=40.0, R=4.0, sites=120, separation=11.0)
    cond = dict(pH=7.0, pKa=5.0, pKb=5.0, pIX_pos=0.8, pIX_neg=0.8, kappa=0.5)
    return s, cond


@pytest.mark.parametrize("learned", [False, True])
def test_fp64_chain_in_a_torch_workspace_bit_exact(learned):
    crmc, torch = _gpu()
    s, cond = _system()
    S = crmc.System(n_replicas=2, lB=2.0, rc=6.0, precision=64, trials_per_cell=2, seed=77)
    for r in range(2):
        S.build_cells(r, L=s["L"], xyz=s["xyz"], kind=s["kind"], core_xyz=s["core_xyz"], core_R=s["core_R"])
    nbytes = S.workspace_size()
    ws = torch.zeros(nbytes, dtype=torch.uint8, device="cuda")
    S.set_workspace(ws)
    rng = np.random.default_rng(2)
    par = rng.normal(0.0, 0.2, 20865).astype(np.float32)
    if learned:
        S.set_proposal_weights(par)
        S.set_proposal(True, 0.2)
    S.sweep_ex([cond, cond], 12)
    mem = S.memory()
    assert mem["own"] == 0, mem
    assert 0 < mem["workspace_used"] <= nbytes
    obs = S.observe(1)
    assert obs["status"] == 0 and sum(obs["accepts"]) > 0
    e = S.energy(1)
    assert S.memory()["own"] == 0
    o = oracle.Oracle(s["L"], obs["n_cells"], 2.0, cond["kappa"], 6.0, seed=77, replica=1)
    o.set_conditions(cond["pH"], cond["pKa"], cond["pKb"], cond["pIX_pos"], cond["pIX_neg"])
    o.set_particles(s["xyz"], s["kind"])
    o.set_cores(s["core_xyz"], s["core_R"])
    o.set_schedule(2)
    if learned:
        o.set_learned(par.astype(np.float64), 0.2)
    ser = o.sweeps(12)
    for a, b in zip(S.particles(1), o.particles()):
        assert np.array_equal(np.asarray(a).astype(np.int64), np.asarray(b).astype(np.int64))
    assert np.array_equal(S.series(1, 0, 12), ser)
    assert e == pytest.approx(o.energy(), rel=1e-9, abs=1e-9)
    # the workspace bytes are the handle's state: clearing the tensor would
    # clear the chain, so the records read back must be non-trivial
    assert int(ws.count_nonzero()) > 0
    S.close()


def test_too_small_workspace_is_reported():
    crmc, torch = _gpu()
    s, cond = _system()
    S = crmc.System(n_replicas=1, lB=2.0, rc=6.0, precision=32, trials_per_cell=2, seed=7)
    S.build_cells(0, L=s["L"], xyz=s["xyz"], kind=s["kind"], core_xyz=s["core_xyz"], core_R=s["core_R"])
    nbytes = S.workspace_size()
    ws = torch.zeros(nbytes // 2, dtype=torch.uint8, device="cuda")
    S.set_workspace(ws)
    with pytest.raises(crmc.CrmcError) as ei:
        S.sweep_ex([cond], 2)
    assert ei.value.code == crmc.CRMC_E_NOMEM
    assert S.memory()["own"] == 0
    S.close()
