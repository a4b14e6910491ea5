"""Checkpoint and resume through the C ABI, and graph replay against eager
launches, compared through the exported state (needs an MI355X).

A chain exported after some sweeps and imported into a handle rebuilt from
the same inputs must continue bit for bit: the state exported after the same
further sweeps is byte-identical to that of the uninterrupted run, and so are
the observables.  States that do not fit the handle are rejected and leave it
unchanged.
"""
import numpy as np
import pytest

from workloads import nanoparticle_pair, random_sites

pytestmark = pytest.mark.gpu
CRMC_E_ARG = -1


def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2109_07527_amd import crmc
    return crmc


def _mixed():
    s = random_sites(12, 10, 24.0, 3, min_dist=1.0)
    s.update(core_xyz=np.array([[12.0, 12.0, 12.0]]), core_R=np.array([3.0]))
    return s


def _pair():
    return nanoparticle_pair(seed=2, L=48.0, R=6.0, sites=300, separation=16.0)


def _cond(pH, kappa=0.5):
    return dict(pH=pH, pKa=5.0, pKb=5.0, pIX_pos=0.7, pIX_neg=0.9, kappa=kappa)


def _system(crmc, s, n_rep, precision, seed=11, learned=False, ion_trials=0):
    S = crmc.System(n_replicas=n_rep, lB=2.0, rc=6.0, eps=1.0, ion_coupling=1, precision=precision,
                    trials_per_cell=2, seed=seed, ion_trials=ion_trials)
    for r in range(n_rep):
        kw = dict(L=s["L"], xyz=s["xyz"], kind=s["kind"], group=s.get("group"))
        if len(s.get("core_R", [])):
            kw.update(core_xyz=s["core_xyz"], core_R=s["core_R"])
        S.build_cells(r, **kw)
    if learned:
        S.init_proposal_weights(5)
        S.set_proposal(1, 0.2)
    return S


def _observables(S, n_rep, sweeps):
    out = []
    for r in range(n_rep):
        obs = S.observe(r)
        X, k, c, sid = S.particles(r)
        out.append((sorted(obs.items()), X.tobytes(), k.tobytes(), c.tobytes(), sid.tobytes(),
                    S.series(r, 0, sweeps).tobytes(), S.occupancy(r).tobytes()))
    return out


@pytest.mark.parametrize("case", ["mixed_fp32", "mixed_fp64_learned", "pair_fp32", "pair_fp64_learned",
                                  "pair_fp32_relocation"])
def test_resume_continues_the_chain_bit_for_bit(case):
    crmc = _gpu()
    make, precision, learned, it = {"mixed_fp32": (_mixed, 32, False, 0), "mixed_fp64_learned": (_mixed, 64, True, 0),
                                    "pair_fp32": (_pair, 32, False, 0), "pair_fp64_learned": (_pair, 64, True, 0),
                                    "pair_fp32_relocation": (_pair, 32, False, 2)}[case]
    s = make()
    conds = [_cond(4.0), _cond(7.5, kappa=0.3)]
    n1, n2 = 3, 7  # odd: the import lands on the second record buffer
    A = _system(crmc, s, 2, precision, learned=learned, ion_trials=it)
    A.sweep_ex(conds, n1)
    state = A.export_state()
    A.sweep_ex(conds, n2)
    final = A.export_state()
    ref = _observables(A, 2, n1 + n2)

    # a fresh handle built from the same inputs, never swept
    B = _system(crmc, s, 2, precision, ion_trials=it)
    B.import_state(state)
    assert B.export_state() == state
    B.sweep_ex(conds, n2)
    assert B.export_state() == final
    assert _observables(B, 2, n1 + n2) == ref
    for r in range(2):
        assert B.energy(r) == A.energy(r)
    if it:
        assert A.observe(0)["relocation_accepts"] > 0

    # a handle that has already run its own sweeps, with the other proposal,
    # is overwritten as well (a network it holds stays allocated, so only the
    # observables are compared)
    C = _system(crmc, s, 2, precision, learned=not learned, ion_trials=it)
    C.sweep_ex([_cond(9.0), _cond(3.0)], 2)
    C.import_state(state)
    C.sweep_ex(conds, n2)
    assert _observables(C, 2, n1 + n2) == ref


def test_states_that_do_not_fit_are_rejected():
    crmc = _gpu()
    s = _mixed()
    A = _system(crmc, s, 2, 32)
    A.sweep_ex([_cond(4.0), _cond(6.0)], 2)
    state = A.export_state()

    B = _system(crmc, s, 2, 32)
    B.sweep_ex([_cond(5.0), _cond(5.0)], 1)
    before = B.export_state()
    bad = [state[:len(state) // 2],                  # truncated
           state + b"\0",                           # trailing bytes
           b"X" + state[1:],                        # not a state
           ]
    for blob in bad:
        with pytest.raises(crmc.CrmcError) as e:
            B.import_state(blob)
        assert e.value.code == CRMC_E_ARG
        assert B.export_state() == before
    for other in (_system(crmc, s, 2, 32, seed=12),   # another seed
                  _system(crmc, s, 2, 64),            # another precision
                  _system(crmc, s, 1, 32),            # another replica count
                  _system(crmc, _pair(), 2, 32)):     # another geometry
        snap = other.export_state()
        with pytest.raises(crmc.CrmcError) as e:
            other.import_state(state)
        assert e.value.code == CRMC_E_ARG
        assert other.export_state() == snap


@pytest.mark.parametrize("case", ["mixed_fp32", "pair_fp64_learned", "pair_fp32_relocation", "chain_fp32_sparse",
                                  "pair_fp64_large_pool"])
def test_graph_replays_equal_eager_launches(case):
    """Sweeps replayed from captured HIP graphs and the same sweeps launched
    one kernel at a time give byte-identical states after every call; the
    calls are interleaved with synchronizing reads, and the graphs are
    replayed many times (single-sweep and multi-sweep graphs)."""
    crmc = _gpu()
    from workloads import config1
    make, precision, learned, it, pool = {
        "mixed_fp32": (_mixed, 32, False, 0, 0),
        "pair_fp64_learned": (_pair, 64, True, 0, 0),
        "pair_fp32_relocation": (_pair, 32, False, 2, 0),
        "chain_fp32_sparse": (config1, 32, False, 0, 0),
        "pair_fp64_large_pool": (_pair, 64, False, 0, 10000)}[case]
    s = make()
    conds = [_cond(4.0), _cond(7.5, kappa=0.3)]
    states = []
    for graph in (True, False):
        S = crmc.System(n_replicas=2, lB=2.0, rc=6.0, eps=1.0, ion_coupling=1, precision=precision,
                        trials_per_cell=2, seed=13, ion_trials=it, use_graph=graph, lds_records=pool)
        for r in range(2):
            kw = dict(L=s["L"], xyz=s["xyz"], kind=s["kind"], group=s.get("group"))
            if len(s.get("core_R", [])):
                kw.update(core_xyz=s["core_xyz"], core_R=s["core_R"])
            S.build_cells(r, **kw)
        if learned:
            S.init_proposal_weights(5)
            S.set_proposal(1, 0.2)
        seq = []
        for n in (1, 7, 40, 3):
            S.sweep_ex(conds, n)
            assert S.observe(0)["status"] == 0
            seq.append(S.export_state())
        states.append(seq)
    for a, b in zip(*states):
        assert a == b


def test_handles_interleaved_on_one_device_are_independent():
    """Two handles with different parameters (precision, schedule, proposal,
    relocation, pool) sweeping in turn end in the states each reaches alone."""
    crmc = _gpu()
    specs = [dict(s=_pair(), precision=32, learned=False, it=2, pool=0, trials=2),
             dict(s=_mixed(), precision=64, learned=True, it=0, pool=6000, trials=3)]
    conds = [_cond(5.0), _cond(8.0, kappa=0.4)]

    def make(sp):
        S = crmc.System(n_replicas=2, lB=2.0, rc=6.0, eps=1.0, ion_coupling=1, precision=sp["precision"],
                        trials_per_cell=sp["trials"], seed=23, ion_trials=sp["it"], lds_records=sp["pool"])
        s = sp["s"]
        for r in range(2):
            kw = dict(L=s["L"], xyz=s["xyz"], kind=s["kind"], group=s.get("group"))
            if len(s.get("core_R", [])):
                kw.update(core_xyz=s["core_xyz"], core_R=s["core_R"])
            S.build_cells(r, **kw)
        if sp["learned"]:
            S.init_proposal_weights(3)
            S.set_proposal(1, 0.3)
        return S

    alone = []
    for sp in specs:
        S = make(sp)
        for n in (5, 20, 5):
            S.sweep_ex(conds, n)
        alone.append(S.export_state())
        S.close()
    A, B = make(specs[0]), make(specs[1])
    for n in (5, 20, 5):
        A.sweep_ex(conds, n)
        B.sweep_ex(conds, n)
    assert A.export_state() == alone[0]
    assert B.export_state() == alone[1]
