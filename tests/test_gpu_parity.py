"""GPU path against the oracle (needs an MI355X).

FP64 runs must reproduce the oracle's cell schedule bit for bit: same final
particles in the same order, same per-sweep series, same move statistics.
FP32 runs must give the same decisions except within 1e-4 of the acceptance
threshold, and every energy change within 1e-5 * max(|dU|, 1 kT).
"""
import math

import numpy as np
import pytest

import oracle
from oracle import closed_forms as cf
from workloads import config1, config2, config3, config5, nanoparticle_pair, random_sites, ring

pytestmark = pytest.mark.gpu

RHO = 0.0269424


def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2109_07527_amd import crmc
    return crmc


def _cond(pH, pKa, pKb, pIXp, pIXm, kappa):
    return dict(pH=pH, pKa=pKa, pKb=pKb, pIX_pos=pIXp, pIX_neg=pIXm, kappa=kappa)


def _mixed(seed=3, L=24.0, with_core=True, charged=False):
    s = random_sites(12, 10, L, seed, min_dist=1.0)
    if with_core:
        s["core_xyz"] = np.array([[L / 2, L / 2, L / 2]])
        s["core_R"] = np.array([3.0])
    if charged:
        s["charged"] = (np.arange(22) % 3 == 0).astype(np.int32)
    return s


def _cutoff_line(L=80.0, rc=6.0, n=12):
    """Acid sites on a line whose neighbours sit at lattice distances just
    inside and just outside the cutoff (alternately floor and ceil of rc in
    lattice units, both within 1e-5 of rc): every flip sums pairs that only the
    exact integer test separates."""
    t = rc / L * 2.0 ** 32
    d_in, d_out = math.floor(t), math.ceil(t)
    assert d_in * d_in < math.ceil(t * t) <= d_out * d_out
    xs = [2 ** 28]
    for k in range(1, n):
        xs.append(xs[-1] + (d_in if k % 2 else d_out))
    pts = np.array([[x, 2 ** 31, 2 ** 31 + 12345] for x in xs], dtype=np.float64)
    xyz = pts * (L / 2.0 ** 32)  # exact: the library maps them back to these lattice points
    return dict(L=L, xyz=xyz, kind=np.ones(n, np.int32), group=np.zeros(n, np.int32),
                core_xyz=np.zeros((0, 3)), core_R=np.zeros(0))


CASES = {
    # name: (system factory, model, condition)
    "cutoff_band": (lambda: _cutoff_line(), dict(lB=2.0, rc=6.0, eps=1.0, ion_coupling=0),
                    _cond(4.5, 4.5, 5.0, 1.0, 1.0, 0.5)),
    "mixed": (lambda: _mixed(), dict(lB=2.0, rc=6.0, eps=1.0, ion_coupling=1),
              _cond(6.0, 5.0, 5.0, 0.5, 0.7, 0.5)),
    "mixed_charged_start": (lambda: _mixed(charged=True), dict(lB=2.0, rc=6.0, eps=1.0, ion_coupling=1),
                            _cond(5.0, 5.5, 6.0, 1.2, 0.9, 0.7)),
    "chain40": (lambda: config1(), dict(lB=2.0, rc=6.0, eps=1.0, ion_coupling=1),
                _cond(4.5, 4.5, 5.0, cf.pIX_from_salt(2.0, 4.5), cf.pIX_from_salt(2.0, 4.5), 0.5)),
    "ring_ideal_ions": (lambda: ring(12, L=24.0), dict(lB=2.0, rc=6.0, eps=1.0, ion_coupling=0),
                        _cond(4.5, 4.5, 5.0, 1.0, 1.0, 0.5)),
    "np_pair_small": (lambda: nanoparticle_pair(seed=4, L=40.0, R=4.0, sites=120, separation=11.0),
                      dict(lB=2.0, rc=6.0, eps=1.0, ion_coupling=1), _cond(7.0, 5.0, 5.0, 0.8, 0.8, 0.5)),
    "salt_only": (lambda: dict(L=24.0, xyz=np.zeros((0, 3)), kind=np.zeros(0, np.int32),
                               group=np.zeros(0, np.int32), core_xyz=np.zeros((0, 3)), core_R=np.zeros(0)),
                  dict(lB=2.0, rc=6.0, eps=1.0, ion_coupling=1), _cond(7.0, 4.5, 5.0, 0.3, 0.3, 0.5)),
}


def _oracle_for(s, model, cond, n_cells, trials, pairing, seed, replica=0, fixed_grid=False, site_trials=0,
                ion_trials=0):
    o = oracle.Oracle(s["L"], n_cells, model["lB"], cond["kappa"], model["rc"], eps=model["eps"],
                      ion_coupling=model["ion_coupling"], seed=seed, replica=replica)
    o.set_conditions(cond["pH"], cond["pKa"], cond["pKb"], cond["pIX_pos"], cond["pIX_neg"])
    o.set_particles(s["xyz"], s["kind"], charged=s.get("charged"))
    if len(s.get("core_R", [])):
        o.set_cores(s["core_xyz"], s["core_R"])
    o.set_schedule(trials, fixed_grid=fixed_grid, pairing=pairing, site_trials=site_trials, ion_trials=ion_trials)
    return o


def _gpu_system(crmc, s, model, n_rep, precision, trials, pairing, seed, lds_records=0, fixed_grid=False,
                site_trials=0, ion_trials=0):
    S = crmc.System(n_replicas=n_rep, lB=model["lB"], rc=model["rc"], eps=model["eps"],
                    ion_coupling=model["ion_coupling"], precision=precision, trials_per_cell=trials,
                    pairing=pairing, seed=seed, lds_records=lds_records, fixed_grid=fixed_grid,
                    site_trials=site_trials, ion_trials=ion_trials)
    for r in range(n_rep):
        kw = dict(L=s["L"], xyz=s["xyz"], kind=s["kind"], charged=s.get("charged"), group=s.get("group"))
        if len(s.get("core_R", [])):
            kw.update(core_xyz=s["core_xyz"], core_R=s["core_R"])
        S.build_cells(r, **kw)
    return S


def _same_state(gpu_particles, orc_particles):
    for a, b, name in zip(gpu_particles, orc_particles, ("xyz", "kind", "charged", "site_id")):
        a = np.asarray(a)
        b = np.asarray(b)
        assert a.shape == b.shape, (name, a.shape, b.shape)
        assert np.array_equal(a.astype(np.int64), b.astype(np.int64)), name


@pytest.mark.parametrize("case", sorted(CASES))
@pytest.mark.parametrize("trials,pairing,site_trials,ion_trials",
                         [(1, True, 0, 0), (2, True, 0, 0), (1, False, 0, 0), (1, True, 12, 0), (1, True, 0, 2),
                          (2, False, 0, 1)])
def test_fp64_bit_exact(case, trials, pairing, site_trials, ion_trials):
    crmc = _gpu()
    make, model, cond = CASES[case]
    s = make()
    nsw = 12
    S = _gpu_system(crmc, s, model, 1, 64, trials, pairing, seed=77, site_trials=site_trials, ion_trials=ion_trials)
    S.sweep_ex([cond], nsw)
    obs = S.observe(0)
    assert obs["status"] == 0 and obs["error_flags"] & 11 == 0
    o = _oracle_for(s, model, cond, obs["n_cells"], trials, pairing, seed=77, site_trials=site_trials,
                    ion_trials=ion_trials)
    ser = o.sweeps(nsw)
    _same_state(S.particles(0), o.particles())
    assert np.array_equal(S.series(0, 0, nsw), ser)
    att, acc = o.move_stats()
    assert list(att) == obs["attempts"] and list(acc) == obs["accepts"]
    assert o.relocation_stats() == (obs["relocation_attempts"], obs["relocation_accepts"])
    if ion_trials and case != "salt_only":
        assert obs["relocation_accepts"] > 0
    assert obs["energy"] == pytest.approx(o.running_energy(), rel=1e-9, abs=1e-9)
    assert S.energy(0) == pytest.approx(o.energy(), rel=1e-9, abs=1e-9)
    assert sum(obs["accepts"]) > 0


def _compare_logs(glog, olog, ftol=1e-5):
    """Walk the oracle's trials in processing order; the GPU must agree until
    the first decision within 1e-4 of threshold, which may differ."""
    key = {(int(r["sweep"]), int(r["cell"]), int(r["trial"])): r for r in glog}
    assert len(key) == len(glog)
    n_checked = 0
    for r in olog:
        g = key[(int(r["sweep"]), int(r["cell"]), int(r["trial"]))]
        assert g["move"] == r["move"]
        if r["status"] == 2:
            assert g["status"] == 2
            continue
        ro, rg = r["dU"], g["dU"]
        if np.isfinite(ro) and ro < 1e3:
            assert abs(rg - ro) <= ftol * max(abs(ro), 1.0), (r, g)
        else:
            assert not np.isfinite(rg) or rg > 1e3
        if g["status"] != r["status"]:
            p = math.exp(min(0.0, r["lnp"]))
            assert abs(r["u"] - p) < 1e-4, (r, g)
            return n_checked, True
        n_checked += 1
    return n_checked, False


@pytest.mark.parametrize("case,ion_trials", [("mixed", 0), ("chain40", 0), ("np_pair_small", 0), ("cutoff_band", 0),
                                             ("np_pair_small", 2), ("chain40", 1)])
def test_fp32_decisions_and_dU(case, ion_trials):
    crmc = _gpu()
    make, model, cond = CASES[case]
    s = make()
    nsw = 10
    S = _gpu_system(crmc, s, model, 1, 32, 2, True, seed=5, ion_trials=ion_trials)
    S.enable_log(2_000_000)
    S.sweep_ex([cond], nsw)
    obs = S.observe(0)
    o = _oracle_for(s, model, cond, obs["n_cells"], 2, True, seed=5, ion_trials=ion_trials)
    o.enable_log(2_000_000)
    o.sweeps(nsw)
    n, diverged = _compare_logs(S.read_log(), o.log())
    assert n > 1000
    if not diverged:
        _same_state(S.particles(0), o.particles())


@pytest.mark.parametrize("light", [1, 65536])
def test_unstaged_neighbours_bit_exact(light):
    """A tiny on-chip pool forces domains to read neighbours from memory;
    results must not change."""
    crmc = _gpu()
    _, model, _ = CASES["mixed"]
    s = _mixed()
    cond = _cond(6.0, 5.0, 5.0, -0.8, -0.8, 0.5)  # dense salt: neighbourhoods outgrow the pool
    S = crmc.System(n_replicas=1, lB=2.0, rc=6.0, eps=1.0, precision=64, trials_per_cell=4, seed=9,
                    lds_records=1, light_neighbours=light)
    S.build_cells(0, L=s["L"], xyz=s["xyz"], kind=s["kind"], core_xyz=s["core_xyz"], core_R=s["core_R"],
                  cell_capacity=160)
    S.sweep_ex([cond], 24)
    obs = S.observe(0)
    assert obs["status"] == 0
    assert obs["error_flags"] & 4  # the slow path was taken
    o = _oracle_for(s, model, cond, obs["n_cells"], 4, True, seed=9)
    o.sweeps(24)
    _same_state(S.particles(0), o.particles())


@pytest.mark.parametrize("case", ["np_pair_small", "mixed_groups"])
def test_observables_equal_those_of_the_oracle_states(case):
    """Per-site occupancy sums and per-group histograms of the number of
    ionized sites (the paper's alpha and particle-charge distributions), both
    sampled at the start of every sweep, equal what the test accumulates from
    the oracle's state before each of its sweeps (FP64 chain).  Groups are the
    caller's ids mapped to dense indices in ascending order."""
    crmc = _gpu()
    if case == "mixed_groups":
        make, model, cond = CASES["mixed"]
        s = make()
        s = dict(s, group=np.array([(7, -2, 30)[i % 3] for i in range(len(s["kind"]))], dtype=np.int32))
    else:
        make, model, cond = CASES[case]
        s = make()
    nsw = 9
    S = _gpu_system(crmc, s, model, 1, 64, 2, True, seed=41)
    S.sweep_ex([cond], nsw)
    obs = S.observe(0)
    assert obs["status"] == 0
    o = _oracle_for(s, model, cond, obs["n_cells"], 2, True, seed=41)
    kind = np.asarray(s["kind"])
    group = np.asarray(s["group"])
    ids = sorted(set(group.tolist()))
    dense = np.array([ids.index(g) for g in group.tolist()])
    sizes = np.bincount(dense, minlength=len(ids))
    occ = np.zeros(len(kind), dtype=np.uint64)
    hist = [np.zeros(n + 1, dtype=np.int64) for n in sizes]
    for _ in range(nsw):
        _, k, c, sid = o.particles()
        on = sid[(sid >= 0) & (c == 1) & ((k == 1) | (k == 2))]
        occ[on] += 1
        cnt = np.bincount(dense[on], minlength=len(ids))
        for g in range(len(ids)):
            hist[g][cnt[g]] += 1
        o.sweeps(1)
    assert occ.sum() > 0
    assert np.array_equal(S.occupancy(0), occ)
    gh = S.group_hist(0)
    assert len(gh) == len(hist)
    for a, b in zip(gh, hist):
        assert np.array_equal(a, b)


@pytest.mark.parametrize("case", ["mixed", "np_pair_small"])
def test_conditions_changing_between_calls_bit_exact(case):
    """A titration-like protocol: pH, pI_X and kappa change between calls
    (a time-dependent reservoir pH, App. B).  The FP64 chain follows the
    oracle given the same changes, and after the kappa change the retained
    energy restarts from the state's energy at the new screening length."""
    crmc = _gpu()
    make, model, c0 = CASES[case]
    s = make()
    steps = [(c0, 4),
             (dict(c0, pH=c0["pH"] + 2.0, pIX_pos=c0["pIX_pos"] + 0.4, pIX_neg=c0["pIX_neg"] - 0.2), 3),
             (dict(c0, pH=c0["pH"] - 1.5, kappa=c0["kappa"] * 0.6), 5),
             (dict(c0, pKa=c0["pKa"] + 1.0, pKb=c0["pKb"] - 0.5), 2)]
    S = _gpu_system(crmc, s, model, 1, 64, 2, True, seed=31)
    for c, n in steps:
        S.sweep_ex([c], n)
    obs = S.observe(0)
    assert obs["status"] == 0
    o = _oracle_for(s, model, c0, obs["n_cells"], 2, True, seed=31)
    ser = []
    for c, n in steps:
        o.set_conditions(c["pH"], c["pKa"], c["pKb"], c["pIX_pos"], c["pIX_neg"], kappa=c["kappa"])
        ser.append(o.sweeps(n))
    nsw = sum(n for _, n in steps)
    _same_state(S.particles(0), o.particles())
    assert np.array_equal(S.series(0, 0, nsw), np.concatenate(ser))
    att, acc = o.move_stats()
    assert list(att) == obs["attempts"] and list(acc) == obs["accepts"]
    assert obs["energy"] == pytest.approx(o.energy(), rel=1e-9, abs=1e-9)
    assert sum(obs["accepts"]) > 0


@pytest.mark.parametrize("case", ["chain40", "mixed"])
def test_four_argument_sweep_bit_exact(case):
    """crmc_sweep(pH, pKa, mu_ion, n): one condition for every replica, with
    pI_X+ = pI_X- = mu_ion and the base pK and kappa taken from the creation
    parameters; FP64 chain against the oracle given the same conditions."""
    crmc = _gpu()
    make, model, _ = CASES[case]
    s = make()
    pH, pKa, mu, pKb, kappa = 5.2, 4.8, cf.pIX_from_salt(1.5, 5.2), 6.3, 0.4
    S = crmc.System(n_replicas=2, lB=model["lB"], rc=model["rc"], eps=model["eps"],
                    ion_coupling=model["ion_coupling"], precision=64, trials_per_cell=2, seed=19, pKb=pKb,
                    kappa=kappa)
    for r in range(2):
        kw = dict(L=s["L"], xyz=s["xyz"], kind=s["kind"])
        if len(s.get("core_R", [])):
            kw.update(core_xyz=s["core_xyz"], core_R=s["core_R"])
        S.build_cells(r, **kw)
    S.sweep(pH, pKa, mu, 10)
    cond = _cond(pH, pKa, pKb, mu, mu, kappa)
    for r in range(2):
        obs = S.observe(r)
        assert obs["status"] == 0
        o = _oracle_for(s, model, cond, obs["n_cells"], 2, True, seed=19, replica=r)
        ser = o.sweeps(10)
        _same_state(S.particles(r), o.particles())
        assert np.array_equal(S.series(r, 0, 10), ser)


def test_thousand_replicas_sampled_bit_exact():
    """1000 replicas of a small system in one handle (every table indexed by
    replica, the end-of-sweep grid over replicas): the first, a middle and the
    last replica against the oracle, FP64."""
    crmc = _gpu()
    make, model, cond = CASES["mixed"]
    s = make()
    n_rep = 1000
    S = crmc.System(n_replicas=n_rep, lB=model["lB"], rc=model["rc"], eps=model["eps"],
                    ion_coupling=model["ion_coupling"], precision=64, trials_per_cell=2, seed=29)
    kw = dict(L=s["L"], xyz=s["xyz"], kind=s["kind"])
    if len(s.get("core_R", [])):
        kw.update(core_xyz=s["core_xyz"], core_R=s["core_R"])
    for r in range(n_rep):
        S.build_cells(r, **kw)
    conds = [dict(cond, pH=cond["pH"] + 0.002 * r) for r in range(n_rep)]
    S.sweep_ex(conds, 6)
    for r in (0, 517, n_rep - 1):
        obs = S.observe(r)
        assert obs["status"] == 0 and obs["sweeps"] == 6
        o = _oracle_for(s, model, conds[r], obs["n_cells"], 2, True, seed=29, replica=r)
        ser = o.sweeps(6)
        _same_state(S.particles(r), o.particles())
        assert np.array_equal(S.series(r, 0, 6), ser)


def test_batched_rebinning_bit_exact():
    """A handle with over 65 536 cells re-bins eight new cells per wavefront:
    1030 small boxes of 64 cells and two nanoparticle pairs whose surface
    cells gather more than 64 records (the one-cell path inside a batch).
    Sampled replicas of both kinds against the oracle, FP64, with their move
    counts."""
    crmc = _gpu()
    small, model, cond = CASES["mixed"]
    _, pair_model, pair_cond = CASES["np_pair_small"]
    assert pair_model == model
    s_small = small()
    s_pair = CASES["np_pair_small"][0]()
    n_small = 1030
    systems = [s_small] * n_small + [s_pair] * 2
    conds = [dict(cond, pH=cond["pH"] + 0.001 * r) for r in range(n_small)] + [pair_cond, dict(pair_cond, pH=8.0)]
    S = crmc.System(n_replicas=len(systems), lB=model["lB"], rc=model["rc"], eps=model["eps"],
                    ion_coupling=model["ion_coupling"], precision=64, trials_per_cell=2, seed=37)
    for r, s in enumerate(systems):
        kw = dict(L=s["L"], xyz=s["xyz"], kind=s["kind"], charged=s.get("charged"), group=s.get("group"))
        if len(s.get("core_R", [])):
            kw.update(core_xyz=s["core_xyz"], core_R=s["core_R"])
        S.build_cells(r, **kw)
    n_cells = [S.observe(r)["n_cells"] for r in (0, n_small)]
    assert n_small * n_cells[0] ** 3 + 2 * n_cells[1] ** 3 >= 65536, n_cells
    nsw = 4
    S.sweep_ex(conds, nsw)
    for r in (0, 1, 515, n_small - 1, n_small, n_small + 1):
        obs = S.observe(r)
        assert obs["status"] == 0 and obs["sweeps"] == nsw
        o = _oracle_for(systems[r], model, conds[r], obs["n_cells"], 2, True, seed=37, replica=r)
        ser = o.sweeps(nsw)
        _same_state(S.particles(r), o.particles())
        assert np.array_equal(S.series(r, 0, nsw), ser), r
        att, acc = o.move_stats()
        assert list(att) == obs["attempts"] and list(acc) == obs["accepts"], r


def test_replica_batch_with_different_conditions():
    """Several replicas of different size and conditions in one launch; each
    matches its own oracle."""
    crmc = _gpu()
    systems = [_mixed(seed=3), _mixed(seed=4, L=32.0), config1(), _mixed(seed=5, with_core=False)]
    conds = [_cond(6.0, 5.0, 5.0, 0.5, 0.7, 0.5), _cond(4.0, 4.5, 6.0, 1.0, 1.0, 0.3),
             _cond(4.5, 4.5, 5.0, 2.0, 2.0, 0.9), _cond(8.0, 5.0, 4.0, 0.2, 0.4, 0.6)]
    model = dict(lB=2.0, rc=6.0, eps=1.0, ion_coupling=1)
    S = crmc.System(n_replicas=4, lB=2.0, rc=6.0, eps=1.0, precision=64, trials_per_cell=1, seed=123)
    for r, s in enumerate(systems):
        kw = dict(L=s["L"], xyz=s["xyz"], kind=s["kind"])
        if len(s.get("core_R", [])):
            kw.update(core_xyz=s["core_xyz"], core_R=s["core_R"])
        S.build_cells(r, **kw)
    S.sweep_ex(conds, 10)
    for r, s in enumerate(systems):
        obs = S.observe(r)
        o = _oracle_for(s, model, conds[r], obs["n_cells"], 1, True, seed=123, replica=r)
        ser = o.sweeps(10)
        _same_state(S.particles(r), o.particles())
        assert np.array_equal(S.series(r, 0, 10), ser)


def test_philox_words_match_oracle():
    crmc = _gpu()
    rng = np.random.default_rng(5)
    ctr = rng.integers(0, 2 ** 32, (1000, 4), dtype=np.uint64).astype(np.uint32)
    k0, k1 = 0x12345678, 0x9ABCDEF0
    g = crmc.crmc_philox(ctr, k0, k1)
    for i in range(0, 1000, 37):
        assert list(g[i]) == list(oracle.philox(ctr[i], [k0, k1]))


def test_capacity_overflow_is_reported():
    """Far more salt than a tiny per-cell capacity allows: the library must
    refuse the extra insertions and report the condition, not corrupt memory."""
    crmc = _gpu()
    s = CASES["salt_only"][0]()
    S = crmc.System(n_replicas=1, lB=2.0, rc=6.0, eps=1.0, precision=32, trials_per_cell=4, seed=1)
    S.build_cells(0, L=s["L"], xyz=s["xyz"], kind=s["kind"], cell_capacity=4)
    S.sweep(7.0, 4.5, -1.5, 5)
    obs = S.observe(0)
    assert obs["status"] == crmc.CRMC_E_CAPACITY
    assert obs["error_flags"] & 2


def test_running_energy_tracks_recomputed_energy_fp32():
    crmc = _gpu()
    make, model, cond = CASES["np_pair_small"]
    s = make()
    S = _gpu_system(crmc, s, model, 1, 32, 2, True, seed=21)
    S.sweep_ex([cond], 30)
    obs = S.observe(0)
    e = S.energy(0)
    assert obs["energy"] == pytest.approx(e, rel=1e-5, abs=1e-3)
    o = _oracle_for(s, model, cond, obs["n_cells"], 2, True, seed=21)
    # the oracle's brute-force energy of the GPU's state (computed on the CPU)
    X, kind, charged, sid = S.particles(0)
    chk = oracle.Oracle(s["L"], obs["n_cells"], model["lB"], cond["kappa"], model["rc"], eps=1.0)
    chk.set_particles(X, kind, charged=charged, sid=sid, fixed=True)
    chk.set_cores(s["core_xyz"], s["core_R"])
    assert e == pytest.approx(chk.energy(), rel=1e-9, abs=1e-9)
    del o


def test_config2_full_size_sampled_replicas():
    """The benchmark workload (two nanoparticles, 4000 sites, L = 120, nine
    pH replicas, FP32) for a few sweeps; replicas 0 and 4 against the oracle."""
    crmc = _gpu()
    c = config2()
    model = dict(lB=c["lB"], rc=c["rc"], eps=1.0, ion_coupling=1)
    conds = [_cond(pH, c["pKa"], c["pKb"], c["pIX"], c["pIX"], c["kappa"]) for pH in c["pH_list"]]
    S = crmc.System(n_replicas=9, lB=c["lB"], rc=c["rc"], eps=1.0, precision=32, trials_per_cell=1, seed=2024)
    for r in range(9):
        S.build_cells(r, c)
    S.enable_log(4_000_000)
    nsw = 2
    S.sweep_ex(conds, nsw)
    glog = S.read_log()
    for r in (0, 4):
        obs = S.observe(r)
        assert obs["status"] == 0
        o = _oracle_for(c, model, conds[r], obs["n_cells"], 1, True, seed=2024, replica=r)
        o.enable_log(2_000_000)
        o.sweeps(nsw)
        n, _ = _compare_logs(glog[glog["replica"] == r], o.log())
        assert n > 1000


def test_config3_full_size_sampled_replicas():
    """The 256 uneven chains (50..2000 sites, L up to 156) in one batch, FP32,
    for two sweeps; the shortest, a median and the longest chain against the
    oracle trial by trial."""
    crmc = _gpu()
    reps = config3()
    model = dict(lB=reps[0]["lB"], rc=reps[0]["rc"], eps=1.0, ion_coupling=1)
    conds = [_cond(r["pH"], r["pKa"], r["pKb"], r["pIX"], r["pIX"], r["kappa"]) for r in reps]
    S = crmc.System(n_replicas=len(reps), lB=model["lB"], rc=model["rc"], eps=1.0, precision=32,
                    trials_per_cell=1, seed=2024)
    for i, r in enumerate(reps):
        S.build_cells(i, r)
    cap = 6_000_000
    S.enable_log(cap)
    nsw = 2
    S.sweep_ex(conds, nsw)
    glog = S.read_log()
    assert len(glog) < cap
    sizes = np.array([len(r["kind"]) for r in reps])
    order = np.argsort(sizes)
    for i in (int(order[0]), int(order[len(order) // 2]), int(order[-1])):
        obs = S.observe(i)
        assert obs["status"] == 0
        o = _oracle_for(reps[i], model, conds[i], obs["n_cells"], 1, True, seed=2024, replica=i)
        o.enable_log(2_000_000)
        o.sweeps(nsw)
        n, _ = _compare_logs(glog[glog["replica"] == i], o.log())
        assert n > 100


@pytest.mark.timeout(400)
def test_config5_full_size_sampled_replica():
    """The 64-nanoparticle suspension (51 200 sites, L = 300, eight pH replicas,
    FP32) for one sweep; the first trials of one replica in the oracle's
    processing order against the oracle trial by trial.  The oracle's initial
    energy is a brute-force sum over all pairs (about a minute here) and its dU
    runs over the whole system, so a full sweep would take minutes."""
    crmc = _gpu()
    c = config5()
    model = dict(lB=c["lB"], rc=c["rc"], eps=1.0, ion_coupling=1)
    conds = [_cond(pH, c["pKa"], c["pKb"], c["pIX"], c["pIX"], c["kappa"]) for pH in c["pH_list"]]
    S = crmc.System(n_replicas=len(conds), lB=c["lB"], rc=c["rc"], eps=1.0, precision=32, trials_per_cell=1,
                    seed=2024)
    for r in range(len(conds)):
        S.build_cells(r, c)
    S.enable_log(4_000_000)
    S.sweep_ex(conds, 1)
    glog = S.read_log()
    r = 4
    obs = S.observe(r)
    assert obs["status"] == 0
    o = _oracle_for(c, model, conds[r], obs["n_cells"], 1, True, seed=2024, replica=r)
    o.enable_log(20_000)
    o.set_trial_limit(3000)
    o.sweeps(1)
    assert len(o.log()) == 3000
    n, _ = _compare_logs(glog[glog["replica"] == r], o.log())
    assert n > 1000


@pytest.mark.parametrize("case", ["mixed", "np_pair_small", "chain40"])
@pytest.mark.parametrize("light", [1, 65536])
@pytest.mark.parametrize("ion_trials", [0, 1])
@pytest.mark.parametrize("trials", [3, 20])
def test_light_and_heavy_domains_bit_exact(case, light, ion_trials, trials):
    """Every domain on a whole workgroup (light_neighbours = 1) or every domain
    that fits on one wavefront: the chain is the oracle's either way.  With 3
    trials per cell the light domains' lists (with room for two insertions per
    trial) fit 64 records and sit in registers; with 20 they do not, and the
    light domains keep them in the LDS pool."""
    crmc = _gpu()
    make, model, cond = CASES[case]
    s = make()
    S = crmc.System(n_replicas=1, lB=model["lB"], rc=model["rc"], eps=model["eps"],
                    ion_coupling=model["ion_coupling"], precision=64, trials_per_cell=trials, seed=41,
                    light_neighbours=light, ion_trials=ion_trials)
    kw = dict(L=s["L"], xyz=s["xyz"], kind=s["kind"])
    if len(s.get("core_R", [])):
        kw.update(core_xyz=s["core_xyz"], core_R=s["core_R"])
    S.build_cells(0, **kw)
    S.sweep_ex([cond], 12)
    obs = S.observe(0)
    assert obs["status"] == 0
    o = _oracle_for(s, model, cond, obs["n_cells"], trials, True, seed=41, ion_trials=ion_trials)
    ser = o.sweeps(12)
    _same_state(S.particles(0), o.particles())
    assert np.array_equal(S.series(0, 0, 12), ser)
    att, acc = o.move_stats()
    assert list(att) == obs["attempts"] and list(acc) == obs["accepts"]


def test_uneven_replica_batch_bit_exact():
    """Replicas of different size, box, screening length and pH advance in the
    same launches; each must follow the oracle with its own Philox key."""
    crmc = _gpu()
    from workloads import random_walk_chain
    sizes = [(30, 24.0), (70, 36.0), (12, 24.0), (45, 30.0), (90, 36.0)]
    systems, conds = [], []
    for i, (n, L) in enumerate(sizes):
        rng = np.random.default_rng([7, i])
        xyz = random_walk_chain(n, L, rng)
        systems.append(dict(L=L, xyz=xyz, kind=np.full(n, 1, np.int32)))
        pH = 3.5 + 0.6 * i
        conds.append(_cond(pH, 4.5, 5.0, cf.pIX_from_salt(1.5, pH), cf.pIX_from_salt(1.5, pH), 0.2 + 0.2 * i))
    model = dict(lB=2.0, rc=6.0, eps=1.0, ion_coupling=1)
    S = crmc.System(n_replicas=len(sizes), lB=2.0, rc=6.0, eps=1.0, precision=64, trials_per_cell=2, seed=31)
    for r, s in enumerate(systems):
        S.build_cells(r, L=s["L"], xyz=s["xyz"], kind=s["kind"])
    nsw = 10
    S.sweep_ex(conds, nsw)
    for r, s in enumerate(systems):
        obs = S.observe(r)
        assert obs["status"] == 0 and obs["error_flags"] & 11 == 0
        o = _oracle_for(s, model, conds[r], obs["n_cells"], 2, True, seed=31, replica=r)
        ser = o.sweeps(nsw)
        _same_state(S.particles(r), o.particles())
        assert np.array_equal(S.series(r, 0, nsw), ser), r
        att, acc = o.move_stats()
        assert list(att) == obs["attempts"] and list(acc) == obs["accepts"]
        assert obs["energy"] == pytest.approx(o.running_energy(), rel=1e-9, abs=1e-9)


def test_autotune_keeps_the_chain():
    """The tuner's sweeps are ordinary sweeps under every launch shape it
    tries: the chain after tuning plus more sweeps is the oracle's."""
    crmc = _gpu()
    make, model, cond = CASES["np_pair_small"]
    s = make()
    S = crmc.System(n_replicas=1, lB=model["lB"], rc=model["rc"], eps=model["eps"], precision=64,
                    trials_per_cell=2, seed=55)
    S.build_cells(0, L=s["L"], xyz=s["xyz"], kind=s["kind"], core_xyz=s["core_xyz"], core_R=s["core_R"])
    res = S.autotune([cond], sweeps_per_candidate=2)
    assert len(res["candidates"]) > 1
    assert (res["light_neighbours"], res["lds_records"]) in [(c[0], c[1]) for c in res["candidates"]]
    assert res["sweeps_used"] == 3 * len(res["candidates"])
    S.sweep_ex([cond], 4)
    obs = S.observe(0)
    assert obs["status"] == 0 and obs["error_flags"] & 11 == 0
    total = res["sweeps_used"] + 4
    o = _oracle_for(s, model, cond, obs["n_cells"], 2, True, seed=55)
    ser = o.sweeps(total)
    _same_state(S.particles(0), o.particles())
    assert np.array_equal(S.series(0, 0, total), ser)
