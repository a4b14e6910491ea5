"""GPU learned proposal against the oracle (needs an MI355X).

The network's BF16 matrix-core forward and backward passes against the FP64
oracle at the same (BF16-rounded) parameters; the FP64 chain with the learned
proposal bit for bit against the oracle's; eps = 1 against the plain chain;
training rows, a short training run, and training from the library's
initial weights.
"""
import numpy as np
import pytest

import oracle
from workloads import random_sites, nanoparticle_pair, config1

pytestmark = pytest.mark.gpu
NP_ = 20865
MLP_B1, MLP_W2, MLP_B2 = 4096, 4224, 4224 + 16384  # W1 [0, 4096), b1, W2 [4224, 20608)


def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2109_07527_amd import crmc
    return crmc


def _params(seed, scale=1.0):
    rng = np.random.default_rng(seed)
    W1 = rng.normal(0, np.sqrt(2.0 / 32), (128, 32)) * scale
    b1 = rng.normal(0, 0.1, 128)
    W2 = rng.normal(0, np.sqrt(2.0 / 128), (128, 128)) * scale
    b2 = rng.normal(0, 0.1, 128)
    w3 = rng.normal(0, np.sqrt(2.0 / 128), 128) * scale
    b3 = rng.normal(0, 0.5, 1)
    return np.concatenate([W1.ravel(), b1, W2.ravel(), b2, w3, b3]).astype(np.float32)


def _bf16(x):
    """round-to-nearest-even to bfloat16, as float64"""
    u = np.asarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16 << 16
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def _bf16_params(p32):
    p = p32.astype(np.float64)
    p[:4096] = _bf16(p32[:4096])
    p[4224:4224 + 16384] = _bf16(p32[4224:4224 + 16384])
    return p


def test_forward_matches_oracle():
    crmc = _gpu()
    S = crmc.System(n_replicas=1)
    p = _params(3)
    S.set_proposal_weights(p)
    assert np.array_equal(S.proposal_weights(), p)
    rng = np.random.default_rng(4)
    X = rng.integers(0, 7, (200, 32)).astype(np.float32)
    z = S.mlp_forward(X)
    pr = _bf16_params(p)
    ref = np.array([oracle.mlp_logit(pr, x) for x in X.astype(np.float64)])
    # BF16 operands (unit roundoff 2^-9) in both products, the hidden layer
    # included: about 4e-3 typical, a few times that at worst
    err = np.abs(z - ref) / np.maximum(1.0, np.abs(ref))
    assert err.mean() < 5e-3 and err.max() < 3e-2, (err.mean(), err.max())


def test_gradient_matches_oracle():
    crmc = _gpu()
    S = crmc.System(n_replicas=1)
    p = _params(5)
    S.set_proposal_weights(p)
    rng = np.random.default_rng(6)
    X = rng.integers(0, 6, (96, 32)).astype(np.float32)
    y = (rng.random(96) < 0.4).astype(np.float32)
    loss, g = S.mlp_gradient(np.concatenate([X, y[:, None]], 1))
    lref, gref = oracle.mlp_loss_grad(_bf16_params(p), X.astype(np.float64), y.astype(np.float64))
    assert loss == pytest.approx(lref, rel=2e-2)
    for lo, hi in ((0, 4096), (4096, 4224), (4224, 20608), (20608, 20736), (20736, 20864), (20864, 20865)):
        d = np.linalg.norm(g[lo:hi] - gref[lo:hi]) / max(np.linalg.norm(gref[lo:hi]), 1e-12)
        assert d < 2e-2, (lo, hi, d)


def _case(name):
    if name == "mixed":
        s = random_sites(12, 10, 24.0, 3, min_dist=1.0)
        s["core_xyz"] = np.array([[12.0, 12.0, 12.0]])
        s["core_R"] = np.array([3.0])
        return s, dict(lB=2.0, rc=6.0), dict(pH=6.0, pKa=5.0, pKb=5.0, pIX_pos=0.5, pIX_neg=0.7, kappa=0.5)
    if name == "np_pair_small":
        s = nanoparticle_pair(seed=4, L=40.0, R=4.0, sites=120, separation=11.0)
        return s, dict(lB=2.0, rc=6.0), dict(pH=7.0, pKa=5.0, pKb=5.0, pIX_pos=0.8, pIX_neg=0.8, kappa=0.5)
    s = config1()
    return s, dict(lB=2.0, rc=6.0), dict(pH=4.5, pKa=4.5, pKb=5.0, pIX_pos=s["pIX"], pIX_neg=s["pIX"], kappa=0.5)


def _run_pair(crmc, name, eps, learned_gpu=True, learned_oracle=True, nsw=12, trials=2, seed=71, scale=2.0,
              offsets=(0.0, 0.0), ion_trials=0):
    s, m, c = _case(name)
    p = _params(9, scale)
    S = crmc.System(n_replicas=1, lB=m["lB"], rc=m["rc"], precision=64, trials_per_cell=trials, seed=seed,
                    ion_trials=ion_trials)
    kw = dict(L=s["L"], xyz=s["xyz"], kind=s["kind"])
    if len(s.get("core_R", [])):
        kw.update(core_xyz=s["core_xyz"], core_R=s["core_R"])
    S.build_cells(0, **kw)
    S.set_proposal_weights(p)
    S.set_proposal_offsets(0, *offsets)
    if learned_gpu:
        S.set_proposal(True, eps)
    S.sweep_ex([c], nsw)
    obs = S.observe(0)
    assert obs["status"] == 0 and obs["error_flags"] & 11 == 0
    o = oracle.Oracle(s["L"], obs["n_cells"], m["lB"], c["kappa"], m["rc"], seed=seed)
    o.set_conditions(c["pH"], c["pKa"], c["pKb"], c["pIX_pos"], c["pIX_neg"])
    o.set_particles(s["xyz"], s["kind"])
    if len(s.get("core_R", [])):
        o.set_cores(s["core_xyz"], s["core_R"])
    o.set_schedule(trials, ion_trials=ion_trials)
    if learned_oracle:
        o.set_learned(p.astype(np.float64), eps)
        o.set_learned_offsets(*offsets)
    ser = o.sweeps(nsw)
    return S, obs, o, ser, nsw


@pytest.mark.parametrize("name,offsets,ion_trials,trials", [("mixed", (0.0, 0.0), 0, 2), ("np_pair_small", (0.0, 0.0), 0, 2),
                                                            ("chain40", (0.0, 0.0), 0, 2),
                                                            ("np_pair_small", (-2.5, 1.5), 0, 2),
                                                            ("np_pair_small", (0.0, 0.0), 2, 2),
                                                            ("np_pair_small", (0.0, 0.0), 0, 20)])
def test_fp64_learned_chain_bit_exact(name, offsets, ion_trials, trials):
    """The FP64 learned chain is the oracle's bit for bit; with 20 trials per
    cell the light domains' lists exceed 64 records with their room and stay
    in the LDS pool instead of registers."""
    crmc = _gpu()
    S, obs, o, ser, nsw = _run_pair(crmc, name, 0.1, offsets=offsets, ion_trials=ion_trials, trials=trials)
    for a, b in zip(S.particles(0), o.particles()):
        assert np.array_equal(np.asarray(a).astype(np.int64), np.asarray(b).astype(np.int64))
    assert np.array_equal(S.series(0, 0, nsw), ser)
    att, acc = o.move_stats()
    assert list(att) == obs["attempts"] and list(acc) == obs["accepts"]
    assert sum(acc[:4]) > 0


def test_uniform_weight_one_is_the_plain_chain():
    crmc = _gpu()
    S, obs, o, ser, nsw = _run_pair(crmc, "np_pair_small", 1.0, learned_oracle=False)
    assert np.array_equal(S.series(0, 0, nsw), ser)
    for a, b in zip(S.particles(0), o.particles()):
        assert np.array_equal(np.asarray(a).astype(np.int64), np.asarray(b).astype(np.int64))


def test_fp32_learned_chain_statistics():
    """BF16 network: picks differ from the FP64 oracle near boundaries, so the
    chains are compared by their means (the nanoparticle pair, 9 acid/base
    sites' worth of statistics per sweep)."""
    crmc = _gpu()
    from paper_2109_07527_amd.stats import mean_se
    s, m, c = _case("np_pair_small")
    p = _params(9, 2.0)
    S = crmc.System(n_replicas=1, lB=2.0, rc=6.0, precision=32, trials_per_cell=4, seed=3, learned=True,
                    learned_eps=0.1)
    S.build_cells(0, L=s["L"], xyz=s["xyz"], kind=s["kind"], core_xyz=s["core_xyz"], core_R=s["core_R"])
    S.set_proposal_weights(p)
    S.sweep_ex([c], 3000)
    g = S.series(0, 300, 2700).astype(float)
    o = oracle.Oracle(s["L"], S.observe(0)["n_cells"], 2.0, 0.5, 6.0, seed=3)
    o.set_conditions(c["pH"], c["pKa"], c["pKb"], c["pIX_pos"], c["pIX_neg"])
    o.set_particles(s["xyz"], s["kind"])
    o.set_cores(s["core_xyz"], s["core_R"])
    o.set_schedule(4)
    o.set_learned(p.astype(np.float64), 0.1)
    r = o.sweeps(1500)[150:].astype(float)
    for col in (0, 1):
        m1, s1, _ = mean_se(g[:, col])
        m2, s2, _ = mean_se(r[:, col])
        assert abs(m1 - m2) < 4.0 * np.hypot(s1, s2), (col, m1, s1, m2, s2)


def test_training_rows_and_a_short_training_run():
    crmc = _gpu()
    s, m, c = _case("np_pair_small")
    S = crmc.System(n_replicas=1, lB=2.0, rc=6.0, precision=32, trials_per_cell=4, seed=3)
    S.build_cells(0, L=s["L"], xyz=s["xyz"], kind=s["kind"], core_xyz=s["core_xyz"], core_R=s["core_R"])
    S.sweep_ex([c], 50)
    S.collect_training(100000)
    S.sweep_ex([c], 40)
    n = S.training_rows()
    assert n == 40 * 240  # every site once per sweep
    rows = S.read_training()
    F, y = rows[:, :32], rows[:, 32]
    assert np.all(F >= 0) and np.array_equal(F, np.round(F)) and set(np.unique(y)) <= {0.0, 1.0}
    assert 0.0 < y.mean() < 1.0
    S.set_proposal_weights(_params(11, 0.5))
    l1 = S.train(1, batch=256, lr=2e-3, seed=1)
    l5 = S.train(6, batch=256, lr=2e-3, seed=2)
    assert np.isfinite(l1) and l5 < l1
    w = S.proposal_weights()
    assert np.isfinite(w).all() and not np.array_equal(w, _params(11, 0.5))


def test_training_from_the_initial_weights_learns_the_features():
    """From the library's initial (He-uniform) weights, training moves the
    hidden layers and fits better than the best constant predictor, whose
    loss is the label entropy; all-zero weights could only move the output
    bias."""
    crmc = _gpu()
    s, m, c = _case("np_pair_small")
    S = crmc.System(n_replicas=1, lB=2.0, rc=6.0, precision=32, trials_per_cell=4, seed=3)
    S.build_cells(0, L=s["L"], xyz=s["xyz"], kind=s["kind"], core_xyz=s["core_xyz"], core_R=s["core_R"])
    S.sweep_ex([c], 50)
    S.collect_training(100000)
    S.sweep_ex([c], 200)
    rows = S.read_training()
    y = rows[:, 32]
    ybar = float(y.mean())
    h_const = -(ybar * np.log(ybar) + (1.0 - ybar) * np.log(1.0 - ybar))
    w0 = S.proposal_weights()
    assert np.abs(w0[:MLP_B1]).max() > 0.1 and np.abs(w0[MLP_W2:MLP_B2]).max() > 0.1
    loss = S.train(20, batch=256, lr=2e-3, seed=4)
    w1 = S.proposal_weights()
    assert np.abs(w1[:MLP_B1] - w0[:MLP_B1]).max() > 1e-3
    assert np.abs(w1[MLP_W2:MLP_B2] - w0[MLP_W2:MLP_B2]).max() > 1e-3
    assert loss < 0.97 * h_const, (loss, h_const)
    z = S.mlp_forward(rows[:2000, :32].astype(np.float32))
    assert np.std(z) > 0.1
    # re-drawing from a seed is deterministic and restarts from those weights
    S.init_proposal_weights(99)
    a = S.proposal_weights()
    S.init_proposal_weights(99)
    assert np.array_equal(a, S.proposal_weights()) and not np.array_equal(a, w1)


def test_site_probabilities_follow_the_network_and_offsets():
    """The p_i the kernels used, read back, against the network evaluated on
    the host (FP64 path): with offsets (a, b) every acid's logit moves by a
    and every base's by b, and the chain with the offsets is still the
    oracle's (bit-exact test above)."""
    crmc = _gpu()
    S0, obs0, _, _, _ = _run_pair(crmc, "np_pair_small", 0.1, learned_oracle=False)
    S1, obs1, _, _, _ = _run_pair(crmc, "np_pair_small", 0.1, learned_oracle=False, nsw=12, offsets=(-2.5, 1.5))
    p0, p1 = S0.site_probabilities(0), S1.site_probabilities(0)
    kind = np.asarray(_case("np_pair_small")[0]["kind"])
    site = (kind == 1) | (kind == 2)
    assert np.all((p0[site] > 0) & (p0[site] < 1)) and np.all((p1[site] > 0) & (p1[site] < 1))
    # the two chains differ, so compare the spread of logits, not site by site
    z0 = np.log(p0[site] / (1 - p0[site]))
    assert np.std(z0) > 0.05
    z1 = np.log(p1[site] / (1 - p1[site]))
    ks = kind[site]
    assert np.median(z1[ks == 1]) < np.median(z0[ks == 1]) - 1.0
    assert np.median(z1[ks == 2]) > np.median(z0[ks == 2]) + 0.5


def _colour0_cells(n):
    """Linear indices of the first colour's cells (all coordinates even)."""
    e = np.arange(0, n, 2)
    cx, cy, cz = np.meshgrid(e, e, e, indexing="ij")
    return (cx + n * (cy + n * cz)).ravel()


def test_fp32_features_and_probabilities_full_size():
    """The FP32 path of the learned proposal (float shell tests with the exact
    integer fallback, BF16 matrix-core network) on the full-size nanoparticle
    pair (4000 sites, L = 120) with ions at the start of three different
    sweeps: every first-phase site's 32 features equal, as integers, the
    oracle's count on the same state, and its p_i equals the logistic of the
    FP64 network at the BF16-rounded weights plus the replica's offset within
    the BF16 tolerance.  Only the first phase of a sweep starts from a state
    the oracle can rebuild exactly (later phases follow FP32 decisions)."""
    crmc = _gpu()
    from workloads import config2
    c = config2()
    cond = dict(pH=7.0, pKa=c["pKa"], pKb=c["pKb"], pIX_pos=c["pIX"], pIX_neg=c["pIX"], kappa=c["kappa"])
    p = _params(13, 1.0)
    off = (-0.7, 0.4)
    S = crmc.System(n_replicas=1, lB=c["lB"], rc=c["rc"], precision=32, trials_per_cell=8, seed=2024,
                    learned=True, learned_eps=0.1)
    S.build_cells(0, c)
    S.set_proposal_weights(p)
    S.set_proposal_offsets(0, *off)
    S.sweep_ex([cond], 40)
    S.record_features(True)
    pr = _bf16_params(p)
    kind = np.asarray(c["kind"])
    checked, z_err, total = 0, [], 0.0
    for rnd in range(3):
        X, k, ch, sid = S.particles(0)
        obs = S.observe(0)
        s0 = obs["sweeps"]
        assert obs["n_xpos"] + obs["n_xneg"] > 100
        S.sweep_ex([cond], 1)
        F = S.site_features(0)
        P = S.site_probabilities(0)
        o = oracle.Oracle(c["L"], obs["n_cells"], c["lB"], c["kappa"], c["rc"], seed=2024)
        o.set_conditions(cond["pH"], cond["pKa"], cond["pKb"], cond["pIX_pos"], cond["pIX_neg"])
        o.set_cores(c["core_xyz"], c["core_R"])
        o.set_learned(pr, 0.1)
        o.load_state(X, k, ch, sid, s0, energy=False)
        o.prepare_sweep()
        for cell in _colour0_cells(obs["n_cells"]):
            ids, Xf = o.cell_site_features(int(cell))
            if len(ids) == 0:
                continue
            assert np.array_equal(F[ids].astype(np.float64), Xf), (rnd, cell)
            for i, x in zip(ids, Xf):
                zo = oracle.mlp_logit(pr, x) + (off[0] if kind[i] == 1 else off[1])
                pg = P[i]
                if 1e-6 < pg < 1 - 1e-6 and abs(zo) < 13.0:
                    zg = np.log(pg / (1.0 - pg))
                    z_err.append(abs(zg - zo) / max(1.0, abs(zo)))
                else:
                    po = 1.0 / (1.0 + np.exp(-zo))
                    assert abs(pg - min(max(po, 1e-6), 1 - 1e-6)) < 1e-4, (i, pg, po)
                checked += 1
            total += Xf.sum()
    z_err = np.array(z_err)
    assert checked > 1000 and total > 10 * checked, (checked, total)
    assert z_err.mean() < 5e-3 and z_err.max() < 3e-2, (z_err.mean(), z_err.max())


def _lcg_shuffle_orders(n, epochs, seed):
    """The minibatch order of crmc_train: per epoch one Fisher-Yates pass
    over the row indices driven by the 64-bit LCG x -> 6364136223846793005 x
    + 1442695040888963407 (Knuth's MMIX constants), seeded with one step from
    the seed; index j = (x >> 33) mod (i + 1)."""
    A, Cc, M = 6364136223846793005, 1442695040888963407, (1 << 64) - 1
    st = (seed * A + Cc) & M
    perm = list(range(n))
    out = []
    for _ in range(epochs):
        for i in range(n - 1, 0, -1):
            st = (st * A + Cc) & M
            j = (st >> 33) % (i + 1)
            perm[i], perm[j] = perm[j], perm[i]
        out.append(list(perm))
    return out


def test_training_steps_match_the_oracle_adam():
    """crmc_train against the oracle step for step: the same minibatches (the
    library's seeded shuffle), the FP64 mean cross-entropy gradient at the
    BF16-rounded weights, and the FP64 Adam step (lr 1e-3, betas 0.9 and
    0.999, bias-corrected moments).  After 16 steps the parameter changes
    agree component by component within a small fraction of the step size
    (a BF16 gradient can differ in sign where the exact gradient is close to
    zero, so a few components may differ by up to 2 lr per step), and the
    last epoch's mean loss agrees."""
    crmc = _gpu()
    rng = np.random.default_rng(17)
    n, batch, epochs, lr, seed = 2048, 256, 2, 1e-3, 5
    X = rng.integers(0, 12, (n, 32)).astype(np.float32)
    wt = rng.normal(0, 0.3, 32)
    y = (rng.random(n) < 1.0 / (1.0 + np.exp(-(X - 5.5) @ wt / 4.0))).astype(np.float32)
    rows = np.concatenate([X, y[:, None]], 1)
    p0 = _params(21, 1.0)
    S = crmc.System(n_replicas=1)
    S.set_proposal_weights(p0)
    S.load_training(rows)
    assert S.training_rows() == n
    loss_gpu = S.train(epochs, batch=batch, lr=lr, seed=seed)
    p_gpu = S.proposal_weights().astype(np.float64)
    # the oracle: FP64 master parameters, BF16 weights for each gradient
    par = p0.astype(np.float64)
    m = np.zeros_like(par)
    v = np.zeros_like(par)
    t = 0
    losses = []
    for order in _lcg_shuffle_orders(n, epochs, seed):
        losses = []
        for b in range(n // batch):
            idx = np.array(order[b * batch:(b + 1) * batch])
            pb = par.copy()
            pb[:4096] = _bf16(par[:4096].astype(np.float32))
            pb[4224:4224 + 16384] = _bf16(par[4224:4224 + 16384].astype(np.float32))
            l, g = oracle.mlp_loss_grad(pb, X[idx].astype(np.float64), y[idx].astype(np.float64))
            losses.append(l)
            t += 1
            oracle.adam_step(par, g, m, v, t, lr)
    assert loss_gpu == pytest.approx(np.mean(losses), rel=1e-2)
    step = lr * t
    d_gpu, d_orc = p_gpu - p0.astype(np.float64), par - p0.astype(np.float64)
    err = np.abs(d_gpu - d_orc)
    assert np.percentile(err, 99) < 0.1 * step, np.percentile(err, 99) / step
    assert err.max() < 2.0 * step
    assert np.abs(d_orc).mean() > 0.1 * step  # the steps are not vanishing
    # the BF16 copies the kernels use follow the trained masters
    Xq = X[:256]
    z1 = S.mlp_forward(Xq)
    S2 = crmc.System(n_replicas=1)
    S2.set_proposal_weights(p_gpu.astype(np.float32))
    assert np.array_equal(z1, S2.mlp_forward(Xq))


def test_training_buffer_reallocated_under_graph_replay():
    """Collecting rows into a buffer of N rows and then of N/2 rows, with the
    sweeps replayed from captured graphs: the second buffer never receives
    more than N/2 rows (the graphs follow every change of a launch argument)."""
    crmc = _gpu()
    s, m, c = _case("np_pair_small")
    S = crmc.System(n_replicas=1, lB=2.0, rc=6.0, precision=32, trials_per_cell=2, seed=3, use_graph=True)
    S.build_cells(0, L=s["L"], xyz=s["xyz"], kind=s["kind"], core_xyz=s["core_xyz"], core_R=s["core_R"])
    S.sweep_ex([c], 20)
    N = 240 * 30
    S.collect_training(N)
    S.sweep_ex([c], 40)
    assert S.training_rows() == N
    S.collect_training(N // 2)
    S.sweep_ex([c], 40)
    assert S.training_rows() == N // 2
    S.collect_training(N)
    S.sweep_ex([c], 16)
    assert S.training_rows() == 16 * 240
    rows = S.read_training()
    assert np.all(rows[:, :32] >= 0) and set(np.unique(rows[:, 32])) <= {0.0, 1.0}
