"""Pins of the oracle's learned site proposal and its network (no GPU).

The network's gradient is checked against central finite differences, its
forward pass against hand-set special cases, the features against a direct
count, and the Metropolis-Hastings-corrected proposal against the exact 2^12
enumeration of the ring (random and strongly biased networks) and against the
plain chain (uniform mixing weight 1).
"""
import numpy as np
import pytest

import oracle
from oracle import closed_forms as cf
from workloads import random_sites, ring

RHO = 0.0269424
NP_ = 20865


def _random_params(seed, scale=1.0):
    """He-style random network: layer weights ~ N(0, 2/fan_in) * scale."""
    rng = np.random.default_rng(seed)
    W1 = rng.normal(0, np.sqrt(2.0 / 32), (128, 32)) * scale
    b1 = rng.normal(0, 0.1, 128)
    W2 = rng.normal(0, np.sqrt(2.0 / 128), (128, 128)) * scale
    b2 = rng.normal(0, 0.1, 128)
    w3 = rng.normal(0, np.sqrt(2.0 / 128), 128) * scale
    b3 = rng.normal(0, 0.5, 1)
    return np.concatenate([W1.ravel(), b1, W2.ravel(), b2, w3, b3])


def test_parameter_count():
    assert oracle.mlp_params() == NP_ == 128 * 32 + 128 + 128 * 128 + 128 + 128 + 1


def test_forward_special_cases():
    par = np.zeros(NP_)
    par[-1] = 0.75                         # b3 only
    assert oracle.mlp_logit(par, np.arange(32.0)) == 0.75
    par = np.zeros(NP_)
    par[0 * 32 + 5] = 2.0                  # W1[0][5]
    par[4096 + 128 + 0 * 128 + 0] = 1.5    # W2[0][0]
    par[4096 + 128 + 16384 + 128 + 0] = -0.5  # w3[0]
    x = np.zeros(32)
    x[5] = 3.0
    assert oracle.mlp_logit(par, x) == pytest.approx(-0.5 * 1.5 * 2.0 * 3.0)
    x[5] = -3.0                            # both ReLUs cut it
    assert oracle.mlp_logit(par, x) == 0.0
    par[4096 + 0] = 10.0                   # b1[0] lifts the first layer
    assert oracle.mlp_logit(par, x) == pytest.approx(-0.5 * 1.5 * (10.0 - 6.0))


def test_gradient_matches_finite_differences():
    rng = np.random.default_rng(3)
    par = _random_params(4)
    X = rng.integers(0, 6, (16, 32)).astype(float)
    y = (rng.random(16) < 0.4).astype(float)
    loss, g = oracle.mlp_loss_grad(par, X, y)
    assert np.isfinite(loss) and loss > 0
    idx = np.concatenate([rng.choice(4096, 60, replace=False), 4096 + rng.choice(128, 20, replace=False),
                          4224 + rng.choice(16384, 80, replace=False), 20608 + rng.choice(128, 20, replace=False),
                          20736 + rng.choice(128, 20, replace=False), [20864]])
    h = 1e-6
    for i in idx:
        pp, pm = par.copy(), par.copy()
        pp[i] += h
        pm[i] -= h
        fd = (oracle.mlp_loss_grad(pp, X, y)[0] - oracle.mlp_loss_grad(pm, X, y)[0]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(g[i])), (i, fd, g[i])


def test_adam_step_by_hand():
    par = np.array([1.0] * NP_)
    g = np.zeros(NP_)
    g[0], g[1] = 0.5, -2.0
    m, v = np.zeros(NP_), np.zeros(NP_)
    oracle.adam_step(par, g, m, v, 1, lr=0.01)
    # first step of Adam moves every parameter with a nonzero gradient by lr * sign(g)
    assert par[0] == pytest.approx(1.0 - 0.01, abs=1e-9)
    assert par[1] == pytest.approx(1.0 + 0.01, abs=1e-9)
    assert par[2] == 1.0
    assert m[0] == pytest.approx(0.05) and v[1] == pytest.approx(0.004)


def test_training_reduces_the_loss():
    """A few hundred Adam steps fit a separable labelling of random features."""
    rng = np.random.default_rng(5)
    X = rng.integers(0, 5, (64, 32)).astype(float)
    y = (X[:, :16].sum(1) > X[:, 16:].sum(1)).astype(float)
    par = _random_params(6, 0.5)
    m, v = np.zeros(NP_), np.zeros(NP_)
    l0 = oracle.mlp_loss_grad(par, X, y)[0]
    for t in range(1, 201):
        _, g = oracle.mlp_loss_grad(par, X, y)
        oracle.adam_step(par, g, m, v, t, lr=3e-3)
    assert oracle.mlp_loss_grad(par, X, y)[0] < 0.3 * l0


def _shell_thresholds(rc, L):
    return [0] + [int(np.ceil(((k * rc / 16.0 / L) * 2.0 ** 32) ** 2)) for k in range(1, 17)]


def test_features_by_direct_count():
    """Features of every site after one sweep against a direct count over all
    charged particles outside the site's own cell (minimum image, integer
    shells)."""
    L, n = 24.0, 4
    s = random_sites(10, 8, L, seed=12, min_dist=1.0)
    charged = (np.arange(18) % 3 == 0).astype(np.int32)
    o = oracle.Oracle(L, n, 2.0, 0.5, 6.0, seed=2)
    o.set_conditions(7.0, 5.0, 5.0, 0.2, 0.2)
    o.set_particles(s["xyz"], s["kind"], charged=charged)
    o.set_learned(_random_params(1), 0.5)
    o.sweeps(1)
    X, kind, ch, sid = o.particles()
    sh = o.shift(0)
    thr = _shell_thresholds(6.0, L)
    q = np.where(kind == 1, -ch, np.where(kind == 2, ch, np.where(kind == 3, 1, np.where(kind == 4, -1, 0))))
    cell = lambda x: tuple(int(((int(x[d]) - int(sh[d])) % 2 ** 32) * n >> 32) for d in range(3))
    seen = 0
    for c in range(n ** 3):
        sids, F = o.cell_site_features(c)
        for k, si in enumerate(sids):
            i = int(np.where(sid == si)[0][0])
            own = cell(X[i])
            qi = -1 if kind[i] == 1 else 1
            ref = np.zeros(32)
            for j in range(len(kind)):
                if j == i or q[j] == 0 or cell(X[j]) == own:
                    continue
                d = [((int(X[j][a]) - int(X[i][a]) + 2 ** 31) % 2 ** 32) - 2 ** 31 for a in range(3)]
                d2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2]
                if d2 >= thr[16]:
                    continue
                shell = max(kk for kk in range(16) if thr[kk] <= d2)
                ref[(0 if q[j] * qi < 0 else 16) + shell] += 1
            assert np.array_equal(F[k], ref), (si, F[k], ref)
            seen += 1
    assert seen == 18


def test_uniform_weight_one_is_the_plain_chain():
    """eps = 1: every pick is uniform, the chain is the plain one."""
    s = random_sites(12, 10, 24.0, 3, min_dist=1.0)
    runs = []
    for learned in (False, True):
        o = oracle.Oracle(24.0, 4, 2.0, 0.5, 6.0, seed=8)
        o.set_conditions(6.0, 5.0, 5.0, 0.5, 0.7)
        o.set_particles(s["xyz"], s["kind"])
        o.set_schedule(2)
        if learned:
            o.set_learned(_random_params(9), 1.0)
        runs.append((o.sweeps(40), o.particles()))
    assert np.array_equal(runs[0][0], runs[1][0])
    for a, b in zip(runs[0][1], runs[1][1]):
        assert np.array_equal(a, b)


def _hist_ok(series, P, k=4.0):
    from paper_2109_07527_amd.stats import tau_int
    n = len(series)
    for v in range(len(P)):
        ind = (series == v).astype(float)
        p = ind.mean()
        tau = tau_int(ind) if 0 < p < 1 else 0.5
        se = np.sqrt(max(P[v] * (1 - P[v]), 1e-12) * 2 * tau / n)
        assert abs(p - P[v]) < k * se + 2.0 / n, (v, p, P[v], se)


def _near_charge_params(a, b):
    """logit = b + a * (opposite charges closer than rc/2): a network that
    singles out sites with a charged partner nearby in another cell."""
    par = np.zeros(NP_)
    par[0:8] = 1.0                    # W1[0][0..7]: opposite charges, inner half of the shells
    par[4224] = 1.0                   # W2[0][0]
    par[20736] = a                    # w3[0]
    par[20864] = b
    return par


@pytest.mark.parametrize("offsets", [(0.0, 0.0), (-3.0, 1.0)])
def test_learned_proposal_keeps_per_site_occupancies(offsets):
    """T-13 with power: four acid sites in one cell, a base (always charged)
    two to four sigma away; the network strongly prefers the two acids
    nearest to the base.  Every per-site occupancy, and the near-minus-far
    difference, must match the exact enumeration; dropping the q_rev / q_fwd
    factor moves that difference by about 8 standard errors (checked when the
    test was written)."""
    from paper_2109_07527_amd.stats import mean_se
    L = 24.0
    xyz = np.array([[12, 12, 12], [13.5, 12, 12], [12, 13.5, 12], [13.5, 13.5, 12], [10, 12, 12]], float)
    kinds = [1, 1, 1, 1, 2]
    X = oracle.to_fixed(xyz, L)
    pH, pKa, pKb = 4.5, 4.5, 2.0
    pIX = cf.pIX_from_salt(2.0, pH)
    _, _, per = cf.enumerate_sites(X, kinds, L, 2.0, 0.5, 6.0, pH, pKa, pKb, pIX, pIX, RHO)
    o = oracle.Oracle(L, 4, 2.0, 0.5, 6.0, eps=1.0, ion_coupling=0, seed=5)
    o.set_conditions(pH, pKa, pKb, pIX, pIX)
    o.set_particles(xyz, np.array(kinds))
    o.set_schedule(8)
    o.set_learned(_near_charge_params(4.0, -2.0), 0.02)
    o.set_learned_offsets(*offsets)
    nsw = 4000
    occ = np.zeros((nsw, 5))
    for t in range(nsw):
        o.sweeps(1, series=False)
        _, _, ch, sid = o.particles()
        m = sid >= 0
        occ[t, sid[m]] = ch[m]
    occ = occ[nsw // 10:]
    for i in range(4):
        mm, se, _ = mean_se(occ[:, i])
        assert abs(mm - per[i]) < 4.0 * se, (i, mm, se, per[i])
    d = occ[:, 0] + occ[:, 2] - occ[:, 1] - occ[:, 3]
    mm, se, _ = mean_se(d)
    ed = per[0] + per[2] - per[1] - per[3]
    assert abs(mm - ed) < 4.0 * se, (mm, se, ed)


@pytest.mark.parametrize("scale,eps", [(4.0, 0.05)])
def test_learned_proposal_keeps_the_exact_distribution(scale, eps):
    """T-13: the ring of 12 interacting acid sites (ideal ions) under the
    learned proposal with random networks, one of them strongly biased,
    against the exact 2^12 enumeration."""
    from paper_2109_07527_amd.stats import mean_se
    L = 24.0
    s = ring(12, L=L)
    X = oracle.to_fixed(s["xyz"], L)
    pIX = cf.pIX_from_salt(1.0, 4.5)
    P, ex, _ = cf.enumerate_sites(X, [1] * 12, L, 2.0, 0.5, 6.0, 4.5, 4.5, 0.0, pIX, pIX, RHO)
    o = oracle.Oracle(L, 4, 2.0, 0.5, 6.0, eps=1.0, ion_coupling=0, seed=21)
    o.set_conditions(4.5, 4.5, 0.0, pIX, pIX)
    o.set_particles(s["xyz"], s["kind"])
    o.set_schedule(16)
    o.set_learned(_random_params(22, scale), eps)
    ser = o.sweeps(3000)
    m, se, _ = mean_se(ser[300:, 0] / 12.0)
    assert abs(m - ex) < 3.5 * se + 1e-3, (m, se, ex)
    _hist_ok(ser[300:, 0], P)
