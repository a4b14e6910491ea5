"""Pins of the exact results (no GPU).

Each closed form is checked against a computation that does not share its
derivation: a direct term-by-term sum of eq. (QQ), a limiting case with a
textbook answer, or a second closed form that must agree in a stated regime.
"""
import json
import math
import os

import numpy as np
import pytest

from oracle import closed_forms as cf

RHO = 0.0269424
GOLD = os.path.join(os.path.dirname(__file__), "golden", "closed_forms.json")


def test_pIX_grouping_relation():
    # eq. (pIXgen): at vanishing salt the combined ion is the dissociated ion
    assert cf.pIX_from_salt(50.0, 4.0) == pytest.approx(4.0, abs=1e-12)
    assert cf.pIX_from_salt(50.0, 9.0) == pytest.approx(5.0, abs=1e-12)
    # at high salt it is the salt
    assert cf.pIX_from_salt(-2.0, 7.0) == pytest.approx(-2.0, abs=1e-8)
    # equal contributions: 10^-pIX = 2 * 10^-x
    assert cf.pIX_from_salt(7.0, 7.0) == pytest.approx(7.0 - math.log10(2.0), abs=1e-12)


@pytest.mark.parametrize("pIS", [1.0, 2.0, 3.0])
def test_ideal_distribution_equals_direct_sum(pIS):
    """Bessel form of the ion sum vs summing eq. (QQ) over nX+ and nX- term by term."""
    pIX = cf.pIX_from_salt(pIS, 4.5)
    a = cf.ideal_distribution(40, 0, 4.5, 4.5, 0.0, pIX, pIX, 64000.0, RHO)[:, 0]
    b = cf.ideal_distribution_bruteforce(40, 4.5, 4.5, pIX, pIX, 64000.0, RHO, nmax=600)
    assert np.abs(a - b).max() < 1e-12


def test_ideal_asymmetric_and_two_species_direct_sum():
    """Acids and bases with pIX+ != pIX-: compare with an explicit triple sum."""
    nA, nB, V = 5, 4, 3000.0
    pH, pKa, pKb, pIXp, pIXm = 6.0, 5.5, 7.5, 1.3, 1.9
    P = cf.ideal_distribution(nA, nB, pH, pKa, pKb, pIXp, pIXm, V, RHO)
    lnKa = (pH - pKa) * math.log(10)
    lnKb = (14 - pH - pKb) * math.log(10)
    a = RHO * V * 10 ** -pIXp
    b = RHO * V * 10 ** -pIXm
    W = np.zeros((nA + 1, nB + 1))
    for i in range(nA + 1):
        for j in range(nB + 1):
            s = 0.0
            for m in range(0, 200):
                n = m + i - j
                if n < 0:
                    continue
                s += math.exp(n * math.log(a) - math.lgamma(n + 1) + m * math.log(b) - math.lgamma(m + 1))
            W[i, j] = math.comb(nA, i) * math.comb(nB, j) * math.exp(i * lnKa + j * lnKb) * s
    W /= W.sum()
    assert np.abs(W - P).max() < 1e-12


def test_high_salt_limit_is_henderson_hasselbalch():
    """alpha -> 1/(1+10^(pKa-pH)) as salt -> infinity (Donnan effect vanishes)."""
    for pH, pKa in [(4.5, 4.5), (5.0, 4.0), (3.0, 4.2)]:
        pIX = cf.pIX_from_salt(-3.0, pH)
        al = cf.ideal_alpha(40, pH, pKa, pIX, pIX, 64000.0, RHO)
        assert al == pytest.approx(1.0 / (1.0 + 10 ** (pKa - pH)), abs=5e-6)


@pytest.mark.parametrize("pIS", [-1.0, 0.0, 1.0, 2.0, 3.0])
def test_donnan_hh_close_to_exact(pIS):
    """The paper's ideal Gibbs-Donnan + Henderson-Hasselbalch curve (App. C) is a
    large-system approximation of the exact ideal result."""
    pIX = cf.pIX_from_salt(pIS, 4.5)
    ex = cf.ideal_alpha(40, 4.5, 4.5, pIX, pIX, 64000.0, RHO)
    dh = cf.donnan_hh_alpha(40, 4.5, 4.5, pIX, pIX, 64000.0, RHO)
    assert abs(ex - dh) < 5e-3


def test_salt_only_mean_matches_series():
    for pIS in [1.0, 2.0, 3.0]:
        pIX = cf.pIX_from_salt(pIS, 7.0)
        a = RHO * 64000.0 * 10 ** -pIX
        n = np.arange(2000)
        from scipy.special import gammaln, logsumexp
        lw = n * 2 * math.log(a) - 2 * gammaln(n + 1)
        w = np.exp(lw - logsumexp(lw))
        assert cf.salt_only_mean(64000.0, RHO, pIX, pIX) == pytest.approx(float((n * w).sum()), rel=1e-12)
    # dilute limit: <n> -> ab for ab -> 0 ; dense limit <n> -> sqrt(ab) - 1/4
    assert cf.salt_only_mean(1.0, RHO, 6.0, 6.0) == pytest.approx((RHO * 1e-6) ** 2, rel=1e-6)
    s = cf.salt_only_mean(1e6, RHO, -1.0, -1.0)
    assert s == pytest.approx(RHO * 1e7 - 0.25, rel=1e-6)


def test_enumeration_without_interactions_is_ideal():
    """2^N enumeration with lB = 0 must reduce to the binomial closed form."""
    import oracle
    from workloads import ring
    s = ring(10)
    X = oracle.to_fixed(s["xyz"], s["L"])
    pIX = cf.pIX_from_salt(1.0, 4.5)
    P, al, _ = cf.enumerate_sites(X, [1] * 10, s["L"], 0.0, 0.5, 6.0, 4.5, 4.5, 0.0, pIX, pIX, RHO)
    Pex = cf.ideal_distribution(10, 0, 4.5, 4.5, 0.0, pIX, pIX, s["L"] ** 3, RHO)[:, 0]
    assert np.abs(P - Pex).max() < 1e-12


def test_enumeration_two_sites_by_hand():
    """Two acid sites at distance r: four states with weights 1, K, K, K^2 e^(-u)
    times the ion factors; written out directly."""
    import oracle
    L = 40.0
    xyz = np.array([[10.0, 10.0, 10.0], [11.7, 10.0, 10.0]])
    X = oracle.to_fixed(xyz, L)
    pIX = 2.0
    P, al, per = cf.enumerate_sites(X, [1, 1], L, 2.0, 0.5, 6.0, 4.0, 4.5, 0.0, pIX, pIX, RHO)
    r = 1.7
    u = 2.0 * math.exp(-0.5 * r) / r
    K = 10 ** (4.0 - 4.5)
    a = RHO * L ** 3 * 10 ** -pIX
    from scipy.special import iv
    z = 2 * a
    w = np.array([iv(0, z), 2 * K * iv(1, z), K * K * math.exp(-u) * iv(2, z)])
    w /= w.sum()
    assert np.abs(P - w).max() < 1e-7


def test_one_site_quadrature_limits():
    pIX = cf.pIX_from_salt(6.0, 7.5)
    z = RHO * 10 ** -pIX
    x = 10 ** 3 * z * 24.0 ** 3
    # no interaction at all: K z V / (1 + K z V)
    assert cf.one_site_ion_probability(24.0, 0.0, 0.5, 6.0, 7.5, 4.5, pIX, RHO, eps=0.0) == pytest.approx(
        x / (1 + x), rel=1e-10)
    # attraction raises the ionized fraction monotonically with lB
    p = [cf.one_site_ion_probability(24.0, lb, 0.5, 6.0, 7.5, 4.5, pIX, RHO) for lb in (0, 2, 4, 8)]
    assert p[0] < p[1] < p[2] < p[3]


def test_golden_values():
    """Stored values (written by tests/golden/make_golden.py from oracle/ only)
    and, where given, the same quantities computed independently while
    surveying the paper (T-1, T-4, T-5, T-6 tables)."""
    with open(GOLD) as f:
        g = json.load(f)
    for row in g["ideal_alpha_nA40_L40"]:
        pIX = cf.pIX_from_salt(row["pIS"], 4.5)
        assert cf.ideal_alpha(40, 4.5, 4.5, pIX, pIX, 64000.0, RHO) == pytest.approx(row["alpha"], abs=1e-12)
    independent = {-1.0: 0.499855, 0.0: 0.498554, 1.0: 0.485896, 2.0: 0.390701, 3.0: 0.180575}
    for pIS, v in independent.items():
        pIX = cf.pIX_from_salt(pIS, 4.5)
        assert cf.ideal_alpha(40, 4.5, 4.5, pIX, pIX, 64000.0, RHO) == pytest.approx(v, abs=1e-6)
    for pIS, v in {1.0: 172.1812, 2.0: 16.9914, 3.0: 1.445797}.items():
        pIX = cf.pIX_from_salt(pIS, 7.0)
        assert cf.salt_only_mean(64000.0, RHO, pIX, pIX) == pytest.approx(v, rel=5e-6)  # printed to 6-7 digits
    pIX = cf.pIX_from_salt(6.0, 7.5)
    for lb, v in {8.0: 0.340383, 4.0: 0.332052, 2.0: 0.330203}.items():
        assert cf.one_site_ion_probability(24.0, lb, 0.5, 6.0, 7.5, 4.5, pIX, RHO) == pytest.approx(v, abs=2e-6)
    assert g["ring12"]["alpha_lB2"] == pytest.approx(0.2778291, abs=1e-7)
    assert g["ring12"]["alpha_lB0"] == pytest.approx(0.4956804, abs=1e-7)
