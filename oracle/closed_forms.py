"""Exact results for CR-MC that the oracle's Monte Carlo is pinned against.

TEST INFRASTRUCTURE ONLY (imported by tests and by the scripts that write the
stored expected values under tests/golden/).

All functions are FP64 numpy/scipy.  Notation follows the paper (Curk, Yuan,
Luijten): pH, pOH = pKw - pH, pKa, pKb, pI_X+ and pI_X- in log10 units,
rho0*NA the reference number density (rho0 = 1 M), V the box volume.

* ``pIX_from_salt``      - combined-ion chemical potential, eq. (pIXgen), App. C.
* ``ideal_distribution`` - exact P(nA-, nB+) of the grand-canonical weight
  eq. (QQ) when the free ions are ideal: summing the two Poisson-like ion factors
  over ion numbers under electroneutrality nX+ - nX- = nA- - nB+ = D gives
  (a/b)^(D/2) I_|D|(2 sqrt(ab)) with a = rho0 NA V 10^-pIX+, b likewise with pIX-.
* ``donnan_hh_alpha``    - the ideal Gibbs-Donnan + Henderson-Hasselbalch
  estimate the paper uses as its dashed reference curves (App. C, Fig. 6).
* ``salt_only_mean``     - <nX+> of a box with no ionizable groups and ideal ions.
* ``enumerate_sites``    - exact 2^N enumeration of the site states of eq. (QQ)
  for fixed site positions with site-site screened Coulomb and ideal ions.
* ``one_site_ion_probability`` - a single acid site with an interacting
  counterion in the dilute limit (quadrature of the site-ion Boltzmann factor).
* ``salt_pair_ratio``    - a box with no ionizable groups and interacting free
  ions: the exact ratio of the weights of the one-pair and the empty state.
"""
from __future__ import annotations

import itertools
import math

import numpy as np
from scipy import integrate, optimize, special

LN10 = math.log(10.0)


def pIX_from_salt(pIS: float, pH: float, pKw: float = 14.0) -> float:
    """eq. (pIXgen): 10^-pIX = 10^-pIS + 10^-min(pH, pOH)."""
    pOH = pKw - pH
    return -math.log10(10.0 ** (-pIS) + 10.0 ** (-min(pH, pOH)))


def _log_bessel_i(order: np.ndarray, z: float) -> np.ndarray:
    """log I_order(z) for integer orders >= 0, stable for large z."""
    return np.log(special.ive(order, z)) + z


def ideal_distribution(nA: int, nB: int, pH: float, pKa: float, pKb: float,
                       pIXp: float, pIXm: float, V: float, rho0NA: float,
                       pKw: float = 14.0) -> np.ndarray:
    """Exact P[nA-, nB+] (shape (nA+1, nB+1)) of eq. (QQ) with ideal ions."""
    pOH = pKw - pH
    lnKa = (pH - pKa) * LN10
    lnKb = (pOH - pKb) * LN10
    lna = math.log(rho0NA * V) - pIXp * LN10
    lnb = math.log(rho0NA * V) - pIXm * LN10
    z = 2.0 * math.exp(0.5 * (lna + lnb))
    i = np.arange(nA + 1)[:, None]
    j = np.arange(nB + 1)[None, :]
    D = i - j
    lnw = (special.gammaln(nA + 1) - special.gammaln(i + 1) - special.gammaln(nA - i + 1)
           + special.gammaln(nB + 1) - special.gammaln(j + 1) - special.gammaln(nB - j + 1)
           + i * lnKa + j * lnKb + 0.5 * D * (lna - lnb) + _log_bessel_i(np.abs(D), z))
    lnw -= lnw.max()
    w = np.exp(lnw)
    return w / w.sum()


def ideal_alpha(nA, pH, pKa, pIXp, pIXm, V, rho0NA, pKw=14.0):
    """<nA->/nA of ``ideal_distribution`` for acids only."""
    P = ideal_distribution(nA, 0, pH, pKa, 0.0, pIXp, pIXm, V, rho0NA, pKw)[:, 0]
    return float((np.arange(nA + 1) * P).sum() / nA)


def ideal_distribution_bruteforce(nA, pH, pKa, pIXp, pIXm, V, rho0NA, nmax=400, pKw=14.0):
    """Acids only: the same distribution by summing eq. (QQ) term by term over
    nA-, nX+ and nX- (nX+ = nX- + nA-), truncated at nX- < nmax."""
    lnKa = (pH - pKa) * LN10
    lna = math.log(rho0NA * V) - pIXp * LN10
    lnb = math.log(rho0NA * V) - pIXm * LN10
    m = np.arange(nmax)
    out = np.zeros(nA + 1)
    logs = []
    for k in range(nA + 1):
        terms = ((m + k) * lna - special.gammaln(m + k + 1) + m * lnb - special.gammaln(m + 1))
        logs.append(special.gammaln(nA + 1) - special.gammaln(k + 1) - special.gammaln(nA - k + 1)
                    + k * lnKa + special.logsumexp(terms))
    logs = np.array(logs)
    out = np.exp(logs - logs.max())
    return out / out.sum()


def donnan_hh_alpha(nA: int, pH: float, pKa: float, pIXp: float, pIXm: float, V: float,
                    rho0NA: float) -> float:
    """Ideal Gibbs-Donnan equilibrium coupled to Henderson-Hasselbalch.

    Inside the box c+ c- = cX+ cX- (reservoir product), c+ - c- = alpha cA
    (electroneutrality) and alpha/(1-alpha) = 10^(pH-pKa) cX+/c+ (the local
    proton activity is raised by the Donnan factor c+/cX+)."""
    cA = nA / V
    cxp = rho0NA * 10.0 ** (-pIXp)
    cxm = rho0NA * 10.0 ** (-pIXm)
    K = 10.0 ** (pH - pKa)

    def f(alpha):
        q = alpha * cA
        cp = 0.5 * (q + math.sqrt(q * q + 4.0 * cxp * cxm))
        return alpha / (1.0 - alpha) - K * cxp / cp

    return optimize.brentq(f, 1e-15, 1.0 - 1e-15, xtol=1e-15)


def salt_only_mean(V: float, rho0NA: float, pIXp: float, pIXm: float) -> float:
    """<nX+> for ideal ions and no ionizable groups: sqrt(ab) I1(2 sqrt(ab))/I0(2 sqrt(ab))."""
    a = rho0NA * V * 10.0 ** (-pIXp)
    b = rho0NA * V * 10.0 ** (-pIXm)
    s = math.sqrt(a * b)
    return float(s * special.ive(1, 2 * s) / special.ive(0, 2 * s))


def _min_image_r(xi, xj, L):
    """distance and exact integer squared distance of two fixed-point points"""
    d = []
    for a, b in zip(xi, xj):
        v = (int(b) - int(a)) & 0xFFFFFFFF
        if v >= 1 << 31:
            v -= 1 << 32
        d.append(v)
    r2i = d[0] * d[0] + d[1] * d[1] + d[2] * d[2]
    s = L / 4294967296.0
    return math.sqrt(r2i) * s, r2i


def enumerate_sites(X, kinds, L, lB, kappa, rc, pH, pKa, pKb, pIXp, pIXm, rho0NA, pKw=14.0):
    """Exact distribution over all 2^N site states (N <= ~14).

    X: fixed-point site coordinates (N,3) uint32; kinds 1 = acid, 2 = base.
    Sites interact by the truncated screened Coulomb (cutoff decided on the
    exact integer squared distance, as in the oracle); ions are ideal.
    Returns (P_nAm: distribution of the number of charged acids,
             mean_alpha: <nA->/nA, per_site: <s_i>)."""
    N = len(kinds)
    V = L ** 3
    pOH = pKw - pH
    lnK = np.array([(pH - pKa) * LN10 if k == 1 else (pOH - pKb) * LN10 for k in kinds])
    sign = np.array([-1 if k == 1 else 1 for k in kinds])
    R2 = math.ceil(((rc / L) * 4294967296.0) ** 2)
    J = np.zeros((N, N))
    for i in range(N):
        for j in range(i + 1, N):
            r, r2i = _min_image_r(X[i], X[j], L)
            if r2i < R2:
                J[i, j] = lB * math.exp(-kappa * r) / r
    lna = math.log(rho0NA * V) - pIXp * LN10
    lnb = math.log(rho0NA * V) - pIXm * LN10
    z = 2.0 * math.exp(0.5 * (lna + lnb))
    states = np.array(list(itertools.product([0, 1], repeat=N)), dtype=np.int64)
    q = states * sign[None, :]
    E = np.einsum("si,ij,sj->s", q.astype(float), J, q.astype(float))
    nAm = (states * (np.array(kinds) == 1)).sum(1)
    nBp = (states * (np.array(kinds) == 2)).sum(1)
    D = nAm - nBp
    lnw = -E + states @ lnK + 0.5 * D * (lna - lnb) + _log_bessel_i(np.abs(D), z)
    w = np.exp(lnw - lnw.max())
    w /= w.sum()
    nA = int((np.array(kinds) == 1).sum())
    P = np.bincount(nAm, weights=w, minlength=nA + 1)
    return P, float((nAm * w).sum() / max(nA, 1)), (states * w[:, None]).sum(0)


def _attractive_pair_J(L, lB, kappa, rc, eps):
    """J = V + 4 pi int_0^rc r^2 (exp(-u(r)) - 1) dr for a pair of opposite
    unit charges: u = -lB exp(-kappa r)/r below rc (truncated) plus the
    shifted WCA below 2^(1/6) when eps > 0, infinite below 1/2 (the hard core
    of the excluded volume)."""
    V = L ** 3

    def u(r):
        e = -lB * math.exp(-kappa * r) / r if lB else 0.0
        if eps > 0.0 and r < 2.0 ** (1.0 / 6.0):
            e += 4.0 * eps * (r ** -12 - r ** -6) + eps
        return e

    def integrand(r):
        if eps > 0.0 and r < 0.5:
            return -r * r
        return r * r * (math.exp(-u(r)) - 1.0)

    val = 0.0
    edges = [0.0, 0.5, 2.0 ** (1.0 / 6.0), rc]
    for a, b in zip(edges[:-1], edges[1:]):
        val += integrate.quad(integrand, a, b, epsabs=1e-13, epsrel=1e-12, limit=200)[0]
    return V + 4.0 * math.pi * val


def salt_pair_ratio(L, lB, kappa, rc, pIXp, pIXm, rho0NA, eps=1.0):
    """P(one X+ X- pair) / P(no free ion) in a periodic box without ionizable
    groups, with interacting free ions.

    Summing eq. (QQ) over the positions of one cation and one anion gives the
    weight (a b / V^2) int int exp(-u(|r1 - r2|)) dr1 dr2 = a b J / V with
    a = rho0 NA V 10^-pIX+, b likewise with pIX-, and J the pair integral of
    ``_attractive_pair_J`` (minimum image, rc < L/2); the empty box has weight
    1.  The ratio is exact: states with more pairs do not enter it."""
    V = L ** 3
    a = rho0NA * V * 10.0 ** (-pIXp)
    b = rho0NA * V * 10.0 ** (-pIXm)
    return a * b * _attractive_pair_J(L, lB, kappa, rc, eps) / V


def one_site_ion_probability(L, lB, kappa, rc, pH, pKa, pIX, rho0NA, eps=1.0):
    """One acid site and its counterion in the dilute-salt limit.

    States: neutral site, no ions (weight 1); charged site plus one X+ anywhere
    (weight K z J with K = 10^(pH-pKa), z = rho0 NA 10^-pIX and
    J = V + 4 pi int_0^rc r^2 (exp(-u(r)) - 1) dr, u the site-ion Coulomb plus
    excluded volume).  Salt pairs enter at O(a^2) with a = rho0 NA V 10^-pIX."""
    V = L ** 3

    def u(r):
        e = -lB * math.exp(-kappa * r) / r if lB else 0.0
        if eps > 0.0 and r < 2.0 ** (1.0 / 6.0):
            e += 4.0 * eps * (r ** -12 - r ** -6) + eps
        return e

    def integrand(r):
        if eps > 0.0 and r < 0.5:  # hard core of the excluded volume
            return -r * r
        return r * r * (math.exp(-u(r)) - 1.0)

    pts = [0.5, 2.0 ** (1.0 / 6.0)]
    val = 0.0
    edges = [0.0] + pts + [rc]
    for a, b in zip(edges[:-1], edges[1:]):
        val += integrate.quad(integrand, a, b, epsabs=1e-13, epsrel=1e-12, limit=200)[0]
    J = V + 4.0 * math.pi * val
    x = 10.0 ** (pH - pKa) * rho0NA * 10.0 ** (-pIX) * J
    return x / (1.0 + x)
