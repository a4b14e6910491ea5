"""Seeded synthetic inputs for CR-MC runs.

This module only builds geometry and condition tables (numpy PCG64 streams);
it holds none of the Monte Carlo arithmetic, so both the GPU path's tests and
the oracle's tests may use it.

Every system is a dict with
  L        box edge (sigma units), periodic cube
  xyz      (n,3) float64 particle positions (sites first, in input order)
  kind     (n,) int32   1 acid, 2 base, 3 free cation, 4 free anion, 5 neutral bead
  group    (n,) int32   group id of each site (chain or nanoparticle index)
  core_xyz (m,3) float64 nanoparticle core centres, core_R (m,) radii
plus the model parameters (lB, kappa, rc) and the conditions it is run at.
"""
from __future__ import annotations

import math

import numpy as np

RHO0NA = 0.0269424  # rho0 NA in sigma^-3 for rho0 = 1 M and sigma = 0.355 nm (lB = 2 sigma)


def pIX_from_salt(pIS: float, pH: float, pKw: float = 14.0) -> float:
    """Combined-ion chemical potential from a symmetric salt pI_S and the pH
    (the grouping relation for a non-neutral reservoir)."""
    return -math.log10(10.0 ** (-pIS) + 10.0 ** (-min(pH, pKw - pH)))


def cells_per_dim(L: float, rc: float) -> int:
    """Largest even number of cells per edge whose width is at least rc."""
    n = int(math.floor(L / rc + 1e-12))
    if n % 2:
        n -= 1
    if n < 4:
        raise ValueError("box too small for the cell schedule (need L >= 4 rc)")
    return n


def random_walk_chain(n: int, L: float, rng: np.random.Generator, step: float = 0.97,
                      min_dist: float = 1.0, max_tries: int = 200) -> np.ndarray:
    """Self-avoiding bead-spring chain: steps of fixed length in random
    directions, rejecting any step that brings the new bead closer than
    min_dist to a non-bonded bead (minimum image)."""
    pos = np.zeros((n, 3))
    pos[0] = rng.uniform(0, L, 3)
    i = 1
    restarts = 0
    while i < n:
        ok = False
        for _ in range(max_tries):
            v = rng.normal(size=3)
            v *= step / np.linalg.norm(v)
            p = pos[i - 1] + v
            if i >= 2:
                d = pos[: i - 1] - p
                d -= L * np.round(d / L)
                if np.min(np.einsum("ij,ij->i", d, d)) < min_dist * min_dist:
                    continue
            ok = True
            break
        if ok:
            pos[i] = p
            i += 1
        else:  # stuck: back off a few beads
            restarts += 1
            i = max(1, i - 5)
            if restarts > 10000:
                raise RuntimeError("chain growth failed")
    return np.mod(pos, L)


def sphere_points(m: int, radius: float, rng: np.random.Generator) -> np.ndarray:
    v = rng.normal(size=(m, 3))
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    return v * radius


def _system(L, xyz, kind, group, core_xyz=None, core_R=None, **kw):
    d = dict(L=float(L), xyz=np.ascontiguousarray(xyz, dtype=np.float64),
             kind=np.ascontiguousarray(kind, dtype=np.int32),
             group=np.ascontiguousarray(group, dtype=np.int32),
             core_xyz=np.zeros((0, 3)) if core_xyz is None else np.asarray(core_xyz, dtype=np.float64),
             core_R=np.zeros(0) if core_R is None else np.asarray(core_R, dtype=np.float64))
    d.update(kw)
    return d


# --------------------------------------------------------------------------
# the five benchmark systems
# --------------------------------------------------------------------------
def config1(seed: int = 1):
    """Single weak-acid chain: 40 acid beads, pKa = pH = 4.5, L = 40,
    lB = 2, kappa = 0.5, rc = 6, salt pI_S = 2."""
    rng = np.random.default_rng(seed)
    L = 40.0
    xyz = random_walk_chain(40, L, rng)
    pH = 4.5
    return _system(L, xyz, np.full(40, 1), np.zeros(40), lB=2.0, kappa=0.5, rc=6.0,
                   pH=pH, pKa=4.5, pKb=5.0, pIX=pIX_from_salt(2.0, pH), name="weak-acid chain, 40 sites")


def nanoparticle_pair(seed: int = 2, L: float = 120.0, R: float = 10.0, sites: int = 2000,
                      separation: float = 25.0):
    """Acid-coated and base-coated spheres (cores of radius R, sites uniform on
    the shell of radius R - 1/2) at the given centre separation."""
    rng = np.random.default_rng(seed)
    c = L / 2.0
    ca = np.array([c - separation / 2, c, c])
    cb = np.array([c + separation / 2, c, c])
    xa = ca + sphere_points(sites, R - 0.5, rng)
    xb = cb + sphere_points(sites, R - 0.5, rng)
    xyz = np.concatenate([xa, xb])
    kind = np.concatenate([np.full(sites, 1), np.full(sites, 2)])
    group = np.concatenate([np.zeros(sites), np.ones(sites)])
    return _system(L, xyz, kind, group, core_xyz=np.stack([ca, cb]), core_R=np.array([R, R]))


def config2(seed: int = 2):
    """Two oppositely charged nanoparticles (R = 10, 2000 acid / 2000 base
    sites, pKa = 5, pKb = 5) at separation 25 in L = 120, rc = 8, ~2x10^4 ions
    (pI_X = 0.668), scanned over pH 3..11."""
    s = nanoparticle_pair(seed)
    s.update(lB=2.0, kappa=0.5, rc=8.0, pKa=5.0, pKb=5.0, pIX=0.668,
             pH_list=[3.0 + i for i in range(9)], name="nanoparticle pair, 4000 sites, pH 3..11")
    return s


def config3(seed: int = 3):
    """256 weak-polyelectrolyte chains of uneven length (50..2000 sites) on a
    16 x 16 grid of pH (2..12) and kappa (0.1..1.0); lB = 2, rc = 6, pKa 4.5,
    pI_S = 2; box edge L_r = 12 ceil(40 (N_r/40)^(1/3) / 12)."""
    rng = np.random.default_rng(seed)
    N = rng.integers(50, 2001, size=256)
    reps = []
    for r in range(256):
        i, j = divmod(r, 16)
        pH = 2.0 + 10.0 * i / 15.0
        kappa = 0.1 + 0.9 * j / 15.0
        n = int(N[r])
        L = 12.0 * math.ceil(40.0 * (n / 40.0) ** (1.0 / 3.0) / 12.0)
        xyz = random_walk_chain(n, L, np.random.default_rng([seed, r]))
        reps.append(_system(L, xyz, np.full(n, 1), np.zeros(n), lB=2.0, kappa=kappa, rc=6.0,
                            pH=pH, pKa=4.5, pKb=5.0, pIX=pIX_from_salt(2.0, pH)))
    return reps


def config5(seed: int = 5, n_np: int = 64, L: float = 300.0, R: float = 8.0, sites: int = 800):
    """Dense suspension: 64 nanoparticles (R = 8, 800 sites each at radius 7.5;
    32 acid-coated, 32 base-coated) with centres >= 18 apart in L = 300;
    rc = 8, kappa = 0.5, lB = 2, pI_X = 0.862, 8 replicas at pH 3..10."""
    rng = np.random.default_rng(seed)
    centres = []
    while len(centres) < n_np:
        p = rng.uniform(0, L, 3)
        ok = True
        for q in centres:
            d = p - q
            d -= L * np.round(d / L)
            if d @ d < 18.0 ** 2:
                ok = False
                break
        if ok:
            centres.append(p)
    centres = np.array(centres)
    xyz, kind, group = [], [], []
    for g, c in enumerate(centres):
        xyz.append(c + sphere_points(sites, R - 0.5, rng))
        kind.append(np.full(sites, 1 if g < n_np // 2 else 2))
        group.append(np.full(sites, g))
    s = _system(L, np.mod(np.concatenate(xyz), L), np.concatenate(kind), np.concatenate(group),
                core_xyz=centres, core_R=np.full(n_np, R))
    s.update(lB=2.0, kappa=0.5, rc=8.0, pKa=5.0, pKb=5.0, pIX=0.862,
             pH_list=[3.0 + i for i in range(8)], name="64-nanoparticle suspension, 51,200 sites")
    return s


# --------------------------------------------------------------------------
# small systems for exact checks
# --------------------------------------------------------------------------
def ring(n: int = 12, radius: float = 2.0, L: float = 40.0):
    """n acid sites on a ring of the given radius in the z = L/2 plane."""
    a = np.arange(n) * 2.0 * np.pi / n
    xyz = np.stack([L / 2 + radius * np.cos(a), L / 2 + radius * np.sin(a), np.full(n, L / 2)], 1)
    return _system(L, xyz, np.full(n, 1), np.zeros(n))


def random_sites(n_acid: int, n_base: int, L: float, seed: int, min_dist: float = 0.0):
    rng = np.random.default_rng(seed)
    pts = []
    while len(pts) < n_acid + n_base:
        p = rng.uniform(0, L, 3)
        if min_dist > 0:
            ok = True
            for q in pts:
                d = p - q
                d -= L * np.round(d / L)
                if d @ d < min_dist ** 2:
                    ok = False
                    break
            if not ok:
                continue
        pts.append(p)
    kind = np.concatenate([np.full(n_acid, 1), np.full(n_base, 2)])
    return _system(L, np.array(pts), kind, np.zeros(n_acid + n_base))
