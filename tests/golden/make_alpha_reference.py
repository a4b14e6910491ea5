"""Writes tests/golden/chain40_alpha.json from oracle/ only.

Reference <alpha> and distribution of the number of ionized sites of the
40-site weak-acid chain with interacting ions
(l_B = 2, kappa = 0.5, rc = 6, WCA on, L = 40, pKa = 4.5, salt pI_S = 2 and
pI_X from eq. pIXgen) at three pH values, from the oracle's paper-mode chain:
the six moves of Sec. II C with participants drawn from the whole box and ions
inserted anywhere in it.  No closed form exists here; the paper-mode chain is
the plainest sampler of eq. (QQ).  Each pH runs independent seeds; a
reference value is the mean of the per-seed values and its standard error the
spread of those values over sqrt(seeds).
Run: python tests/golden/make_alpha_reference.py   (about a minute on 8 cores)
"""
import json
import os
import sys
from multiprocessing import Pool

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle  # noqa: E402
from oracle import closed_forms as cf  # noqa: E402
from workloads import config1  # noqa: E402

PH = [3.5, 4.5, 5.5]
SEEDS = 8
TRIALS = 3_000_000
EVERY = 100


def one(args):
    pH, seed = args
    c = config1()
    pIX = cf.pIX_from_salt(2.0, pH)
    o = oracle.Oracle(c["L"], 6, c["lB"], c["kappa"], c["rc"], eps=1.0, seed=1000 + seed)
    o.set_conditions(pH, c["pKa"], c["pKb"], pIX, pIX)
    o.set_particles(c["xyz"], c["kind"])
    s = o.paper_trials(TRIALS, EVERY)
    n = s[len(s) // 10:, 0]
    hist = np.bincount(n, minlength=len(c["kind"]) + 1) / len(n)
    return float(n.mean() / len(c["kind"])), hist.tolist()


def main():
    jobs = [(pH, k) for pH in PH for k in range(SEEDS)]
    with Pool(min(8, os.cpu_count() or 1)) as p:
        res = p.map(one, jobs)
    out = {"system": "config1 geometry (40 acid sites, random walk, seed 1), lB 2, kappa 0.5, rc 6, eps 1, "
                     "L 40, pKa 4.5, pI_S 2", "sampler": "oracle paper mode", "trials_per_seed": TRIALS,
           "seeds": SEEDS, "burn_in_fraction": 0.1, "points": []}
    for i, pH in enumerate(PH):
        m = np.array([a for a, _ in res[i * SEEDS:(i + 1) * SEEDS]])
        h = np.array([q for _, q in res[i * SEEDS:(i + 1) * SEEDS]])
        out["points"].append({"pH": pH, "pIX": cf.pIX_from_salt(2.0, pH), "alpha": float(m.mean()),
                              "se": float(m.std(ddof=1) / np.sqrt(SEEDS)),
                              "P_nA": h.mean(axis=0).tolist(),
                              "P_nA_se": (h.std(axis=0, ddof=1) / np.sqrt(SEEDS)).tolist()})
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "chain40_alpha.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
