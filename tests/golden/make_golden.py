"""Writes tests/golden/closed_forms.json from oracle/ only.

Exact values of the grand-canonical weight eq. (QQ) used by the tests:
the ideal-ion degree of ionisation of 40 acid sites in L = 40 (pKa = pH = 4.5,
salt pI_S -1..3) and the exact 2^12 enumeration of a 12-site acid ring
(radius 2, L = 40, lB = 2 and 0, kappa = 0.5, rc = 6, pI_S = 1).
Run: python tests/golden/make_golden.py
"""
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from oracle import closed_forms as cf  # noqa: E402
from workloads import ring  # noqa: E402

RHO = 0.0269424


def main():
    out = {"ideal_alpha_nA40_L40": []}
    for pIS in [-1.0, 0.0, 1.0, 2.0, 3.0]:
        pIX = cf.pIX_from_salt(pIS, 4.5)
        out["ideal_alpha_nA40_L40"].append(
            {"pIS": pIS, "pIX": pIX, "alpha": cf.ideal_alpha(40, 4.5, 4.5, pIX, pIX, 64000.0, RHO),
             "alpha_donnan_hh": cf.donnan_hh_alpha(40, 4.5, 4.5, pIX, pIX, 64000.0, RHO)})
    s = ring(12)
    X = oracle.to_fixed(s["xyz"], s["L"])
    pIX = cf.pIX_from_salt(1.0, 4.5)
    P2, a2, _ = cf.enumerate_sites(X, [1] * 12, 40.0, 2.0, 0.5, 6.0, 4.5, 4.5, 0.0, pIX, pIX, RHO)
    P0, a0, _ = cf.enumerate_sites(X, [1] * 12, 40.0, 0.0, 0.5, 6.0, 4.5, 4.5, 0.0, pIX, pIX, RHO)
    out["ring12"] = {"alpha_lB2": a2, "alpha_lB0": a0, "P_lB2": P2.tolist(), "P_lB0": P0.tolist(),
                     "pIX": pIX}
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "closed_forms.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
