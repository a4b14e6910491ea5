"""What the trained network changes (needs an MI355X).

The learned proposal on the nanoparticle pair (nine pH replicas, the
training recipe of the benchmark: 10^6 rows from plain sweeps, three
epochs, per-replica logit offsets) against the plain chain of the same
handle.  Plain and learned blocks of equal length alternate after a long
equilibration, so a slow drift cannot favour either; the standard error of
the per-sweep mixing sum_r 1/tau_r is taken from the scatter between blocks
(the tau of the extreme-pH replicas has a heavy-tailed estimate, which the
asymptotic formula understates).

Checked: the network fits the labels better than the best constant
predictor; both chains give the same <alpha> per replica; the learned
chain mixes at least as fast per sweep (within three standard errors);
a learned sweep costs more than a plain one.  Printed: the mixing gain,
the sweep cost and their net effect on independent samples/s.
"""
import importlib.util
import math
import os
import time

import numpy as np
import pytest

from workloads import config2

pytestmark = pytest.mark.gpu
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.timeout(600)
def test_learned_proposal_against_plain_on_the_pair():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2109_07527_amd import crmc
    from paper_2109_07527_amd.stats import blocking_se, mean_se, tau_int
    spec = importlib.util.spec_from_file_location("bench", os.path.join(ROOT, "bench.py"))
    bench = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(bench)
    c = config2()
    conds = [dict(pH=pH, pKa=c["pKa"], pKb=c["pKb"], pIX_pos=c["pIX"], pIX_neg=c["pIX"], kappa=c["kappa"])
             for pH in c["pH_list"]]
    R = len(conds)
    S = crmc.System(n_replicas=R, lB=c["lB"], rc=c["rc"], precision=32, trials_per_cell=8, seed=77)
    for r in range(R):
        S.build_cells(r, c)
    neq = 1000
    S.sweep_ex(conds, neq)

    kind = np.asarray(c["kind"])
    rows_per = R * int(((kind == 1) | (kind == 2)).sum())
    S.collect_training(1_000_000)
    first_row = S.observe(0)["sweeps"]
    S.sweep_ex(conds, -(-1_000_000 // rows_per))
    y = S.read_training()[:, 32]
    yb = float(y.mean())
    h_const = -(yb * math.log(yb) + (1 - yb) * math.log(1 - yb))
    S.init_proposal_weights(7)
    loss = S.train(3, batch=1024, lr=1e-3, seed=7)
    assert loss < 0.98 * h_const, (loss, h_const)
    S.collect_training(0)
    S.set_proposal(True, 0.1)
    S.sweep_ex(conds, 1)
    bench.calibrate_offsets(S, [c] * R, first_row - neq // 2, neq // 2)

    nst, nblk = 2000, 3
    out = {m: dict(dt=0.0, inv=[], ser=[]) for m in ("plain", "learned")}
    for _ in range(nblk):
        for mode in ("plain", "learned"):
            S.set_proposal(mode == "learned", 0.1)
            S.sweep_ex(conds, 20)
            f0 = S.observe(0)["sweeps"]
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            S.sweep_ex(conds, nst)
            torch.cuda.synchronize()
            out[mode]["dt"] += time.perf_counter() - t0
            ser = [S.series(r, f0, nst).astype(np.float64) for r in range(R)]
            taus = np.array([tau_int(s[:, 0] + s[:, 1]) for s in ser])
            out[mode]["inv"].append(float((1.0 / taus).sum()))
            out[mode]["ser"].append(ser)
    P, L = out["plain"], out["learned"]
    for r in range(R):
        for k in range(2):
            x1 = np.concatenate([b[r][:, k] for b in L["ser"]]) / 2000.0
            x2 = np.concatenate([b[r][:, k] for b in P["ser"]]) / 2000.0
            (m1, s1, _), (m2, s2, _) = mean_se(x1), mean_se(x2)
            s1, s2 = max(s1, blocking_se(x1)), max(s2, blocking_se(x2))
            assert abs(m1 - m2) < 3.5 * math.hypot(s1, s2) + 1e-12, (r, k, m1, s1, m2, s2)
    mp, ml = float(np.mean(P["inv"])), float(np.mean(L["inv"]))
    sp = float(np.std(P["inv"], ddof=1)) / math.sqrt(nblk)
    sl = float(np.std(L["inv"], ddof=1)) / math.sqrt(nblk)
    assert ml > mp - 3.0 * math.hypot(sp, sl), (L["inv"], P["inv"])
    cost = L["dt"] / P["dt"]
    assert 1.0 < cost < 1.6, cost
    ratio = (ml / L["dt"]) / (mp / P["dt"])
    print("sum 1/tau per block: plain %s, learned %s; means %.3f +- %.3f and %.3f +- %.3f (gain x%.3f); "
          "sweep cost x%.3f; independent samples/s ratio %.3f"
          % (np.round(P["inv"], 3).tolist(), np.round(L["inv"], 3).tolist(), mp, sp, ml, sl, ml / mp, cost, ratio),
          flush=True)
