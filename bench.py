#!/usr/bin/env python
"""Benchmark of the CR-MC hot path on one MI355X.

Workload (default, --workload suspension): 64 nanoparticles (radius 8, 800
surface sites each; 32 acid-coated with pKa 5, 32 base-coated with pKb 5) in
a periodic box L = 300 with about 2x10^5 free ions per replica (pI_X =
0.862), lB = 2, kappa = 0.5, rc = 8, as eight pH replicas (3..10) advanced
together; FP32 pair terms, FP64 sums and acceptance; the learned site
proposal (a 32-128-128-1 network trained on the GPU from rows of the plain
chain) with the plain chain's figures reported beside it.

--workload pair: two oppositely charged nanoparticles (R = 10, 2000 acid
and 2000 base sites, separation 25, L = 120, ~2x10^4 ions), nine pH replicas.
--workload chains: the 256-replica batch of uneven weak-acid chains over a
pH x kappa grid, all replicas advanced by the same launches.

A step is one sweep of every replica: re-binning into the shifted cell grid
plus the eight colour phases (every cell gets `trials` trials; with the
learned proposal each phase starts with the feature-and-network kernel)
plus the end-of-sweep bookkeeping.

Order of a run: build, launch-shape autotuning, --equilibrate plain sweeps
from the neutral start, a plain statistics pass of --stats-sweeps sweeps,
(learned: row collection, training, offset calibration, 100 sweeps, a
learned statistics pass of --stats-sweeps sweeps), --warmup sweeps, then the
timed region of exactly --steps sweeps bracketed by device synchronisation,
then a per-kernel HIP-event pass.  The statistics passes fix tau_int and
<alpha> whatever --steps and --warmup are.

Printed (one JSON line): trial moves/s over the timed region (value);
effectively independent samples/s = sum over replicas of (timed sweeps/s) /
(2 tau_int), tau_int (Sokal, c = 5) of the number of ionized sites from the
statistics pass (null if that pass is shorter than 50 tau_int); <alpha> with
standard errors; the plain chain's figures and the largest deviation of the
learned chain's <alpha> from the plain one in standard errors; the roofline
of the phase kernel measured with HIP events around its launches; and the
oracle's own rate on a bounded sample on the host cores.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
SERIES_WINDOW = 16384  # sweeps of the per-sweep series the library retains
sys.path.insert(0, ROOT)

METRIC = "CR-MC trial moves/s and indep. samples/s at matched <alpha>; % HBM roofline"
HBM_PEAK_GBS = 8000.0
PHASE_SOURCES = ["paper_2109_07527_amd/csrc/crmc_kernels.hip"]


def phase_source_hash() -> str:
    h = hashlib.sha256()
    for p in PHASE_SOURCES:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def stencil_bytes_per_sweep(n_records: float, n_cells: int) -> float:
    """Algorithmic bytes the phase kernels move per sweep with the 27-cell
    neighbourhood method: every record is read once as a member of its own
    cell, 26 times as a neighbour and written back once (16 B each); every
    cell count is read 27 times and written once (4 B)."""
    return n_records * 16.0 * 28.0 + n_cells * 4.0 * 28.0


def read_traffic(args, path, tuned):
    """HBM bytes per phase launch from the committed counter summary, if it
    was taken on this kernel source with this launch configuration."""
    if not path or not os.path.exists(path):
        return None
    kv = {}
    with open(path) as f:
        for line in f:
            if line.startswith("- ") and ": " in line:
                k, v = line[2:].split(": ", 1)
                kv[k.strip()] = v.strip().strip("`")
    lds = tuned["lds_records"] if tuned else args.lds_records
    light = tuned["light_neighbours"] if tuned else args.light_neighbours
    want = {"source_hash": phase_source_hash(), "trials_per_cell": str(args.trials),
            "precision": str(args.precision), "lds_records": str(lds),
            "site_trials": str(args.site_trials), "light_neighbours": str(light)}
    if args.ion_trials:
        return None  # the counters were taken on the paper's six moves only
    if any(kv.get(k) != v for k, v in want.items()) or "bytes_per_launch" not in kv:
        return None
    return float(kv["bytes_per_launch"])


def calibrate_offsets(S, systems, first, count):
    """Per replica and site kind, the logit offset d with mean over the
    replica's acid (base) sites of logistic(z_i + d) equal to their ionized
    fraction over the given sweeps; z_i are the logits the kernels used in
    the latest sweep.  Any fixed offsets keep the chain exact."""
    import numpy as np
    out = []
    for r, sy in enumerate(systems):
        p = S.site_probabilities(r)
        ser = S.series(r, first, count).astype(np.float64)
        kind = np.asarray(sy["kind"])
        pair = []
        for col, k in ((0, 1), (1, 2)):
            m = kind[:p.size] == k
            if not m.any():
                pair.append(0.0)
                continue
            z = np.log(p[m] / (1.0 - p[m]))
            target = min(max(ser[:, col].mean() / m.sum(), 1e-4), 1.0 - 1e-4)
            lo, hi = -30.0, 30.0
            for _ in range(60):
                mid = 0.5 * (lo + hi)
                if np.mean(1.0 / (1.0 + np.exp(-(z + mid)))) < target:
                    lo = mid
                else:
                    hi = mid
            pair.append(round(0.5 * (lo + hi), 4))
        S.set_proposal_offsets(r, pair[0], pair[1])
        out.append(pair)
    return out


def cpu_baseline(system, cond, trials, site_trials, seconds, replica=4, pairing=True, ion_trials=0, trial_chunk=0):
    """The oracle as it stands (plain FP64 C, one core) on the same system at
    one pH, started from the same neutral state; rate over the sweeps of the
    last half of the sample.  The oracle's trial costs O(N): it copies the
    domain's particles into one array and sums the energy change over every
    particle of the system.  With trial_chunk > 0 each sweep runs only its
    first trial_chunk trials (a bounded sample of a sweep that would take
    minutes)."""
    import oracle
    o = oracle.Oracle(system["L"], system["n_cells"], system["lB"], cond["kappa"], system["rc"],
                      eps=1.0, seed=2024, replica=replica)
    o.set_conditions(cond["pH"], cond["pKa"], cond["pKb"], cond["pIX_pos"], cond["pIX_neg"])
    o.set_particles(system["xyz"], system["kind"])
    if len(system.get("core_R", [])):
        o.set_cores(system["core_xyz"], system["core_R"])
    o.set_schedule(trials, pairing=pairing, site_trials=site_trials, ion_trials=ion_trials)
    t_start = time.perf_counter()
    marks = []

    def attempted_o():
        return int(sum(o.move_stats()[0])) + o.relocation_stats()[0]
    while True:
        a0 = attempted_o()
        if trial_chunk:
            o.set_trial_limit(trial_chunk)
        t0 = time.perf_counter()
        o.sweeps(1, series=False)
        t1 = time.perf_counter()
        marks.append((t1 - t0, attempted_o() - a0))
        if t1 - t_start > seconds:
            break
    tail = marks[len(marks) // 2:]
    dt = sum(m[0] for m in tail)
    n = sum(m[1] for m in tail)
    c = o.counts()
    what = ("the first %d trials of each sweep" % trial_chunk) if trial_chunk else "whole sweeps"
    return {"value": n / dt, "unit": "trial moves/s", "cores": 1, "kind": "oracle",
            "sample": "one replica (pH %.0f) of the same system from the neutral start, %s, %d sweeps in %.0f s; "
                      "rate over the last %d sweeps (%d free ions at the end); the oracle's trial is O(N) in the "
                      "particle count (whole-system copy and energy sum)"
                      % (cond["pH"], what, len(marks), time.perf_counter() - t_start, len(tail),
                         c["nXp"] + c["nXm"])}


def host_cpu():
    """The host's CPU model and logical CPU count, for the baseline's record."""
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return "%s; %d logical CPUs, %d in this process's share" % (model or "unknown CPU", os.cpu_count() or 0,
                                                                 len(os.sched_getaffinity(0)))


def cpu_worker(spec):
    """One oracle baseline run in a process of its own (no GPU use): one
    replica of the chain batch, printed as a JSON line."""
    from workloads import config3
    r = spec["replica"]
    sysd = dict(config3()[r])
    sysd["n_cells"] = spec["n_cells"]
    cond = dict(pH=sysd["pH"], pKa=sysd["pKa"], pKb=sysd["pKb"], pIX_pos=sysd["pIX"], pIX_neg=sysd["pIX"],
                kappa=sysd["kappa"])
    res = cpu_baseline(sysd, cond, spec["trials"], spec["site_trials"], spec["seconds"], replica=r,
                       pairing=spec["pairing"], ion_trials=spec["ion_trials"])
    res["replica"], res["sites"] = r, len(sysd["kind"])
    print(json.dumps(res), flush=True)


def cpu_baseline_cores(systems, after, args, cores):
    """The chain batch on the host: one replica per core (chains spread over
    the length range), each timed like cpu_baseline in a child process; the
    host's rate is the sum of the per-core rates."""
    import subprocess
    import numpy as np
    order = np.argsort([len(sy["kind"]) for sy in systems])
    picks = [int(order[round(i * (len(order) - 1) / max(cores - 1, 1))]) for i in range(cores)]
    env = dict(os.environ, OMP_NUM_THREADS="1")
    procs = []
    for r in picks:
        spec = dict(replica=r, n_cells=after[r]["n_cells"], trials=args.trials, site_trials=args.site_trials,
                    ion_trials=args.ion_trials, seconds=args.cpu_seconds, pairing=not args.no_pairing)
        procs.append(subprocess.Popen([sys.executable, os.path.abspath(__file__), "--cpu-worker", json.dumps(spec)],
                                      stdout=subprocess.PIPE, env=env, cwd=ROOT))
    outs = []
    for p in procs:
        out, _ = p.communicate()
        if p.returncode != 0:
            raise RuntimeError("oracle baseline worker failed")
        outs.append(json.loads(out.decode().strip().splitlines()[-1]))
    sizes = sorted(o["sites"] for o in outs)
    return {"value": sum(o["value"] for o in outs), "unit": "trial moves/s", "cores": len(outs), "kind": "oracle",
            "sample": "one chain per core (%d chains of %d..%d sites spread over the length range), each from the "
                      "neutral start for about %.0f s; per-core rate over the last half of its sweeps, summed"
                      % (len(outs), sizes[0], sizes[-1], args.cpu_seconds)}


WORKLOADS = {
    "pair": "nanoparticle pair: 2000 acid + 2000 base sites, R=10, separation 25, L=120, ~2e4 ions "
            "(pI_X=0.668), lB=2, kappa=0.5, rc=8; 9 replicas pH 3..11",
    "chains": "256 weak-acid chains of seeded uneven length 50..2000 (pKa 4.5, pI_S 2), 16x16 grid of "
              "pH 2..12 x kappa 0.1..1.0, lB=2, rc=6, L_r = 12 ceil(40 (N_r/40)^(1/3) / 12); one launch per phase",
    "suspension": "64 nanoparticles (R=8, 800 sites each, 32 acid- and 32 base-coated, pKa=pKb=5) in L=300, "
                  "~2e5 ions (pI_X=0.862), lB=2, kappa=0.5, rc=8; 8 replicas pH 3..10",
}
TRAFFIC_FILES = {
    ("pair", False): os.path.join(ROOT, "profiles", "k_phase_nanoparticle_pair_traffic.md"),
    ("suspension", True): os.path.join(ROOT, "profiles", "k_phase_suspension_learned_traffic.md"),
    ("suspension", False): os.path.join(ROOT, "profiles", "k_phase_suspension_plain_traffic.md"),
}


def phase_kernel_name(precision, learned, reloc):
    """The phase kernel a sweep of this configuration launches (as rocprofv3 names it)."""
    m = "true" if reloc else "false"
    if learned and precision == 32:
        return "k_phase_learned32<%s>" % m
    return "k_phase<%s, %s, %s>" % ("float" if precision == 32 else "double", "true" if learned else "false", m)


def load_workload(name):
    """(systems, per-replica conditions, model constants) of a workload."""
    from workloads import config2, config3, config5
    if name in ("pair", "suspension"):
        c = config2() if name == "pair" else config5()
        conds = [dict(pH=pH, pKa=c["pKa"], pKb=c["pKb"], pIX_pos=c["pIX"], pIX_neg=c["pIX"], kappa=c["kappa"])
                 for pH in c["pH_list"]]
        return [c] * len(conds), conds, dict(lB=c["lB"], rc=c["rc"])
    reps = config3()
    conds = [dict(pH=r["pH"], pKa=r["pKa"], pKb=r["pKb"], pIX_pos=r["pIX"], pIX_neg=r["pIX"], kappa=r["kappa"])
             for r in reps]
    return reps, conds, dict(lB=reps[0]["lB"], rc=reps[0]["rc"])


def attempted(obs):
    return sum(o["attempts"][i] for o in obs for i in range(6)) + sum(o["relocation_attempts"] for o in obs)


def stats_pass(S, conds, systems, sweeps, torch):
    """An untimed-for-the-headline pass of fixed length: per replica tau_int
    (Sokal, c = 5) of n_A- + n_B+ in sweeps, <alpha> of the acid and the base
    sites with standard errors, and the pass's own trial moves/s and
    sweeps/s (graph replay, device-synchronised).  tau is reported as null
    when the pass is shorter than 50 tau."""
    import numpy as np
    from paper_2109_07527_amd.stats import mean_se, tau_int
    R = len(conds)
    before = [S.observe(r) for r in range(R)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    S.sweep_ex(conds, sweeps)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    after = [S.observe(r) for r in range(R)]
    for o in after:
        if o["status"] != 0:
            raise SystemExit("device error: %s" % o)
    first = before[0]["sweeps"]
    out = {"sweeps": sweeps, "seconds": round(dt, 3), "trial_moves_per_s": round((attempted(after) - attempted(before)) / dt, 1),
           "sweeps_per_s": round(sweeps / dt, 3), "tau_int_sweeps": [], "alpha_acid": [], "alpha_acid_se": [],
           "alpha_base": [], "alpha_base_se": []}
    samples, valid = 0.0, True
    for r in range(R):
        ser = S.series(r, first, sweeps).astype(np.float64)
        t = tau_int(ser[:, 0] + ser[:, 1])
        if sweeps < 50.0 * t:
            valid = False
        out["tau_int_sweeps"].append(round(t, 2))
        samples += (sweeps / dt) / (2.0 * t)
        nA, nB = max(after[r]["n_acid"], 1), max(after[r]["n_base"], 1)
        ma, sa, _ = mean_se(ser[:, 0] / nA)
        mb, sb, _ = mean_se(ser[:, 1] / nB)
        out["alpha_acid"].append(round(ma, 6))
        out["alpha_acid_se"].append(round(sa, 6))
        out["alpha_base"].append(round(mb, 6))
        out["alpha_base_se"].append(round(sb, 6))
    out["independent_samples_per_s"] = round(samples, 2) if valid else None
    out["window_over_50_tau"] = valid
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--workload", choices=sorted(WORKLOADS), default="suspension")
    ap.add_argument("--steps", type=int, default=None, help="timed sweeps (default 300 suspension, 3000 pair, "
                                                            "1000 chains)")
    ap.add_argument("--warmup", type=int, default=20, help="untimed sweeps right before the timed region")
    ap.add_argument("--equilibrate", type=int, default=None,
                    help="plain sweeps from the neutral start before any measurement (default 600 suspension, "
                         "300 otherwise); independent of --warmup")
    ap.add_argument("--stats-sweeps", type=int, default=None,
                    help="length of each fixed statistics pass (tau_int, <alpha>; default 2500 suspension, "
                         "6000 pair, 1000 chains); independent of --steps")
    ap.add_argument("--trials", type=int, default=8, help="trials per cell per sweep")
    ap.add_argument("--precision", type=int, default=32, choices=(32, 64))
    ap.add_argument("--site-trials", type=int, default=0, help="extra trials per 16 sites of a domain")
    ap.add_argument("--ion-trials", type=int, default=0,
                    help="ion relocation trials per cell of a domain per phase (not one of the paper's moves; "
                         "default 0)")
    ap.add_argument("--lds-records", type=int, default=0, help="LDS pool per phase workgroup in records (0 = default)")
    ap.add_argument("--no-graph", action="store_true", help="launch kernels one by one in the timed region")
    ap.add_argument("--md-steps", type=int, default=0, metavar="N",
                    help="after the timed sweeps, time one hybrid-MD block of N Langevin steps (dt 0.005, "
                         "gamma 1) of the free ions and report it under 'md'")
    ap.add_argument("--tune-schedule", type=int, default=0, metavar="SWEEPS",
                    help="first choose trials per cell (4, 8, 16) and pairing by independent samples/s, each "
                         "candidate a chain of its own timed over SWEEPS sweeps (plain proposal)")
    ap.add_argument("--no-pairing", action="store_true",
                    help="single-cell domains instead of reflection-paired cell pairs")
    ap.add_argument("--kernel-steps", type=int, default=200, help="sweeps of the per-kernel event timing pass")
    ap.add_argument("--light-neighbours", type=int, default=0,
                    help="neighbour records up to which a domain runs on one wavefront (0 = library default)")
    ap.add_argument("--autotune", type=int, default=None, metavar="SWEEPS",
                    help="before equilibration, time SWEEPS sweeps per launch shape and keep the fastest "
                         "(default: 5 for the chain batch and the suspension, 0 for the pair)")
    ap.add_argument("--plain", action="store_true",
                    help="time the plain (uniform-pick) chain; the default for the suspension is the learned "
                         "proposal, with the plain chain's figures reported beside it")
    ap.add_argument("--learned", action="store_true", help="learned proposal for the pair or the chain batch")
    ap.add_argument("--train-rows", type=int, default=1_000_000)
    ap.add_argument("--epochs", type=int, default=3)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--learned-eps", type=float, default=0.1)
    ap.add_argument("--no-calibrate", action="store_true",
                    help="leave the per-replica logit offsets at zero (by default they match the mean network "
                         "output of the acid and of the base sites to their ionized fractions)")
    ap.add_argument("--cpu-seconds", type=float, default=20.0)
    ap.add_argument("--cpu-cores", type=int, default=0,
                    help="host cores of the oracle baseline for the chain batch (0 = the process's CPU share, "
                         "at most 16); the single-system workloads use one core")
    ap.add_argument("--cpu-worker", default=None, help=argparse.SUPPRESS)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB ten times (counter calibration) and exit")
    args = ap.parse_args()
    if args.cpu_worker is not None:
        cpu_worker(json.loads(args.cpu_worker))
        return
    wl = args.workload
    if args.steps is None:
        args.steps = {"pair": 3000, "chains": 1000, "suspension": 300}[wl]
    if args.equilibrate is None:
        args.equilibrate = 600 if wl == "suspension" else 300
    if args.stats_sweeps is None:
        args.stats_sweeps = {"pair": 6000, "chains": 1000, "suspension": 2500}[wl]
    if args.autotune is None:
        args.autotune = 0 if wl == "pair" else 5
    if not 0 <= args.stats_sweeps <= SERIES_WINDOW:
        raise SystemExit("--stats-sweeps must lie in 0..%d (the retained series)" % SERIES_WINDOW)
    use_learned = (wl == "suspension" and not args.plain) or args.learned

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py runs on one GPU only: the CR-MC replicas of this workload fit one MI355X "
              "and no multi-GPU path is built (requested --gpus %d, WORLD_SIZE %d)" % (args.gpus, world),
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2109_07527_amd import crmc

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    if args.copy_probe:
        n = args.copy_probe << 20
        src = torch.ones(n, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(10):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes": n, "launches": 10}), flush=True)
        return

    def progress(msg):
        print("[bench] %s" % msg, file=sys.stderr, flush=True)

    systems, conds, model = load_workload(wl)
    R = len(conds)
    schedule = None
    if args.tune_schedule:
        from paper_2109_07527_amd.tune import search_schedule
        schedule = search_schedule(systems, conds, model, trials=(4, 8, 16), pairing=(True, False),
                                   window=args.tune_schedule, equilibrate=args.equilibrate,
                                   precision=args.precision, shape_sweeps=args.autotune)
        args.trials = schedule["best"]["trials_per_cell"]
        args.no_pairing = not schedule["best"]["pairing"]
        progress("schedule: %d trials per cell, %s domains" % (args.trials, "paired" if not args.no_pairing
                                                                 else "single-cell"))
    S = crmc.System(n_replicas=R, lB=model["lB"], rc=model["rc"], eps=1.0, precision=args.precision,
                    trials_per_cell=args.trials, pairing=not args.no_pairing, seed=2024, site_trials=args.site_trials,
                    ion_trials=args.ion_trials,
                    lds_records=args.lds_records, use_graph=not args.no_graph,
                    light_neighbours=args.light_neighbours)
    for r in range(R):
        S.build_cells(r, systems[r])
    tuned = None
    if args.autotune:
        tuned = S.autotune(conds, args.autotune)
        progress("autotuned: %s" % {k: tuned[k] for k in ("light_neighbours", "lds_records")})
    S.sweep_ex(conds, args.equilibrate)
    torch.cuda.synchronize()
    progress("equilibrated (%d sweeps)" % args.equilibrate)

    # the plain chain: its own fixed statistics pass (reported beside a learned headline)
    plain = None
    if args.stats_sweeps:
        plain = stats_pass(S, conds, systems, args.stats_sweeps, torch)
        progress("plain statistics pass done")
    learned, lstats = None, None
    if use_learned:
        # rows from plain sweeps, BF16 matrix-core training, then the learned proposal
        per_sweep = sum(int(((sy["kind"] == 1) | (sy["kind"] == 2)).sum()) for sy in systems)
        S.collect_training(args.train_rows)
        n_collect = max(1, -(-args.train_rows // max(per_sweep, 1)))
        first_row_sweep = S.observe(0)["sweeps"]
        S.sweep_ex(conds, n_collect)
        rows = S.training_rows()
        S.init_proposal_weights(7)
        torch.cuda.synchronize()
        tt = time.perf_counter()
        loss = S.train(args.epochs, batch=1024, lr=args.lr, seed=7)
        torch.cuda.synchronize()
        train_s = time.perf_counter() - tt
        S.collect_training(0)
        S.set_proposal(True, args.learned_eps)
        offsets = None
        if not args.no_calibrate:
            S.sweep_ex(conds, 1)
            # the ionized fractions of the plain statistics pass (or of the collection sweeps)
            if plain is not None:
                offsets = calibrate_offsets(S, systems, first_row_sweep - args.stats_sweeps, args.stats_sweeps)
            else:
                offsets = calibrate_offsets(S, systems, first_row_sweep, n_collect)
        S.sweep_ex(conds, 100)
        torch.cuda.synchronize()
        learned = {"train_rows": int(rows), "epochs": args.epochs, "batch": 1024, "lr": args.lr,
                   "final_loss": round(loss, 5), "train_seconds": round(train_s, 3), "eps": args.learned_eps,
                   "logit_offsets": offsets}
        progress("trained (loss %.4f); learned statistics pass" % loss)
        lstats = stats_pass(S, conds, systems, args.stats_sweeps, torch) if args.stats_sweeps else None
        progress("learned statistics pass done")

    S.sweep_ex(conds, args.warmup)
    before = [S.observe(r) for r in range(R)]
    # timed region: exactly --steps sweeps, replayed as captured graphs
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    S.sweep_ex(conds, args.steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    after = [S.observe(r) for r in range(R)]
    for o in after:
        if o["status"] != 0:
            raise SystemExit("device error: %s" % o)
    elapsed = t1 - t0
    progress("timed region: %d sweeps in %.3f s" % (args.steps, elapsed))

    # kernel durations: the same kernels launched one by one, each bracketed
    # by HIP events on the library's stream
    n_kern = min(max(args.steps, 20), args.kernel_steps)
    crmc.crmc_set_timing(S.h, True)
    S.sweep_ex(conds, n_kern)
    torch.cuda.synchronize()
    ms, launches = crmc.crmc_get_timing(S.h)
    crmc.crmc_set_timing(S.h, False)
    trials = attempted(after) - attempted(before)
    accepts = sum(sum(a["accepts"]) - sum(b["accepts"]) for a, b in zip(after, before))
    rate = trials / elapsed
    sweeps_per_s = args.steps / elapsed

    # roofline of the phase kernel
    n_rec = [0.5 * (a["n_acid"] + a["n_base"] + a["n_xpos"] + a["n_xneg"]
                    + b["n_acid"] + b["n_base"] + b["n_xpos"] + b["n_xneg"]) for a, b in zip(after, before)]
    cells = [a["n_cells"] ** 3 for a in after]
    bytes_sweep = sum(stencil_bytes_per_sweep(n, k) for n, k in zip(n_rec, cells))
    bytes_launch = bytes_sweep / 8.0
    phase_avg_ms = ms[1] / max(launches[1], 1)
    achieved = bytes_launch / (phase_avg_ms * 1e-3) / 1e9
    traffic = read_traffic(args, TRAFFIC_FILES.get((wl, use_learned)), tuned)
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                "kernel": phase_kernel_name(args.precision, use_learned, args.ion_trials > 0),
                "bytes_per_launch": round(bytes_launch), "avg_launch_ms": round(phase_avg_ms, 5),
                "timed_launches": int(launches[1])}

    config = {"workload": WORKLOADS[wl] + ("; learned proposal (MLP 32-128-128-1, BF16/FP32)" if use_learned else ""),
              "replicas": R, "trials_per_cell": args.trials,
              "site_trials_per_16": args.site_trials, "ion_trials_per_cell": args.ion_trials,
              "graph": not args.no_graph,
              "light_neighbours": args.light_neighbours, "lds_records": args.lds_records,
              "schedule": "shifted cells, " + ("single-cell domains" if args.no_pairing else "paired domains"),
              "proposal": "learned" if use_learned else "uniform",
              "cells_total": int(sum(cells)), "records_mean": round(float(sum(n_rec)), 1),
              "equilibrate_sweeps": args.equilibrate, "stats_sweeps": args.stats_sweeps}
    if learned is not None:
        config["learned_proposal"] = learned
    if tuned is not None:
        config["autotuned"] = {"light_neighbours": tuned["light_neighbours"], "lds_records": tuned["lds_records"],
                               "candidates": len(tuned["candidates"]),
                               "best_ms_per_sweep": round(tuned["best_ms_per_sweep"], 4)}
    if wl != "chains":
        config.update(cells_per_edge=after[0]["n_cells"], cell_capacity=after[0]["cell_capacity"])
    if schedule is not None:
        config["schedule_search"] = [{k: c[k] for k in ("trials_per_cell", "pairing", "ms_per_sweep",
                                                        "independent_samples_per_s", "window_over_50_tau")}
                                     for c in schedule["candidates"]]
    head = lstats if use_learned else plain
    samples = None
    if head is not None and head["independent_samples_per_s"] is not None:
        # tau from the statistics pass, sweeps/s from the timed region
        samples = round(sum(sweeps_per_s / (2.0 * t) for t in head["tau_int_sweeps"]), 2)
    line = {
        "metric": METRIC, "value": round(rate, 1), "unit": "trial moves/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(elapsed / args.steps * 1e3, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32" if args.precision == 32 else "f64", "data": "synthetic",
        "config": config,
        "independent_samples_per_s": samples,
        "acceptance": round(accepts / max(trials, 1), 4),
        "kernel_ms": {"bin_plan_learn": round(ms[0] / max(launches[0], 1), 5), "phase": round(phase_avg_ms, 5),
                      "sweep_end": round(ms[2] / max(launches[2], 1), 5)},
        "roofline": roofline,
        "cpu_baseline": None,
    }
    if args.md_steps:
        # one block of the hybrid protocol: start velocities, N velocity-Verlet steps with the
        # Langevin thermostat, re-binning after every drift, and the energy restart at the end
        S.md(10, 0.005, 1.0)
        torch.cuda.synchronize()
        ions = sum(S.observe(r)["n_xpos"] + S.observe(r)["n_xneg"] for r in range(R))
        t0 = time.perf_counter()
        S.md(args.md_steps, 0.005, 1.0)
        torch.cuda.synchronize()
        md_s = time.perf_counter() - t0
        line["md"] = {"steps": args.md_steps, "dt": 0.005, "gamma": 1.0, "ions": int(ions),
                      "ms_per_block": round(1e3 * md_s, 3), "ms_per_step": round(1e3 * md_s / args.md_steps, 4),
                      "ion_steps_per_s": round(ions * args.md_steps / md_s, 1)}
    if head is not None:
        line["stats"] = head
    if use_learned and plain is not None and lstats is not None:
        line["plain"] = plain
        # matched <alpha>: the learned chain against the plain one, replica by replica
        dev = []
        for key in ("alpha_acid", "alpha_base"):
            for r in range(R):
                se = math.hypot(lstats[key + "_se"][r], plain[key + "_se"][r])
                dev.append(abs(lstats[key][r] - plain[key][r]) / se if se > 0 else 0.0)
        line["matched_alpha_max_dev_se"] = round(max(dev), 2)
        if plain["independent_samples_per_s"] and samples:
            line["learned_vs_plain_samples"] = round(samples / plain["independent_samples_per_s"], 3)
    if not args.no_cpu_baseline:
        rb = {"pair": 4, "suspension": 4}.get(wl)
        if rb is None:
            rb = int(np.argsort([len(sy["kind"]) for sy in systems])[R // 2])
        sysd = dict(systems[rb])
        sysd["n_cells"] = after[rb]["n_cells"]
        sysd["lB"], sysd["rc"] = model["lB"], model["rc"]
        progress("oracle baseline on the host")
        if wl == "chains":
            cores = args.cpu_cores or min(16, len(os.sched_getaffinity(0)))
            line["cpu_baseline"] = cpu_baseline_cores(systems, after, args, cores)
        else:
            line["cpu_baseline"] = cpu_baseline(sysd, conds[rb], args.trials, args.site_trials, args.cpu_seconds,
                                                replica=rb, pairing=not args.no_pairing, ion_trials=args.ion_trials,
                                                trial_chunk=2000 if wl == "suspension" else 0)
        line["cpu_baseline"]["host"] = host_cpu()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
