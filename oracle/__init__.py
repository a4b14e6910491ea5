"""FP64 CPU oracle for charge-regulation Monte Carlo (CR-MC).

TEST INFRASTRUCTURE ONLY: tests, the smoke check and the benchmark's CPU
baseline use it; the product library never imports it.  It shares no code with
the GPU path.

``Oracle`` wraps the plain C implementation in ``crmc_oracle.c`` (paper schedule
and cell schedule, brute-force energies, Philox4x32-10).  ``closed_forms``
holds the exact results the oracle is pinned against.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "crmc_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

ACID, BASE, XPOS, XNEG, NEUTRAL = 1, 2, 3, 4, 5
MOVES = ("acid_fwd", "acid_back", "base_fwd", "base_back", "salt_ins", "salt_del")


def build(force: bool = True) -> str:
    """Compile the oracle with plain gcc (-O2, no SIMD intrinsics)."""
    if force or not os.path.exists(_LIB):
        tmp = "%s.tmp%d" % (_LIB, os.getpid())
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-Wall", "-shared", "-fPIC",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class TrialRecord(C.Structure):
    _fields_ = [("sweep", C.c_int64), ("cell", C.c_int64), ("trial", C.c_int64),
                ("move", C.c_int32), ("status", C.c_int32),
                ("dU", C.c_double), ("lnp", C.c_double), ("u", C.c_double)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        L = C.CDLL(_LIB)
        vp, d, i32, u32, u64, i64 = C.c_void_p, C.c_double, C.c_int32, C.c_uint32, C.c_uint64, C.c_int64
        P = C.POINTER
        L.orc_create.restype = vp
        L.orc_create.argtypes = [d, C.c_int, d, d, d, d, d, C.c_int, u64, u32]
        L.orc_destroy.argtypes = [vp]
        L.orc_set_conditions.argtypes = [vp, d, d, d, d, d, d]
        L.orc_set_kappa.argtypes = [vp, d]
        L.orc_set_schedule.argtypes = [vp, C.c_int, C.c_int, C.c_int, C.c_int]
        L.orc_partner.restype = u32
        L.orc_partner.argtypes = [vp, u64, C.c_int, u32, u32]
        L.orc_set_log.argtypes = [vp, vp, i64]
        L.orc_log_count.restype = i64
        L.orc_log_count.argtypes = [vp]
        L.orc_set_check.argtypes = [vp, C.c_int]
        L.orc_set_trial_limit.argtypes = [vp, i64]
        L.orc_set_ion_trials.argtypes = [vp, C.c_int]
        L.orc_relocation_stats.argtypes = [vp, P(i64)]
        L.orc_max_dU_err.restype = d
        L.orc_max_dU_err.argtypes = [vp]
        L.orc_set_particles.argtypes = [vp, C.c_int, P(u32), P(i32), P(i32), P(i32)]
        L.orc_set_cores.argtypes = [vp, C.c_int, P(u32), P(d)]
        L.orc_num_particles.restype = C.c_int
        L.orc_num_particles.argtypes = [vp]
        L.orc_get_particles.restype = C.c_int
        L.orc_get_particles.argtypes = [vp, C.c_int, P(u32), P(i32), P(i32), P(i32)]
        L.orc_counts.argtypes = [vp, P(i64)]
        L.orc_running_energy.restype = d
        L.orc_running_energy.argtypes = [vp]
        L.orc_energy.restype = d
        L.orc_energy.argtypes = [vp]
        L.orc_sweep_index.restype = u64
        L.orc_sweep_index.argtypes = [vp]
        L.orc_move_stats.argtypes = [vp, P(i64), P(i64)]
        L.orc_sweeps.argtypes = [vp, i64, P(i32)]
        L.orc_paper_trials.argtypes = [vp, i64, i64, P(i32)]
        L.orc_philox.argtypes = [P(u32), P(u32), P(u32)]
        L.orc_cutoff_R2.restype = u64
        L.orc_cutoff_R2.argtypes = [d, d]
        L.orc_to_fixed.argtypes = [i64, P(d), d, P(u32)]
        L.orc_shift.argtypes = [vp, u64, P(u32)]
        L.orc_mlp_params.restype = C.c_int
        L.orc_mlp_logit.restype = d
        L.orc_mlp_logit.argtypes = [P(d), P(d)]
        L.orc_mlp_loss_grad.restype = d
        L.orc_mlp_loss_grad.argtypes = [P(d), P(d), P(d), C.c_int, P(d)]
        L.orc_adam_step.argtypes = [P(d), P(d), P(d), P(d), i64, d, d, d, d]
        L.orc_set_learned.restype = C.c_int
        L.orc_set_learned.argtypes = [vp, P(d), d, C.c_int]
        L.orc_set_learned_offsets.restype = None
        L.orc_set_learned_offsets.argtypes = [vp, d, d]
        L.orc_load_state.restype = C.c_int
        L.orc_load_state.argtypes = [vp, C.c_int, P(u32), P(i32), P(i32), P(i32), u64, C.c_int]
        L.orc_prepare_sweep.argtypes = [vp]
        L.orc_set_domain_filter.argtypes = [vp, C.c_int, P(i32)]
        L.orc_ungroup.argtypes = [vp, P(d), u64, P(i64), P(i32)]
        L.orc_md.restype = d
        L.orc_md.argtypes = [vp, i64, d, d]
        L.orc_forces.argtypes = [vp, P(d)]
        L.orc_features_of_cell_sites.restype = C.c_int
        L.orc_features_of_cell_sites.argtypes = [vp, C.c_int, C.c_int, P(i32), P(d)]
        _lib = L
    return _lib


def _ptr(a, ctype):
    return a.ctypes.data_as(C.POINTER(ctype))


def philox(ctr, key):
    """Philox4x32-10 of one counter block: four 32-bit words."""
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib().orc_philox(_ptr(c, C.c_uint32), _ptr(k, C.c_uint32), _ptr(out, C.c_uint32))
    return out


def to_fixed(xyz, L):
    x = np.ascontiguousarray(xyz, dtype=np.float64).reshape(-1)
    out = np.zeros(x.size, dtype=np.uint32)
    lib().orc_to_fixed(x.size, _ptr(x, C.c_double), float(L), _ptr(out, C.c_uint32))
    return out.reshape(-1, 3)


def cutoff_R2(rc, L):
    return int(lib().orc_cutoff_R2(float(rc), float(L)))


MLP_IN, MLP_H = 32, 128


def mlp_params():
    """Number of network parameters: W1[128][32], b1[128], W2[128][128],
    b2[128], w3[128], b3 in that order."""
    return int(lib().orc_mlp_params())


def mlp_logit(par, x):
    """Network logit for one 32-vector of features (FP64)."""
    par = np.ascontiguousarray(par, dtype=np.float64)
    x = np.ascontiguousarray(x, dtype=np.float64)
    return float(lib().orc_mlp_logit(_ptr(par, C.c_double), _ptr(x, C.c_double)))


def mlp_loss_grad(par, X, y):
    """Mean binary cross-entropy over the rows of X (labels y) and its gradient."""
    par = np.ascontiguousarray(par, dtype=np.float64)
    X = np.ascontiguousarray(X, dtype=np.float64).reshape(-1, MLP_IN)
    y = np.ascontiguousarray(y, dtype=np.float64)
    g = np.zeros(par.size)
    loss = lib().orc_mlp_loss_grad(_ptr(par, C.c_double), _ptr(X, C.c_double), _ptr(y, C.c_double),
                                   X.shape[0], _ptr(g, C.c_double))
    return float(loss), g


def adam_step(par, grad, m, v, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """In place: one Adam step of par (FP64) with moments m, v at step t >= 1."""
    for a in (par, grad, m, v):
        assert a.dtype == np.float64 and a.flags.c_contiguous
    lib().orc_adam_step(_ptr(par, C.c_double), _ptr(grad, C.c_double), _ptr(m, C.c_double),
                        _ptr(v, C.c_double), int(t), lr, b1, b2, eps)


class Oracle:
    """One replica of a CR-MC system on the CPU (FP64).

    ``n_cells`` is the number of cells per box edge used by the cell schedule
    (even, >= 4, L/n_cells >= rc); the paper schedule ignores it.
    """

    def __init__(self, L, n_cells, lB, kappa, rc, eps=1.0, rho0NA=0.0269424,
                 ion_coupling=1, seed=1234, replica=0):
        self._L = lib()
        self.h = self._L.orc_create(float(L), int(n_cells), float(lB), float(kappa), float(rc),
                                    float(eps), float(rho0NA), int(ion_coupling),
                                    int(seed) & 0xFFFFFFFFFFFFFFFF, int(replica))
        self.box = float(L)
        self._log = None

    def __del__(self):
        if getattr(self, "h", None):
            self._L.orc_destroy(self.h)
            self.h = None

    # -- set-up ----------------------------------------------------------
    def set_conditions(self, pH, pKa, pKb=0.0, pIXp=0.0, pIXm=None, pKw=14.0, kappa=None):
        if pIXm is None:
            pIXm = pIXp
        self._L.orc_set_conditions(self.h, pH, pKa, pKb, pIXp, pIXm, pKw)
        if kappa is not None:
            self._L.orc_set_kappa(self.h, float(kappa))

    def set_schedule(self, trials_per_cell=1, fixed_grid=False, pairing=True, site_trials=0, ion_trials=0):
        """Cell schedule: trials per active cell per phase, plus site_trials/16
        extra trials per ionizable site of a domain (rounded up), then
        ion_trials ion relocation trials per cell of the domain; fixed_grid
        turns the per-sweep random shift off (a planted mistake for the negative
        control); pairing lets a trial act on two reflection-paired cells."""
        self._L.orc_set_schedule(self.h, int(trials_per_cell), int(bool(fixed_grid)), int(bool(pairing)),
                                 int(site_trials))
        self._L.orc_set_ion_trials(self.h, int(ion_trials))

    def relocation_stats(self):
        """(attempts, accepts) of the ion relocation trials."""
        out = np.zeros(2, dtype=np.int64)
        self._L.orc_relocation_stats(self.h, _ptr(out, C.c_int64))
        return int(out[0]), int(out[1])

    def partner(self, sweep, colour, a, M):
        return int(self._L.orc_partner(self.h, int(sweep), int(colour), int(a), int(M)))

    def set_particles(self, xyz, kind, charged=None, sid=None, fixed=False):
        kind = np.ascontiguousarray(kind, dtype=np.int32)
        n = kind.size
        if fixed:
            X = np.ascontiguousarray(xyz, dtype=np.uint32).reshape(n, 3)
        else:
            X = to_fixed(xyz, self.box)
        X = np.ascontiguousarray(X.reshape(-1))
        ch = None if charged is None else np.ascontiguousarray(charged, dtype=np.int32)
        sd = None if sid is None else np.ascontiguousarray(sid, dtype=np.int32)
        self._L.orc_set_particles(self.h, n, _ptr(X, C.c_uint32), _ptr(kind, C.c_int32),
                                  None if ch is None else _ptr(ch, C.c_int32),
                                  None if sd is None else _ptr(sd, C.c_int32))

    def load_state(self, xyz, kind, charged, sid, sweep, energy=True):
        """Test aid: continue a chain another program ran.  Fixed-point
        positions, kinds, charged flags and site ids in that program's
        particle order (which the next sweep's stable binning starts from), at
        the start of sweep `sweep`.  The running energy restarts from a
        brute-force sum (NaN with energy=False: the sum is quadratic in the
        particle count) and the move counters from zero; no arithmetic
        changes.  Call set_cores first when the system has cores."""
        kind = np.ascontiguousarray(kind, dtype=np.int32)
        n = kind.size
        X = np.ascontiguousarray(np.asarray(xyz, dtype=np.uint32).reshape(-1))
        ch = np.ascontiguousarray(charged, dtype=np.int32)
        sd = np.ascontiguousarray(sid, dtype=np.int32)
        self._L.orc_load_state(self.h, n, _ptr(X, C.c_uint32), _ptr(kind, C.c_int32), _ptr(ch, C.c_int32),
                               _ptr(sd, C.c_int32), int(sweep), int(bool(energy)))

    def prepare_sweep(self):
        """Test aid: bin into the current sweep's shifted grid without
        running trials (cell_site_features then reads that grid)."""
        self._L.orc_prepare_sweep(self.h)

    def set_domain_filter(self, first_cells):
        """Test aid: later sweeps run only the listed domains (first cell of
        each) of their first colour phase and skip the other phases; None
        turns it off.  Domains of one colour do not interact, so the listed
        domains' trials are exactly those of the full sweep."""
        if first_cells is None:
            self._L.orc_set_domain_filter(self.h, -1, None)
            return
        a = np.ascontiguousarray(first_cells, dtype=np.int32)
        self._L.orc_set_domain_filter(self.h, a.size, _ptr(a, C.c_int32))

    def set_cores(self, xyz, radius):
        radius = np.ascontiguousarray(radius, dtype=np.float64)
        X = np.ascontiguousarray(to_fixed(xyz, self.box).reshape(-1))
        self._L.orc_set_cores(self.h, radius.size, _ptr(X, C.c_uint32), _ptr(radius, C.c_double))

    def set_learned(self, par, eps=0.1, on=True):
        """Learned site proposal with network parameters par (FP64 values)
        mixed with the uniform pick at weight eps."""
        par = np.ascontiguousarray(par, dtype=np.float64)
        assert par.size == mlp_params()
        rc = self._L.orc_set_learned(self.h, _ptr(par, C.c_double), float(eps), int(bool(on)))
        if rc:
            raise ValueError("eps must lie in (0, 1]")

    def set_learned_offsets(self, acid=0.0, base=0.0):
        """Offsets added to the network's logit of acid and base sites."""
        self._L.orc_set_learned_offsets(self.h, float(acid), float(base))

    def cell_site_features(self, cell, cap=4096):
        """(site ids, features) of the sites in one cell of the last sweep's grid."""
        sid = np.zeros(cap, dtype=np.int32)
        X = np.zeros((cap, MLP_IN))
        n = self._L.orc_features_of_cell_sites(self.h, int(cell), cap, _ptr(sid, C.c_int32), _ptr(X, C.c_double))
        n = min(n, cap)
        return sid[:n], X[:n]

    def enable_log(self, cap):
        self._log = (TrialRecord * int(cap))()
        self._L.orc_set_log(self.h, C.cast(self._log, C.c_void_p), int(cap))

    def log(self):
        n = self._L.orc_log_count(self.h)
        if self._log is None:
            return np.zeros(0)
        a = np.ctypeslib.as_array(self._log)[:n]
        return np.array(a.tolist(), dtype=[("sweep", "i8"), ("cell", "i8"), ("trial", "i8"),
                                          ("move", "i4"), ("status", "i4"), ("dU", "f8"),
                                          ("lnp", "f8"), ("u", "f8")])

    def set_check(self, on=True):
        self._L.orc_set_check(self.h, int(on))

    def set_trial_limit(self, n):
        """Run only the next n trials in processing order (n < 0: no limit);
        later trials of the sweeps are skipped, so the state is the one after
        those n trials.  For comparing a prefix of a long run."""
        self._L.orc_set_trial_limit(self.h, int(n))

    def max_dU_err(self):
        return self._L.orc_max_dU_err(self.h)

    # -- running ---------------------------------------------------------
    def sweeps(self, n, series=True):
        s = np.zeros((int(n), 4), dtype=np.int32) if series else None
        self._L.orc_sweeps(self.h, int(n), None if s is None else _ptr(s, C.c_int32))
        return s

    def paper_trials(self, n, sample_every=0):
        rows = int(n) // int(sample_every) if sample_every else 0
        s = np.zeros((max(rows, 1), 4), dtype=np.int32)
        self._L.orc_paper_trials(self.h, int(n), int(sample_every), _ptr(s, C.c_int32))
        return s[:rows]

    # -- state -----------------------------------------------------------
    def particles(self):
        n = self._L.orc_num_particles(self.h)
        X = np.zeros(3 * max(n, 1), dtype=np.uint32)
        k = np.zeros(max(n, 1), dtype=np.int32)
        c = np.zeros(max(n, 1), dtype=np.int32)
        s = np.zeros(max(n, 1), dtype=np.int32)
        self._L.orc_get_particles(self.h, n, _ptr(X, C.c_uint32), _ptr(k, C.c_int32),
                                  _ptr(c, C.c_int32), _ptr(s, C.c_int32))
        return X[:3 * n].reshape(n, 3), k[:n], c[:n], s[:n]

    def counts(self):
        out = np.zeros(6, dtype=np.int64)
        self._L.orc_counts(self.h, _ptr(out, C.c_int64))
        return dict(zip(("nA", "nAm", "nB", "nBp", "nXp", "nXm"), out.tolist()))

    def energy(self):
        """Brute-force total energy of the current state (kT)."""
        return self._L.orc_energy(self.h)

    def running_energy(self):
        return self._L.orc_running_energy(self.h)

    def sweep_index(self):
        return int(self._L.orc_sweep_index(self.h))

    def move_stats(self):
        a = np.zeros(6, dtype=np.int64)
        b = np.zeros(6, dtype=np.int64)
        self._L.orc_move_stats(self.h, _ptr(a, C.c_int64), _ptr(b, C.c_int64))
        return a, b

    def md(self, nsteps, dt=0.005, gamma=1.0):
        """A block of Langevin molecular dynamics of the free ions (velocity
        Verlet, Maxwell-Boltzmann start, friction gamma; units sigma, kT, ion
        mass).  Returns the mean v^2 per component over ions and steps."""
        return float(self._L.orc_md(self.h, int(nsteps), float(dt), float(gamma)))

    def forces(self):
        """Forces on the free ions (zero rows for other particles), global order."""
        n = self._L.orc_num_particles(self.h)
        F = np.zeros((max(n, 1), 3))
        self._L.orc_forces(self.h, _ptr(F, C.c_double))
        return F[:n]

    def ungroup(self, frac, draw):
        """Ungrouping (Sec. II D): each free ion of the current state, in
        global order, becomes a salt ion with probability frac[0] (cations) or
        frac[2] (anions), H+ / OH- with frac[1] / frac[3], else another
        reservoir ion; the uniforms come from Philox counters (draw, particle
        index, tag 5).  Returns (labels per particle: 0 not an ion, 1 salt,
        2 H+ or OH-, 3 other; counts [S+, H+, other+, S-, OH-, other-])."""
        f = np.ascontiguousarray(frac, dtype=np.float64)
        n = self._L.orc_num_particles(self.h)
        lab = np.zeros(max(n, 1), dtype=np.int32)
        cnt = np.zeros(6, dtype=np.int64)
        self._L.orc_ungroup(self.h, _ptr(f, C.c_double), int(draw), _ptr(cnt, C.c_int64), _ptr(lab, C.c_int32))
        return lab[:n], cnt

    def shift(self, sweep):
        o = np.zeros(3, dtype=np.uint32)
        self._L.orc_shift(self.h, int(sweep), _ptr(o, C.c_uint32))
        return o
