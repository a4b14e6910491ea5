"""ctypes binding of libcrmc.so (include/crmc.h): argument marshalling only.

The functions carry the C names; ``System`` is a small convenience wrapper over
them.  Every step of the Monte Carlo runs in the HIP library: if the library
is missing or cannot be loaded this module raises, it never falls back.
PyTorch (optional here) only supplies the HIP stream the calls are ordered on.
"""
from __future__ import annotations

import ctypes as C
import os
import re

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libcrmc.so")
HEADER = os.path.join(os.path.dirname(_HERE), "include", "crmc.h")

CRMC_OK, CRMC_E_ARG, CRMC_E_NOMEM, CRMC_E_DEVICE, CRMC_E_CAPACITY, CRMC_E_STATE = 0, -1, -2, -3, -4, -5
ACID, BASE, XPOS, XNEG, NEUTRAL = 1, 2, 3, 4, 5
MOVES = ("acid_fwd", "acid_back", "base_fwd", "base_back", "salt_in", "salt_out")


class CrmcError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("crmc error %d: %s" % (code, msg))
        self.code = code


class crmc_params(C.Structure):
    _fields_ = [("n_replicas", C.c_int32), ("precision", C.c_int32), ("trials_per_cell", C.c_int32),
                ("pairing", C.c_int32), ("ion_coupling", C.c_int32), ("lds_records", C.c_int32),
                ("fixed_grid", C.c_int32), ("site_trials", C.c_int32),
                ("light_neighbours", C.c_int32), ("use_graph", C.c_int32),
                ("learned_proposal", C.c_int32), ("ion_trials", C.c_int32),
                ("lB", C.c_double), ("rc", C.c_double), ("eps_wca", C.c_double), ("rho0NA", C.c_double),
                ("pKw", C.c_double), ("kappa", C.c_double), ("pKb", C.c_double), ("learned_eps", C.c_double),
                ("seed", C.c_uint64), ("stream", C.c_void_p), ("workspace", C.c_void_p),
                ("workspace_bytes", C.c_int64)]


class crmc_cond(C.Structure):
    _fields_ = [("pH", C.c_double), ("pKa", C.c_double), ("pKb", C.c_double),
                ("pIX_pos", C.c_double), ("pIX_neg", C.c_double), ("kappa", C.c_double)]


class crmc_obs(C.Structure):
    _fields_ = [("sweeps", C.c_int64), ("n_acid", C.c_int64), ("n_acid_charged", C.c_int64),
                ("n_base", C.c_int64), ("n_base_charged", C.c_int64), ("n_xpos", C.c_int64),
                ("n_xneg", C.c_int64), ("energy", C.c_double), ("attempts", C.c_int64 * 6),
                ("accepts", C.c_int64 * 6), ("error_flags", C.c_uint32), ("n_cells", C.c_int32),
                ("cell_capacity", C.c_int32), ("max_cell_count", C.c_int32),
                ("relocation_attempts", C.c_int64), ("relocation_accepts", C.c_int64)]


class crmc_trial_rec(C.Structure):
    _fields_ = [("sweep", C.c_int64), ("cell", C.c_int64), ("trial", C.c_int32), ("replica", C.c_int32),
                ("move", C.c_int32), ("status", C.c_int32),
                ("dU", C.c_double), ("lnp", C.c_double), ("u", C.c_double)]


TUNE_MAX = 32


class crmc_tune(C.Structure):
    _fields_ = [("light_neighbours", C.c_int32), ("lds_records", C.c_int32), ("n_candidates", C.c_int32),
                ("reserved", C.c_int32), ("sweeps_used", C.c_int64), ("best_ms_per_sweep", C.c_double),
                ("ms_per_sweep", C.c_double * TUNE_MAX), ("cand_light", C.c_int32 * TUNE_MAX),
                ("cand_lds", C.c_int32 * TUNE_MAX)]


TRIAL_DTYPE = np.dtype([("sweep", "i8"), ("cell", "i8"), ("trial", "i4"), ("replica", "i4"), ("move", "i4"),
                        ("status", "i4"), ("dU", "f8"), ("lnp", "f8"), ("u", "f8")])

_lib = None


def load():
    """Load libcrmc.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("libcrmc.so is not built (run __graft_entry__.build() or "
                           "python -m paper_2109_07527_amd.build)")
    L = C.CDLL(LIB_PATH)
    P, vp, d, i32, i64, u32, u64 = C.POINTER, C.c_void_p, C.c_double, C.c_int32, C.c_int64, C.c_uint32, C.c_uint64
    sig = {
        "crmc_create": (C.c_int, [P(crmc_params), P(vp)]),
        "crmc_workspace_size": (C.c_int, [vp, P(i64)]),
        "crmc_set_workspace": (C.c_int, [vp, vp, i64]),
        "crmc_memory": (C.c_int, [vp, P(i64), P(i64), P(i64)]),
        "crmc_build_cells": (C.c_int, [vp, i32, d, i32, i32, i32, P(d), P(i32), P(i32), P(i32), i32, P(d), P(d)]),
        "crmc_sweep": (C.c_int, [vp, d, d, d, i64]),
        "crmc_sweep_ex": (C.c_int, [vp, P(crmc_cond), i64]),
        "crmc_sweep_recover": (C.c_int, [vp, P(crmc_cond), i64, i64, P(i32)]),
        "crmc_md": (C.c_int, [vp, i64, d, d]),
        "crmc_autotune": (C.c_int, [vp, P(crmc_cond), i32, P(crmc_tune)]),
        "crmc_set_proposal": (C.c_int, [vp, i32, d]),
        "crmc_set_proposal_weights": (C.c_int, [vp, P(C.c_float), i64]),
        "crmc_get_proposal_weights": (C.c_int, [vp, P(C.c_float), i64]),
        "crmc_init_proposal_weights": (C.c_int, [vp, u64]),
        "crmc_set_proposal_offsets": (C.c_int, [vp, i32, d, d]),
        "crmc_get_site_probabilities": (C.c_int, [vp, i32, P(d), i64]),
        "crmc_collect_training": (C.c_int, [vp, i64]),
        "crmc_training_rows": (C.c_int, [vp, P(i64)]),
        "crmc_read_training": (C.c_int, [vp, i64, i64, P(C.c_float)]),
        "crmc_train": (C.c_int, [vp, i32, i32, d, u64, P(d)]),
        "crmc_mlp_forward": (C.c_int, [vp, P(C.c_float), i32, P(C.c_float)]),
        "crmc_load_training": (C.c_int, [vp, P(C.c_float), i64]),
        "crmc_record_features": (C.c_int, [vp, i32]),
        "crmc_get_site_features": (C.c_int, [vp, i32, P(C.c_float), i64]),
        "crmc_mlp_gradient": (C.c_int, [vp, P(C.c_float), i32, P(C.c_float), P(d)]),
        "crmc_observe": (C.c_int, [vp, i32, P(crmc_obs)]),
        "crmc_get_series": (C.c_int, [vp, i32, i64, i64, P(i32)]),
        "crmc_get_particles": (C.c_int, [vp, i32, i32, P(u32), P(i32), P(i32), P(i32), P(i32)]),
        "crmc_energy": (C.c_int, [vp, i32, P(d)]),
        "crmc_energy_noalloc": (C.c_int, [vp, i32, P(d)]),
        "crmc_export_state": (C.c_int, [vp, vp, P(i64)]),
        "crmc_import_state": (C.c_int, [vp, vp, i64]),
        "crmc_get_occupancy": (C.c_int, [vp, i32, i64, P(u64), P(i64)]),
        "crmc_get_group_hist": (C.c_int, [vp, i32, i64, P(i64), i32, P(i32), P(i32)]),
        "crmc_enable_log": (C.c_int, [vp, i64]),
        "crmc_read_log": (C.c_int, [vp, i64, P(crmc_trial_rec), P(i64)]),
        "crmc_philox": (C.c_int, [i64, P(u32), u32, u32, P(u32)]),
        "crmc_set_timing": (C.c_int, [vp, i32]),
        "crmc_enable_trace": (C.c_int, [vp, i64]),
        "crmc_read_trace": (C.c_int, [vp, i64, vp, P(i64)]),
        "crmc_get_timing": (C.c_int, [vp, P(d), P(i64)]),
        "crmc_pIX_from_salt": (d, [d, d, d]),
        "crmc_ungroup_fractions": (C.c_int, [d, d, d, d, d, d, P(d)]),
        "crmc_ungroup": (C.c_int, [vp, i32, P(d), u64, P(i64), P(C.c_int8), i64, P(i64)]),
        "crmc_last_error": (C.c_char_p, [vp]),
        "crmc_destroy": (None, [vp]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def header_symbols():
    """Function names declared in include/crmc.h."""
    with open(HEADER) as f:
        text = f.read()
    decl = r"^\s*(?:int|void|double|const\s+char\s*\*)\s*(crmc_\w+)\s*\("
    return sorted(set(re.findall(decl, text, flags=re.M)))


def _p(a, ct):
    return None if a is None else a.ctypes.data_as(C.POINTER(ct))


def _check(h, rc):
    if rc != CRMC_OK:
        msg = load().crmc_last_error(h)
        raise CrmcError(rc, msg.decode() if msg else "")
    return rc


# --------------------------------------------------------------------------
# the C functions, same names
# --------------------------------------------------------------------------
def crmc_create(params: crmc_params):
    h = C.c_void_p()
    rc = load().crmc_create(C.byref(params), C.byref(h))
    if rc != CRMC_OK:
        raise CrmcError(rc, "crmc_create rejected the parameters")
    return h


def crmc_build_cells(h, replica, L, xyz, kind, charged=None, group=None, core_xyz=None, core_R=None,
                     n_cells=0, cell_capacity=0):
    xyz = np.ascontiguousarray(xyz, dtype=np.float64).reshape(-1, 3)
    kind = np.ascontiguousarray(kind, dtype=np.int32)
    n = kind.size
    ch = None if charged is None else np.ascontiguousarray(charged, dtype=np.int32)
    gr = None if group is None else np.ascontiguousarray(group, dtype=np.int32)
    if core_xyz is None or len(core_R) == 0:
        cx, cr, nc = None, None, 0
    else:
        cx = np.ascontiguousarray(core_xyz, dtype=np.float64).reshape(-1, 3)
        cr = np.ascontiguousarray(core_R, dtype=np.float64)
        nc = cr.size
    return _check(h, load().crmc_build_cells(h, int(replica), float(L), int(n_cells), int(cell_capacity), n,
                                             _p(xyz, C.c_double), _p(kind, C.c_int32), _p(ch, C.c_int32),
                                             _p(gr, C.c_int32), nc, _p(cx, C.c_double), _p(cr, C.c_double)))


def crmc_workspace_size(h):
    n = C.c_int64(0)
    _check(h, load().crmc_workspace_size(h, C.byref(n)))
    return n.value


def crmc_set_workspace(h, ptr, nbytes):
    """Hand over caller-owned device memory (a device pointer, e.g. a torch
    uint8 tensor's data_ptr()) for the handle's state."""
    return _check(h, load().crmc_set_workspace(h, C.c_void_p(int(ptr)), int(nbytes)))


def crmc_memory(h):
    """{own, workspace_used, workspace_largest_free} device bytes of the handle."""
    a, b, c = C.c_int64(0), C.c_int64(0), C.c_int64(0)
    _check(h, load().crmc_memory(h, C.byref(a), C.byref(b), C.byref(c)))
    return dict(own=a.value, workspace_used=b.value, workspace_largest_free=c.value)


def crmc_sweep(h, pH, pKa, mu_ion, n_sweeps):
    return _check(h, load().crmc_sweep(h, float(pH), float(pKa), float(mu_ion), int(n_sweeps)))


def crmc_sweep_ex(h, conds, n_sweeps):
    arr = (crmc_cond * len(conds))()
    for i, c in enumerate(conds):
        arr[i] = crmc_cond(*[float(c[k]) for k in ("pH", "pKa", "pKb", "pIX_pos", "pIX_neg", "kappa")])
    return _check(h, load().crmc_sweep_ex(h, arr, int(n_sweeps)))


def crmc_sweep_recover(h, conds, n_sweeps, chunk):
    """crmc_sweep_ex in chunks with recovery from cell-capacity overflow;
    returns the number of capacity enlargements."""
    arr = (crmc_cond * len(conds))()
    for i, c in enumerate(conds):
        arr[i] = crmc_cond(*[float(c[k]) for k in ("pH", "pKa", "pKb", "pIX_pos", "pIX_neg", "kappa")])
    n = C.c_int32(0)
    _check(h, load().crmc_sweep_recover(h, arr, int(n_sweeps), int(chunk), C.byref(n)))
    return n.value


def crmc_md(h, n_steps, dt=0.005, gamma=1.0):
    return _check(h, load().crmc_md(h, int(n_steps), float(dt), float(gamma)))


def crmc_observe(h, replica):
    o = crmc_obs()
    rc = load().crmc_observe(h, int(replica), C.byref(o))
    out = {k: getattr(o, k) for k, _ in crmc_obs._fields_ if k not in ("attempts", "accepts")}
    out["attempts"] = list(o.attempts)
    out["accepts"] = list(o.accepts)
    out["status"] = rc
    return out


def crmc_get_series(h, replica, first, count):
    out = np.zeros((int(count), 4), dtype=np.int32)
    _check(h, load().crmc_get_series(h, int(replica), int(first), int(count), _p(out, C.c_int32)))
    return out


def crmc_get_particles(h, replica, cap=None):
    n = C.c_int32(0)
    if cap is None:
        _check(h, load().crmc_get_particles(h, int(replica), 0, None, None, None, None, C.byref(n)))
        cap = n.value
    X = np.zeros((max(cap, 1), 3), dtype=np.uint32)
    k = np.zeros(max(cap, 1), dtype=np.int32)
    c = np.zeros(max(cap, 1), dtype=np.int32)
    s = np.zeros(max(cap, 1), dtype=np.int32)
    _check(h, load().crmc_get_particles(h, int(replica), int(cap), _p(X, C.c_uint32), _p(k, C.c_int32),
                                        _p(c, C.c_int32), _p(s, C.c_int32), C.byref(n)))
    m = min(n.value, cap)
    return X[:m], k[:m], c[:m], s[:m]


def crmc_export_state(h):
    """The chain's state as bytes (see crmc_import_state)."""
    n = C.c_int64(0)
    _check(h, load().crmc_export_state(h, None, C.byref(n)))
    buf = C.create_string_buffer(max(n.value, 1))
    _check(h, load().crmc_export_state(h, buf, C.byref(n)))
    return buf.raw[:n.value]


def crmc_import_state(h, state):
    buf = C.create_string_buffer(bytes(state), len(state))
    _check(h, load().crmc_import_state(h, buf, len(state)))


def crmc_energy(h, replica):
    e = C.c_double(0.0)
    _check(h, load().crmc_energy(h, int(replica), C.byref(e)))
    return e.value


def crmc_energy_noalloc(h, replica):
    e = C.c_double(0.0)
    _check(h, load().crmc_energy_noalloc(h, int(replica), C.byref(e)))
    return e.value


def crmc_get_occupancy(h, replica):
    n = C.c_int64(0)
    _check(h, load().crmc_get_occupancy(h, int(replica), 0, None, C.byref(n)))
    out = np.zeros(max(n.value, 1), dtype=np.uint64)
    _check(h, load().crmc_get_occupancy(h, int(replica), n.value, _p(out, C.c_uint64), C.byref(n)))
    return out[:n.value]


def crmc_get_group_hist(h, replica):
    ng = C.c_int32(0)
    _check(h, load().crmc_get_group_hist(h, int(replica), 0, None, 0, None, C.byref(ng)))
    off = np.zeros(ng.value + 1, dtype=np.int32)
    _check(h, load().crmc_get_group_hist(h, int(replica), 0, None, ng.value + 1, _p(off, C.c_int32), C.byref(ng)))
    out = np.zeros(max(int(off[-1]), 1), dtype=np.int64)
    _check(h, load().crmc_get_group_hist(h, int(replica), int(off[-1]), _p(out, C.c_int64), ng.value + 1,
                                         _p(off, C.c_int32), C.byref(ng)))
    return [out[off[g]:off[g + 1]] for g in range(ng.value)]


def crmc_enable_log(h, capacity):
    return _check(h, load().crmc_enable_log(h, int(capacity)))


def crmc_read_log(h, cap):
    n = C.c_int64(0)
    buf = np.zeros(max(int(cap), 1), dtype=TRIAL_DTYPE)
    _check(h, load().crmc_read_log(h, int(cap), buf.ctypes.data_as(C.POINTER(crmc_trial_rec)), C.byref(n)))
    return buf[:min(n.value, int(cap))], n.value


def crmc_philox(ctr, k0, k1):
    ctr = np.ascontiguousarray(ctr, dtype=np.uint32).reshape(-1, 4)
    out = np.zeros_like(ctr)
    rc = load().crmc_philox(ctr.shape[0], _p(ctr, C.c_uint32), int(k0), int(k1), _p(out, C.c_uint32))
    if rc != CRMC_OK:
        raise CrmcError(rc, "crmc_philox failed")
    return out


def crmc_autotune(h, conds, sweeps_per_candidate):
    arr = (crmc_cond * len(conds))()
    for i, c in enumerate(conds):
        arr[i] = crmc_cond(*[float(c[k]) for k in ("pH", "pKa", "pKb", "pIX_pos", "pIX_neg", "kappa")])
    t = crmc_tune()
    _check(h, load().crmc_autotune(h, arr, int(sweeps_per_candidate), C.byref(t)))
    n = t.n_candidates
    return {"light_neighbours": t.light_neighbours, "lds_records": t.lds_records, "sweeps_used": t.sweeps_used,
            "best_ms_per_sweep": t.best_ms_per_sweep, "cached": bool(t.reserved),
            "candidates": [(t.cand_light[i], t.cand_lds[i], t.ms_per_sweep[i]) for i in range(n)]}


MLP_PARAMS = 20865


def crmc_set_proposal(h, learned, eps=0.1):
    return _check(h, load().crmc_set_proposal(h, int(bool(learned)), float(eps)))


def crmc_set_proposal_weights(h, w):
    w = np.ascontiguousarray(w, dtype=np.float32)
    return _check(h, load().crmc_set_proposal_weights(h, _p(w, C.c_float), w.size))


def crmc_get_proposal_weights(h):
    w = np.zeros(MLP_PARAMS, dtype=np.float32)
    _check(h, load().crmc_get_proposal_weights(h, _p(w, C.c_float), w.size))
    return w


def crmc_init_proposal_weights(h, seed):
    return _check(h, load().crmc_init_proposal_weights(h, int(seed) & (2**64 - 1)))


def crmc_set_proposal_offsets(h, replica, acid, base):
    return _check(h, load().crmc_set_proposal_offsets(h, int(replica), float(acid), float(base)))


def crmc_get_site_probabilities(h, replica):
    n = C.c_int64(0)
    _check(h, load().crmc_get_occupancy(h, int(replica), 0, None, C.byref(n)))  # particle count
    out = np.zeros(max(n.value, 1), dtype=np.float64)
    _check(h, load().crmc_get_site_probabilities(h, int(replica), _p(out, C.c_double), out.size))
    return out[:n.value]


def crmc_collect_training(h, capacity):
    return _check(h, load().crmc_collect_training(h, int(capacity)))


def crmc_training_rows(h):
    n = C.c_int64()
    _check(h, load().crmc_training_rows(h, C.byref(n)))
    return n.value


def crmc_read_training(h, first=0, count=None):
    if count is None:
        count = crmc_training_rows(h) - first
    out = np.zeros((int(count), 33), dtype=np.float32)
    _check(h, load().crmc_read_training(h, int(first), int(count), _p(out, C.c_float)))
    return out


def crmc_load_training(h, rows):
    rows = np.ascontiguousarray(rows, dtype=np.float32).reshape(-1, 33)
    return _check(h, load().crmc_load_training(h, _p(rows, C.c_float), rows.shape[0]))


def crmc_record_features(h, on):
    return _check(h, load().crmc_record_features(h, int(bool(on))))


def crmc_get_site_features(h, replica):
    n = C.c_int64(0)
    _check(h, load().crmc_get_occupancy(h, int(replica), 0, None, C.byref(n)))  # particle count
    out = np.zeros((max(n.value, 1), 32), dtype=np.float32)
    _check(h, load().crmc_get_site_features(h, int(replica), _p(out, C.c_float), out.size))
    return out[:n.value]


def crmc_train(h, epochs, batch=256, lr=1e-3, seed=1):
    loss = C.c_double()
    _check(h, load().crmc_train(h, int(epochs), int(batch), float(lr), int(seed), C.byref(loss)))
    return loss.value


def crmc_mlp_forward(h, X):
    X = np.ascontiguousarray(X, dtype=np.float32).reshape(-1, 32)
    out = np.zeros(X.shape[0], dtype=np.float32)
    _check(h, load().crmc_mlp_forward(h, _p(X, C.c_float), X.shape[0], _p(out, C.c_float)))
    return out


def crmc_mlp_gradient(h, rows):
    rows = np.ascontiguousarray(rows, dtype=np.float32).reshape(-1, 33)
    g = np.zeros(MLP_PARAMS, dtype=np.float32)
    loss = C.c_double()
    _check(h, load().crmc_mlp_gradient(h, _p(rows, C.c_float), rows.shape[0], _p(g, C.c_float), C.byref(loss)))
    return loss.value, g


def crmc_set_timing(h, on):
    return _check(h, load().crmc_set_timing(h, int(bool(on))))


def crmc_get_timing(h):
    """(milliseconds, launches) per kernel kind: re-binning, trial phases, end of sweep."""
    ms = np.zeros(3, dtype=np.float64)
    n = np.zeros(3, dtype=np.int64)
    _check(h, load().crmc_get_timing(h, _p(ms, C.c_double), _p(n, C.c_int64)))
    return ms, n


TRACE_DTYPE = np.dtype([("t0", "u8"), ("t1", "u8"), ("sweep", "u4"), ("domain", "u4"), ("colour", "i4"),
                        ("trials", "i4"), ("neighbours", "i4"), ("own", "i4"), ("staged", "i4"), ("hw_id", "i4")])


def crmc_enable_trace(h, capacity):
    return _check(h, load().crmc_enable_trace(h, int(capacity)))


def crmc_read_trace(h, cap):
    n = C.c_int64(0)
    buf = np.zeros(max(int(cap), 1), dtype=TRACE_DTYPE)
    _check(h, load().crmc_read_trace(h, int(cap), C.c_void_p(buf.ctypes.data), C.byref(n)))
    return buf[:min(n.value, int(cap))], n.value


def crmc_pIX_from_salt(pIS, pH, pKw=14.0):
    return load().crmc_pIX_from_salt(float(pIS), float(pH), float(pKw))


def crmc_ungroup_fractions(pH, pIS_pos, pIS_neg, pIX_pos, pIX_neg, pKw=14.0):
    """{S+, H+} shares of X+ and {S-, OH-} shares of X- (a dict)."""
    out = np.zeros(4)
    rc = load().crmc_ungroup_fractions(float(pH), float(pKw), float(pIS_pos), float(pIS_neg), float(pIX_pos),
                                       float(pIX_neg), _p(out, C.c_double))
    if rc:
        raise CrmcError(rc, "invalid arguments")
    return dict(S_pos=out[0], H=out[1], S_neg=out[2], OH=out[3])


def crmc_ungroup(h, replica, frac, draw):
    """(labels per particle in the library's order, counts [S+, H+, other+,
    S-, OH-, other-]) of one ungrouping of the current state."""
    f = np.ascontiguousarray(frac, dtype=np.float64)
    cnt = np.zeros(6, dtype=np.int64)
    n = C.c_int64(0)
    _check(h, load().crmc_ungroup(h, int(replica), _p(f, C.c_double), int(draw), _p(cnt, C.c_int64), None, 0,
                                  C.byref(n)))
    lab = np.zeros(max(n.value, 1), dtype=np.int8)
    _check(h, load().crmc_ungroup(h, int(replica), _p(f, C.c_double), int(draw), _p(cnt, C.c_int64),
                                  _p(lab, C.c_int8), lab.size, C.byref(n)))
    return lab[:n.value], cnt


def crmc_destroy(h):
    load().crmc_destroy(h)


def current_stream():
    """The current torch HIP stream handle (None when torch has no GPU)."""
    try:
        import torch
        if torch.cuda.is_available():
            return C.c_void_p(torch.cuda.current_stream().cuda_stream)
    except Exception:
        pass
    return None


# --------------------------------------------------------------------------
# convenience wrapper
# --------------------------------------------------------------------------
class System:
    """A batch of CR-MC replicas on the GPU (one handle of the C library)."""

    def __init__(self, n_replicas=1, lB=2.0, rc=6.0, eps=1.0, rho0NA=0.0269424, pKw=14.0, kappa=0.5,
                 pKb=5.0, seed=1234, precision=32, trials_per_cell=1, pairing=True, ion_coupling=True,
                 lds_records=0, fixed_grid=False, site_trials=0, ion_trials=0, light_neighbours=0, use_graph=True,
                 learned=False, learned_eps=0.1, stream="torch"):
        p = crmc_params()
        p.n_replicas = int(n_replicas)
        p.precision = int(precision)
        p.trials_per_cell = int(trials_per_cell)
        p.pairing = int(bool(pairing))
        p.ion_coupling = int(bool(ion_coupling))
        p.lds_records = int(lds_records)
        p.fixed_grid = int(bool(fixed_grid))
        p.site_trials = int(site_trials)
        p.ion_trials = int(ion_trials)
        p.light_neighbours = int(light_neighbours)
        p.use_graph = int(bool(use_graph))
        p.learned_proposal = int(bool(learned))
        p.learned_eps = float(learned_eps)
        p.lB, p.rc, p.eps_wca, p.rho0NA, p.pKw, p.kappa, p.pKb = lB, rc, eps, rho0NA, pKw, kappa, pKb
        p.seed = int(seed) & 0xFFFFFFFFFFFFFFFF
        s = current_stream() if stream == "torch" else stream
        p.stream = s.value if isinstance(s, C.c_void_p) else s
        self.params = p
        self.n_replicas = int(n_replicas)
        self.pKw, self.kappa, self.pKb = pKw, kappa, pKb
        self.h = crmc_create(p)

    def close(self):
        if getattr(self, "h", None) is not None:
            crmc_destroy(self.h)
            self.h = None
        self._workspace = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def build_cells(self, replica, system=None, **kw):
        if system is not None:
            kw.setdefault("L", system["L"])
            kw.setdefault("xyz", system["xyz"])
            kw.setdefault("kind", system["kind"])
            kw.setdefault("group", system.get("group"))
            if len(system.get("core_R", [])):
                kw.setdefault("core_xyz", system["core_xyz"])
                kw.setdefault("core_R", system["core_R"])
        return crmc_build_cells(self.h, replica, **kw)

    def workspace_size(self):
        return crmc_workspace_size(self.h)

    def set_workspace(self, tensor):
        """Place the handle's device state in a caller-owned torch uint8
        tensor (kept referenced here until close())."""
        self._workspace = tensor
        return crmc_set_workspace(self.h, tensor.data_ptr(), tensor.numel() * tensor.element_size())

    def memory(self):
        return crmc_memory(self.h)

    def sweep(self, pH, pKa, mu_ion, n_sweeps):
        return crmc_sweep(self.h, pH, pKa, mu_ion, n_sweeps)

    def sweep_ex(self, conds, n_sweeps):
        return crmc_sweep_ex(self.h, conds, n_sweeps)

    def md(self, n_steps, dt=0.005, gamma=1.0):
        """A block of Langevin molecular dynamics of the free ions."""
        return crmc_md(self.h, n_steps, dt, gamma)

    def sweep_recover(self, conds, n_sweeps, chunk=16):
        return crmc_sweep_recover(self.h, conds, n_sweeps, chunk)

    def set_proposal(self, learned, eps=0.1):
        return crmc_set_proposal(self.h, learned, eps)

    def set_proposal_weights(self, w):
        return crmc_set_proposal_weights(self.h, w)

    def proposal_weights(self):
        return crmc_get_proposal_weights(self.h)

    def init_proposal_weights(self, seed):
        return crmc_init_proposal_weights(self.h, seed)

    def set_proposal_offsets(self, replica, acid, base):
        return crmc_set_proposal_offsets(self.h, replica, acid, base)

    def site_probabilities(self, replica):
        return crmc_get_site_probabilities(self.h, replica)

    def collect_training(self, capacity):
        return crmc_collect_training(self.h, capacity)

    def training_rows(self):
        return crmc_training_rows(self.h)

    def read_training(self, first=0, count=None):
        return crmc_read_training(self.h, first, count)

    def load_training(self, rows):
        return crmc_load_training(self.h, rows)

    def record_features(self, on=True):
        return crmc_record_features(self.h, on)

    def site_features(self, replica):
        return crmc_get_site_features(self.h, replica)

    def train(self, epochs, batch=256, lr=1e-3, seed=1):
        return crmc_train(self.h, epochs, batch, lr, seed)

    def mlp_forward(self, X):
        return crmc_mlp_forward(self.h, X)

    def mlp_gradient(self, rows):
        return crmc_mlp_gradient(self.h, rows)

    def autotune(self, conds, sweeps_per_candidate=10):
        return crmc_autotune(self.h, conds, sweeps_per_candidate)

    def observe(self, replica=0):
        return crmc_observe(self.h, replica)

    def series(self, replica, first, count):
        return crmc_get_series(self.h, replica, first, count)

    def particles(self, replica=0):
        return crmc_get_particles(self.h, replica)

    def energy(self, replica=0):
        return crmc_energy(self.h, replica)

    def export_state(self):
        return crmc_export_state(self.h)

    def import_state(self, state):
        return crmc_import_state(self.h, state)

    def occupancy(self, replica=0):
        return crmc_get_occupancy(self.h, replica)

    def group_hist(self, replica=0):
        return crmc_get_group_hist(self.h, replica)

    def enable_log(self, capacity):
        return crmc_enable_log(self.h, capacity)

    def read_log(self, cap=None):
        if cap is None:
            _, n = crmc_read_log(self.h, 0)
            cap = n
        return crmc_read_log(self.h, cap)[0]
