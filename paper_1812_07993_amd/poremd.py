"""ctypes binding of libporemd.so (the C interface in include/poremd.h).

Every function here only marshals arguments: all of the method's work runs
in the library's HIP kernels.  Importing this module fails loudly if the
library has not been built (run ``python -m paper_1812_07993_amd.build`` or
``__graft_entry__.build()``); there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("PMD_LIBRARY") or os.path.join(_HERE, "_build", "libporemd.so")

PMD_OK, PMD_EINVAL, PMD_ENOMEM, PMD_EHIP, PMD_ENUMERIC, PMD_EAGAIN, PMD_ESTATE = (
    0, -1, -2, -3, -4, -5, -6)
PMD_FP64, PMD_MIXED = 0, 1
PORE_KINDS = {"none": 0, "slab": 1, "cylinder": 2, "slit": 3, "cone": 4, "inkbottle": 5}
PRECISIONS = {"fp64": PMD_FP64, "mixed": PMD_MIXED}


class PmdError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("poremd error %d: %s" % (code, msg))
        self.code = code


class pmd_params(ctypes.Structure):
    _fields_ = [("box", ctypes.c_double * 3), ("sigma", ctypes.c_double),
                ("epsilon", ctypes.c_double), ("mass", ctypes.c_double),
                ("cutoff", ctypes.c_double), ("dt", ctypes.c_double),
                ("sigma_wall", ctypes.c_double), ("epsilon_wall", ctypes.c_double),
                ("precision", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("thermostat_tau", ctypes.c_double), ("thermostat_t0", ctypes.c_double)]


class pmd_pore(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("lattice_a", ctypes.c_double), ("slab_center_z", ctypes.c_double),
                ("slab_thickness", ctypes.c_double), ("r0", ctypes.c_double),
                ("r1", ctypes.c_double), ("slit_gap", ctypes.c_double)]


class pmd_energies(ctypes.Structure):
    _fields_ = [("step", ctypes.c_int64), ("ke", ctypes.c_double),
                ("pe_vv", ctypes.c_double), ("pe_vw", ctypes.c_double),
                ("etotal", ctypes.c_double), ("temperature", ctypes.c_double),
                ("virial_vv", ctypes.c_double), ("virial_vw", ctypes.c_double),
                ("ke_pore", ctypes.c_double), ("virial_pore", ctypes.c_double),
                ("n_pore", ctypes.c_int64), ("pore_volume", ctypes.c_double),
                ("pressure", ctypes.c_double)]


class pmd_tuning(ctypes.Structure):
    _fields_ = [("skin", ctypes.c_double), ("rebin_every", ctypes.c_int32),
                ("block", ctypes.c_int32), ("list_cap", ctypes.c_int32),
                ("energy_every", ctypes.c_int32), ("use_graph", ctypes.c_int32),
                ("brick_atoms", ctypes.c_int32), ("brick_order", ctypes.c_int32),
                ("virial", ctypes.c_int32)]


_lib = None

class pmd_pm_model(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("lx", ctypes.c_double), ("ly", ctypes.c_double), ("lz", ctypes.c_double),
                ("k", ctypes.c_double), ("sigma", ctypes.c_double), ("epsilon", ctypes.c_double),
                ("mass", ctypes.c_double), ("dt", ctypes.c_double),
                ("thermostat_tau", ctypes.c_double), ("thermostat_t0", ctypes.c_double)]


class pmd_pm_record(ctypes.Structure):
    _fields_ = [("step", ctypes.c_int64), ("ke", ctypes.c_double), ("pe", ctypes.c_double),
                ("etotal", ctypes.c_double), ("temperature", ctypes.c_double),
                ("pressure", ctypes.c_double), ("n_pore", ctypes.c_int64), ("reflections", ctypes.c_int64),
                ("n_outside", ctypes.c_int64)]


PM_RECORD_DTYPE = np.dtype([("step", np.int64), ("ke", np.float64), ("pe", np.float64),
                            ("etotal", np.float64), ("temperature", np.float64),
                            ("pressure", np.float64), ("n_pore", np.int64), ("reflections", np.int64),
                            ("n_outside", np.int64)])


# name -> (restype, argtypes)
_P, _vp, _i64, _i32, _d = ctypes.POINTER, ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_double
_SIGS = {
    "pmd_last_error": (ctypes.c_char_p, []),
    "pmd_version": (ctypes.c_int, []),
    "pmd_wall_count": (ctypes.c_int, [_P(pmd_params), _P(pmd_pore), _P(_i64)]),
    "pmd_footprint_bytes": (ctypes.c_int, [_P(pmd_params), _P(pmd_pore), _i64, _P(pmd_tuning),
                                           _P(ctypes.c_size_t)]),
    "pmd_create_system": (ctypes.c_int, [_P(pmd_params), _P(pmd_pore), _i64, _vp, _vp, _i64, _vp,
                                         _vp, _P(pmd_tuning), _P(_vp)]),
    "pmd_step": (ctypes.c_int, [_vp, _i64]),
    "pmd_sync": (ctypes.c_int, [_vp]),
    "pmd_get_positions": (ctypes.c_int, [_vp, _vp, _i64]),
    "pmd_get_velocities": (ctypes.c_int, [_vp, _vp, _i64]),
    "pmd_get_forces": (ctypes.c_int, [_vp, _vp, _i64]),
    "pmd_get_energies": (ctypes.c_int, [_vp, _P(pmd_energies)]),
    "pmd_get_energy_history": (ctypes.c_int, [_vp, _vp, _i64, _P(_i64)]),
    "pmd_get_wall_positions": (ctypes.c_int, [_vp, _vp, _i64]),
    "pmd_get_counts": (ctypes.c_int, [_vp, _P(_i64), _P(_i64)]),
    "pmd_get_step": (_i64, [_vp]),
    "pmd_get_positions_device": (ctypes.c_int, [_vp, _vp, _i64, _vp]),
    "pmd_set_tuning": (ctypes.c_int, [_vp, _P(pmd_tuning)]),
    "pmd_get_tuning": (ctypes.c_int, [_vp, _P(pmd_tuning)]),
    "pmd_set_state": (ctypes.c_int, [_vp, _vp, _vp, _i64, _i64]),
    "pmd_autotune_grid": (ctypes.c_int, [_P(pmd_params), _i64, _vp, _i32, _P(_i32)]),
    "pmd_autotune": (ctypes.c_int, [_P(pmd_params), _P(pmd_pore), _i64, _vp, _vp, _i64, _vp, _vp,
                                    _vp, _i32, _i64, _vp, _P(_i32)]),
    "pmd_destroy": (ctypes.c_int, [_vp]),
    "pmd_timing_enable": (ctypes.c_int, [_vp, ctypes.c_int]),
    "pmd_kernel_time": (ctypes.c_int, [_vp, _P(_i64), _P(_d)]),
    "pmd_kernel_times": (ctypes.c_int, [_vp, _vp, _i64, _P(_i64)]),
    "pmd_debug_cells": (ctypes.c_int, [_vp, _vp, _i64, _vp, _i64, _vp, _vp, _vp]),
    "pmd_debug_pairs": (ctypes.c_int, [_vp, _vp, _i64, _P(_i64), _vp, _P(_i64)]),
    "pmd_debug_lists": (ctypes.c_int, [_vp, _P(_i64), _P(_i64)]),
    "pmd_batch_create": (ctypes.c_int, [ctypes.c_size_t, ctypes.c_int, _vp, _P(_vp)]),
    "pmd_batch_admit": (ctypes.c_int, [_vp, _vp, _i64, _P(ctypes.c_int)]),
    "pmd_batch_advance": (ctypes.c_int, [_vp, _i64]),
    "pmd_batch_poll": (ctypes.c_int, [_vp, _vp, ctypes.c_int, _P(ctypes.c_int)]),
    "pmd_batch_poll_async": (ctypes.c_int, [_vp, _vp, ctypes.c_int, _P(ctypes.c_int)]),
    "pmd_batch_release": (ctypes.c_int, [_vp, ctypes.c_int, _P(_vp)]),
    "pmd_batch_info": (ctypes.c_int, [_vp, _P(ctypes.c_int), _P(ctypes.c_size_t),
                                      _P(ctypes.c_size_t)]),
    "pmd_batch_destroy": (ctypes.c_int, [_vp]),
    "pmd_batch_wall_room": (ctypes.c_int, [_i64, _i64]),
    "pmd_pore_volume": (ctypes.c_int, [_P(pmd_params), _P(pmd_pore), _P(_d)]),
    "pmd_allpairs_forces": (ctypes.c_int, [ctypes.c_int, _i64, _vp, _P(_d), _d, _d, _vp, _vp, _vp, _vp]),
    "pmd_pm_record_rows": (_i64, [_i64, _i64]),
    "pmd_pm_run": (ctypes.c_int, [_P(pmd_pm_model), _i64, _vp, _vp, _vp, _i64, _i64, _vp, _i64, _vp]),
    "pmd_pm_run_noalloc": (ctypes.c_int, [_P(pmd_pm_model), _i64, _vp, _vp, _vp, _i64, _i64, _vp,
                                          _i64, _vp]),
}


def load():
    """Load libporemd.so; raises if it is missing (no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError("libporemd.so not built at %s; run __graft_entry__.build()" % LIB_PATH)
    # One HIP runtime per process: PyTorch ships its own copy of the HIP
    # runtime under the same soname; loading it first makes the library bind
    # to that copy, so streams and device pointers from torch are valid here.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in _SIGS.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _check(code):
    if code != PMD_OK:
        raise PmdError(code, load().pmd_last_error().decode())
    return code


def _f64(a, n3=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if n3 is not None:
        a = a.reshape(n3, 3)
    return a


def _ptr(a):
    return ctypes.c_void_p(a.ctypes.data) if a is not None else None


# ---------------------------------------------------------------------------
# Struct builders
# ---------------------------------------------------------------------------

def make_params(box, precision="fp64", sigma=1.0, epsilon=1.0, mass=1.0, cutoff=2.5,
                dt=0.005, sigma_wall=1.0, epsilon_wall=1.5, thermostat_tau=0.0,
                thermostat_t0=0.0) -> pmd_params:
    p = pmd_params()
    b = np.broadcast_to(np.asarray(box, dtype=np.float64), (3,))
    for k in range(3):
        p.box[k] = float(b[k])
    p.sigma, p.epsilon, p.mass, p.cutoff, p.dt = sigma, epsilon, mass, cutoff, dt
    p.sigma_wall, p.epsilon_wall = sigma_wall, epsilon_wall
    p.precision = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    p.thermostat_tau, p.thermostat_t0 = thermostat_tau, thermostat_t0
    return p


def make_pore(kind="none", lattice_a=1.0, slab_center_z=0.0, slab_thickness=0.0, r0=0.0,
              r1=0.0, slit_gap=0.0) -> pmd_pore:
    q = pmd_pore()
    q.kind = PORE_KINDS[kind] if isinstance(kind, str) else int(kind)
    q.lattice_a, q.slab_center_z, q.slab_thickness = lattice_a, slab_center_z, slab_thickness
    q.r0, q.r1, q.slit_gap = r0, r1, slit_gap
    return q


def make_tuning(skin=0.0, rebin_every=0, block=0, list_cap=0, energy_every=0,
                use_graph=1, brick_atoms=0, brick_order=0, virial=0) -> pmd_tuning:
    t = pmd_tuning()
    t.skin, t.rebin_every, t.block, t.list_cap = skin, rebin_every, block, list_cap
    t.energy_every, t.use_graph, t.brick_atoms = energy_every, use_graph, brick_atoms
    t.brick_order, t.virial = brick_order, virial
    return t


# ---------------------------------------------------------------------------
# C functions under their own names
# ---------------------------------------------------------------------------

def pmd_version():
    return int(load().pmd_version())


def pmd_last_error():
    return load().pmd_last_error().decode()


def pmd_wall_count(params, pore):
    n = ctypes.c_int64()
    _check(load().pmd_wall_count(ctypes.byref(params), ctypes.byref(pore), ctypes.byref(n)))
    return n.value


def pmd_footprint_bytes(params, pore, n_vapor, tuning=None):
    out = ctypes.c_size_t()
    _check(load().pmd_footprint_bytes(ctypes.byref(params), ctypes.byref(pore), int(n_vapor),
                                      ctypes.byref(tuning) if tuning else None,
                                      ctypes.byref(out)))
    return out.value


def pmd_create_system(params, pore, pos, vel, wall_pos=None, stream=None, tuning=None):
    pos = _f64(pos, -1)
    vel = _f64(vel, -1)
    n = pos.shape[0]
    w = _f64(wall_pos, -1) if wall_pos is not None else None
    h = ctypes.c_void_p()
    _check(load().pmd_create_system(ctypes.byref(params), ctypes.byref(pore), n, _ptr(pos),
                                    _ptr(vel), 0 if w is None else w.shape[0], _ptr(w),
                                    ctypes.c_void_p(stream) if stream else None,
                                    ctypes.byref(tuning) if tuning else None, ctypes.byref(h)))
    return h


def pmd_step(h, nsteps):
    _check(load().pmd_step(h, int(nsteps)))


def pmd_sync(h):
    _check(load().pmd_sync(h))


def pmd_get_counts(h):
    a, b = ctypes.c_int64(), ctypes.c_int64()
    _check(load().pmd_get_counts(h, ctypes.byref(a), ctypes.byref(b)))
    return a.value, b.value


def _get3(fn, h, n):
    out = np.empty((n, 3), dtype=np.float64)
    _check(fn(h, _ptr(out), n))
    return out


def pmd_get_positions(h):
    return _get3(load().pmd_get_positions, h, pmd_get_counts(h)[0])


def pmd_get_velocities(h):
    return _get3(load().pmd_get_velocities, h, pmd_get_counts(h)[0])


def pmd_get_forces(h):
    return _get3(load().pmd_get_forces, h, pmd_get_counts(h)[0])


def pmd_get_wall_positions(h):
    return _get3(load().pmd_get_wall_positions, h, pmd_get_counts(h)[1])


def _energy_dict(e):
    return dict(step=e.step, ke=e.ke, pe_vv=e.pe_vv, pe_vw=e.pe_vw, etotal=e.etotal,
                temperature=e.temperature, virial_vv=e.virial_vv, virial_vw=e.virial_vw,
                ke_pore=e.ke_pore, virial_pore=e.virial_pore, n_pore=e.n_pore,
                pore_volume=e.pore_volume, pressure=e.pressure)


def pmd_get_energies(h):
    e = pmd_energies()
    _check(load().pmd_get_energies(h, ctypes.byref(e)))
    return _energy_dict(e)


def pmd_get_energy_history(h, cap=1 << 20):
    """Recorded energies as a structured array (step, ke, pe_vv, pe_vw, etotal,
    temperature, virial_vv, virial_vw, ke_pore, virial_pore, n_pore,
    pore_volume, pressure)."""
    dt = np.dtype([("step", np.int64), ("ke", np.float64), ("pe_vv", np.float64),
                   ("pe_vw", np.float64), ("etotal", np.float64), ("temperature", np.float64),
                   ("virial_vv", np.float64), ("virial_vw", np.float64),
                   ("ke_pore", np.float64), ("virial_pore", np.float64), ("n_pore", np.int64),
                   ("pore_volume", np.float64), ("pressure", np.float64)])
    out = np.zeros(cap, dtype=dt)
    n = ctypes.c_int64()
    _check(load().pmd_get_energy_history(h, ctypes.c_void_p(out.ctypes.data), cap,
                                         ctypes.byref(n)))
    return out[:n.value]


def pmd_get_step(h):
    return int(load().pmd_get_step(h))


def pmd_get_positions_device(h, dev_ptr, n, stream=None):
    _check(load().pmd_get_positions_device(h, ctypes.c_void_p(dev_ptr), int(n),
                                           ctypes.c_void_p(stream) if stream else None))


def pmd_pore_volume(params, pore):
    v = ctypes.c_double()
    _check(load().pmd_pore_volume(ctypes.byref(params), ctypes.byref(pore), ctypes.byref(v)))
    return v.value


def pmd_batch_wall_room(resident_walls, new_walls):
    """PMD_OK if a batch holding resident_walls wall slots can take
    new_walls more; raises PmdError (PMD_EAGAIN) if not."""
    return _check(load().pmd_batch_wall_room(int(resident_walls), int(new_walls)))


def pmd_allpairs_forces(precision, n, x_ptr, box, epsilon, sigma, f_ptr, u_ptr, e_ptr, stream=None):
    """All-pairs forces on device buffers given by address (see the header)."""
    prec = {"mixed": 1, "fp64": 2}.get(precision, precision)
    b = (ctypes.c_double * 3)(*[float(v) for v in box])
    _check(load().pmd_allpairs_forces(int(prec), int(n), ctypes.c_void_p(x_ptr or None), b,
                                      float(epsilon), float(sigma), ctypes.c_void_p(f_ptr or None),
                                      ctypes.c_void_p(u_ptr or None), ctypes.c_void_p(e_ptr or None),
                                      ctypes.c_void_p(stream) if stream else None))


def pmd_set_tuning(h, tuning):
    _check(load().pmd_set_tuning(h, ctypes.byref(tuning)))


def pmd_get_tuning(h):
    t = pmd_tuning()
    _check(load().pmd_get_tuning(h, ctypes.byref(t)))
    return t


def pmd_set_state(h, pos, vel, step=0):
    pos = _f64(pos, -1)
    vel = _f64(vel, -1)
    _check(load().pmd_set_state(h, _ptr(pos), _ptr(vel), pos.shape[0], int(step)))


def pmd_autotune_grid(params, n_vapor):
    n = ctypes.c_int32()
    _check(load().pmd_autotune_grid(ctypes.byref(params), int(n_vapor), None, 0, ctypes.byref(n)))
    out = (pmd_tuning * n.value)()
    _check(load().pmd_autotune_grid(ctypes.byref(params), int(n_vapor), out, n.value,
                                    ctypes.byref(n)))
    return list(out)


def pmd_autotune(params, pore, pos, vel, candidates, trial_steps=200, wall_pos=None, stream=None):
    """Returns (index of the fastest candidate, microseconds per step of each)."""
    pos = _f64(pos, -1)
    vel = _f64(vel, -1)
    w = _f64(wall_pos, -1) if wall_pos is not None else None
    cand = (pmd_tuning * len(candidates))(*candidates)
    us = np.zeros(len(candidates), dtype=np.float64)
    best = ctypes.c_int32()
    _check(load().pmd_autotune(ctypes.byref(params), ctypes.byref(pore), pos.shape[0], _ptr(pos),
                               _ptr(vel), 0 if w is None else w.shape[0], _ptr(w),
                               ctypes.c_void_p(stream) if stream else None, cand, len(candidates),
                               int(trial_steps), _ptr(us), ctypes.byref(best)))
    return best.value, us


def pmd_destroy(h):
    if h:
        _check(load().pmd_destroy(h))


def pmd_timing_enable(h, enable=True):
    _check(load().pmd_timing_enable(h, 1 if enable else 0))


def pmd_kernel_time(h):
    n, ms = ctypes.c_int64(), ctypes.c_double()
    _check(load().pmd_kernel_time(h, ctypes.byref(n), ctypes.byref(ms)))
    return n.value, ms.value


def pmd_kernel_times(h):
    n = ctypes.c_int64()
    _check(load().pmd_kernel_times(h, None, 0, ctypes.byref(n)))
    out = np.zeros(n.value, dtype=np.float64)
    _check(load().pmd_kernel_times(h, _ptr(out), n.value, ctypes.byref(n)))
    return out


def pmd_debug_cells(h):
    nv, _ = pmd_get_counts(h)
    nc = np.zeros(3, dtype=np.int32)
    inv = np.zeros(3, dtype=np.float64)
    _check(load().pmd_debug_cells(h, None, 0, None, 0, None, _ptr(nc), _ptr(inv)))
    ncell = int(np.prod(nc))
    cell = np.zeros(nv, dtype=np.int32)
    start = np.zeros(ncell + 1, dtype=np.int32)
    perm = np.zeros(nv, dtype=np.int32)
    _check(load().pmd_debug_cells(h, _ptr(cell), nv, _ptr(start), ncell + 1, _ptr(perm),
                                  _ptr(nc), _ptr(inv)))
    return cell, start, perm, nc, inv


def pmd_debug_pairs(h):
    a, b = ctypes.c_int64(), ctypes.c_int64()
    _check(load().pmd_debug_pairs(h, None, 0, ctypes.byref(a), None, ctypes.byref(b)))
    cap = max(a.value, b.value, 1)
    vv = np.zeros((cap, 2), dtype=np.int32)
    vw = np.zeros((cap, 2), dtype=np.int32)
    _check(load().pmd_debug_pairs(h, _ptr(vv), cap, ctypes.byref(a), _ptr(vw), ctypes.byref(b)))
    return vv[:a.value], vw[:b.value]


def pmd_debug_lists(h):
    a, b = ctypes.c_int64(), ctypes.c_int64()
    _check(load().pmd_debug_lists(h, ctypes.byref(a), ctypes.byref(b)))
    return a.value, b.value


def pmd_batch_create(hbm_budget=0, max_slots=256, stream=None):
    h = ctypes.c_void_p()
    _check(load().pmd_batch_create(int(hbm_budget), int(max_slots),
                                   ctypes.c_void_p(stream) if stream else None, ctypes.byref(h)))
    return h


def pmd_batch_admit(b, sys_h, nsteps):
    """Returns the slot, or None if the batch has no room now (PMD_EAGAIN)."""
    slot = ctypes.c_int()
    code = load().pmd_batch_admit(b, sys_h, int(nsteps), ctypes.byref(slot))
    if code == PMD_EAGAIN:
        return None
    _check(code)
    return slot.value


def pmd_batch_advance(b, chunk_steps):
    _check(load().pmd_batch_advance(b, int(chunk_steps)))


def _poll(fn, b, cap):
    out = (ctypes.c_int * max(cap, 1))()
    n = ctypes.c_int()
    _check(fn(b, out, cap, ctypes.byref(n)))
    return [out[k] for k in range(n.value)]


def pmd_batch_poll(b, cap=4096):
    return _poll(load().pmd_batch_poll, b, cap)


def pmd_batch_poll_async(b, cap=4096):
    return _poll(load().pmd_batch_poll_async, b, cap)


def pmd_batch_release(b, slot):
    h = ctypes.c_void_p()
    _check(load().pmd_batch_release(b, int(slot), ctypes.byref(h)))
    return h


def pmd_batch_info(b):
    r, u, g = ctypes.c_int(), ctypes.c_size_t(), ctypes.c_size_t()
    _check(load().pmd_batch_info(b, ctypes.byref(r), ctypes.byref(u), ctypes.byref(g)))
    return r.value, u.value, g.value


def pmd_batch_destroy(b):
    if b:
        _check(load().pmd_batch_destroy(b))


# ---------------------------------------------------------------------------
# Convenience wrapper over a handle
# ---------------------------------------------------------------------------

def params_of(sysdesc, precision=None):
    """C structs from an input-generator system description."""
    p = sysdesc.params
    q = sysdesc.pore
    params = make_params(p.box, precision or p.precision, p.sigma, p.epsilon, p.mass, p.cutoff,
                         p.dt, p.sigma_wall, p.epsilon_wall)
    pore = make_pore(q.kind, q.lattice_a, q.slab_center_z, q.slab_thickness, q.r0, q.r1,
                     q.slit_gap)
    return params, pore


class System:
    """Owns one pmd_system handle."""

    def __init__(self, params, pore, pos, vel, wall_pos=None, stream=None, tuning=None):
        self.h = pmd_create_system(params, pore, pos, vel, wall_pos, stream, tuning)
        self.n, self.n_wall = pmd_get_counts(self.h)

    @classmethod
    def from_desc(cls, sysdesc, precision=None, tuning=None, stream=None, walls_from_lib=True):
        params, pore = params_of(sysdesc, precision)
        w = None if walls_from_lib else sysdesc.walls
        return cls(params, pore, sysdesc.x, sysdesc.v, w, stream, tuning)

    def step(self, n):
        pmd_step(self.h, n)

    def sync(self):
        pmd_sync(self.h)

    def positions(self):
        return pmd_get_positions(self.h)

    def velocities(self):
        return pmd_get_velocities(self.h)

    def forces(self):
        return pmd_get_forces(self.h)

    def walls(self):
        return pmd_get_wall_positions(self.h)

    def energies(self):
        return pmd_get_energies(self.h)

    def energy_history(self):
        return pmd_get_energy_history(self.h)

    def step_count(self):
        return pmd_get_step(self.h)

    def set_state(self, pos, vel, step=0):
        pmd_set_state(self.h, pos, vel, step)

    def set_tuning(self, tuning):
        pmd_set_tuning(self.h, tuning)

    def close(self):
        if self.h:
            pmd_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---------------------------------------------------------------------------
# The paper's pore model
# ---------------------------------------------------------------------------

def make_pm_model(dim, lx, ly, lz=0.0, k=1.0, precision="fp64", sigma=1.0, epsilon=1.0,
                  mass=1.0, dt=0.005, thermostat_tau=0.0, thermostat_t0=0.0) -> pmd_pm_model:
    m = pmd_pm_model()
    m.dim = int(dim)
    m.precision = {"mixed": 1, "fp32": 1, "fp64": 2}[precision] if isinstance(precision, str) \
        else int(precision)
    m.lx, m.ly, m.lz, m.k = float(lx), float(ly), float(lz), float(k)
    m.sigma, m.epsilon, m.mass, m.dt = float(sigma), float(epsilon), float(mass), float(dt)
    m.thermostat_tau, m.thermostat_t0 = float(thermostat_tau), float(thermostat_t0)
    return m


def pmd_pm_record_rows(nsteps, energy_every):
    return int(load().pmd_pm_record_rows(int(nsteps), int(energy_every)))


def pmd_pm_run(model, n, x_ptr, v_ptr, a_ptr, nsteps, energy_every, rec_ptr, rec_cap, stream=None):
    """Device pointers in, in place; a_ptr and rec_ptr may be 0 (not wanted)."""
    return _check(load().pmd_pm_run(ctypes.byref(model), int(n), ctypes.c_void_p(x_ptr or None),
                                    ctypes.c_void_p(v_ptr or None), ctypes.c_void_p(a_ptr or None),
                                    int(nsteps), int(energy_every),
                                    ctypes.c_void_p(rec_ptr or None), int(rec_cap),
                                    ctypes.c_void_p(stream or None)))


def pmd_pm_run_noalloc(model, n, x_ptr, v_ptr, a_ptr, nsteps, energy_every, rec_ptr, rec_cap,
                       stream=None):
    """pmd_pm_run with the library's static working memory (n <= 65536)."""
    return _check(load().pmd_pm_run_noalloc(ctypes.byref(model), int(n),
                                            ctypes.c_void_p(x_ptr or None),
                                            ctypes.c_void_p(v_ptr or None),
                                            ctypes.c_void_p(a_ptr or None), int(nsteps),
                                            int(energy_every), ctypes.c_void_p(rec_ptr or None),
                                            int(rec_cap), ctypes.c_void_p(stream or None)))
