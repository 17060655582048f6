"""Plain FP64 CPU oracle for the pore molecular-dynamics hot path.

TEST INFRASTRUCTURE ONLY.  This package is the checker that the GPU library
is compared against.  Only the tests, the smoke check and the benchmark's
CPU-baseline leg may import it; the product path never does.  It shares no
code with the GPU library: the arithmetic lives in ``oracle.c`` (built by
``oracle/build.py`` into ``oracle/_build/liboracle.so``), and this module only
marshals numpy arrays.

What each function follows in arXiv:1812.07993:
  * ``pair``           -- the Lennard-Jones potential named in Sec. 2;
  * ``forces``         -- eq. 2, f_i = -dU/dr_i + f_i^ex, over all pairs (the
                          paper's F1 visits every pair, Sec. 3);
  * ``forces_subset``  -- eq. 2 for chosen atoms only (sampled checks);
  * ``run``            -- velocity Verlet in the order F2, F1, F3 (Sec. 3);
  * ``allpairs``       -- the force function as stated in Sec. 3: every
                          pair, no cutoff, no shift (minimum image);
  * ``wall_lattice``   -- the pore walls (the paper's walls are boundary
                          conditions, Secs. 4-5; the lattice is a reading);
  * ``cell_sort``, ``pairs`` -- the integer work of binning and neighbour
                          search, written as their plain definitions;
  * ``pm_forces``, ``pm_trace``, ``pm_run`` -- the paper's own pore model
                          (Secs. 4-5): all-pairs forces in 2D or 3D, a
                          pore with reflecting walls opening into a
                          periodic outer space, velocity Verlet F2, F1, F3
                          and the Berendsen F4.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "_build", "liboracle.so")
_lib = None

PORE_KINDS = {"none": 0, "slab": 1, "cylinder": 2, "slit": 3, "cone": 4,
              "inkbottle": 5}


class Params(ctypes.Structure):
    _fields_ = [("box", ctypes.c_double * 3), ("sigma", ctypes.c_double),
                ("epsilon", ctypes.c_double), ("mass", ctypes.c_double),
                ("cutoff", ctypes.c_double), ("dt", ctypes.c_double),
                ("sigma_wall", ctypes.c_double),
                ("epsilon_wall", ctypes.c_double)]


class PmModel(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int32), ("pad_", ctypes.c_int32),
                ("lx", ctypes.c_double), ("ly", ctypes.c_double), ("lz", ctypes.c_double),
                ("k", ctypes.c_double), ("sigma", ctypes.c_double),
                ("epsilon", ctypes.c_double), ("mass", ctypes.c_double),
                ("dt", ctypes.c_double), ("tau", ctypes.c_double), ("t0", ctypes.c_double)]


class Pore(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("pad_", ctypes.c_int32),
                ("lattice_a", ctypes.c_double),
                ("slab_center_z", ctypes.c_double),
                ("slab_thickness", ctypes.c_double),
                ("r0", ctypes.c_double), ("r1", ctypes.c_double),
                ("slit_gap", ctypes.c_double)]


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        from . import build as _build
        _build.build()
    lib = ctypes.CDLL(_LIB_PATH)
    P = ctypes.POINTER
    d, i64, i32 = ctypes.c_double, ctypes.c_int64, ctypes.c_int32
    vp = ctypes.c_void_p
    lib.orc_num_threads.restype = ctypes.c_int
    lib.orc_set_threads.argtypes = [ctypes.c_int]
    lib.orc_pair.argtypes = [d, d, d, d, P(d), P(d)]
    lib.orc_forces.argtypes = [i64, vp, i64, vp, P(Params), vp, P(d), P(d), vp]
    lib.orc_forces_subset.argtypes = [i64, vp, i64, vp, P(Params), i64, vp, vp, vp]
    lib.orc_run.argtypes = [i64, vp, vp, vp, ctypes.c_int, i64, vp, P(Params),
                            i64, i64, vp, d, d]
    lib.orc_run.restype = i64
    lib.orc_virial.argtypes = [i64, vp, i64, vp, P(Params), P(d), P(d)]
    lib.orc_allpairs.argtypes = [i64, vp, vp, d, d, vp, vp, P(d)]
    lib.orc_wall_lattice.argtypes = [P(Pore), vp, vp, i64]
    lib.orc_wall_lattice.restype = i64
    lib.orc_cell_sort.argtypes = [i64, vp, vp, vp, vp, vp, vp]
    lib.orc_pairs.argtypes = [i64, vp, i64, vp, vp, d, i64, vp, P(i64), vp, P(i64)]
    lib.orc_pore_volume.argtypes = [P(Pore), vp]
    lib.orc_pore_volume.restype = d
    lib.orc_pore_pressure.argtypes = [i64, vp, vp, P(Params), P(Pore), vp]
    lib.orc_pore_count.argtypes = [i64, vp, vp, P(Pore)]
    lib.orc_pore_count.restype = i64
    lib.orc_pm_forces.argtypes = [P(PmModel), i64, vp, vp, vp, P(d)]
    lib.orc_pm_trace.argtypes = [P(PmModel), vp, vp, vp]
    lib.orc_pm_trace.restype = ctypes.c_int
    lib.orc_pm_run.argtypes = [P(PmModel), i64, vp, vp, i64, i64, vp]
    lib.orc_pm_run.restype = i64
    _lib = lib
    return lib


def _f64(a, shape=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if shape is not None:
        a = a.reshape(shape)
    return a


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None else None


def make_params(box, sigma=1.0, epsilon=1.0, mass=1.0, cutoff=2.5, dt=0.005,
                sigma_wall=1.0, epsilon_wall=1.5) -> Params:
    p = Params()
    b = np.broadcast_to(np.asarray(box, dtype=np.float64), (3,))
    for k in range(3):
        p.box[k] = float(b[k])
    p.sigma, p.epsilon, p.mass = sigma, epsilon, mass
    p.cutoff, p.dt = cutoff, dt
    p.sigma_wall, p.epsilon_wall = sigma_wall, epsilon_wall
    return p


def make_pore(kind="none", lattice_a=1.0, slab_center_z=0.0,
              slab_thickness=0.0, r0=0.0, r1=0.0, slit_gap=0.0) -> Pore:
    q = Pore()
    q.kind = PORE_KINDS[kind] if isinstance(kind, str) else int(kind)
    q.lattice_a, q.slab_center_z, q.slab_thickness = lattice_a, slab_center_z, slab_thickness
    q.r0, q.r1, q.slit_gap = r0, r1, slit_gap
    return q


def set_threads(n: int) -> None:
    _load().orc_set_threads(int(n))


def num_threads() -> int:
    return int(_load().orc_num_threads())


def pair(r: float, sigma=1.0, epsilon=1.0, cutoff=2.5):
    """(u, w) of one pair at distance r; force on i = w * (r_i - r_j)."""
    u, w = ctypes.c_double(), ctypes.c_double()
    _load().orc_pair(float(r), float(sigma), float(epsilon), float(cutoff),
                     ctypes.byref(u), ctypes.byref(w))
    return u.value, w.value


def forces(x, walls, params: Params, wall_reaction=False):
    """Forces on all vapour atoms (eq. 2).  Returns (F, pe_vv, pe_vw) or, with
    wall_reaction, (F, pe_vv, pe_vw, F_on_walls)."""
    x = _f64(x, (-1, 3))
    w = _f64(walls if walls is not None else np.zeros((0, 3)), (-1, 3))
    F = np.zeros_like(x)
    Fw = np.zeros_like(w) if wall_reaction else None
    evv, evw = ctypes.c_double(), ctypes.c_double()
    _load().orc_forces(x.shape[0], _ptr(x), w.shape[0], _ptr(w),
                       ctypes.byref(params), _ptr(F), ctypes.byref(evv),
                       ctypes.byref(evw), _ptr(Fw))
    if wall_reaction:
        return F, evv.value, evw.value, Fw
    return F, evv.value, evw.value


def forces_subset(x, walls, params: Params, sel):
    """Forces (m, 3) and per-atom energies (m,) on the vapour atoms sel."""
    x = _f64(x, (-1, 3))
    w = _f64(walls if walls is not None else np.zeros((0, 3)), (-1, 3))
    sel = np.ascontiguousarray(sel, dtype=np.int64)
    F = np.zeros((sel.shape[0], 3))
    pe = np.zeros(sel.shape[0])
    _load().orc_forces_subset(x.shape[0], _ptr(x), w.shape[0], _ptr(w),
                              ctypes.byref(params), sel.shape[0], _ptr(sel),
                              _ptr(F), _ptr(pe))
    return F, pe


def run(x, v, walls, params: Params, nsteps: int, every=1, a=None, tau=0.0, t0=0.0):
    """Velocity Verlet for nsteps (F2, F1, F3; with tau > 0 also F4, the
    Berendsen scaling towards temperature t0 with rise time tau, Sec. 2 and
    Sec. 3).  Returns (x, v, a, energies) with energies rows (ke, pe_vv,
    pe_vw) at step 0, every `every` steps and at the last step (ke as the
    thermostat measured it, before its scaling)."""
    x = _f64(x, (-1, 3)).copy()
    v = _f64(v, (-1, 3)).copy()
    w = _f64(walls if walls is not None else np.zeros((0, 3)), (-1, 3))
    have_a = a is not None
    acc = _f64(a, (-1, 3)).copy() if have_a else np.zeros_like(x)
    cap = 2 + (nsteps // every if every > 0 else 0) + 1
    E = np.zeros((cap, 3))
    rows = _load().orc_run(x.shape[0], _ptr(x), _ptr(v), _ptr(acc),
                           int(have_a), w.shape[0], _ptr(w),
                           ctypes.byref(params), int(nsteps), int(every),
                           _ptr(E), float(tau), float(t0))
    return x, v, acc, E[:rows]


def virial(x, walls, params: Params):
    """Virial sums (w_vv, w_vw) of the pressure formula (Sec. 2): sum over
    vapour pairs i < j and over vapour-wall pairs of r_ij . f_ij (f the force
    on the first atom, minimum image, inside the cutoff)."""
    x = _f64(x, (-1, 3))
    w = _f64(walls if walls is not None else np.zeros((0, 3)), (-1, 3))
    wvv, wvw = ctypes.c_double(), ctypes.c_double()
    _load().orc_virial(x.shape[0], _ptr(x), w.shape[0], _ptr(w), ctypes.byref(params),
                       ctypes.byref(wvv), ctypes.byref(wvw))
    return wvv.value, wvw.value


def allpairs(x, box, epsilon=1.0, sigma=1.0):
    """All-pairs Lennard-Jones forces as the paper's force function states
    them (Sec. 3): every pair, no cutoff, no shift; minimum image on the axes
    with box[k] > 0.  Returns (forces [n, 3], per-atom half shares of the
    energy [n], total energy)."""
    x = _f64(x, (-1, 3))
    b = _f64(np.asarray(box, dtype=np.float64).reshape(3), (3,))
    n = x.shape[0]
    f = np.zeros((n, 3))
    u = np.zeros(n)
    e = ctypes.c_double()
    _load().orc_allpairs(n, _ptr(x), _ptr(b), float(epsilon), float(sigma), _ptr(f), _ptr(u),
                         ctypes.byref(e))
    return f, u, e.value


def pore_volume(pore: Pore, box):
    """Volume of the pore's void (closed form per shape; the whole box for
    no walls, 0 for a plain slab)."""
    b = _f64(np.broadcast_to(np.asarray(box, dtype=np.float64), (3,)))
    return float(_load().orc_pore_volume(ctypes.byref(pore), _ptr(b)))


def pore_count(x, box, pore: Pore):
    """How many of the points lie in the pore's void."""
    x = _f64(x, (-1, 3))
    b = _f64(np.broadcast_to(np.asarray(box, dtype=np.float64), (3,)))
    return int(_load().orc_pore_count(x.shape[0], _ptr(x), _ptr(b), ctypes.byref(pore)))


def pore_pressure(x, v, params: Params, pore: Pore):
    """Pressure in the pore by the formula of Sec. 2 with V the pore volume:
    dict(ke_pore, virial_pore, n_pore, volume, pressure) with
    P = (2 ke_pore + virial_pore) / (3 V), the virial over vapour pairs
    inside the cutoff, each pair split equally between its molecules."""
    x = _f64(x, (-1, 3))
    v = _f64(v, (-1, 3))
    out = np.zeros(5)
    _load().orc_pore_pressure(x.shape[0], _ptr(x), _ptr(v), ctypes.byref(params),
                              ctypes.byref(pore), _ptr(out))
    return dict(ke_pore=out[0], virial_pore=out[1], n_pore=int(out[2]), volume=out[3],
                pressure=out[4])


def wall_lattice(pore: Pore, box):
    """Wall sites (n, 3) of a pore in canonical order (layer, y, x)."""
    b = _f64(np.broadcast_to(np.asarray(box, dtype=np.float64), (3,)))
    lib = _load()
    n = lib.orc_wall_lattice(ctypes.byref(pore), _ptr(b), None, 0)
    out = np.zeros((max(n, 1), 3))
    lib.orc_wall_lattice(ctypes.byref(pore), _ptr(b), _ptr(out), n)
    return out[:n]


def cell_sort(x, inv, nc):
    """Stable counting sort into cells: (cell[n], cell_start[ncells+1], perm[n])."""
    x = _f64(x, (-1, 3))
    inv = _f64(inv)
    nc = np.ascontiguousarray(nc, dtype=np.int32)
    n = x.shape[0]
    ncell = int(nc[0]) * int(nc[1]) * int(nc[2])
    cell = np.zeros(n, dtype=np.int32)
    start = np.zeros(ncell + 1, dtype=np.int32)
    perm = np.zeros(n, dtype=np.int32)
    _load().orc_cell_sort(n, _ptr(x), _ptr(inv), _ptr(nc), _ptr(cell),
                          _ptr(start), _ptr(perm))
    return cell, start, perm


def pairs(x, walls, box, cutoff):
    """In-cutoff pair sets: vv (k, 2) with i < j and vw (k, 2) as (i, wall)."""
    x = _f64(x, (-1, 3))
    w = _f64(walls if walls is not None else np.zeros((0, 3)), (-1, 3))
    b = _f64(np.broadcast_to(np.asarray(box, dtype=np.float64), (3,)))
    lib = _load()
    nvv, nvw = ctypes.c_int64(), ctypes.c_int64()
    lib.orc_pairs(x.shape[0], _ptr(x), w.shape[0], _ptr(w), _ptr(b),
                  float(cutoff), 0, None, ctypes.byref(nvv), None,
                  ctypes.byref(nvw))
    cap = max(nvv.value, nvw.value, 1)
    vv = np.zeros((cap, 2), dtype=np.int32)
    vw = np.zeros((cap, 2), dtype=np.int32)
    lib.orc_pairs(x.shape[0], _ptr(x), w.shape[0], _ptr(w), _ptr(b),
                  float(cutoff), cap, _ptr(vv), ctypes.byref(nvv), _ptr(vw),
                  ctypes.byref(nvw))
    return vv[:nvv.value], vw[:nvw.value]


# ---------------------------------------------------------------------------
# The paper's pore model (Secs. 4-5)
# ---------------------------------------------------------------------------

def pm_model(dim, lx, ly, lz=0.0, k=1.0, sigma=1.0, epsilon=1.0, mass=1.0, dt=0.005,
             tau=0.0, t0=0.0) -> PmModel:
    """The pore [0, lx) x [0, ly) (x [0, lz)) with reflecting walls, open at
    x = lx into an outer space k lx long and (2k+1) times as wide on each
    transverse axis, periodic; all-pairs Lennard-Jones forces without
    cutoff; Berendsen thermostat if tau > 0."""
    m = PmModel()
    m.dim, m.lx, m.ly, m.lz, m.k = int(dim), float(lx), float(ly), float(lz), float(k)
    m.sigma, m.epsilon, m.mass, m.dt = float(sigma), float(epsilon), float(mass), float(dt)
    m.tau, m.t0 = float(tau), float(t0)
    return m


def pm_forces(model: PmModel, x):
    """All-pairs forces (plain differences, no images) in model.dim
    dimensions: (forces [n, d], per-atom half shares [n], total energy)."""
    d = model.dim
    x = _f64(x, (-1, d))
    n = x.shape[0]
    f = np.zeros((n, d))
    u = np.zeros(n)
    e = ctypes.c_double()
    _load().orc_pm_forces(ctypes.byref(model), n, _ptr(x), _ptr(f), _ptr(u), ctypes.byref(e))
    return f, u, e.value


def pm_trace(model: PmModel, p, dl, v):
    """One particle carried along the drift dl through the model's
    boundaries: (new position, new velocity, reflections)."""
    p3 = np.zeros(3)
    d3 = np.zeros(3)
    v3 = np.zeros(3)
    p3[:model.dim] = p
    d3[:model.dim] = dl
    v3[:model.dim] = v
    r = _load().orc_pm_trace(ctypes.byref(model), _ptr(p3), _ptr(d3), _ptr(v3))
    if r < 0:
        raise RuntimeError("drift could not be traced")
    return p3[:model.dim].copy(), v3[:model.dim].copy(), int(r)


def pm_run(model: PmModel, x, v, nsteps: int, every=1):
    """nsteps velocity-Verlet steps of the pore model (F2 with the boundary
    trace, F1, F3, and F4 if model.tau > 0).  Returns (x, v, records) with
    records rows (step, ke, pe, atoms in the pore, reflections so far,
    pressure in the pore) at step 0, every `every` steps and the last
    step."""
    d = model.dim
    x = _f64(x, (-1, d)).copy()
    v = _f64(v, (-1, d)).copy()
    cap = 2 + (nsteps // every if every > 0 else 0) + 1
    rec = np.zeros((cap, 6))
    rows = _load().orc_pm_run(ctypes.byref(model), x.shape[0], _ptr(x), _ptr(v), int(nsteps),
                              int(every), _ptr(rec))
    if rows < 0:
        raise RuntimeError("a drift could not be traced")
    return x, v, rec[:rows]
