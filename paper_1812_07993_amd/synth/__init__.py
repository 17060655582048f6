"""Seeded synthetic inputs for pore molecular-dynamics runs.

Input tooling shared by the tests, the benchmark and the serving demo.  It
holds none of the method's arithmetic (no forces, energies or integration):
it lays out wall sites only to keep new vapour atoms clear of them, places
vapour atoms by random sequential addition with a minimum distance, and draws
Maxwell velocities.  The paper sets its initial state from tabulated vapour
densities (Sec. 2) that are not reproduced here; the workloads below are
synthetic stand-ins in reduced Lennard-Jones units.

Seeds: numpy.random.SeedSequence([1812, 7993, workload, replica]) spawns
independent streams for placement and velocities, so every input is a pure
function of (workload, replica).
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "_build", "librsa.so")
_lib = None

SEED_ROOT = (1812, 7993)


def build(verbose: bool = False) -> str:
    os.makedirs(os.path.dirname(_LIB_PATH), exist_ok=True)
    tmp = _LIB_PATH + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O2", "-fPIC", "-shared", "-std=c11", "-Wall", "-o", tmp,
           os.path.join(_HERE, "rsa.c"), "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        lib = ctypes.CDLL(_LIB_PATH)
        vp, i64, d = ctypes.c_void_p, ctypes.c_int64, ctypes.c_double
        lib.rsa_create.argtypes = [vp, d, i64]
        lib.rsa_create.restype = vp
        lib.rsa_destroy.argtypes = [vp]
        lib.rsa_add_obstacles.argtypes = [vp, vp, i64]
        lib.rsa_add_obstacles.restype = i64
        lib.rsa_try.argtypes = [vp, vp, i64, vp, i64, ctypes.POINTER(i64)]
        lib.rsa_try.restype = i64
        _lib = lib
    return _lib


# ---------------------------------------------------------------------------
# Descriptions of a system
# ---------------------------------------------------------------------------

@dataclass
class Pore:
    """Pore geometry.  kind: none | slab | cylinder | slit | cone | inkbottle.
    Walls are simple-cubic slabs of spacing lattice_a.  One slab of thickness
    slab_thickness is centred at slab_center_z, except for a slit, which has
    two slabs whose facing surfaces are slit_gap apart around slab_center_z.
    The pore axis runs along z through (Lx/2, Ly/2); r0 is the cylinder
    radius, the cone radius at the lower face or the ink-bottle neck radius;
    r1 is the cone radius at the upper face or the ink-bottle cavity radius."""
    kind: str = "none"
    lattice_a: float = 1.0
    slab_center_z: float = 0.0
    slab_thickness: float = 0.0
    r0: float = 0.0
    r1: float = 0.0
    slit_gap: float = 0.0


@dataclass
class Params:
    """Model parameters (reduced Lennard-Jones units)."""
    box: tuple = (32.0, 32.0, 32.0)
    sigma: float = 1.0
    epsilon: float = 1.0
    mass: float = 1.0
    cutoff: float = 2.5
    dt: float = 0.005
    sigma_wall: float = 1.0
    epsilon_wall: float = 1.5
    precision: str = "fp64"  # "fp64" or "mixed"


@dataclass
class System:
    name: str
    params: Params
    pore: Pore
    x: np.ndarray          # (n, 3) vapour positions in [0, L)
    v: np.ndarray          # (n, 3) vapour velocities
    walls: np.ndarray      # (m, 3) wall sites (for exclusion and reference)
    steps: int = 0
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.x.shape[0])


# ---------------------------------------------------------------------------
# Wall sites (only to keep vapour atoms clear of them)
# ---------------------------------------------------------------------------

def _slab(pore: Pore, box, z_lo: float, t: float) -> np.ndarray:
    a = pore.lattice_a
    nx, ny, nz = (int(round(box[0] / a)), int(round(box[1] / a)),
                  int(round(t / a)))
    xs = (np.arange(nx) + 0.5) * a
    ys = (np.arange(ny) + 0.5) * a
    out = []
    for k in range(nz):
        h = (k + 0.5) * a
        if pore.kind == "cylinder":
            r = pore.r0
        elif pore.kind == "cone":
            r = pore.r0 + (pore.r1 - pore.r0) * (h / t)
        elif pore.kind == "inkbottle":
            r = pore.r0 if (h < 0.25 * t or h >= 0.75 * t) else pore.r1
        else:
            r = 0.0
        X, Y = np.meshgrid(xs, ys, indexing="xy")
        keep = (X - 0.5 * box[0]) ** 2 + (Y - 0.5 * box[1]) ** 2 >= r * r
        pts = np.stack([X[keep], Y[keep], np.full(int(keep.sum()), z_lo + h)], 1)
        out.append(pts)
    return np.concatenate(out, 0) if out else np.zeros((0, 3))


def wall_sites(pore: Pore, box) -> np.ndarray:
    """Wall sites in order (layer, y, x); lower slab first for a slit."""
    box = tuple(float(b) for b in box)
    t, c = pore.slab_thickness, pore.slab_center_z
    if pore.kind == "none":
        return np.zeros((0, 3))
    if pore.kind == "slit":
        return np.concatenate([_slab(pore, box, c - 0.5 * pore.slit_gap - t, t),
                               _slab(pore, box, c + 0.5 * pore.slit_gap, t)], 0)
    return _slab(pore, box, c - 0.5 * t, t)


# ---------------------------------------------------------------------------
# Placement and velocities
# ---------------------------------------------------------------------------

def rsa_place(rng: np.random.Generator, box, n: int, obstacles: np.ndarray,
              dmin: float = 0.9, z_exclude=None, max_tries_per_atom=200):
    """Random sequential addition of n points, each at least dmin from every
    obstacle and every earlier point (minimum image).  z_exclude=(lo, hi)
    keeps candidates out of lo <= z < hi (uniform over the rest)."""
    box = np.asarray(box, dtype=np.float64)
    lib = _load()
    obstacles = np.ascontiguousarray(obstacles, dtype=np.float64).reshape(-1, 3)
    g = lib.rsa_create(box.ctypes.data_as(ctypes.c_void_p), float(dmin),
                       int(n + obstacles.shape[0]))
    if not g:
        raise MemoryError("rsa grid")
    try:
        if obstacles.shape[0]:
            lib.rsa_add_obstacles(g, obstacles.ctypes.data_as(ctypes.c_void_p),
                                  obstacles.shape[0])
        out = np.zeros((n, 3))
        got, tried = 0, 0
        while got < n:
            if tried > max_tries_per_atom * max(n, 1):
                raise RuntimeError("placement failed: %d of %d after %d tries"
                                   % (got, n, tried))
            m = max(4096, 2 * (n - got))
            c = rng.random((m, 3)) * box
            if z_exclude is not None:
                lo, hi = z_exclude
                zz = rng.random(m) * (box[2] - (hi - lo))
                c[:, 2] = np.where(zz < lo, zz, zz + (hi - lo))
            c = np.ascontiguousarray(c)
            used = ctypes.c_int64()
            k = lib.rsa_try(g, c.ctypes.data_as(ctypes.c_void_p), m,
                            out[got:].ctypes.data_as(ctypes.c_void_p),
                            n - got, ctypes.byref(used))
            got += int(k)
            tried += int(used.value)
        return out
    finally:
        lib.rsa_destroy(g)


def maxwell(rng: np.random.Generator, n: int, temperature: float,
            mass: float = 1.0) -> np.ndarray:
    """Gaussian components of variance T/m, centre-of-mass velocity removed,
    rescaled so that 2 KE / (3n - 3) equals T exactly (k_B = 1)."""
    v = rng.standard_normal((n, 3)) * math.sqrt(temperature / mass)
    if n > 1:
        v -= v.mean(axis=0, keepdims=True)
        ke2 = mass * float(np.sum(v * v))
        v *= math.sqrt(temperature * (3 * n - 3) / ke2)
    return v


def _streams(*key):
    ss = np.random.SeedSequence(list(SEED_ROOT) + [int(k) for k in key])
    a, b = ss.spawn(2)
    return np.random.default_rng(a), np.random.default_rng(b)


# ---------------------------------------------------------------------------
# Workloads
# ---------------------------------------------------------------------------

T_STAR = 1.2
DT = 0.005
RHO_SMALL = 0.1


def make_system(name, box, pore: Pore, n: int, precision: str, key,
                steps=0, z_exclude=None, temperature=T_STAR, meta=None) -> System:
    rng_x, rng_v = _streams(*key)
    walls = wall_sites(pore, box)
    x = rsa_place(rng_x, box, n, walls, 0.9, z_exclude)
    v = maxwell(rng_v, n, temperature)
    p = Params(box=tuple(float(b) for b in box), dt=DT, precision=precision)
    return System(name, p, pore, x, v, walls, steps, dict(meta or {}))


def cylinder_slab_small(n=1536, seed=0, precision="fp64") -> System:
    """32^3 box, mid-plane slab 4 thick (z in [14, 18)) with a cylindrical
    pore of radius 3; vapour only above and below the slab; 200 steps."""
    pore = Pore("cylinder", 1.0, 16.0, 4.0, 3.0, 0.0, 0.0)
    return make_system("cylinder-slab-32", (32.0, 32.0, 32.0), pore, n,
                       precision, (0, seed), 200, z_exclude=(14.0, 18.0))


def slit_large(precision="mixed", seed=0, n=262144, box=128.0) -> System:
    """128^3 box, slit of gap 8 between two slabs 4 thick; 262144 vapour
    atoms anywhere clear of the walls; 10000 steps."""
    pore = Pore("slit", 1.0, 0.5 * box, 4.0, 0.0, 0.0, 8.0)
    return make_system("slit-128", (box, box, box), pore, n, precision,
                       (1, seed), 10000)


def pore_sweep(variant="cylinder", precision="mixed", seed=0, n=4194304,
               box=(256.0, 256.0, 128.0)) -> System:
    """256 x 256 x 128 box, slab 8 thick around z = 64 with a cylindrical
    (r = 6), conical (4 -> 12) or ink-bottle (neck 3, cavity 10) pore;
    4194304 vapour atoms; 2000 steps."""
    r = {"cylinder": (6.0, 0.0), "cone": (4.0, 12.0), "inkbottle": (3.0, 10.0)}
    r0, r1 = r[variant]
    pore = Pore(variant, 1.0, 0.5 * box[2], 8.0, r0, r1, 0.0)
    vid = {"cylinder": 0, "cone": 1, "inkbottle": 2}[variant]
    return make_system("%s-256" % variant, box, pore, n, precision,
                       (2, vid, seed), 2000)


def _pore_for(shape: str, r: float, L: float) -> Pore:
    """Pore of the batched and served workloads: slab 4 thick at mid-height;
    slit gap 2r; cone r -> 3r; ink-bottle neck r, cavity 10r/3; every radius
    clamped to at most L/2 - 2."""
    rmax = 0.5 * L - 2.0
    clamp = lambda q: min(q, rmax)
    if shape == "cylinder":
        return Pore("cylinder", 1.0, 0.5 * L, 4.0, clamp(r))
    if shape == "slit":
        return Pore("slit", 1.0, 0.5 * L, 4.0, 0.0, 0.0, 2.0 * r)
    if shape == "cone":
        return Pore("cone", 1.0, 0.5 * L, 4.0, clamp(r), clamp(3.0 * r))
    return Pore("inkbottle", 1.0, 0.5 * L, 4.0, clamp(r), clamp(10.0 * r / 3.0))


def replica_specs(count=256, n_lo=1000, n_hi=64000, seed=0):
    """Descriptions (n, shape, r, L) of the batched replicas: n log-uniform in
    [n_lo, n_hi], shape uniform over {cylinder, slit, cone}, r uniform in
    [2, 8], L = round((n / 0.1)^(1/3))."""
    rng = np.random.default_rng(np.random.SeedSequence(list(SEED_ROOT) + [3, seed, 999]))
    shapes = ("cylinder", "slit", "cone")
    out = []
    for k in range(count):
        n = int(round(math.exp(rng.uniform(math.log(n_lo), math.log(n_hi)))))
        shape = shapes[int(rng.integers(0, 3))]
        r = float(rng.uniform(2.0, 8.0))
        L = float(round((n / RHO_SMALL) ** (1.0 / 3.0)))
        out.append(dict(index=k, n=n, shape=shape, r=r, L=L))
    return out


def replica(spec, precision="mixed", steps=5000, seed=0) -> System:
    L = spec["L"]
    pore = _pore_for(spec["shape"], spec["r"], L)
    return make_system("replica-%d" % spec["index"], (L, L, L), pore, spec["n"],
                       precision, (3, seed, spec["index"]), steps, meta=dict(spec))


def request_trace(count=256, rate=200.0, n_lo=2000, n_hi=500000, steps_lo=1000,
                  steps_hi=20000, seed=0):
    """Served requests: Poisson arrivals at `rate` per second; n log-uniform
    in [n_lo, n_hi]; shape uniform over {cylinder, slit, cone, inkbottle};
    r uniform in [2, 8]; steps uniform in [steps_lo, steps_hi]; precision
    mixed or fp64 with probability 1/2 each."""
    rng = np.random.default_rng(np.random.SeedSequence(list(SEED_ROOT) + [4, seed, 999]))
    shapes = ("cylinder", "slit", "cone", "inkbottle")
    t = 0.0
    out = []
    for k in range(count):
        t += float(rng.exponential(1.0 / rate))
        n = int(round(math.exp(rng.uniform(math.log(n_lo), math.log(n_hi)))))
        shape = shapes[int(rng.integers(0, 4))]
        r = float(rng.uniform(2.0, 8.0))
        steps = int(rng.integers(steps_lo, steps_hi + 1))
        prec = "mixed" if rng.random() < 0.5 else "fp64"
        L = float(round((n / RHO_SMALL) ** (1.0 / 3.0)))
        out.append(dict(index=k, arrival=t, n=n, shape=shape, r=r, L=L,
                        steps=steps, precision=prec))
    return out


def request_system(spec, seed=0) -> System:
    L = spec["L"]
    pore = _pore_for(spec["shape"], spec["r"], L)
    return make_system("request-%d" % spec["index"], (L, L, L), pore, spec["n"],
                       spec["precision"], (4, seed, spec["index"]), spec["steps"],
                       meta=dict(spec))


# ---------------------------------------------------------------------------
# The paper's pore model (Secs. 4-5), in reduced units of its own molecule
# ---------------------------------------------------------------------------

# The paper's Lennard-Jones parameters for water (Sec. 2): sigma = 3.17 A,
# epsilon = 6.74e-3 eV; molecular mass 18.015 u.  Reduced units follow:
# tau = sigma sqrt(m / epsilon) = 1.66846 ps, epsilon / k_B = 78.21 K.
PAPER_SIGMA_NM = 0.317
PAPER_TAU_PS = 1.66846
PAPER_EPS_K = 78.21


def paper_model_geometry(dim: int):
    """(lx, ly, lz, k, T*, dt) of the paper's models in reduced units: the
    2D pore 1 um x 1 um with k = 3 at 35 C (Sec. 4), the 3D prism
    500 x 50 x 50 nm with an outer prism of 9 pore volumes (k = 1) at 25 C
    (Sec. 5); dt = 0.016 ps in both."""
    dt = 0.016 / PAPER_TAU_PS
    if dim == 2:
        l = 1000.0 / PAPER_SIGMA_NM
        return l, l, 0.0, 3.0, 308.15 / PAPER_EPS_K, dt
    return 500.0 / PAPER_SIGMA_NM, 50.0 / PAPER_SIGMA_NM, 50.0 / PAPER_SIGMA_NM, 1.0, \
        298.15 / PAPER_EPS_K, dt


def pore_model_state(dim, lx, ly, lz, k, n_pore, n_outer, temperature, seed=0,
                     dmin=0.9, key=5):
    """Positions [n][dim]: n_pore molecules uniform in the pore, then n_outer
    uniform in the outer space, redrawn until no two are closer than dmin
    (plain distance); velocities Gaussian with variance T/m per component,
    rescaled so that 2 KE / (dim n) = T exactly (the walls break momentum
    conservation, so the mean is not removed)."""
    from scipy.spatial import cKDTree

    rng_x, rng_v = _streams(key, dim, n_pore, seed)
    lo_p = np.array([0.0, 0.0, 0.0])[:dim]
    hi_p = np.array([lx, ly, lz])[:dim]
    lo_o = np.array([lx, -k * ly, -k * lz])[:dim]
    hi_o = np.array([(k + 1) * lx, (k + 1) * ly, (k + 1) * lz])[:dim]
    n = n_pore + n_outer
    lo = np.concatenate([np.tile(lo_p, (n_pore, 1)), np.tile(lo_o, (n_outer, 1))]).reshape(n, dim)
    hi = np.concatenate([np.tile(hi_p, (n_pore, 1)), np.tile(hi_o, (n_outer, 1))]).reshape(n, dim)
    x = lo + rng_x.random((n, dim)) * (hi - lo)
    for _ in range(1000):
        bad = sorted({j for _, j in cKDTree(x).query_pairs(dmin)})
        if not bad:
            break
        x[bad] = lo[bad] + rng_x.random((len(bad), dim)) * (hi[bad] - lo[bad])
    else:
        raise RuntimeError("placement failed")
    v = rng_v.standard_normal((n, dim)) * math.sqrt(temperature)
    if n:
        v *= math.sqrt(temperature * dim * n / float(np.sum(v * v)))
    return x, v


def paper_model_system(dim: int, n_pore: int, seed=0):
    """The paper's workload at one pore population: n_pore molecules in the
    pore and, at a fifth of the pore's density, k (2k+1)^(dim-1) n_pore / 5
    in the outer space (1764 for 420 in 2D, 1800 for 1000 in 3D).  Returns
    (x, v, dict of the model's geometry and state)."""
    lx, ly, lz, k, T, dt = paper_model_geometry(dim)
    n_outer = int(round(k * (2 * k + 1) ** (dim - 1) * n_pore / 5.0))
    x, v = pore_model_state(dim, lx, ly, lz, k, n_pore, n_outer, T, seed)
    return x, v, dict(dim=dim, lx=lx, ly=ly, lz=lz, k=k, temperature=T, dt=dt,
                      n_pore=n_pore, n_outer=n_outer)
