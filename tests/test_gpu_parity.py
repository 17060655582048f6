"""GPU parity: the HIP path through the C interface against the FP64 oracle.

Tolerances (stated per result): relative force error ||F - F_ref|| / ||F_ref||
<= 1e-12 in FP64 mode and <= 1e-5 in mixed mode at identical positions, and
the per-atom error max_i |dF_i| / rms |F| <= 1e-11 (FP64) and 1e-4 (mixed)
(tests/forcecheck.py); 10-step trajectories agree to 1e-10 (FP64) and 1e-5
(mixed) in position; integer work (wall lattice, cell binning, in-cutoff
pair sets) bit-exact.  The reference side (walls included) comes from the
oracle alone.
"""
import numpy as np
import pytest

import oracle
from paper_1812_07993_amd import poremd, synth
from forcecheck import TOL_F, check_forces

pytestmark = pytest.mark.gpu

TOL_X = {"fp64": 1e-10, "mixed": 1e-5}


def opore_of(p: synth.Pore):
    return oracle.make_pore(p.kind, p.lattice_a, p.slab_center_z, p.slab_thickness, p.r0, p.r1,
                            p.slit_gap)


def small(n, L, pore, seed, dmin=0.9, box=None):
    """Seeded input (placement and velocities from the input generator) and
    the oracle's own wall lattice for the reference side."""
    box = box or (L, L, L)
    rng = np.random.default_rng(seed)
    x = synth.rsa_place(rng, box, n, synth.wall_sites(pore, box), dmin)
    v = synth.maxwell(rng, n, 1.2)
    walls = oracle.wall_lattice(opore_of(pore), box)
    return x, v, walls


def rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def mi(d, L):
    L = np.broadcast_to(np.asarray(L, dtype=np.float64), (3,))
    return d - L * np.rint(d / L)


def make(x, v, box, pore, prec, **tune):
    params = poremd.make_params(box, prec)
    cp = poremd.make_pore(pore.kind, pore.lattice_a, pore.slab_center_z, pore.slab_thickness,
                          pore.r0, pore.r1, pore.slit_gap)
    t = poremd.make_tuning(**tune) if tune else None
    return poremd.System(params, cp, x, v, tuning=t)


PORES = [
    ("cylinder", synth.Pore("cylinder", 1.0, 8.0, 4.0, 2.5)),
    ("slit", synth.Pore("slit", 1.0, 8.0, 2.0, slit_gap=4.0)),
    ("cone", synth.Pore("cone", 1.0, 8.0, 4.0, 1.5, 4.5)),
    ("inkbottle", synth.Pore("inkbottle", 1.0, 8.0, 4.0, 1.5, 4.0)),
    ("slab", synth.Pore("slab", 1.0, 8.0, 2.0)),
    ("none", synth.Pore("none")),
]


@pytest.mark.parametrize("name,pore", PORES)
def test_wall_lattice_bit_exact(name, pore):
    L = 16.0
    x, v, _ = small(300, L, pore, 1)
    s = make(x, v, L, pore, "mixed")
    w = s.walls()
    ref = oracle.wall_lattice(opore_of(pore), (L, L, L))
    assert w.shape == ref.shape
    assert np.array_equal(w, ref)


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
@pytest.mark.parametrize("n", [1, 37, 256, 300, 1000])
@pytest.mark.parametrize("name,pore", PORES[:3] + PORES[5:])
def test_forces_energies_at_create(prec, n, name, pore):
    L = 16.0
    x, v, walls = small(n, L, pore, 100 + n)
    s = make(x, v, L, pore, prec)
    F = s.forces()
    op = oracle.make_params(L)
    F_ref, evv, evw = oracle.forces(x, walls, op)
    if np.linalg.norm(F_ref) > 0:
        check_forces(F, F_ref, prec, what="create %s n=%d" % (name, n))
    else:
        assert np.abs(F).max() == 0.0
    e = s.energies()
    assert e["step"] == 0
    assert e["pe_vv"] == pytest.approx(evv, rel=TOL_F[prec] * 10, abs=1e-12)
    assert e["pe_vw"] == pytest.approx(evw, rel=TOL_F[prec] * 10, abs=1e-12)
    assert e["ke"] == pytest.approx(0.5 * np.sum(v * v), rel=1e-13)


@pytest.mark.parametrize("block", [64, 128, 256, 320, 512, 1024])
@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_trajectory_10_steps(prec, block):
    """Ten velocity-Verlet steps from the same start; also crosses a rebuild
    (rebin_every = 4) inside the run."""
    L = 16.0
    pore = PORES[0][1]
    x, v, walls = small(700, L, pore, 7)
    s = make(x, v, L, pore, prec, block=block, rebin_every=4)
    s.step(10)
    X = s.positions()
    V = s.velocities()
    F = s.forces()
    op = oracle.make_params(L)
    xr, vr, ar, E = oracle.run(x, v, walls, op, 10)
    assert np.abs(mi(X - xr, L)).max() <= TOL_X[prec]
    assert np.abs(V - vr).max() <= TOL_X[prec] * 10
    # forces after 10 steps: the trajectories differ by grown rounding
    check_forces(F, ar, prec, factor=1e3, what="after 10 steps")
    # ... and at the GPU's own positions they are exact to the gates
    Fx, _, _ = oracle.forces(X, walls, op)
    check_forces(F, Fx, prec, what="at step 10, block %d" % block)
    assert np.all((X >= 0) & (X < L))
    e = s.energies()
    assert e["step"] == 10
    tot = E[-1].sum()
    assert e["etotal"] == pytest.approx(tot, rel=1e-9 if prec == "fp64" else 1e-6)


def test_steps_split_across_calls_match_one_call():
    L = 16.0
    pore = PORES[1][1]
    x, v, _ = small(500, L, pore, 9)
    a = make(x, v, L, pore, "fp64", rebin_every=5)
    b = make(x, v, L, pore, "fp64", rebin_every=5)
    a.step(12)
    b.step(5)
    b.step(7)
    # same positions up to rounding (the rebuild schedule restarts per call)
    assert np.abs(mi(a.positions() - b.positions(), L)).max() < 1e-11


def test_cells_bit_exact_vs_counting_sort():
    L = 16.0
    pore = PORES[0][1]
    x, v, _ = small(900, L, pore, 3)
    s = make(x, v, L, pore, "fp64")
    cell, start, perm, nc, inv = poremd.pmd_debug_cells(s.h)
    assert np.array_equal(inv, nc / L)
    rc, rs, rp = oracle.cell_sort(x, inv, nc)
    assert np.array_equal(cell, rc)
    # storage groups cells brick by brick; inside every cell the atoms must
    # be exactly the counting sort's, in ascending caller order
    assert start[-1] == len(x)
    assert sorted(perm.tolist()) == list(range(len(x)))
    for c in range(int(np.prod(nc))):
        k = rs[c + 1] - rs[c]
        assert np.array_equal(perm[start[c]:start[c] + k], rp[rs[c]:rs[c + 1]])


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_pair_sets_bit_exact(prec):
    L = 13.0
    pore = PORES[3][1]
    box = (L, L, L)
    pore = synth.Pore("inkbottle", 1.0, 6.5, 4.0, 1.5, 4.0)
    x, v, walls = small(400, L, pore, 21)
    s = make(x, v, L, pore, prec, rebin_every=3)
    for nsteps in (0, 7):
        if nsteps:
            s.step(nsteps)
        X = s.positions()
        vv, vw = poremd.pmd_debug_pairs(s.h)
        rvv, rvw = oracle.pairs(X, walls, box, 2.5)
        assert np.array_equal(vv, rvv)
        assert np.array_equal(vw, rvw)
        assert len(rvv) > 100 and len(rvw) > 10


def test_single_atom_ballistic():
    L = 16.0
    pore = synth.Pore("none")
    x = np.array([[15.5, 0.25, 8.0]])
    v = np.array([[1.0, -0.5, 0.25]])
    params = poremd.make_params(L, "fp64", dt=1.0 / 256.0)
    s = poremd.System(params, poremd.make_pore("none"), x, v)
    s.step(300)
    X = s.positions()
    assert np.array_equal(X, np.mod(x + v * 300 / 256.0, L))
    assert np.array_equal(s.velocities(), v)


def test_momentum_conserved_without_walls():
    L = 14.0
    pore = synth.Pore("none")
    x, v, _ = small(600, L, pore, 5)
    s = make(x, v, L, pore, "mixed")
    s.step(200)
    assert np.abs(s.velocities().sum(axis=0) - v.sum(axis=0)).max() < 1e-10


def test_reversibility_fp64():
    L = 16.0
    pore = PORES[0][1]
    x, v, _ = small(500, L, pore, 13)
    s = make(x, v, L, pore, "fp64")
    s.step(100)
    X1, V1 = s.positions(), s.velocities()
    t = make(X1, -V1, L, pore, "fp64")
    t.step(100)
    assert np.abs(mi(t.positions() - x, L)).max() < 1e-8


def test_invalid_inputs_rejected():
    L = 16.0
    pore = poremd.make_pore("none")
    p = poremd.make_params(L, "fp64")
    x = np.array([[1.0, 2.0, 3.0], [np.nan, 1.0, 1.0]])
    v = np.zeros((2, 3))
    with pytest.raises(poremd.PmdError) as e:
        poremd.System(p, pore, x, v)
    assert e.value.code == poremd.PMD_EINVAL
    with pytest.raises(poremd.PmdError):
        poremd.System(p, pore, np.array([[1.0, 2.0, 16.0]]), np.zeros((1, 3)))
    small_box = poremd.make_params(7.0, "fp64")
    with pytest.raises(poremd.PmdError):
        poremd.System(small_box, pore, np.array([[1.0, 2.0, 3.0]]), np.zeros((1, 3)))


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_pairs_at_the_cutoff(prec):
    """A simple cubic lattice of spacing r_c, each site moved by at most 2e-6:
    every atom has six partners within the band around the cutoff where the
    mixed path leaves the decision to FP64 (more than the two entries the
    pair loops record, so the pass rescans the list), each on either side
    of r_c at random (the closest lies 4e-9 from r_c^2, far beyond FP64
    rounding).  Forces against the oracle's all-pairs sums."""
    rc, m = 2.5, 10
    L = rc * m
    g = (np.arange(m) + 0.5) * rc
    x = np.stack(np.meshgrid(g, g, g, indexing="ij"), axis=-1).reshape(-1, 3)
    rng = np.random.default_rng(21)
    x = x + rng.uniform(-2e-6, 2e-6, size=x.shape)
    v = np.zeros_like(x)
    s = make(x, v, L, synth.Pore("none"), prec)
    p = oracle.make_params(L)
    Fr, _, _ = oracle.forces(x, None, p)
    d = x[:, None, :] - x[None, :, :]
    d -= L * np.rint(d / L)
    r2 = (d * d).sum(-1)
    inside = (r2 < rc * rc) & (r2 > 0)
    assert 0 < inside.sum() < 6 * len(x)  # both sides of r_c occur
    check_forces(s.forces(), Fr, prec, what="cutoff-band lattice")
    s.close()
