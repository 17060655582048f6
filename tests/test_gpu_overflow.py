"""GPU tests of the capacity paths: neighbour lists that outgrow their
capacity, and a dense cluster whose halo outgrows the staged LDS tile.  The
step that finds an overflow is discarded and redone after the buffer grows
(or the bricks shrink), so the results are those of a run that never
overflowed: bit-identical for the list capacity, and within the parity
tolerances against the oracle for the dense cluster."""
import numpy as np
import pytest

import oracle
from paper_1812_07993_amd import poremd, synth

pytestmark = pytest.mark.gpu

TOL_F = {"fp64": 1e-12, "mixed": 1e-5}


@pytest.mark.parametrize("prec", ["mixed", "fp64"])
def test_small_list_capacity_grows(prec):
    d = synth.replica(dict(index=0, n=2000, shape="slit", r=2.5, L=27.0), precision=prec,
                      steps=0, seed=9)
    a = poremd.System.from_desc(d, tuning=poremd.make_tuning(rebin_every=8, list_cap=16))
    b = poremd.System.from_desc(d, tuning=poremd.make_tuning(rebin_every=8))
    assert poremd.pmd_get_tuning(a.h).list_cap > 16
    a.step(40)
    b.step(40)
    assert np.array_equal(a.positions(), b.positions())
    assert np.array_equal(a.velocities(), b.velocities())
    a.close()
    b.close()


def _cluster(n, side, box, seed):
    rng = np.random.default_rng(seed)
    x = synth.rsa_place(rng, (side, side, side), n, np.zeros((0, 3)), 0.9)
    x = x + (box - side) / 2.0
    v = synth.maxwell(rng, n, 1.2)
    return x, v


@pytest.mark.parametrize("prec", ["mixed", "fp64"])
def test_dense_cluster_outgrows_the_tile(prec):
    """2000 atoms packed into a 14-sigma cube inside a 44-sigma box: the mean
    occupancy sizes the tile far below the cluster's halo (the FP64 tile
    cannot hold it at its largest, so the bricks shrink as well)."""
    L = 44.0
    x, v = _cluster(2000, 14.0, L, 4)
    params = poremd.make_params(L, prec)
    s = poremd.System(params, poremd.make_pore("none"), x, v)
    # the initial force evaluation had to be redone after the tile grew
    rebuilds, _ = poremd.pmd_debug_lists(s.h)
    assert rebuilds >= 2
    p = oracle.make_params(L)
    Fr, _, _ = oracle.forces(x, None, p)
    F = s.forces()
    assert np.linalg.norm(F - Fr) / np.linalg.norm(Fr) <= TOL_F[prec]
    s.step(10)
    X = s.positions()
    Fr, _, _ = oracle.forces(X, None, p)
    assert np.linalg.norm(s.forces() - Fr) / np.linalg.norm(Fr) <= TOL_F[prec]
    s.close()


@pytest.mark.parametrize("prec", ["mixed", "fp64"])
def test_lists_overflow_in_the_middle_of_a_run(prec):
    """An imploding gas (velocities toward the box centre) outgrows its
    neighbour lists part-way through one step() call that queued 50
    replays.  The replay whose rebuild overflowed stalls the system, the
    queued replays behind it skip their rebuilds and steps, the host grows
    the lists and the run resumes: the result is bit-identical to a run that
    had room from the start, with one extra rebuild per overflow."""
    L = 30.0
    rng = np.random.default_rng(5)
    x = synth.rsa_place(rng, (L, L, L), 2000, np.zeros((0, 3)), 0.9)
    v = -0.3 * (x - L / 2.0)
    params = poremd.make_params(L, prec)
    a = poremd.System(params, poremd.make_pore("none"), x, v,
                      tuning=poremd.make_tuning(rebin_every=4, list_cap=16))
    b = poremd.System(params, poremd.make_pore("none"), x, v,
                      tuning=poremd.make_tuning(rebin_every=4, list_cap=256))
    cap0 = poremd.pmd_get_tuning(a.h).list_cap
    a.step(200)
    b.step(200)
    assert np.array_equal(a.positions(), b.positions())  # (waits for the run)
    assert np.array_equal(a.velocities(), b.velocities())
    assert poremd.pmd_get_tuning(a.h).list_cap > cap0
    ra, _ = poremd.pmd_debug_lists(a.h)
    rb, _ = poremd.pmd_debug_lists(b.h)
    assert rb < ra <= rb + 4, (ra, rb)
    a.close()
    b.close()
