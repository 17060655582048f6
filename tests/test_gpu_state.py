"""GPU tests of checkpoint/restart (pmd_set_state) and of the autotuner.

A restart loads the positions and velocities read back at step s and
recomputes the forces there, so the continued trajectory matches the
uninterrupted one to rounding only: the gate is the 10-step trajectory
tolerance of the parity tests (1e-10 FP64, 1e-5 mixed, in sigma).  Forces
right after a restart are checked against the oracle at the same tolerance
as at creation.
"""
import numpy as np
import pytest

import oracle
from paper_1812_07993_amd import poremd, synth

pytestmark = pytest.mark.gpu

TOL_X = {"fp64": 1e-10, "mixed": 1e-5}
TOL_F = {"fp64": 1e-12, "mixed": 1e-5}


def _desc():
    return synth.replica(dict(index=0, n=1200, shape="cone", r=2.0, L=24.0), precision="fp64",
                         steps=0, seed=5)


def _oracle_walls(desc):
    q = desc.pore
    return oracle.wall_lattice(oracle.make_pore(q.kind, q.lattice_a, q.slab_center_z,
                                                q.slab_thickness, q.r0, q.r1, q.slit_gap),
                               desc.params.box)


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_restart_continues_the_trajectory(prec):
    desc = _desc()
    tun = poremd.make_tuning(rebin_every=6)
    a = poremd.System.from_desc(desc, precision=prec, tuning=tun)
    a.step(25)
    x25, v25, s25 = a.positions(), a.velocities(), a.step_count()
    assert s25 == 25
    a.step(10)
    xa, va = a.positions(), a.velocities()
    ea = a.energies()

    b = poremd.System.from_desc(desc, precision=prec, tuning=tun)
    b.step(3)
    b.set_state(x25, v25, s25)
    assert b.step_count() == 25
    hist = b.energy_history()
    assert len(hist) == 1 and hist["step"][0] == 25
    # forces at the restart point against the oracle
    p = oracle.make_params(desc.params.box)
    Fr, _, _ = oracle.forces(x25, _oracle_walls(desc), p)
    F = b.forces()
    assert np.linalg.norm(F - Fr) / np.linalg.norm(Fr) <= TOL_F[prec]
    b.step(10)
    assert b.step_count() == 35
    d = b.positions() - xa
    d -= np.asarray(desc.params.box) * np.rint(d / np.asarray(desc.params.box))
    assert np.abs(d).max() <= TOL_X[prec]
    assert np.abs(b.velocities() - va).max() <= 10 * TOL_X[prec]
    assert b.energies()["step"] == ea["step"] == 35
    a.close()
    b.close()


def test_restart_rejects_bad_input():
    desc = _desc()
    s = poremd.System.from_desc(desc)
    x, v = s.positions(), s.velocities()
    with pytest.raises(poremd.PmdError) as e:
        s.set_state(x[:-1], v[:-1], 0)
    assert e.value.code == poremd.PMD_EINVAL
    bad = x.copy()
    bad[3, 1] = np.nan
    with pytest.raises(poremd.PmdError):
        s.set_state(bad, v, 0)
    with pytest.raises(poremd.PmdError):
        s.set_state(x, v, -1)
    # the system is still usable and unchanged by the rejected calls
    s.step(2)
    assert s.step_count() == 2
    s.close()


def test_autotune_picks_a_runnable_candidate():
    desc = _desc()
    params, pore = poremd.params_of(desc, "mixed")
    cands = [poremd.make_tuning(skin=sk, rebin_every=r) for sk, r in
             [(0.3, 4), (0.5, 10), (0.8, 15), (6.0, 10)]]
    best, us = poremd.pmd_autotune(params, pore, desc.x, desc.v, cands, trial_steps=40)
    # skin 6 leaves fewer than 3 cells per axis of a 24-sigma box: not runnable
    assert np.isinf(us[3])
    assert np.all(np.isfinite(us[:3])) and np.all(us[:3] > 0)
    # the fastest, or the largest skin within 2% of it
    ok = np.flatnonzero(us <= 1.02 * us.min())
    assert best in ok
    assert cands[best].skin == max(cands[i].skin for i in ok)
    # the caller's arrays are untouched and a system made with the winner runs
    s = poremd.System.from_desc(desc, precision="mixed", tuning=cands[best])
    s.step(20)
    assert s.step_count() == 20
    s.close()


def test_kernel_timing_mode():
    """Timing mode times whole replays of R back-to-back step launches and
    leaves the trajectory unchanged (same kernels, no graph)."""
    desc = _desc()
    tun = poremd.make_tuning(rebin_every=5, skin=0.8)
    a = poremd.System.from_desc(desc, tuning=tun)
    b = poremd.System.from_desc(desc, tuning=tun)
    poremd.pmd_timing_enable(a.h, True)
    a.step(20)
    b.step(20)
    n, ms = poremd.pmd_kernel_time(a.h)
    t = poremd.pmd_kernel_times(a.h)
    assert 0 < len(t) <= n <= 20 and np.all(t > 0)
    assert ms > 0 and t.min() * (1 - 1e-9) <= ms <= t.max() * (1 + 1e-9)
    poremd.pmd_timing_enable(a.h, False)
    assert poremd.pmd_kernel_time(a.h) == (0, 0.0)
    assert a.step_count() == b.step_count() == 20
    assert np.array_equal(a.positions(), b.positions())
    a.close()
    b.close()
