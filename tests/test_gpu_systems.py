"""GPU tests at the workloads' real shapes, batching and energy conservation.

Tolerances: relative force error <= 1e-5 (mixed) and <= 1e-12 (FP64) at
identical positions; energy drift trend <= 1e-4 over 1000 steps after a
100-step burn-in (the same gate the oracle meets, see its pins); a system
run inside a batch gives the same positions as when run alone (the per-atom
summation order does not depend on the batch, so they agree bit for bit;
the gate is 1e-12).
"""
import numpy as np
import pytest

import oracle
from paper_1812_07993_amd import poremd, synth
from forcecheck import check_forces

pytestmark = pytest.mark.gpu


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def oracle_walls(desc):
    q = desc.pore
    return oracle.wall_lattice(oracle.make_pore(q.kind, q.lattice_a, q.slab_center_z,
                                                q.slab_thickness, q.r0, q.r1, q.slit_gap),
                               desc.params.box)


def energy_drift(tot, burn=100, window=1000):
    seg = np.asarray(tot[burn:burn + window + 1], dtype=np.float64)
    t = np.arange(seg.shape[0], dtype=np.float64)
    slope = np.polyfit(t, seg, 1)[0]
    return abs(slope) * window / abs(seg[0]), float(np.abs(seg - seg[0]).max() / abs(seg[0]))


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_nve_drift_cylinder_slab(prec):
    desc = synth.cylinder_slab_small()
    s = poremd.System.from_desc(desc, precision=prec,
                                tuning=poremd.make_tuning(energy_every=1))
    s.step(1100)
    E = s.energy_history()
    assert E["step"][0] == 0 and E["step"][-1] == 1100 and len(E) == 1101
    trend, maxdev = energy_drift(E["etotal"])
    assert trend <= 1e-4, trend
    assert maxdev <= 2e-4, maxdev
    assert np.isclose(E["ke"][0], 0.5 * (3 * desc.n - 3) * 1.2, rtol=1e-12)


# (skin, rebuild period, block, atoms per brick): the library default and
# the shapes the benchmark's tuning chose for this workload (256-thread
# bricks of 4 x 4 x 4 cells in mixed precision, 512-thread ones in FP64)
SLIT_TUNINGS = [None, (0.7, 10, 256, 270), (0.7, 10, 512, 460)]


@pytest.mark.parametrize("tune", SLIT_TUNINGS)
@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_slit_128_sampled_forces(prec, tune):
    """262144 vapour + 131072 wall atoms: forces of 2048 sampled atoms against
    the oracle's all-pairs sums, at creation and after 60 steps, with the
    default tuning and with the benchmark's launch configurations."""
    desc = synth.slit_large()
    t = None
    if tune is not None:
        t = poremd.make_tuning(skin=tune[0], rebin_every=tune[1], block=tune[2], brick_atoms=tune[3])
    s = poremd.System.from_desc(desc, precision=prec, tuning=t)
    walls = oracle_walls(desc)
    assert s.n_wall == walls.shape[0] == 131072
    p = oracle.make_params(desc.params.box)
    rng = np.random.default_rng(7)
    sel = np.sort(rng.choice(desc.n, 2048, replace=False))
    F = s.forces()
    Fr, _ = oracle.forces_subset(desc.x, walls, p, sel)
    check_forces(F[sel], Fr, prec, what="slit 128^3 at creation")
    s.step(60)
    X = s.positions()
    F = s.forces()
    Fr, _ = oracle.forces_subset(X, walls, p, sel)
    check_forces(F[sel], Fr, prec, what="slit 128^3 after 60 steps")
    s.close()


_SWEEP = {}


def _sweep_desc(variant):
    # one placement of 4194304 atoms per pore variant, shared by both precisions
    if variant not in _SWEEP:
        _SWEEP.clear()
        _SWEEP[variant] = synth.pore_sweep(variant)
    return _SWEEP[variant]


@pytest.mark.parametrize("variant,n_wall,prec",
                         [(v, nw, p) for v, nw in (("cylinder", 523392), ("cone", 522612),
                                                   ("inkbottle", 522896))
                          for p in ("mixed", "fp64")])
def test_pore_sweep_4m_sampled_forces(variant, n_wall, prec):
    """4194304 vapour atoms in a 256 x 256 x 128 box with an 8-thick slab and
    each of the three pores, in both precisions, at the benchmark's launch
    configuration: the wall count derived by hand, and the forces of 256
    sampled atoms (half of them drawn from the atoms within 3 sigma of a wall
    site) against the oracle's all-pairs sums, at creation and after 20
    steps, at the GPU's positions."""
    desc = _sweep_desc(variant)
    # the launch configuration the benchmark's tuning chose for this workload
    t = poremd.make_tuning(skin=0.4, rebin_every=6, block=512, brick_atoms=460)
    s = poremd.System.from_desc(desc, precision=prec, tuning=t)
    assert s.n_wall == n_wall
    walls = oracle_walls(desc)
    assert walls.shape[0] == n_wall
    p = oracle.make_params(desc.params.box)
    rng = np.random.default_rng(3)
    z = desc.x[:, 2]
    zc, half = desc.pore.slab_center_z, 0.5 * desc.pore.slab_thickness
    near = np.flatnonzero(np.abs(z - zc) < half + 3.0)
    sel = np.unique(np.concatenate([rng.choice(desc.n, 128, replace=False),
                                    rng.choice(near, 128, replace=False)]))
    F = s.forces()
    Fr, _ = oracle.forces_subset(desc.x, walls, p, sel)
    check_forces(F[sel], Fr, prec, what="%s 4M at creation" % variant)
    s.step(20)
    e = s.energies()
    assert e["step"] == 20 and np.isfinite(e["etotal"])
    X = s.positions()
    assert np.all((X >= 0) & (X < np.asarray(desc.params.box)))
    F = s.forces()
    Fr, _ = oracle.forces_subset(X, walls, p, sel)
    check_forces(F[sel], Fr, prec, what="%s 4M after 20 steps" % variant)
    s.close()


def _small_systems(prec):
    specs = [dict(index=0, n=900, shape="cylinder", r=3.0, L=22.0),
             dict(index=1, n=2500, shape="slit", r=2.5, L=30.0),
             dict(index=2, n=1400, shape="cone", r=2.0, L=25.0),
             dict(index=3, n=600, shape="cylinder", r=5.0, L=22.0)]
    return [synth.replica(sp, precision=prec, steps=0, seed=11) for sp in specs]


@pytest.mark.parametrize("prec", ["mixed", "fp64"])
def test_batch_matches_alone(prec):
    descs = _small_systems(prec)
    steps = [37, 50, 23, 64]
    tun = poremd.make_tuning(rebin_every=7)
    alone = []
    for d, n in zip(descs, steps):
        s = poremd.System.from_desc(d, tuning=tun)
        s.step(n)
        alone.append((s.positions(), s.velocities(), s.energies()))
        s.close()
    b = poremd.pmd_batch_create(0, 8)
    handles = [poremd.System.from_desc(d, tuning=tun) for d in descs]
    slots = [poremd.pmd_batch_admit(b, h.h, n) for h, n in zip(handles, steps)]
    assert sorted(slots) == [0, 1, 2, 3]
    done = set()
    for _ in range(200):
        poremd.pmd_batch_advance(b, 14)
        done |= set(poremd.pmd_batch_poll(b))
        if len(done) == 4:
            break
    assert done == {0, 1, 2, 3}
    for h, sl, (X, V, E), n in zip(handles, slots, alone, steps):
        poremd.pmd_batch_release(b, sl)
        Xb = h.positions()
        assert np.abs(Xb - X).max() <= 1e-12
        assert np.abs(h.velocities() - V).max() <= 1e-12
        e = h.energies()
        assert e["step"] == n
        assert e["etotal"] == pytest.approx(E["etotal"], rel=1e-12)
        h.close()
    poremd.pmd_batch_destroy(b)


def test_batch_admission_by_budget():
    descs = _small_systems("mixed")
    need = [poremd.pmd_footprint_bytes(*poremd.params_of(d), d.n) for d in descs]
    b = poremd.pmd_batch_create(need[0] + need[3] + need[3] // 2, 8)
    h0 = poremd.System.from_desc(descs[0])
    h1 = poremd.System.from_desc(descs[1])
    h3 = poremd.System.from_desc(descs[3])
    assert poremd.pmd_batch_admit(b, h0.h, 10) is not None
    assert poremd.pmd_batch_admit(b, h1.h, 10) is None  # over budget: EAGAIN
    assert poremd.pmd_batch_admit(b, h3.h, 10) is not None
    resident, used, budget = poremd.pmd_batch_info(b)
    assert resident == 2 and used <= budget
    for _ in range(20):
        poremd.pmd_batch_advance(b, 7)
        if len(poremd.pmd_batch_poll(b)) == 2:
            break
    poremd.pmd_batch_release(b, 0)
    resident2, used2, _ = poremd.pmd_batch_info(b)
    assert resident2 == 1 and used2 < used
    poremd.pmd_batch_destroy(b)
    for h in (h0, h1, h3):
        h.close()


@pytest.mark.parametrize("prec", ["mixed", "fp64"])
def test_runs_are_reproducible(prec):
    """The same inputs give bit-identical trajectories: no floating-point
    atomics, fixed summation orders, and every workgroup reads the positions
    as of the start of the step (cutoff-edge re-tests read partners' master
    positions while other workgroups write the next ones)."""
    for d in _small_systems(prec):
        runs = []
        for _ in range(2):
            s = poremd.System.from_desc(d, tuning=poremd.make_tuning(rebin_every=9))
            s.step(150)
            runs.append((s.positions(), s.velocities(), s.energies()["etotal"]))
            s.close()
        assert np.array_equal(runs[0][0], runs[1][0])
        assert np.array_equal(runs[0][1], runs[1][1])
        assert runs[0][2] == runs[1][2]


def test_batch_with_one_system_asking_for_the_virial():
    """A pool runs the virial-summing step kernel when any resident system asks
    for the sums: the other system's trajectory is the same bit for bit as
    when it runs alone on the plain kernel, and its sums read 0; the asking
    system's sums match its own run alone (to 1e-12, the batch gate for
    energies) and the oracle at its positions (1e-10, the FP64 gate)."""
    descs = _small_systems("fp64")[:2]
    steps = [30, 44]
    tuns = [poremd.make_tuning(rebin_every=7, energy_every=1, virial=1),
            poremd.make_tuning(rebin_every=7, energy_every=1)]
    alone = []
    for d, n, t in zip(descs, steps, tuns):
        s = poremd.System.from_desc(d, tuning=t)
        s.step(n)
        alone.append((s.positions(), s.energies()))
        s.close()
    b = poremd.pmd_batch_create(0, 4)
    handles = [poremd.System.from_desc(d, tuning=t) for d, t in zip(descs, tuns)]
    slots = [poremd.pmd_batch_admit(b, h.h, n) for h, n in zip(handles, steps)]
    done = set()
    for _ in range(100):
        poremd.pmd_batch_advance(b, 9)
        done |= set(poremd.pmd_batch_poll(b))
        if len(done) == 2:
            break
    assert done == set(slots)
    for k, (h, sl, (X, E)) in enumerate(zip(handles, slots, alone)):
        poremd.pmd_batch_release(b, sl)
        assert np.array_equal(h.positions(), X)
        e = h.energies()
        if k == 0:
            assert e["virial_vv"] == pytest.approx(E["virial_vv"], rel=1e-12)
            assert e["virial_vw"] == pytest.approx(E["virial_vw"], rel=1e-12, abs=1e-14)
            wvv, wvw = oracle.virial(X, oracle_walls(descs[0]), oracle.make_params(descs[0].params.box))
            assert e["virial_vv"] == pytest.approx(wvv, rel=1e-10)
            assert e["virial_vw"] == pytest.approx(wvw, rel=1e-10, abs=1e-12)
        else:
            assert e["virial_vv"] == 0.0 and e["virial_vw"] == 0.0
        h.close()
    poremd.pmd_batch_destroy(b)


def test_batch_of_16_replicas_matches_alone():
    """16 replicas of the batched workload (vapour N log-uniform in [1k, 64k],
    cylinder, slit or cone pores), each with its own step count: every
    system's positions, velocities and energies after the batch equal its
    run alone bit for bit (the per-atom sums do not depend on the batch)."""
    specs = synth.replica_specs(count=16, seed=5)
    assert max(sp["n"] for sp in specs) > 30000
    descs = [synth.replica(sp, precision="mixed", steps=0, seed=5) for sp in specs]
    steps = [60 + 13 * k for k in range(len(descs))]
    tun = poremd.make_tuning(rebin_every=8)
    alone = []
    for d, n in zip(descs, steps):
        s = poremd.System.from_desc(d, tuning=tun)
        s.step(n)
        alone.append((s.positions(), s.velocities(), s.energies()["etotal"]))
        s.close()
    b = poremd.pmd_batch_create(0, 16)
    handles = [poremd.System.from_desc(d, tuning=tun) for d in descs]
    slots = [poremd.pmd_batch_admit(b, h.h, n) for h, n in zip(handles, steps)]
    done = set()
    for _ in range(100):
        poremd.pmd_batch_advance(b, 40)
        done |= set(poremd.pmd_batch_poll(b))
        if len(done) == len(descs):
            break
    assert done == set(slots)
    for h, sl, (X, V, E) in zip(handles, slots, alone):
        poremd.pmd_batch_release(b, sl)
        assert np.array_equal(h.positions(), X)
        assert np.array_equal(h.velocities(), V)
        assert h.energies()["etotal"] == E
        h.close()
    poremd.pmd_batch_destroy(b)
