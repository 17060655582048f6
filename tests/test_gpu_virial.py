"""GPU parity of the virial sums of the pressure formula (Sec. 2) against
the FP64 oracle at the same positions: at creation and after 30 steps that
cross rebuilds.  Tolerance: relative 1e-10 (FP64) and 1e-4 (mixed).  The
mixed bound is looser than the force bound because r . f = w r^2 with
w = r^-8 (12 A r^-6 - 6 B) cancels near the LJ minimum, where adsorbed
atoms sit next to the wall lattice: an FP32 pair term there carries an
absolute error of about 1e-6, and a few hundred of them sum to a few 1e-4
on a wall virial of about -17."""
import numpy as np
import pytest

import oracle
from paper_1812_07993_amd import poremd, synth

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-10, "mixed": 1e-4}


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
@pytest.mark.parametrize("shape", ["cylinder", "slit"])
def test_virial_sums_match_the_oracle(prec, shape):
    L = 16.0
    pore = (synth.Pore("cylinder", 1.0, 8.0, 4.0, 2.5) if shape == "cylinder"
            else synth.Pore("slit", 1.0, 8.0, 2.0, slit_gap=4.0))
    walls = synth.wall_sites(pore, (L, L, L))
    rng = np.random.default_rng(17)
    x = synth.rsa_place(rng, (L, L, L), 900, walls, 0.9)
    v = synth.maxwell(rng, 900, 1.2)
    params = poremd.make_params(L, prec)
    cp = poremd.make_pore(pore.kind, pore.lattice_a, pore.slab_center_z, pore.slab_thickness,
                          pore.r0, pore.r1, pore.slit_gap)
    s = poremd.System(params, cp, x, v,
                      tuning=poremd.make_tuning(energy_every=10, rebin_every=4, virial=1))
    op = oracle.make_params(L)
    e0 = s.energies()
    wvv, wvw = oracle.virial(x, walls, op)
    assert e0["virial_vv"] == pytest.approx(wvv, rel=TOL[prec])
    assert e0["virial_vw"] == pytest.approx(wvw, rel=TOL[prec])
    s.step(30)
    X = s.positions()
    e1 = s.energies()
    assert e1["step"] == 30
    wvv, wvw = oracle.virial(X, walls, op)
    assert e1["virial_vv"] == pytest.approx(wvv, rel=TOL[prec])
    assert e1["virial_vw"] == pytest.approx(wvw, rel=TOL[prec])
    # the pressure the paper's formula gives, over the box volume here
    P = (2.0 * e1["ke"] + e1["virial_vv"]) / (3.0 * L ** 3)
    assert np.isfinite(P)
    # switched off by a retune: the sums read 0 and the trajectory goes on
    s.set_tuning(poremd.make_tuning(energy_every=10, rebin_every=4))
    s.step(10)
    e2 = s.energies()
    assert e2["step"] == 40 and e2["virial_vv"] == 0.0 and e2["virial_vw"] == 0.0
    s.close()


def test_virial_sums_are_off_by_default():
    L = 12.0
    rng = np.random.default_rng(5)
    x = synth.rsa_place(rng, (L, L, L), 300, np.zeros((0, 3)), 0.9)
    s = poremd.System(poremd.make_params(L, "mixed"), poremd.make_pore("none"), x,
                      np.zeros_like(x), tuning=poremd.make_tuning(energy_every=5))
    s.step(10)
    e = s.energies()
    assert e["virial_vv"] == 0.0 and e["virial_vw"] == 0.0 and e["pe_vv"] < 0.0
    s.close()


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
@pytest.mark.parametrize("shape", ["cylinder", "cone", "inkbottle", "slit", "none"])
def test_pressure_in_the_pore_matches_the_oracle(prec, shape):
    """The pressure in the pore (Sec. 2's formula with V the pore's void
    volume, over the molecules inside the void) at creation and after 30
    steps: molecule count exact, kinetic energy to 1e-12, virial share to the
    virial tolerance, volume to rounding."""
    L = 16.0
    pore = {"cylinder": synth.Pore("cylinder", 1.0, 8.0, 4.0, 3.5),
            "cone": synth.Pore("cone", 1.0, 8.0, 4.0, 2.0, 5.0),
            "inkbottle": synth.Pore("inkbottle", 1.0, 8.0, 4.0, 2.0, 5.0),
            "slit": synth.Pore("slit", 1.0, 8.0, 2.0, slit_gap=4.0),
            "none": synth.Pore("none")}[shape]
    walls = synth.wall_sites(pore, (L, L, L))
    rng = np.random.default_rng(23)
    x = synth.rsa_place(rng, (L, L, L), 1000, walls, 0.9)
    v = synth.maxwell(rng, 1000, 1.2)
    params = poremd.make_params(L, prec)
    cp = poremd.make_pore(pore.kind, pore.lattice_a, pore.slab_center_z, pore.slab_thickness,
                          pore.r0, pore.r1, pore.slit_gap)
    op = oracle.make_params(L)
    oq = oracle.make_pore(pore.kind, pore.lattice_a, pore.slab_center_z, pore.slab_thickness,
                          pore.r0, pore.r1, pore.slit_gap)
    V = poremd.pmd_pore_volume(params, cp)
    assert V == pytest.approx(oracle.pore_volume(oq, (L, L, L)), rel=1e-15)
    s = poremd.System(params, cp, x, v,
                      tuning=poremd.make_tuning(energy_every=10, rebin_every=4, virial=1))
    for nsteps in (0, 30):
        if nsteps:
            s.step(nsteps)
        X, Vv, e = s.positions(), s.velocities(), s.energies()
        r = oracle.pore_pressure(X, Vv, op, oq)
        assert e["n_pore"] == r["n_pore"] > 10
        assert e["pore_volume"] == pytest.approx(r["volume"], rel=1e-15)
        assert e["ke_pore"] == pytest.approx(r["ke_pore"], rel=1e-12)
        assert e["virial_pore"] == pytest.approx(r["virial_pore"], rel=TOL[prec], abs=1e-12)
        scale = (2 * r["ke_pore"] + abs(r["virial_pore"])) / (3 * r["volume"])
        assert abs(e["pressure"] - r["pressure"]) <= TOL[prec] * scale
    s.close()
