"""GPU tests of the Berendsen thermostat (F4) through the C interface,
against the FP64 oracle's F2, F1, F3, F4 step.

Tolerances: the free gas (no pair forces) follows the closed-form geometric
relaxation of the temperature to 1e-12 relative in both precisions (its
velocities change only by the FP64 scaling); an interacting system with
walls matches the oracle's trajectory over 20 steps to 1e-10 (FP64) and
1e-5 (mixed) in position, and its recorded kinetic energies to 1e-10 and
1e-5 relative.
"""
import numpy as np
import pytest

import oracle
from paper_1812_07993_amd import poremd, synth

pytestmark = pytest.mark.gpu

TOL_X = {"fp64": 1e-10, "mixed": 1e-5}


def mi(d, L):
    return d - L * np.rint(d / L)


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_free_gas_relaxes_geometrically(prec):
    """epsilon = 0: T_n = t0 + (T_0 - t0)(1 - dt/tau)^(n - 1) at step n >= 1
    (measured before that step's scaling), as the oracle's pin states."""
    L, n = 20.0, 300
    rng = np.random.default_rng(4)
    x = rng.uniform(0.0, L, size=(n, 3))
    v = rng.normal(0.0, 1.0, size=(n, 3))
    v -= v.mean(axis=0)
    tau, t0, steps = 0.1, 2.0, 60
    params = poremd.make_params(L, prec, epsilon=0.0, thermostat_tau=tau, thermostat_t0=t0)
    s = poremd.System(params, poremd.make_pore("none"), x, v,
                      tuning=poremd.make_tuning(energy_every=1, rebin_every=7))
    s.step(steps)
    E = s.energy_history()
    dof = 3 * n - 3
    T0 = np.sum(v * v) / dof
    k = np.maximum(np.asarray(E["step"]) - 1, 0)
    want = t0 + (T0 - t0) * (1.0 - 0.005 / tau) ** k
    assert len(E) == steps + 1
    assert np.allclose(E["temperature"], want, rtol=1e-12, atol=0.0)
    s.close()


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_thermostat_trajectory_matches_the_oracle(prec):
    """A vapour with a cylindrical pore heated from T = 1.2 towards t0 = 2
    with tau = 0.05 (ten steps): 20 steps that cross rebuilds
    (rebin_every = 4), against the oracle."""
    L = 16.0
    pore = synth.Pore("cylinder", 1.0, 8.0, 4.0, 2.5)
    walls = synth.wall_sites(pore, (L, L, L))
    rng = np.random.default_rng(13)
    x = synth.rsa_place(rng, (L, L, L), 700, walls, 0.9)
    v = synth.maxwell(rng, 700, 1.2)
    tau, t0, steps = 0.05, 2.0, 20
    params = poremd.make_params(L, prec, thermostat_tau=tau, thermostat_t0=t0)
    cp = poremd.make_pore(pore.kind, pore.lattice_a, pore.slab_center_z, pore.slab_thickness,
                          pore.r0, pore.r1, pore.slit_gap)
    s = poremd.System(params, cp, x, v, tuning=poremd.make_tuning(energy_every=1, rebin_every=4))
    s.step(steps)
    X, V = s.positions(), s.velocities()
    E = s.energy_history()
    xr, vr, _, Er = oracle.run(x, v, walls, oracle.make_params(L), steps, every=1, tau=tau, t0=t0)
    assert np.abs(mi(X - xr, L)).max() <= TOL_X[prec]
    assert np.abs(V - vr).max() <= TOL_X[prec] * 10
    ke = np.asarray(E["ke"])
    assert np.allclose(ke, Er[:, 0], rtol=TOL_X[prec], atol=0.0)
    # the run did heat up
    assert E["temperature"][-1] > 1.4
    s.close()


def test_rejects_a_rise_time_below_dt():
    params = poremd.make_params(16.0, "fp64", thermostat_tau=0.001, thermostat_t0=1.0)
    x = np.array([[1.0, 1.0, 1.0], [5.0, 5.0, 5.0]])
    with pytest.raises(poremd.PmdError):
        poremd.System(params, poremd.make_pore("none"), x, np.zeros_like(x))
