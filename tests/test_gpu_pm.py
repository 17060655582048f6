"""GPU parity of the paper's pore model (all-pairs forces, reflecting pore
walls, periodic outer space, 2D and 3D, velocity Verlet F2-F1-F3 and the
Berendsen F4) against the FP64 oracle, through the C interface on device
buffers.

Gates: accelerations at the final positions by the force gates of
tests/forcecheck.py (relative 1e-12 FP64, 1e-5 mixed; per atom 1e-11,
1e-4); positions and velocities after 10-20 steps within 1e-10 (FP64) and
1e-6 (mixed) of the oracle's, relative to the largest velocity for v;
records: energies to 1e-12 (FP64) and 1e-6 (mixed) of the kinetic energy,
the pressure in the pore to the same fraction of its scale, and the integer
fields (molecules in the pore, wall reflections, molecules
outside the domain) exactly."""
import numpy as np
import pytest
import torch

import oracle
from paper_1812_07993_amd import poremd, synth
from forcecheck import check_forces

pytestmark = pytest.mark.gpu

TOL_X = {"fp64": 1e-10, "mixed": 1e-6}
TOL_E = {"fp64": 1e-12, "mixed": 1e-6}


def gpu_run(x, v, model, nsteps, every=1):
    dev = torch.device("cuda:0")
    n, d = x.shape
    xd = torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float64, device=dev).clone()
    vd = torch.as_tensor(np.ascontiguousarray(v), dtype=torch.float64, device=dev).clone()
    ad = torch.full((max(n, 1), d), float("nan"), dtype=torch.float64, device=dev)
    rows = poremd.pmd_pm_record_rows(nsteps, every)
    rec = torch.zeros((rows, poremd.PM_RECORD_DTYPE.itemsize // 8), dtype=torch.float64, device=dev)
    s = torch.cuda.current_stream()
    poremd.pmd_pm_run(model, n, xd.data_ptr() if n else 0, vd.data_ptr() if n else 0,
                      ad.data_ptr(), nsteps, every, rec.data_ptr(), rows, s.cuda_stream)
    s.synchronize()
    r = rec.cpu().numpy().view(poremd.PM_RECORD_DTYPE).reshape(rows)
    return xd.cpu().numpy(), vd.cpu().numpy(), ad.cpu().numpy()[:n], r


def models(dim, prec, **kw):
    base = dict(lx=12.0, ly=8.0, lz=6.0, k=1.0, dt=0.002)
    base.update(kw)
    g = poremd.make_pm_model(dim, base["lx"], base["ly"], base["lz"], base["k"], prec,
                             dt=base["dt"], thermostat_tau=base.get("tau", 0.0),
                             thermostat_t0=base.get("t0", 0.0))
    o = oracle.pm_model(dim, base["lx"], base["ly"], base["lz"], k=base["k"], dt=base["dt"],
                        tau=base.get("tau", 0.0), t0=base.get("t0", 0.0))
    return g, o, base


def dense_state(dim, n_pore, n_outer, base, seed, T=1.0):
    return synth.pore_model_state(dim, base["lx"], base["ly"], base["lz"], base["k"], n_pore,
                                  n_outer, T, seed=seed)


def compare(xg, vg, ag, rg, xo, vo, ro, model_o, prec, what):
    n = xg.shape[0]
    assert np.abs(xg - xo).max() <= TOL_X[prec] * max(1.0, np.abs(xo).max()), what
    assert np.abs(vg - vo).max() <= TOL_X[prec] * max(1.0, np.abs(vo).max()), what
    fo, _, _ = oracle.pm_forces(model_o, xg)
    check_forces(ag, fo, prec, what=what)
    assert len(rg) == len(ro)
    assert np.array_equal(rg["step"], ro[:, 0].astype(np.int64))
    ke = max(abs(ro[0, 1]), 1e-300)
    assert np.abs(rg["ke"] - ro[:, 1]).max() <= TOL_E[prec] * ke, what
    assert np.abs(rg["pe"] - ro[:, 2]).max() <= TOL_E[prec] * ke, what
    assert np.array_equal(rg["n_pore"], ro[:, 3].astype(np.int64)), what
    assert np.array_equal(rg["reflections"], ro[:, 4].astype(np.int64)), what
    assert np.all(rg["n_outside"] == 0), what
    assert np.allclose(rg["temperature"], 2.0 * rg["ke"] / (xg.shape[1] * n), rtol=1e-14)
    d = xg.shape[1]
    vol = model_o.lx * model_o.ly * (model_o.lz if d == 3 else 1.0)
    pscale = np.abs(ro[:, 5]).max() + np.abs(ro[:, 1]).max() / (d * vol)
    assert np.abs(rg["pressure"] - ro[:, 5]).max() <= TOL_E[prec] * pscale, what


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("n_pore,n_outer,vscale", [(1, 0, 3.0), (2, 3, 3.0), (60, 10, 3.0),
                                                   (30, 6, 6.0)])
def test_dense_pore_matches_the_oracle(dim, prec, n_pore, n_outer, vscale):
    """A small pore crowded enough that molecules interact and hit the walls
    within 60 steps (dt 0.002, T = 9 or 36; in the last case a molecule
    leaves through the mouth), with a sparse outer space: forces use plain
    differences, so a molecule wrapping through a periodic face can land
    next to another one, and a dense outer space would make such jumps (and
    an ill-conditioned comparison) common.  The oracle's own total energy
    moves by under 1% in every case."""
    g, o, base = models(dim, prec)
    x, v = dense_state(dim, n_pore, n_outer, base, seed=n_pore + 7 * dim)
    v *= vscale
    xg, vg, ag, rg = gpu_run(x, v, g, 60, every=1)
    xo, vo, ro = oracle.pm_run(o, x, v, 60, every=1)
    eo = ro[:, 1] + ro[:, 2]
    assert np.abs(eo - eo[0]).max() <= 1e-2 * max(abs(eo[0]), ro[0, 1])
    if x.shape[0] > 1:
        compare(xg, vg, ag, rg, xo, vo, ro, o, prec, "dense dim=%d n=%d" % (dim, x.shape[0]))
    else:
        assert np.allclose(xg, xo, rtol=0, atol=1e-12) and np.all(ag == 0.0)
    if n_pore >= 30:
        assert rg["reflections"][-1] > 0
    if vscale > 3.0:
        assert rg["n_pore"].min() < n_pore  # the mouth was crossed


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
@pytest.mark.parametrize("dim", [2, 3])
def test_paper_workload_matches_the_oracle(dim, prec):
    """The paper's models at their own sizes (2D: 420 + 1764 molecules in a
    1 um pore; 3D: 1000 + 1800 in a 500 x 50 x 50 nm prism), 30 steps with
    the thermostat on (tau = 1 ps, t0 the paper's temperature)."""
    n_pore = 420 if dim == 2 else 1000
    x, v, geo = synth.paper_model_system(dim, n_pore)
    tau = 1.0 / synth.PAPER_TAU_PS
    g = poremd.make_pm_model(dim, geo["lx"], geo["ly"], geo["lz"], geo["k"], prec, dt=geo["dt"],
                             thermostat_tau=tau, thermostat_t0=geo["temperature"])
    o = oracle.pm_model(dim, geo["lx"], geo["ly"], geo["lz"], k=geo["k"], dt=geo["dt"], tau=tau,
                        t0=geo["temperature"])
    xg, vg, ag, rg = gpu_run(x, v, g, 30, every=10)
    xo, vo, ro = oracle.pm_run(o, x, v, 30, every=10)
    compare(xg, vg, ag, rg, xo, vo, ro, o, prec, "paper dim=%d" % dim)
    assert rg["n_pore"][0] == n_pore


@pytest.mark.parametrize("dim", [2, 3])
def test_free_gas_thermostat_closed_form(dim):
    """Non-interacting molecules (epsilon = 0) under the thermostat: the
    temperature measured at step s is t0 + (1 - dt/tau)^(s-1) (T_1 - t0)."""
    g, o, base = models(dim, "fp64", dt=0.01, tau=0.25, t0=1.5)
    g.epsilon = 0.0
    x, v = dense_state(dim, 80, 120, base, seed=3, T=1.0)
    v *= 2.0
    _, _, _, rg = gpu_run(x, v, g, 60, every=1)
    T1 = float(np.sum(v * v)) / (dim * x.shape[0])
    s = np.arange(1, 61)
    assert np.allclose(rg["temperature"][1:], 1.5 + (1 - 0.01 / 0.25) ** (s - 1) * (T1 - 1.5),
                       rtol=1e-12)


@pytest.mark.parametrize("dim", [2, 3])
def test_free_molecules_keep_their_speeds_and_stay_inside(dim):
    """3000 steps of non-interacting molecules (epsilon = 0, so the motion is
    ballistic between boundary events): every wall reflection and periodic
    wrap keeps |v|, no molecule leaves the domain, and the positions, the
    pore counts and the number of reflections are the oracle's."""
    g, o, base = models(dim, "fp64", dt=0.01)
    g.epsilon = 0.0
    o.epsilon = 0.0
    x, v = dense_state(dim, 60, 150, base, seed=4)
    v *= 3.0
    xg, vg, _, rg = gpu_run(x, v, g, 3000, every=1000)
    xo, vo, ro = oracle.pm_run(o, x, v, 3000, every=1000)
    assert np.allclose(np.linalg.norm(vg, axis=1), np.linalg.norm(v, axis=1), rtol=1e-13)
    assert np.all(rg["n_outside"] == 0) and rg["reflections"][-1] > 300
    assert rg["n_pore"][-1] == int(np.sum(xg[:, 0] < base["lx"]))
    assert np.array_equal(rg["n_pore"], ro[:, 3].astype(np.int64))
    assert np.array_equal(rg["reflections"], ro[:, 4].astype(np.int64))
    assert np.abs(xg - xo).max() <= 1e-9 and np.abs(vg - vo).max() <= 1e-12


def test_empty_and_repeatable():
    g, o, base = models(3, "mixed")
    _, _, _, r = gpu_run(np.zeros((0, 3)), np.zeros((0, 3)), g, 5, every=1)
    assert len(r) == 6 and np.all(r["ke"] == 0.0) and np.all(r["pe"] == 0.0)
    x, v = dense_state(3, 100, 150, base, seed=9)
    a = gpu_run(x, v, g, 25, every=5)
    b = gpu_run(x, v, g, 25, every=5)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1]) and np.array_equal(a[3], b[3])
