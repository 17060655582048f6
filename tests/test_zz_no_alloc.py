"""The allocation-free pore-model entry point (pmd_pm_run_noalloc, static
device working memory) against the allocating one (pmd_pm_run) through the
C interface: two calls in a row, the second on a smaller input (2D after
3D), each giving the same positions, velocities, accelerations and records
bit for bit (same kernels, same arithmetic, fixed summation orders)."""
import numpy as np
import pytest
import torch

from paper_1812_07993_amd import poremd, synth

pytestmark = pytest.mark.gpu


def _run(fn, model, x, v, nsteps, every):
    dev = torch.device("cuda:0")
    n, d = x.shape
    xd = torch.as_tensor(x, dtype=torch.float64, device=dev).clone()
    vd = torch.as_tensor(v, dtype=torch.float64, device=dev).clone()
    ad = torch.full((n, d), float("nan"), dtype=torch.float64, device=dev)
    rows = poremd.pmd_pm_record_rows(nsteps, every)
    rec = torch.zeros((rows, poremd.PM_RECORD_DTYPE.itemsize // 8), dtype=torch.float64, device=dev)
    s = torch.cuda.current_stream()
    fn(model, n, xd.data_ptr(), vd.data_ptr(), ad.data_ptr(), nsteps, every, rec.data_ptr(), rows,
       s.cuda_stream)
    s.synchronize()
    return xd.cpu().numpy(), vd.cpu().numpy(), ad.cpu().numpy(), rec.cpu().numpy()


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_noalloc_matches_the_allocating_entry(prec):
    cases = []
    for dim, n_pore, n_outer in ((3, 1800, 1200), (2, 300, 400)):
        lx, ly, lz, k = 40.0, 20.0, 20.0, 1.0
        x, v = synth.pore_model_state(dim, lx, ly, lz, k, n_pore, n_outer, 1.5, seed=dim)
        m = poremd.make_pm_model(dim, lx, ly, lz, k, prec, dt=0.004, thermostat_tau=0.5,
                                 thermostat_t0=1.2)
        cases.append((m, x, v))
    for m, x, v in cases:  # the second call is the smaller input
        a = _run(poremd.pmd_pm_run_noalloc, m, x, v, 40, 10)
        b = _run(poremd.pmd_pm_run, m, x, v, 40, 10)
        for p, q in zip(a, b):
            assert np.array_equal(p, q)
        assert np.all(np.isfinite(a[0]))


def test_noalloc_rejects_more_than_its_working_memory():
    m = poremd.make_pm_model(3, 40.0, 20.0, 20.0, 1.0, "fp64")
    with pytest.raises(poremd.PmdError) as e:
        poremd.pmd_pm_run_noalloc(m, 65537, 0x1000, 0x1000, 0, 1, 1, 0, 0)
    assert e.value.code == poremd.PMD_EINVAL
    assert "static working memory" in poremd.pmd_last_error()
