"""GPU parity of the all-pairs forces (the force function as stated in
Sec. 3: every pair, no cutoff, no shift, minimum image) against the FP64
oracle, through the C interface on device buffers.

Sizes up to N = 7800, the largest the benchmark times (N_pore = 1500).
Forces: the relative error ||F - F_ref|| / ||F_ref|| <= 1e-12 (FP64) and
<= 1e-5 (mixed: FP32 pair terms from FP64 differences, FP64 sums), and the
per-atom error max_i |dF_i| / rms |F| <= 1e-11 and 1e-4 (tests/forcecheck.py).
Energies: each atom's share and the total within the same relative gate of
the sum of the per-atom energy magnitudes."""
import numpy as np
import pytest
import torch

import oracle
from paper_1812_07993_amd import poremd, synth
from forcecheck import TOL_F, check_forces

pytestmark = pytest.mark.gpu


def _run(x, box, prec, eps=1.0, sig=1.0):
    dev = torch.device("cuda:0")
    n = x.shape[0]
    xd = torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float64, device=dev)
    f = torch.full((max(n, 1), 3), float("nan"), dtype=torch.float64, device=dev)
    u = torch.full((max(n, 1),), float("nan"), dtype=torch.float64, device=dev)
    e = torch.full((1,), float("nan"), dtype=torch.float64, device=dev)
    s = torch.cuda.current_stream()
    poremd.pmd_allpairs_forces(prec, n, xd.data_ptr() if n else 0, box, eps, sig, f.data_ptr(),
                               u.data_ptr(), e.data_ptr(), s.cuda_stream)
    s.synchronize()
    return f.cpu().numpy()[:n], u.cpu().numpy()[:n], float(e.cpu()[0])


def _config(n, seed):
    L = (n / 0.05) ** (1.0 / 3.0) if n > 1 else 4.0
    rng = np.random.default_rng(seed)
    return synth.rsa_place(rng, (L, L, L), n, np.zeros((0, 3)), 0.9), L


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
@pytest.mark.parametrize("periodic", [True, False])
@pytest.mark.parametrize("n", [1, 2, 17, 64, 65, 1000, 1531, 7800])
def test_allpairs_matches_the_oracle(n, periodic, prec):
    x, L = _config(n, 100 + n)
    box = (L, L, L) if periodic else (0.0, 0.0, 0.0)
    f, u, e = _run(x, box, prec, 1.1, 0.97)
    fr, ur, er = oracle.allpairs(x, box, 1.1, 0.97)
    if n > 1:
        check_forces(f, fr, prec, what="all-pairs n=%d periodic=%s" % (n, periodic))
    else:
        assert np.all(f == 0.0) and np.all(u == 0.0) and e == 0.0
    us = max(np.abs(ur).sum(), 1e-300)
    assert np.abs(u - ur).max() <= TOL_F[prec] * us
    assert abs(e - er) <= TOL_F[prec] * us


def test_allpairs_empty_and_repeatable():
    f, u, e = _run(np.zeros((0, 3)), (5.0, 5.0, 5.0), "fp64")
    assert e == 0.0 and f.shape == (0, 3)
    x, L = _config(700, 5)
    a = _run(x, (L, L, L), "mixed")
    b = _run(x, (L, L, L), "mixed")
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1]) and a[2] == b[2]
