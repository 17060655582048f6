"""Pins of the oracle's pressure in the pore of the cell-list workloads
(Sec. 2's virial formula with V the pore volume): the closed-form void
volumes against a Monte Carlo count of the region test, the ideal-gas limit,
the whole-box case against the pinned virial sums, and a dimer in the slit
against its closed form.  CPU only."""
import math

import numpy as np
import pytest

import oracle

BOX = (24.0, 24.0, 24.0)
PORES = [
    ("cylinder", oracle.make_pore("cylinder", 1.0, 12.0, 8.0, 4.0)),
    ("cone", oracle.make_pore("cone", 1.0, 12.0, 8.0, 2.0, 6.0)),
    ("inkbottle", oracle.make_pore("inkbottle", 1.0, 12.0, 8.0, 2.0, 7.0)),
    ("slit", oracle.make_pore("slit", 1.0, 12.0, 4.0, slit_gap=6.0)),
    ("none", oracle.make_pore("none")),
]


@pytest.mark.parametrize("name,pore", PORES)
def test_void_volume_matches_a_monte_carlo_count(name, pore):
    """4M uniform points in the box: the fraction inside the region test
    times the box volume agrees with the closed form within 4 standard
    errors of the count."""
    rng = np.random.default_rng(11)
    n = 4_000_000
    x = rng.random((n, 3)) * np.asarray(BOX)
    c = oracle.pore_count(x, BOX, pore)
    Vb = np.prod(BOX)
    V = oracle.pore_volume(pore, BOX)
    p = V / Vb
    assert abs(c / n - p) <= 4.0 * math.sqrt(p * (1 - p) / n) + 1e-12
    closed = {"cylinder": math.pi * 16 * 8, "cone": math.pi * 8 * (4 + 12 + 36) / 3,
              "inkbottle": math.pi * 4 * (4 + 49), "slit": 24 * 24 * 6, "none": Vb}[name]
    assert V == pytest.approx(closed, rel=1e-15)


def test_plain_slab_has_no_pore():
    q = oracle.make_pore("slab", 1.0, 12.0, 4.0)
    assert oracle.pore_volume(q, BOX) == 0.0
    assert oracle.pore_count(np.full((1, 3), 12.0), BOX, q) == 0


def _gas(n, seed):
    rng = np.random.default_rng(seed)
    g = np.stack(np.meshgrid(*[np.arange(8)] * 3, indexing="ij"), -1).reshape(-1, 3)
    x = (0.5 + 3.0 * g[:n] + rng.uniform(-0.4, 0.4, (n, 3))) % 24.0
    v = rng.normal(0.0, 1.1, (n, 3))
    return x, v


@pytest.mark.parametrize("name,pore", PORES)
def test_ideal_gas_limit(name, pore):
    """epsilon = 0: P = 2 K_pore / (3 V) = n_pore T_pore / V."""
    x, v = _gas(400, 1)
    p = oracle.make_params(BOX, epsilon=0.0)
    r = oracle.pore_pressure(x, v, p, pore)
    inside = np.array([oracle.pore_count(x[i:i + 1], BOX, pore) for i in range(len(x))], bool)
    assert r["n_pore"] == inside.sum() > 0
    assert r["virial_pore"] == 0.0
    T = np.sum(v[inside] ** 2) / (3 * inside.sum())
    assert r["pressure"] == pytest.approx(inside.sum() * T / r["volume"], rel=1e-13)


def test_whole_box_virial_equals_the_pinned_sums():
    """Without walls the pore is the whole box: W_pore is the vapour virial
    sum of orc_virial, pinned by its closed forms."""
    x, v = _gas(500, 2)
    p = oracle.make_params(BOX)
    r = oracle.pore_pressure(x, v, p, PORES[4][1])
    wvv, _ = oracle.virial(x, None, p)
    assert r["n_pore"] == 500
    assert r["virial_pore"] == pytest.approx(wvv, rel=1e-12)
    assert r["pressure"] == pytest.approx((2 * 0.5 * np.sum(v * v) + wvv) / (3 * np.prod(BOX)), rel=1e-12)


def test_dimer_in_the_slit():
    """Two molecules at rest r apart inside the slit gap: W = r f(r) =
    24 (2 r^-12 - r^-6); with one of them outside the gap, half of that."""
    q = PORES[3][1]  # gap z in [9, 15)
    p = oracle.make_params(BOX)
    for r in (0.95, 1.2, 2.0):
        rf = 24.0 * (2 * r ** -12 - r ** -6)
        x = np.array([[5.0, 5.0, 12.0], [5.0, 5.0, 12.0 + r]])
        out = oracle.pore_pressure(x, np.zeros_like(x), p, q)
        assert out["virial_pore"] == pytest.approx(rf, rel=1e-13)
        assert out["pressure"] == pytest.approx(rf / (3 * 24 * 24 * 6), rel=1e-13)
        x = np.array([[5.0, 5.0, 14.8], [5.0, 5.0, 14.8 + r]])
        out = oracle.pore_pressure(x, np.zeros_like(x), p, q)
        assert out["n_pore"] == 1 and out["virial_pore"] == pytest.approx(0.5 * rf, rel=1e-13)
