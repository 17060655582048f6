"""Seeded input generator: exclusion distance, temperature, determinism."""
import numpy as np
import pytest
from scipy.spatial import cKDTree

from paper_1812_07993_amd import synth


def test_rsa_exclusion_and_walls():
    s = synth.cylinder_slab_small()
    assert s.n == 1536 and s.walls.shape[0] == 3968
    L = 32.0
    tree = cKDTree(np.concatenate([s.x, s.walls]) % L, boxsize=L)
    pairs = tree.query_pairs(0.9 - 1e-12)
    # no vapour atom within 0.9 of another vapour atom or of a wall site
    assert all(i >= s.n and j >= s.n for i, j in pairs)
    # config rule: vapour only outside the slab's z-range
    assert np.all((s.x[:, 2] < 14.0) | (s.x[:, 2] >= 18.0))
    assert np.all((s.x >= 0) & (s.x < L))


def test_maxwell_temperature_exact():
    rng = np.random.default_rng(0)
    v = synth.maxwell(rng, 1000, 1.2)
    assert np.abs(v.sum(axis=0)).max() < 1e-10
    assert np.sum(v * v) / (3 * 1000 - 3) == pytest.approx(1.2, rel=1e-13)


def test_seeded_determinism():
    a = synth.cylinder_slab_small()
    b = synth.cylinder_slab_small()
    assert np.array_equal(a.x, b.x) and np.array_equal(a.v, b.v)
    c = synth.cylinder_slab_small(seed=1)
    assert not np.array_equal(a.x, c.x)


def test_replica_and_request_samplers():
    specs = synth.replica_specs(256)
    ns = np.array([s["n"] for s in specs])
    assert ns.min() >= 1000 and ns.max() <= 64000
    assert {s["shape"] for s in specs} == {"cylinder", "slit", "cone"}
    reqs = synth.request_trace(64)
    t = np.array([r["arrival"] for r in reqs])
    assert np.all(np.diff(t) > 0)
    assert {r["precision"] for r in reqs} == {"mixed", "fp64"}
    small = synth.replica(dict(index=0, n=1000, shape="cone", r=3.0, L=22.0), steps=10)
    assert small.n == 1000 and small.walls.shape[0] > 0
