"""Serving on the GPU: requests that arrive while others run are admitted
into the resident batches and finish with the same result as when run
alone (positions and velocities agree to 1e-12; bit for bit by design)."""
import numpy as np
import pytest

from paper_1812_07993_amd import poremd, serve, synth

pytestmark = pytest.mark.gpu


def trace():
    specs = [dict(index=0, arrival=0.0, n=1500, shape="cylinder", r=3.0, L=26.0, steps=90, precision="mixed"),
             dict(index=1, arrival=0.0, n=800, shape="slit", r=2.5, L=22.0, steps=40, precision="fp64"),
             dict(index=2, arrival=0.01, n=2200, shape="cone", r=2.0, L=28.0, steps=120, precision="mixed"),
             dict(index=3, arrival=0.02, n=600, shape="inkbottle", r=2.0, L=22.0, steps=60, precision="mixed"),
             dict(index=4, arrival=0.03, n=1000, shape="cylinder", r=4.0, L=23.0, steps=75, precision="fp64"),
             dict(index=5, arrival=0.05, n=1200, shape="slit", r=3.0, L=24.0, steps=33, precision="mixed")]
    out = []
    for sp in specs:
        d = synth.request_system(sp, seed=5)
        out.append(serve.Request(sp["index"], sp["arrival"], sp["precision"], sp["steps"], sp["n"], d))
    return out


def test_served_results_match_alone():
    reqs = trace()
    be = serve.PoremdBackend(hbm_budget=0, max_slots=3, keep_positions=True)
    res = serve.Server(be, chunk_steps=20).run(reqs)
    assert [r.status for r in res] == ["ok"] * len(reqs)
    for req, r in zip(reqs, res):
        s = poremd.System.from_desc(req.payload, precision=req.precision)
        s.step(req.steps)
        X, V = s.positions(), s.velocities()
        assert np.abs(r.output["positions"] - X).max() <= 1e-12, req.index
        assert np.abs(r.output["velocities"] - V).max() <= 1e-12, req.index
        e = s.energies()
        assert r.output["energies"]["step"] == req.steps
        assert r.output["energies"]["etotal"] == pytest.approx(e["etotal"], rel=1e-12)
        s.close()
    summ = serve.summarize(res)
    assert summ["p99_s"] >= summ["p50_s"] > 0


def test_served_mix_with_a_large_request_matches_alone():
    """Three requests, one of them 120,000 vapour atoms, arriving while the
    others run: each served result equals its run alone bit for bit."""
    specs = [dict(index=0, arrival=0.0, n=120000, shape="slit", r=3.0, L=106.0, steps=150, precision="mixed"),
             dict(index=1, arrival=0.005, n=3000, shape="cone", r=2.5, L=31.0, steps=220, precision="mixed"),
             dict(index=2, arrival=0.01, n=5000, shape="inkbottle", r=3.0, L=37.0, steps=90, precision="fp64")]
    reqs = []
    for sp in specs:
        d = synth.request_system(sp, seed=9)
        reqs.append(serve.Request(sp["index"], sp["arrival"], sp["precision"], sp["steps"], sp["n"], d))
    be = serve.PoremdBackend(hbm_budget=0, max_slots=4, keep_positions=True)
    res = serve.Server(be, chunk_steps=25, create_workers=2).run(reqs)
    assert [r.status for r in res] == ["ok"] * len(reqs)
    for req, r in zip(reqs, res):
        s = poremd.System.from_desc(req.payload, precision=req.precision)
        s.step(req.steps)
        assert np.array_equal(r.output["positions"], s.positions()), req.index
        assert np.array_equal(r.output["velocities"], s.velocities()), req.index
        assert r.output["energies"]["etotal"] == s.energies()["etotal"]
        s.close()
