"""Batched sweep of many independent D2Q9 instances (lbm_batch_*).

* each instance of a batch equals the same instance run alone on the GPU
  (same kernel arithmetic: bit-identical), for every launch shape;
* instances against the CPU oracle (FP64 <= 1e-12, FP32 <= 1e-5);
* the 512-instance workload: autotuned shape, every instance against its
  single-instance GPU run, a seeded subset of 32 against the oracle;
* two time steps per launch (source-free batches): bit-identical to the
  instances run alone, for every two-step shape.
"""
import sys

import numpy as np
import pytest

import oracle as orc
from paper_1603_09577_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def small_batch(prec="f64", count=11, seed=31):
    rng = np.random.default_rng(seed)
    specs, phis = [], []
    for i in range(count):
        nx, ny = int(rng.integers(5, 90)), int(rng.integers(3, 70))
        k = np.diag(rng.uniform(0.005, 0.05, 2))
        sp = W.spec_nonlinear_2d(nx, ny, bcoef=float(rng.uniform(0, 1)), k0=k, source=True,
                                 precision=prec)
        specs.append(sp)
        phis.append(W.noise_field((ny, nx), 1000 + i))
    return specs, phis


def single_runs(specs, phis, steps):
    from paper_1603_09577_amd import lbm
    out = []
    for sp, ph in zip(specs, phis):
        s = lbm.Lbm(sp).init(ph)
        s.step(steps)
        out.append(s.phi())
    return out


def test_small_batch_matches_single_and_oracle():
    from paper_1603_09577_amd import lbm
    specs, phis = small_batch()
    say("[gpu batch] 11 ragged instances, f64")
    b = lbm.Batch(specs).init(phis)
    b.step(40)
    got = b.unpack(b.phi())
    ref = single_runs(specs, phis, 40)
    for i, (g, r) in enumerate(zip(got, ref)):
        assert torch.equal(g, r), i
    for i in (0, 3, 7):
        o, _ = orc.run(orc.params_from_spec(specs[i]), phis[i], 40)
        e = float(np.linalg.norm(got[i].cpu().numpy() - o) / np.linalg.norm(o))
        say(f"    instance {i} {specs[i]['shape']}: rel L2 vs oracle {e:.2e}")
        assert e <= 1e-12


@pytest.mark.parametrize("shape", [0, 1, 2, 3])
@pytest.mark.parametrize("grid,remap", [(0, 1), (0, 0), (64, 1), (1024, 0)])
def test_every_launch_shape_identical(shape, grid, remap):
    from paper_1603_09577_amd import lbm
    specs, phis = small_batch("f32", 9, seed=32)
    say(f"[gpu batch] shape {shape} grid {grid} remap {remap}")
    b = lbm.Batch(specs).init(phis)
    b.set_shape(shape, grid, remap)
    b.step(37)
    got = b.unpack(b.phi())
    ref = single_runs(specs, phis, 37)
    for i, (g, r) in enumerate(zip(got, ref)):
        assert torch.equal(g, r), i


def test_batch_workload_512_instances():
    from paper_1603_09577_amd import lbm
    items = W.batch_specs()
    specs = [s for s, _ in items]
    phis = [p for _, p in items]
    say(f"[gpu batch] 512 instances, {sum(p.size for p in phis)} nodes, f32")
    b = lbm.Batch(specs).init(phis)
    rep = b.tune(reps=3)
    say("    tuner: " + rep.splitlines()[-1])
    b.step(64)
    got = b.unpack(b.phi())
    assert all(torch.isfinite(g).all().item() for g in got)
    ref = single_runs(specs, phis, 64)
    for i, (g, r) in enumerate(zip(got, ref)):
        assert torch.equal(g, r), i
    rng = np.random.default_rng(4)
    for i in sorted(rng.choice(len(specs), 32, replace=False)):
        sp = dict(specs[i], precision="f64")
        o, _ = orc.run(orc.params_from_spec(sp), phis[i], 64)
        e = float(np.linalg.norm(got[i].cpu().numpy() - o) / np.linalg.norm(o))
        assert e <= 1e-5, (i, e)


def sourcefree_batch(prec, count=10, seed=33):
    rng = np.random.default_rng(seed)
    specs, phis = [], []
    for i in range(count):
        nx, ny = int(rng.integers(5, 150)), int(rng.integers(3, 60))
        k = np.diag(rng.uniform(0.005, 0.05, 2))
        specs.append(W.spec_nonlinear_2d(nx, ny, bcoef=float(rng.uniform(0, 1)), k0=k, source=False,
                                         precision=prec))
        phis.append(W.noise_field((ny, nx), 2000 + i))
    return specs, phis


@pytest.mark.parametrize("prec,shape", [("f32", 4), ("f32", 5), ("f16", 4), ("f64", 4)])
@pytest.mark.parametrize("remap", [1, 0])
def test_two_step_batch_identical(prec, shape, remap):
    """Two time steps per launch over a ragged source-free batch (instances
    narrower and lower than a tile included) against each instance run alone:
    bit-identical after an odd number of steps, with graph replays."""
    from paper_1603_09577_amd import lbm
    specs, phis = sourcefree_batch(prec)
    say(f"[gpu batch] two steps per launch, {prec} shape {shape} remap {remap}")
    b = lbm.Batch(specs).init(phis)
    b.set_shape(shape, 0, remap)
    sh = b.get_shape()
    assert sh["npt"] < 0 and sh["wg"] % 64 == 0
    b.step(71)
    got = b.unpack(b.phi())
    ref = single_runs(specs, phis, 71)
    for i, (g, r) in enumerate(zip(got, ref)):
        assert torch.equal(g, r), (i, specs[i]["shape"])


def test_two_step_batch_refused_with_a_source():
    from paper_1603_09577_amd import lbm
    specs, phis = small_batch("f32", 3, seed=34)
    b = lbm.Batch(specs)
    with pytest.raises(lbm.LbmError) as ei:
        b.set_shape(4, 0, 1)
    assert ei.value.code == lbm.LBM_E_INVALID


def test_tuner_cache_roundtrip(tmp_path, monkeypatch):
    """The batch tuner's decision is appended to $LBM_TUNE_CACHE (missing
    directories created) and read back by the next tune of the same batch."""
    from paper_1603_09577_amd import lbm
    path = tmp_path / "a" / "b" / "tune.txt"
    monkeypatch.setenv("LBM_TUNE_CACHE", str(path))
    specs, phis = sourcefree_batch("f32", 4, seed=35)
    b = lbm.Batch(specs).init(phis)
    first = b.tune(reps=1, use_cache=True)
    assert path.exists() and "chosen" in first.splitlines()[-1]
    shape = b.get_shape()
    b2 = lbm.Batch(specs).init(phis)
    second = b2.tune(reps=1, use_cache=True)
    assert second.startswith("cached")
    assert b2.get_shape() == shape
