"""The batched form: many cavities of uneven size and parameters stepped by one launch per step
(replayed from a HIP graph), with the launch shape picked by the autotuner.

Each cavity of a batch must equal its own plain run bitwise (the per-node arithmetic is the
plain step's), and a subset is compared with the FP64 CPU oracle (1e-12 FP64 after short runs).
"""
import os

import numpy as np
import pytest
import torch

from oracle import ref
from paper_1308_2071_amd import Batch, Cavity, workloads
from pressure_gauge import phip_gauged

pytestmark = pytest.mark.gpu

FIELDS = ("ux", "uy", "p", "T")


def small_batch(dtype):
    specs = [
        (64, 64, 1e3, 1.0, 1e-2, 0.6),
        (96, 40, 3e5, 0.71, 1e-3, 0.35),
        (33, 70, 1e4, 7.0, 5e-2, 0.8),
        (300, 17, 1e6, 1.0, 1e-4, 0.25),
        (128, 128, 5e4, 0.71, 2e-2, 0.45),
        (5, 5, 1e5, 1.0, 1e-2, 0.5),
    ]
    params, phis = [], []
    for nx, ny, Ra, Pr, Da, phi in specs:
        params.append(workloads.cavity(nx, ny, Ra=Ra, Pr=Pr, Da=Da, dtype=dtype))
        phis.append(phi)
    return params, phis


@pytest.mark.parametrize("spl", [1, 2])
@pytest.mark.parametrize("dtype", ["fp32", "fp64", "fp32_f64"])
def test_batch_equals_standalone_runs_bitwise(dtype, spl, tmp_path):
    """One step per launch and two (the batched two-step kernel, forced through the first
    cavity's steps_per_launch), through graph replays and an odd remainder."""
    params, phis = small_batch(dtype)
    params[0] = dict(params[0], steps_per_launch=spl)
    b = Batch(params, phis, tune_cache_path=str(tmp_path / "tune.txt"))
    assert b.shape()[4] == spl
    b.step(151)           # graph replays + remainder (odd: ends with one single step)
    s, obs = b.observables()
    assert s == 0
    for i, (p, phi) in enumerate(zip(params, phis)):
        c = Cavity(p, phi_uniform=phi)
        c.step(151)
        ref_obs = c.observables()
        got = b.fields(i)
        for k in FIELDS:
            assert torch.equal(got[k], ref_obs[k]), (i, k)
        assert obs[i]["nu_hot"] == ref_obs["nu_hot"]
        assert obs[i]["step"] == 151
        c.close()
    b.close()


def test_batch_subset_against_oracle():
    params, phis = small_batch("fp64")
    b = Batch(params, phis)
    b.step(40)
    for i in (0, 2, 3, 5):
        p = dict(params[i])
        p.pop("dtype")
        lat = ref.RefLattice(phi_uniform=phis[i], **p)
        lat.step(40)
        r = lat.observables(dynamic_pressure=True)
        g = b.fields(i)
        for k in FIELDS:
            assert np.abs(g[k].cpu().numpy() - r[k]).max() <= 1e-12, (i, k)
    b.close()


def test_graph_replay_equals_single_steps():
    params, phis = small_batch("fp32")
    a = Batch(params, phis)
    c = Batch(params, phis)
    a.step(64)
    for _ in range(64):
        c.step(1)
    for i in range(len(params)):
        fa, fc = a.fields(i), c.fields(i)
        for k in FIELDS:
            assert torch.equal(fa[k], fc[k]), (i, k)


def test_autotuner_caches_its_choice(tmp_path):
    path = str(tmp_path / "tune.txt")
    params, phis = small_batch("fp32")
    a = Batch(params, phis, tune_cache_path=path)
    shape = a.shape()
    lines = open(path).read().splitlines()
    # key: format version | device architecture | dtype | hash of the shapes | steps setting;
    # then rows per tile, segments per work-item, work-groups, two-step rows per segment and
    # strips per work-group
    assert len(lines) == 1 and len(lines[0].split()) == 6
    key = lines[0].split()[0].split("|")
    assert key[0] == "v3" and key[1].startswith(("gfx", "unknown")) and key[2] == "fp32"
    assert key[4] == "s0" and int(lines[0].split()[4]) in (0, 2, 3, 4, 5, 6, 8, 12)
    assert int(lines[0].split()[5]) in (1, 2, 4)
    b = Batch(params, phis, tune_cache_path=path)       # served from the cache
    assert b.shape() == shape
    assert len(open(path).read().splitlines()) == 1
    # a different set of cavities gets its own entry
    Batch(params[:3], phis[:3], tune_cache_path=path)
    assert len(open(path).read().splitlines()) == 2
    wg, npt = shape[1], shape[0]
    assert wg in (64, 128, 256, 512) and npt in (1, 2, 4) and shape[3] % 2 == 0
    assert shape[4] in (1, 2) and (shape[5] > 0) == (shape[4] == 2)


@pytest.mark.parametrize("dtype", ["fp32", "fp64"])
def test_every_two_step_shape_the_tuner_tries_equals_standalone_runs(dtype, tmp_path):
    """Every segment height (2, 3, 4, 5, 6, 8, 12 rows) and strip count (1, 2, 4 per
    work-group) the autotuner may pick, forced through its cache file, steps each cavity
    bitwise like its own plain run (odd step count: graph replays, then one single step)."""
    params, phis = small_batch(dtype)
    params[0] = dict(params[0], steps_per_launch=2)
    path = tmp_path / "tune.txt"
    Batch(params, phis, tune_cache_path=str(path)).close()
    line = path.read_text().split()
    want = []
    for p, phi in zip(params, phis):
        c = Cavity(p, phi_uniform=phi)
        c.step(77)
        want.append(c.observables())
        c.close()
    for rows in (2, 3, 4, 5, 6, 8, 12):
        for strips in (1, 2, 4):
            path.write_text(" ".join(line[:4] + [str(rows), str(strips)]) + "\n")
            b = Batch(params, phis, tune_cache_path=str(path))
            assert b.shape()[5] == rows, (rows, b.shape())
            b.step(77)
            for i, ref_obs in enumerate(want):
                got = b.fields(i)
                for k in FIELDS:
                    assert torch.equal(got[k], ref_obs[k]), (rows, strips, i, k)
            b.close()


def test_batch_rejects_mixed_dtypes_and_tapes():
    params, phis = small_batch("fp32")
    bad = list(params)
    bad[1] = dict(bad[1], dtype="fp64")
    with pytest.raises(RuntimeError, match="LBM_E_INVAL"):
        Batch(bad, phis)
    bad = list(params)
    bad[0] = dict(bad[0], checkpoint_every=10)
    with pytest.raises(RuntimeError, match="LBM_E_UNSUPPORTED"):
        Batch(bad, phis)


def test_batch64_workload_runs_and_matches_plain_on_sampled_cavities(tmp_path):
    """The 64-cavity workload at its full size for a few hundred steps: every cavity stays finite,
    and seven cavities (one per side length) equal their plain runs bitwise and the FP64 oracle
    within 1e-4 of each field's range (p up to a constant) and Nu within 1e-3."""
    cav = workloads.batch64()
    params = [dict(c["params"], dtype="fp32") for c in cav]
    phis = [c["phi"] for c in cav]
    b = Batch(params, phis, tune_cache_path=str(tmp_path / "tune.txt"))
    b.step(300)
    s, obs = b.observables()
    assert s == 0 and not any(o["diverged"] for o in obs)
    seen = {}
    for i, p in enumerate(params):
        seen.setdefault(p["nx"], i)
    for nx, i in sorted(seen.items()):
        c = Cavity(params[i], phi_uniform=phis[i])
        c.step(300)
        r = c.observables()
        g = b.fields(i)
        for k in FIELDS:
            assert torch.equal(g[k], r[k]), (nx, k)
        c.close()
        p = {k: v for k, v in params[i].items() if k != "dtype"}
        ref.set_threads(len(os.sched_getaffinity(0)))
        lat = ref.RefLattice(phi_uniform=float(np.float32(phis[i])), **p)
        lat.step(300)
        o = lat.observables(dynamic_pressure=True)
        lat.close()
        for k in FIELDS:
            d = g[k].double().cpu().numpy() - o[k]
            if k == "p":
                d = phip_gauged(d, float(np.float32(phis[i])))   # the free phi p level
            rng = max(o[k].max() - o[k].min(), 1e-2 * np.abs(o[k]).max())
            assert np.abs(d).max() <= 1e-4 * rng, (nx, k, np.abs(d).max() / rng)
        assert abs(obs[i]["nu_hot"] - o["nu_hot"]) <= 1e-3, (nx, obs[i]["nu_hot"], o["nu_hot"])


def read_stability():
    """The oracle's record of the batched workload over its 10,000 steps (written by
    tests/golden/make_batch64_stability.py, oracle only)."""
    rows = {}
    with open(os.path.join(os.path.dirname(__file__), "golden", "batch64_stability.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            v = line.split()
            rows[int(v[0])] = dict(first_flag=int(v[7]), nu_hot=float(v[8]),
                                   nu_cold=float(v[9]), max_speed=float(v[10]))
    return rows


def test_batch64_full_10k_steps_against_the_oracle_record(tmp_path):
    """All 10,000 steps of the batched workload in FP32, in the graph-replayed form the
    benchmark times: the cavities the library flags as diverged are exactly those the FP64
    oracle flags (0 and 9, whose tau_v lies beyond the step's linear stability limit), and every
    other cavity's Nusselt numbers are within 1e-3 of the oracle's and its max |u| within 1e-3
    of it relative."""
    rec = read_stability()
    cav = workloads.batch64()
    params = [dict(c["params"], dtype="fp32") for c in cav]
    b = Batch(params, [c["phi"] for c in cav], tune_cache_path=str(tmp_path / "tune.txt"))
    b.step(10000)
    s, obs = b.observables()
    flagged = sorted(i for i, o in enumerate(obs) if o["diverged"])
    want = sorted(i for i, r in rec.items() if r["first_flag"] >= 0)
    assert flagged == want == [0, 9]
    assert s == -4
    worst = 0.0
    for i, o in enumerate(obs):
        if i in want:
            continue
        r = rec[i]
        e = max(abs(o["nu_hot"] - r["nu_hot"]), abs(o["nu_cold"] - r["nu_cold"]))
        worst = max(worst, e)
        assert e <= 1e-3, (i, o["nu_hot"], r["nu_hot"], o["nu_cold"], r["nu_cold"])
        assert abs(o["max_speed"] - r["max_speed"]) <= 1e-3 * r["max_speed"], i
    print(f"batch64 10k steps: flagged {flagged}, worst |dNu| of the rest {worst:.2e}")

