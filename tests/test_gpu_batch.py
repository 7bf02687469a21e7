"""Batched parameter sweep on the GPU (C ABI lbm_batch_*): every case of a
batch equals the same case run alone (bit for bit, any schedule), matches
the FP64 oracle, and the autotuner leaves the state untouched."""
import numpy as np
import pytest
import torch

import workloads as W
from oracle import lbm2d as L

pytestmark = pytest.mark.gpu


def _lbm():
    from paper_2103_01444_amd import lbm
    return lbm


def _cases(n=5):
    return W.batched_cases()[:n]


def test_batch_cases_equal_single_contexts_bitwise():
    lbm = _lbm()
    cases = _cases()
    b = lbm.BatchedSweep(cases)
    b.step(150)
    obs = b.observables()
    for i, w in enumerate(cases):
        single = lbm.Cathode.from_workload(w)
        single.step(150)
        assert torch.equal(b.populations(i), single.populations()), w["name"]
        o = single.observables()
        assert obs[i]["current_density"] == o["current_density"], w["name"]
        assert obs[i]["sum_c"] == o["sum_c"]



def test_persistent_barrier_timeout_is_an_error_then_recovers():
    """A persistent launch whose grid-barrier waits are bounded at zero (the
    condition forced from the host: one tick of the device clock) gives up
    at a barrier: every workgroup leaves the kernel, the next synchronising
    call raises the device error, and after re-initialisation with the
    default bound the batch steps bit-identically to an untouched one."""
    lbm = _lbm()
    cases = _cases(3)
    b = lbm.BatchedSweep(cases)
    ref = lbm.BatchedSweep(cases)
    b.set_schedule(256, 1, 1)
    b.set_barrier_timeout(0.0)
    b.step(8)
    with pytest.raises(lbm.LbmError, match="timed out"):
        b.synchronize()
    with pytest.raises(lbm.LbmError, match="invalid argument"):
        b.set_barrier_timeout(-1.0)
    b.set_barrier_timeout(4.0)
    b.init_equilibrium()
    b.step(30)
    ref.step(30)
    b.synchronize()
    for i in range(len(cases)):
        assert torch.equal(b.populations(i), ref.populations(i)), i
    b.close()
    ref.close()


@pytest.mark.parametrize("sched", [(64, 4, 0), (512, 2, 0), (128, 2, 1), (256, 1, 1), (64, 16, 1), (128, 1, 0, 128),
                                   (32, 2, 0, 64), (128, 1, 0, 0), (64, 12, 0, 960)])
def test_every_schedule_gives_identical_results(sched):
    lbm = _lbm()
    cases = _cases()
    ref = lbm.BatchedSweep(cases)
    ref.step(60)
    b = lbm.BatchedSweep(cases)
    b.set_schedule(*sched)
    b.step(23)
    b.step(37)
    assert b.step_count == 60
    for i in range(len(cases)):
        assert torch.equal(b.populations(i), ref.populations(i)), (sched, i)


def test_autotune_keeps_state_and_is_cached(tmp_path):
    lbm = _lbm()
    cases = _cases(4)
    b = lbm.BatchedSweep(cases)
    b.step(40)
    before = [b.populations(i).clone() for i in range(len(cases))]
    res = b.autotune(trial_steps=3, cache_path=str(tmp_path / "tune.json"))
    assert not res["cached"] and res["ms_per_step"] > 0
    assert b.step_count == 40
    for i in range(len(cases)):
        assert torch.equal(b.populations(i), before[i])
    assert b.schedule == {k: res[k] for k in ("tile_x", "tile_y", "persistent", "block")}
    b2 = lbm.BatchedSweep(cases)
    res2 = b2.autotune(trial_steps=3, cache_path=str(tmp_path / "tune.json"))
    assert res2["cached"] and b2.schedule == b.schedule
    # the library's cache file: JSON, one entry keyed by arch, precision and the case sizes
    import json
    tune = json.loads((tmp_path / "tune.json").read_text())
    (key, entry), = tune.items()
    assert key.endswith("|fp32|" + ",".join(f"{w['nx']}x{w['ny']}" for w in cases))
    assert {k: entry[k] for k in ("tile_x", "tile_y", "persistent", "block")} == b.schedule
    # another batch adds its own entry; a file in another form is neither used nor rewritten
    b3 = lbm.BatchedSweep(cases[:2])
    assert not b3.autotune(trial_steps=3, cache_path=str(tmp_path / "tune.json"))["cached"]
    assert len(json.loads((tmp_path / "tune.json").read_text())) == 2
    foreign = tmp_path / "other.json"
    foreign.write_text('{"something": [1, 2, 3]}\n')
    assert not b3.autotune(trial_steps=3, cache_path=str(foreign))["cached"]
    assert foreign.read_text() == '{"something": [1, 2, 3]}\n'


def test_batch_case_matches_oracle():
    lbm = _lbm()
    cases = [w for w in W.batched_cases() if w["nx"] * w["ny"] <= 256 * 64][:1]
    if not cases:
        cases = [dict(W.batched_cases()[0], nx=256, ny=64, ny_channel=32, ny_gdl=29, ny_cl=3)]
    w = cases[0]
    b = lbm.BatchedSweep([w])
    b.step(300)
    m = L.Model(L.geometry_from_workload(w), L.Params.from_workload(w))
    s = m.run(m.initial_state(), 300)
    single = lbm.Cathode.from_workload(w)
    single.step(300)
    assert torch.equal(single.populations(), b.populations(0))
    fg, fo = single.fields(), m.fields(s)
    for key in ("ux", "uy", "theta", "c"):
        err = float((fg[key].double().cpu() - fo[key]).abs().max() / fo[key].abs().max())
        print(f"{w['name']} {key}: rel err vs oracle {err:.2e}", flush=True)
        assert err < 1e-4, key
    og = b.observables()[0]
    oo = m.observables(s)
    assert abs(og["current_density"] / float(oo["current_density"]) - 1) < 1e-4


def test_full_sweep_64_cases_launch_shape():
    """The 64-case sweep in the launch shape the benchmark times (autotuned):
    a short run, every case finite, two cases equal to single contexts."""
    lbm = _lbm()
    cases = W.batched_cases()
    b = lbm.BatchedSweep(cases)
    res = b.autotune(trial_steps=3)
    print("autotuned schedule:", res, flush=True)
    b.step(20)
    obs = b.observables()
    assert all(np.isfinite(o["current_density"]) and o["current_density"] > 0 for o in obs)
    for i in (0, 37):
        single = lbm.Cathode.from_workload(cases[i])
        single.step(20)
        assert torch.equal(b.populations(i), single.populations()), i


def _perturbed_fields(lbm, w, gen, which):
    """Per-cell fields for a case: its layer-derived ones (as a context with
    independent_fields = 1 holds them) scaled by seeded factors in the porous
    rows; `which` names the ones returned."""
    base = {k: v.double().cpu() for k, v in lbm.Cathode.from_workload(w, independent_fields=1).material().items()}
    ny, nx = w["ny"], w["nx"]
    porous = torch.zeros(ny, nx, dtype=torch.bool)
    porous[w["ny_channel"]:] = True

    def factor(lo, hi):
        return lo + (hi - lo) * torch.rand(ny, nx, generator=gen, dtype=torch.float64)

    out = {"phi": torch.where(porous, (base["phi"] * factor(0.85, 1.15)).clamp(0.3, 0.95), base["phi"]),
           "inv_k": torch.where(porous, base["inv_k"] * factor(0.5, 2.0), base["inv_k"]),
           "d_eff": torch.where(porous, base["d_eff"] * factor(0.8, 1.0), base["d_eff"])}
    return {k: out[k] for k in which}


@pytest.mark.parametrize("sched,precision", [((128, 1, 0, 0), 32), ((256, 1, 1, 0), 32), ((64, 4, 0, 0), 32),
                                             ((256, 1, 0, 0), 64), ((128, 2, 1, 0), 64), ((64, 12, 0, 960), 32),
                                             ((64, 12, 0, 960), 64)])
def test_cases_with_per_cell_fields_equal_single_contexts_bitwise(sched, precision):
    """A batch whose cases carry per-cell fields (LBM_CELL_FIELDS): case 0
    gets porosity, 1/K and D_eff, case 1 porosity only, case 2 none (derived
    from its layers).  Each equals a single context with independent_fields
    = 1 given the same arrays, bit for bit, under per-step and persistent
    schedules."""
    lbm = _lbm()
    cases = [dict(w, precision=precision) for w in _cases(3)]
    gen = torch.Generator().manual_seed(2103)
    fields = [_perturbed_fields(lbm, cases[0], gen, ("phi", "inv_k", "d_eff")),
              _perturbed_fields(lbm, cases[1], gen, ("phi",)), None]
    b = lbm.BatchedSweep(cases, fields=fields)
    b.step(10)
    b.autotune(trial_steps=2)  # trials from the live state, restored after (fields untouched)
    b.set_schedule(*sched)
    b.step(50)
    obs = b.observables()
    for i, w in enumerate(cases):
        single = lbm.Cathode.from_workload(w, independent_fields=1, **(fields[i] or {}))
        single.step(60)
        assert torch.equal(b.populations(i), single.populations()), (sched, precision, w["name"])
        o = single.observables()
        assert obs[i]["current_density"] == o["current_density"], (sched, precision, w["name"])
        assert obs[i]["heat_rate"] == o["heat_rate"], (sched, precision, w["name"])
        single.close()
    b.close()


def test_per_cell_fields_need_the_flag_and_valid_values():
    """lbm_batch_set_fields refuses a layered batch (LBM_ERR_STATE) and a
    porosity outside (0, 1] (LBM_ERR_UNSTABLE_PARAMS)."""
    lbm = _lbm()
    cases = _cases(2)
    layered = lbm.BatchedSweep(cases)
    with pytest.raises(lbm.LbmError, match="LBM_CELL_FIELDS"):
        layered.set_fields(0, phi=torch.full((cases[0]["ny"], cases[0]["nx"]), 0.5))
    layered.close()
    b = lbm.BatchedSweep(cases, fields=[None, None])
    bad = torch.full((cases[1]["ny"], cases[1]["nx"]), 0.5)
    bad[-1, 3] = 1.5
    with pytest.raises(lbm.LbmError, match="porosity"):
        b.set_fields(1, phi=bad)
    b.close()


def test_two_step_schedule_limits():
    """The two-step form (960-thread workgroups) takes 64 x 12 tiles and no
    persistent launch; a batch with a thin-film CL case and the
    pressure-driven polarisation cases take it and equal their single
    contexts bit for bit over odd step counts."""
    lbm = _lbm()
    cases = _cases(3)
    b = lbm.BatchedSweep(cases)
    for bad in ((64, 8, 0, 960), (128, 12, 0, 960), (64, 12, 1, 960)):
        with pytest.raises(lbm.LbmError, match="invalid argument"):
            b.set_schedule(*bad)
    b.close()
    thin = dict(cases[0], thin_cl=True, ny_gdl=cases[0]["ny_gdl"] + cases[0]["ny_cl"], ny_cl=0)
    t = lbm.BatchedSweep([thin, cases[1]])
    t.set_schedule(64, 12, 0, 960)
    t.step(21)
    for i, w in enumerate((thin, cases[1])):
        single = lbm.Cathode.from_workload(w)
        single.step(21)
        assert torch.equal(t.populations(i), single.populations()), w["name"]
        single.close()
    t.close()
    pol = W.polarisation_sweep(steps=200)[:4]
    b = lbm.BatchedSweep(pol)
    b.set_schedule(64, 12, 0, 960)
    b.step(33)
    for i, w in enumerate(pol):
        single = lbm.Cathode.from_workload(w)
        single.step(33)
        assert torch.equal(b.populations(i), single.populations()), w["name"]
        single.close()
    b.close()
