"""The pressure-driven inlet (LBM_PRESSURE_INLET, Section 4's pressure
difference between inlet and outlet) on the GPU against the FP64 oracle, in
single contexts and in the batched sweep, and the polarisation sweep that
uses it (the Section 5 trends)."""
import numpy as np
import pytest
import torch

import workloads as W
from oracle import lbm2d as L

pytestmark = pytest.mark.gpu
DT = torch.float64


def _lbm():
    from paper_2103_01444_amd import lbm
    return lbm


def _case(precision=64, **over):
    w = W.polarisation_sweep()[5]
    w = dict(w, precision=precision)
    w.update(over)
    return w


def test_pressure_driven_channel_is_exact_poiseuille_on_gpu():
    lbm = _lbm()
    nx, H, p_in = 40, 9, 2e-3
    w = dict(_case(), nx=nx, ny=H, ny_channel=H, ny_gdl=0, ny_cl=0, p_in=p_in, tau_f=1.0)
    gpu = lbm.Cathode.from_workload(w, flags=lbm.LBM_NO_REACTION, dx_cm=1e-3)
    gpu.step(6000)
    f = gpu.fields()
    nu = (1.0 - 0.5) / 3.0
    y = torch.arange(H, dtype=DT)
    exact = p_in / (nx - 1) / (2 * nu) * (y + 0.5) * (H - 0.5 - y)
    err = float((f["ux"].cpu() - exact.view(H, 1)).abs().max() / exact.max())
    print(f"pressure-driven Poiseuille on GPU: rel err {err:.1e}", flush=True)
    assert err < 1e-11


@pytest.mark.parametrize("mode", ["layered", "phi", "full"])
@pytest.mark.parametrize("precision", [64, 32])
def test_one_step_from_arbitrary_state_pressure_inlet(mode, precision):
    lbm = _lbm()
    nx, ny, layers = 203, 37, (18, 15, 4)
    w = _case(precision, nx=nx, ny=ny, ny_channel=layers[0], ny_gdl=layers[1], ny_cl=layers[2], p_in=3e-3)
    rng = np.random.default_rng(500 + precision)
    phi = inv_k = d_eff = None
    if mode != "layered":
        phi = np.ones((ny, nx))
        phi[layers[0]:] = rng.uniform(0.4, 0.8, size=(ny - layers[0], nx))
        w["dp_over_hgdl"] = 0.3325
    if mode == "full":
        inv_k = np.zeros((ny, nx))
        inv_k[layers[0]:] = rng.uniform(0.0, 2.0, size=(ny - layers[0], nx))
        d_eff = rng.uniform(0.001, 0.02, size=(ny, nx))
    pops = W.random_populations(ny, nx, 700 + precision)
    if precision == 32:
        r = lambda a: None if a is None else a.astype(np.float32).astype(np.float64)
        phi, inv_k, d_eff, pops = r(phi), r(inv_k), r(d_eff), r(pops)
    gpu = lbm.Cathode.from_workload(w, phi=phi, inv_k=inv_k, d_eff=d_eff)
    t = lambda a: None if a is None else torch.as_tensor(a, dtype=DT)
    m = L.Model(L.geometry_from_workload(w), L.Params.from_workload(w), phi=t(phi), inv_k=t(inv_k), d_eff=t(d_eff))
    pops = torch.from_numpy(pops)
    gpu.set_populations(pops)
    gpu.step(1)
    out = gpu.populations().double().cpu()
    ref = m.step(pops)
    err = float((out - ref).abs().max())
    print(f"pressure inlet one step {mode} fp{precision}: max |df| = {err:.2e}", flush=True)
    assert err < (1e-13 if precision == 64 else 1e-5 * float(ref.abs().max()))


def test_fp64_pressure_driven_cathode_run_and_observables():
    lbm = _lbm()
    w = _case(64)
    gpu = lbm.Cathode.from_workload(w)
    m = L.Model(L.geometry_from_workload(w), L.Params.from_workload(w))
    s = m.initial_state()
    for chunk in (400, 600):
        gpu.step(chunk)
        s = m.run(s, chunk)
    fg, fo = gpu.fields(), m.fields(s)
    us = max(float(fo["ux"].abs().max()), float(fo["uy"].abs().max()))
    for key in ("ux", "uy"):
        assert float((fg[key].cpu() - fo[key]).abs().max()) / us < 1e-12, key
    for key in ("p", "theta", "c"):
        assert float((fg[key].cpu() - fo[key]).abs().max() / fo[key].abs().max()) < 1e-11, key
    og, oo = gpu.observables(), m.observables(s)
    for key in ("current_density", "heat_rate", "o2_utilisation", "inlet_flux", "T_max", "sum_c", "consumed_c"):
        ref = float(oo[key])
        e = abs(og[key] - ref) / abs(ref)
        print(f"pressure obs {key}: gpu {og[key]:.12e} oracle {ref:.12e} rel {e:.1e}", flush=True)
        assert e < 1e-12, key


def test_pressure_and_velocity_cases_in_one_batch_equal_single_contexts():
    lbm = _lbm()
    cases = [dict(c, nx=96) for c in W.polarisation_sweep()[::6]]
    vel = dict(W.batched_cases(2)[0])
    cases.append(vel)
    b = lbm.BatchedSweep(cases)
    b.set_schedule(256, 1, 0)
    b.step(150)
    obs = b.observables()
    for i, w in enumerate(cases):
        s = lbm.Cathode.from_workload(w)
        s.step(150)
        assert torch.equal(b.populations(i), s.populations()), w["name"]
        o = s.observables()
        assert o["inlet_flux"] == obs[i]["inlet_flux"] and o["o2_utilisation"] == obs[i]["o2_utilisation"]


def test_adjoint_rejects_the_pressure_inlet():
    lbm = _lbm()
    w = _case(64, nx=40, ny=10, ny_channel=5, ny_gdl=4, ny_cl=1)
    sim = lbm.Cathode.from_workload(w, independent_fields=1)
    with pytest.raises(lbm.LbmError, match="PRESSURE_INLET"):
        sim.forward_checkpointed(10, 5)


def test_polarisation_sweep_trends():
    """Section 5 trends on the 39-case sweep after 6000 steps: the current
    density rises as the voltage falls, and at low voltage it rises with
    the flow rate (inlet pressure)."""
    lbm = _lbm()
    cases = W.polarisation_sweep()
    b = lbm.BatchedSweep(cases)
    b.autotune(trial_steps=5)
    b.step(6000)
    I = np.array([o["current_density"] for o in b.observables()]).reshape(len(W.POLARISATION_P_IN), -1)
    flux = np.array([o["inlet_flux"] for o in b.observables()]).reshape(len(W.POLARISATION_P_IN), -1)
    print("I(V) per inlet pressure:", np.array2string(I, precision=3), flush=True)
    assert np.all(np.diff(I, axis=1) < 0)          # voltages ascend along axis 1
    assert np.all(np.diff(I[:, 0]) > 0)            # more flow, more current at 0.30 V
    assert np.all(np.diff(flux[:, 0]) > 0)         # more pressure, more flow
