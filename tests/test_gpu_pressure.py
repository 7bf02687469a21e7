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


@pytest.mark.parametrize("p_in,p_out", [(2e-3, 0.0), (5e-3, 3e-3)])
def test_pressure_driven_channel_is_exact_poiseuille_on_gpu(p_in, p_out):
    lbm = _lbm()
    nx, H = 40, 9
    w = dict(_case(), nx=nx, ny=H, ny_channel=H, ny_gdl=0, ny_cl=0, p_in=p_in, p_out=p_out, tau_f=1.0)
    gpu = lbm.Cathode.from_workload(w, flags=lbm.LBM_NO_REACTION, dx_cm=1e-3)
    gpu.step(6000)
    f = gpu.fields()
    nu = (1.0 - 0.5) / 3.0
    y = torch.arange(H, dtype=DT)
    exact = (p_in - p_out) / (nx - 1) / (2 * nu) * (y + 0.5) * (H - 0.5 - y)
    err = float((f["ux"].cpu() - exact.view(H, 1)).abs().max() / exact.max())
    x = torch.arange(nx, dtype=DT)
    perr = float((f["p"].cpu() - (p_in + (p_out - p_in) * x / (nx - 1))).abs().max())
    print(f"pressure-driven Poiseuille on GPU: rel err {err:.1e}, pressure err {perr:.1e}", flush=True)
    assert err < 1e-12 and perr < 1e-13


@pytest.mark.parametrize("mode", ["layered", "phi", "full"])
@pytest.mark.parametrize("precision", [64, 32])
def test_one_step_from_arbitrary_state_pressure_inlet(mode, precision):
    lbm = _lbm()
    nx, ny, layers = 203, 37, (18, 15, 4)
    w = _case(precision, nx=nx, ny=ny, ny_channel=layers[0], ny_gdl=layers[1], ny_cl=layers[2], p_in=3e-3, p_out=1e-3)
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
        e = float((fg[key].cpu() - fo[key]).abs().max() / fo[key].abs().max())
        print(f"pressure {key}: rel err {e:.2e}", flush=True)
        assert e < 1e-12, key
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


def test_polarisation_sweep_trends():
    """Section 5 trends on the 39-case sweep after 30000 steps: from 0.6 V up
    the current density falls with the voltage (kinetic region); below it
    the curve flattens at a transport-limited plateau; at every voltage up
    to 0.55 V the current rises with the flow rate (lower outlet pressure)."""
    lbm = _lbm()
    cases = W.polarisation_sweep()
    b = lbm.BatchedSweep(cases)
    b.autotune(trial_steps=5)
    b.step(30000)
    obs = b.observables()
    I = np.array([o["current_density"] for o in obs]).reshape(len(W.POLARISATION_P_OUT), -1)
    flux = np.array([o["inlet_flux"] for o in obs]).reshape(len(W.POLARISATION_P_OUT), -1)
    print("I(V) per outlet pressure:", np.array2string(I, precision=3), flush=True)
    v = np.array(W.POLARISATION_V)
    kinetic, plateau = v >= 0.599, v <= 0.551
    assert np.all(np.diff(I[:, kinetic], axis=1) < 0)              # voltages ascend along axis 1
    assert np.all(I[:, plateau].min(1) > 0.9 * I.max(1))            # mass-transport plateau
    assert np.all(np.diff(I[:, plateau], axis=0) > 0)               # more flow, more current
    assert np.all(np.diff(flux[:, 0]) > 0)                           # larger pressure drop, more flow


def test_section5_parameter_trends():
    """Section 5 trends at 0.5 V (mid flow rate, 30000 steps, one batch):
    the current density rises with the operating temperature and with the
    GDL O2 diffusivity, hardly changes with the GDL porosity at fixed
    diffusivity, and changes far less than the permeability; at low
    voltage the CL O2 concentration and the local current fall toward the
    outlet."""
    lbm = _lbm()
    base = dict(W.polarisation_sweep()[len(W.POLARISATION_V) + 4], deff_ratio_gdl=0.4 ** 1.5)
    assert base["V_op"] == 0.5 and base["p_out"] == W.POLARISATION_P_OUT[1]
    variants = [{}, dict(T_in=323.0), dict(T_in=373.0), dict(deff_ratio_gdl=0.5 * 0.4 ** 1.5),
                dict(deff_ratio_gdl=2 * 0.4 ** 1.5), dict(phi_gdl=0.3), dict(phi_gdl=0.6),
                dict(Da_gdl=0.1 * base["Da_gdl"]), dict(Da_gdl=10 * base["Da_gdl"])]
    b = lbm.BatchedSweep([dict(base, **v) for v in variants])
    b.step(30000)
    I = [o["current_density"] for o in b.observables()]
    print("I:", np.round(I, 4), flush=True)
    i0, t323, t373, dlo, dhi, plo, phi_hi, klo, khi = I
    assert t323 < i0 < t373
    assert dlo < i0 < dhi
    assert abs(plo / i0 - 1) < 0.05 and abs(phi_hi / i0 - 1) < 0.05
    assert abs(klo / i0 - 1) < 0.1 and abs(khi / i0 - 1) < 0.5       # 100x in K
    s = lbm.Cathode.from_workload(base)
    s.step(30000)
    o = s.observables()
    n = len(o["c_profile"])
    head, tail = slice(1, n // 10), slice(n - n // 10, n - 1)
    assert o["c_profile"][head].mean() > o["c_profile"][tail].mean()
    assert o["i_profile"][head].mean() > o["i_profile"][tail].mean()


def test_3d_rejects_an_outlet_pressure():
    lbm = _lbm()
    w3 = W.cathode3d_scaled(16, 6, 10, precision=64, sphere_radius=1.5, filter_box=3, Re=1.0)
    with pytest.raises(lbm.LbmError, match="p_outlet"):
        lbm.Cathode3D.from_workload(dict(w3, p_out=1e-3))
