"""3D solver (D3Q19 + 2 x D3Q7, C ABI lbm3d_*) against the FP64 3D oracle.

Tolerances as in 2D: FP64 kernels 1e-12 relative on fields and observables
(populations 1e-13 absolute after one step); FP32 kernels 1e-4 relative on
velocity, temperature and O2.  Inputs are seeded and synthetic
(``workloads``), FP32 cases feed both sides the same rounded inputs.
"""
import numpy as np
import pytest
import torch

import workloads as W
from oracle import lbm3d as L3

pytestmark = pytest.mark.gpu

DT = torch.float64
OBS_KEYS = ("current_density", "power_density", "heat_rate", "o2_utilisation", "T_max", "sum_f", "sum_theta",
            "sum_c", "consumed_c", "heat_added")


def _lbm():
    from paper_2103_01444_amd import lbm
    return lbm


def _r32(a):
    return None if a is None else a.astype(np.float32).astype(np.float64)


def rel(a, b):
    a = torch.as_tensor(a, dtype=DT).cpu()
    b = torch.as_tensor(b, dtype=DT).cpu()
    s = float(b.abs().max())
    return float((a - b).abs().max()) / (s if s > 0 else 1.0)


def oracle3(w, phi=None, inv_k=None, d_eff=None, flags=0, **over):
    g = L3.geometry_from_workload(w, periodic_x=bool(flags & 1), periodic_y=bool(flags & 2),
                                  periodic_z=bool(flags & 16))
    p = L3.params_from_workload(w)
    for k, v in over.items():
        setattr(p, k, v)
    t = lambda a: None if a is None else torch.as_tensor(a, dtype=DT)
    return L3.Model3D(g, p, phi=t(phi), inv_k=t(inv_k), d_eff=t(d_eff))


def compare_fields3(fg, fo, tol, label=""):
    us = max(float(fo[k].abs().max()) for k in ("ux", "uy", "uz"))
    eu = max(float((fg[k].double().cpu() - fo[k]).abs().max()) for k in ("ux", "uy", "uz")) / us
    th = fg["theta"].double().cpu()
    eth = rel(th, fo["theta"]) if float(fo["theta"].abs().max()) > 0 else float(th.abs().max())
    eT, ec = rel(fg["T"], fo["T"]), rel(fg["c"], fo["c"])
    print(f"{label} rel err: u {eu:.2e} theta {eth:.2e} T {eT:.2e} c {ec:.2e}", flush=True)
    assert eu < tol and eth < tol and eT < tol and ec < tol, (eu, eth, eT, ec)


def _case(nx, ny, nz, layers, mode, precision, seed, flags=0, bfx=0.0, bfy=0.0, **over):
    lbm = _lbm()
    w = W.cathode3d_scaled(nx, ny, nz, precision=precision, nz_channel=layers[0], nz_gdl=layers[1],
                           nz_cl=layers[2], Re=0.2 * max(layers[0], 1), **over)
    rng = np.random.default_rng(seed)
    phi = inv_k = d_eff = None
    if mode in ("phi", "full"):
        phi = np.ones((nz, ny, nx))
        phi[layers[0]:] = rng.uniform(0.3, 0.9, size=(nz - layers[0], ny, nx))
    else:
        w["dp_lat"] = 0.0
        w["Da_gdl"] = 1e-3
    if mode == "full":
        inv_k = np.zeros((nz, ny, nx))
        inv_k[layers[0]:] = rng.uniform(0.0, 2.0, size=(nz - layers[0], ny, nx))
        d_eff = rng.uniform(0.001, 0.02, size=(nz, ny, nx))
    if precision == 32:
        phi, inv_k, d_eff = _r32(phi), _r32(inv_k), _r32(d_eff)
    pops = W.random_populations3d(nz, ny, nx, seed + 1)
    if precision == 32:
        pops = _r32(pops)
    gpu = lbm.Cathode3D.from_workload(w, phi=phi, inv_k=inv_k, d_eff=d_eff, flags=flags, body_force_x=bfx,
                                      body_force_y=bfy)
    m = oracle3(w, phi, inv_k, d_eff, flags=flags, body_force=(bfx, bfy), reaction=not (flags & 8))
    return gpu, m, torch.from_numpy(pops)


@pytest.mark.parametrize("mode", ["layered", "phi", "full"])
@pytest.mark.parametrize("precision", [64, 32])
@pytest.mark.parametrize("shape", [(21, 7, 10, (4, 4, 2)), (300, 5, 6, (3, 2, 1)), (5, 3, 4, (2, 1, 1))])
def test_one_step_from_arbitrary_state_3d(mode, precision, shape):
    """One update of an arbitrary state: every population of every node,
    inlet, outlet, walls and a ragged x tile (nx = 300) included."""
    nx, ny, nz, layers = shape
    gpu, m, pops = _case(nx, ny, nz, layers, mode, precision, seed=300 + nx)
    gpu.set_populations(pops)
    compare_fields3(gpu.fields(), m.fields(pops), 1e-12 if precision == 64 else 1e-4,
                    f"3d fields {mode} fp{precision} {nx}x{ny}x{nz}")
    gpu.step(1)
    out = gpu.populations().double().cpu()
    ref = m.step(pops)
    err = float((out - ref).abs().max())
    print(f"3d one step {mode} fp{precision} {nx}x{ny}x{nz}: max |df| = {err:.2e}", flush=True)
    # FP32: rounding (6e-8) of populations up to ~2, amplified ~50x by the
    # Arrhenius / Tafel exponent of the CL source (an argument of ~50 whose
    # absolute FP32 error sets the relative error of the rate constant).
    assert err < (1e-13 if precision == 64 else 1e-5 * float(ref.abs().max()))


@pytest.mark.parametrize("flags", [1 | 2 | 16 | 4, 1 | 4 | 8, 2 | 16])
def test_one_step_periodic_and_body_force_modes_3d(flags):
    gpu, m, pops = _case(12, 6, 8, (4, 3, 1), "phi", 64, seed=77 + flags, flags=flags,
                         bfx=2e-5 if flags & 4 else 0.0, bfy=-1e-5 if flags & 4 else 0.0)
    gpu.set_populations(pops)
    gpu.step(1)
    err = float((gpu.populations().double().cpu() - m.step(pops)).abs().max())
    print(f"3d flags {flags}: max |df| = {err:.2e}", flush=True)
    assert err < 1e-13


def test_fp64_cathode3d_run_and_observables():
    """A 48x10x12 FP64 cathode (sphere pack of radius 2, 5^3 filter) from
    equilibrium over 400 steps: fields and every observable."""
    lbm = _lbm()
    w = W.cathode3d_scaled(48, 10, 12, precision=64, sphere_radius=2.0, filter_box=5, Re=2.0)
    phi = W.sphere_pack_porosity(w)
    gpu = lbm.Cathode3D.from_workload(w, phi=phi)
    m = oracle3(w, phi)
    s = m.initial_state()
    for chunk in (150, 250):
        gpu.step(chunk)
        s = m.run(s, chunk)
        fo = m.fields(s)
        fg = gpu.fields()
        compare_fields3(fg, fo, 1e-12, f"3d fp64 step {gpu.step_count}")
        ep = rel(fg["p"], fo["p"])
        print(f"3d fp64 step {gpu.step_count} p rel err {ep:.2e}", flush=True)
        assert ep < 1e-12
    og, oo = gpu.observables(), m.observables(s)
    for key in OBS_KEYS:
        e = abs(og[key] - float(oo[key])) / abs(float(oo[key]))
        print(f"3d obs {key}: gpu {og[key]:.12e} oracle {float(oo[key]):.12e} rel {e:.1e}", flush=True)
        assert e < 1e-12, key


def test_fp32_sphere_pack_run_64x16x16():
    lbm = _lbm()
    w = W.cathode3d_scaled(64, 16, 16, precision=32, sphere_radius=2.0, filter_box=5, Re=3.0)
    phi = _r32(W.sphere_pack_porosity(w))
    gpu = lbm.Cathode3D.from_workload(w, phi=phi)
    m = oracle3(w, phi)
    gpu.step(300)
    s = m.run(m.initial_state(), 300)
    compare_fields3(gpu.fields(), m.fields(s), 1e-4, "3d fp32 64x16x16 step 300")
    og, oo = gpu.observables(), m.observables(s)
    for key in ("current_density", "o2_utilisation", "T_max", "sum_c"):
        e = abs(og[key] - float(oo[key])) / abs(float(oo[key]))
        print(f"3d fp32 obs {key}: rel {e:.1e}", flush=True)
        assert e < 1e-4, key


def test_material_export_matches_oracle_3d():
    lbm = _lbm()
    w = W.cathode3d_scaled(40, 8, 12, precision=64, sphere_radius=2.0, filter_box=5, Re=2.0)
    phi = W.sphere_pack_porosity(w)
    gpu = lbm.Cathode3D.from_workload(w, phi=phi)
    m = oracle3(w, phi)
    mat = gpu.material()
    assert rel(mat["phi"], m.phi) < 1e-15
    assert rel(mat["inv_k"], m.inv_k) < 1e-13
    assert rel(mat["d_eff"], m.d_eff) < 1e-13


# ------------------------------------------------ full size, bench launch shape
def _full3():
    w = W.cathode3d_256x128x64()
    return w, _r32(W.sphere_pack_porosity(w))


def test_full_size_3d_one_step_from_arbitrary_state():
    """256x128x64 FP32 sphere pack: one update of an arbitrary state over
    the whole lattice (the kernel and launch order the benchmark times)."""
    lbm = _lbm()
    w, phi = _full3()
    pops = _r32(W.random_populations3d(w["nz"], w["ny"], w["nx"], 4343))
    gpu = lbm.Cathode3D.from_workload(w, phi=phi)
    gpu.set_populations(torch.from_numpy(pops))
    gpu.step(1)
    out = gpu.populations().double().cpu()
    del gpu
    ref = oracle3(w, phi).step(torch.from_numpy(pops))
    err = float((out - ref).abs().max())
    print(f"3d full size one step: max |df| = {err:.2e}", flush=True)
    assert err < 2e-6


def test_full_size_3d_inlet_and_outlet_windows():
    """256x128x64 FP32 from equilibrium for 16 steps; 12-column windows at
    the inlet and the outlet against light-cone oracle runs over all (y, z)."""
    lbm = _lbm()
    w, phi = _full3()
    n = 16
    gpu = lbm.Cathode3D.from_workload(w, phi=phi)
    gpu.step(n)
    fg = {k: v.double().cpu() for k, v in gpu.fields().items()}
    del gpu
    dx = oracle3(w, phi).dx
    h = 2 * n + 2
    for x0 in (0, w["nx"] - 12):
        xa, xb = max(0, x0 - h), min(w["nx"], x0 + 12 + h)
        ww = dict(w, nx=xb - xa)
        m = oracle3(ww, phi[..., xa:xb], dx_cm=dx)
        fo = m.fields(m.run(m.initial_state(), n))
        for key in ("ux", "uy", "uz", "c", "T", "theta"):
            a = fg[key][..., x0:x0 + 12]
            b = fo[key][..., x0 - xa:x0 - xa + 12]
            e = float((a - b).abs().max()) / max(float(b.abs().max()), 1e-12)
            print(f"3d window x0={x0} {key}: rel {e:.2e}", flush=True)
            assert e < 1e-4, (x0, key, e)


def test_full_size_3d_run_stays_bounded():
    """The 5000-step 256x128x64 run: finite observables, O2 between 0 and
    its inlet value times the largest diffusivity ratio, temperature rise
    non-negative."""
    lbm = _lbm()
    w, phi = _full3()
    gpu = lbm.Cathode3D.from_workload(w, phi=phi)
    gpu.step(w["steps"])
    o = gpu.observables()
    f = gpu.fields()
    print(f"3d 5000 steps: I = {o['current_density']:.4e} A/cm^2, T_max = {o['T_max']:.3f} K, "
          f"util = {o['o2_utilisation']:.3e}", flush=True)
    assert o["current_density"] > 0 and o["T_max"] >= w["T_in"]
    assert float(f["c"].min()) >= 0.0
    assert float(f["theta"].min()) > -1e-6 * float(f["theta"].max())  # FP32 rounding of a non-negative field


def test_parameter_validation_3d():
    lbm = _lbm()
    w = W.cathode3d_scaled(32, 8, 12, precision=32, sphere_radius=2.0, filter_box=5)
    for over in (dict(tau_f=0.5), dict(D_f_lat=0.2), dict(Re=60.0)):
        with pytest.raises(lbm.LbmError, match="stable range"):
            lbm.Cathode3D.from_workload(w, **over)
    phi = np.ones((12, 8, 32))
    phi[8, 3, 3] = 0.0
    with pytest.raises(lbm.LbmError, match="stable range"):
        lbm.Cathode3D.from_workload(w, phi=phi)
