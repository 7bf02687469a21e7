"""Boussinesq buoyancy (LBM_BUOYANCY) on the GPU against the FP64 oracle and
the closed-form buoyant shear wave: one step of arbitrary states in every
material mode (also with the test-mode body force), a buoyant cathode run
with its observables, and the batched solver.  The adjoint with buoyancy
is tested with the other adjoint parity cases."""
import math

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


def _r32(a):
    return None if a is None else a.astype(np.float32).astype(np.float64)


@pytest.mark.parametrize("mode", ["layered", "phi", "full"])
@pytest.mark.parametrize("precision", [64, 32])
@pytest.mark.parametrize("body", [False, True])
def test_one_step_buoyancy(mode, precision, body):
    lbm = _lbm()
    nx, ny, layers = 150, 29, (12, 14, 3)
    w = dict(W.cathode2d_200x40(), nx=nx, ny=ny, ny_channel=layers[0], ny_gdl=layers[1], ny_cl=layers[2],
             precision=precision, Re=4.0, buoyancy=(3e-4, -5e-4))
    rng = np.random.default_rng(1100 + precision)
    phi = inv_k = d_eff = None
    if mode != "layered":
        phi = np.ones((ny, nx))
        phi[layers[0]:] = rng.uniform(0.4, 0.8, size=(ny - layers[0], nx))
        w["dp_over_hgdl"] = 0.3325
    if mode == "full":
        inv_k = np.zeros((ny, nx))
        inv_k[layers[0]:] = rng.uniform(0.0, 2.0, size=(ny - layers[0], nx))
        d_eff = rng.uniform(0.001, 0.02, size=(ny, nx))
    pops = W.random_populations(ny, nx, 1110 + precision)
    if precision == 32:
        phi, inv_k, d_eff, pops = _r32(phi), _r32(inv_k), _r32(d_eff), _r32(pops)
    bf = (2e-5, 1e-5) if body else (0.0, 0.0)
    gpu = lbm.Cathode.from_workload(w, phi=phi, inv_k=inv_k, d_eff=d_eff, flags=lbm.LBM_BODY_FORCE if body else 0,
                                    body_force_x=bf[0], body_force_y=bf[1])
    t = lambda a: None if a is None else torch.as_tensor(a, dtype=DT)
    pr = L.Params.from_workload(w)
    pr.body_force = bf
    assert pr.buoyancy == (3e-4, -5e-4)
    m = L.Model(L.geometry_from_workload(w), pr, phi=t(phi), inv_k=t(inv_k), d_eff=t(d_eff))
    pops = torch.from_numpy(pops)
    gpu.set_populations(pops)
    gpu.step(1)
    out = gpu.populations().double().cpu()
    ref = m.step(pops)
    err = float((out - ref).abs().max())
    print(f"buoyancy one step {mode} fp{precision} body={body}: max |df| = {err:.2e}", flush=True)
    assert err < (1e-13 if precision == 64 else 1e-5 * float(ref.abs().max()))


def test_buoyant_shear_wave_on_gpu():
    """Fully periodic clear box, theta = sin(k x), buoyancy along y: u_y
    grows and decays as the closed form of the coupled diffusion equations
    (the oracle's pin), and FP64 GPU = oracle."""
    lbm = _lbm()
    nx, ny, b = 32, 3, 1e-6
    w = dict(W.cathode2d_200x40(), nx=nx, ny=ny, ny_channel=ny, ny_gdl=0, ny_cl=0, precision=64, buoyancy=(0.0, b))
    flags = lbm.LBM_PERIODIC_X | lbm.LBM_PERIODIC_Y | lbm.LBM_NO_REACTION
    gpu = lbm.Cathode.from_workload(w, flags=flags, dx_cm=1e-3)
    pr = L.Params.from_workload(w)
    pr.reaction, pr.dx_cm = False, 1e-3
    m = L.Model(L.Geometry(nx, ny, ny, 0, 0, periodic_x=True, periodic_y=True), pr)
    k = 2 * math.pi / nx
    x = torch.arange(nx, dtype=DT).view(1, nx).expand(ny, nx)
    z = torch.zeros(ny, nx, dtype=DT)
    s = m.equilibrium_state(z, z, z, torch.sin(k * x), torch.ones(ny, nx, dtype=DT))
    gpu.set_populations(s)
    n = int(0.25 / (m.nu * k * k))
    gpu.step(n)
    s = m.run(s, n)
    fg, fo = gpu.fields(), m.fields(s)
    scale = float(fo["uy"].abs().max())
    e = float((fg["uy"].cpu() - fo["uy"]).abs().max()) / scale
    print(f"shear wave uy rel err {e:.2e}", flush=True)
    assert e < 1e-12
    A = float((fg["uy"].cpu().mean(0) * torch.sin(k * x[0])).sum() * 2 / nx)
    alpha = float(m.alpha[0, 0])
    exact = b * (math.exp(-alpha * k * k * n) - math.exp(-m.nu * k * k * n)) / ((m.nu - alpha) * k * k)
    print(f"shear wave amplitude gpu {A:.6e} closed form {exact:.6e}", flush=True)
    assert abs(A / exact - 1) < 5e-3


def test_fp64_buoyant_cathode_run_and_observables():
    lbm = _lbm()
    w = dict(W.cathode2d_200x40(), nx=60, ny=20, ny_channel=10, ny_gdl=8, ny_cl=2, precision=64, Re=3.0,
             V_op=0.45, buoyancy=(0.0, -2e-4))
    gpu = lbm.Cathode.from_workload(w)
    m = L.Model(L.geometry_from_workload(w), L.Params.from_workload(w))
    s = m.initial_state()
    for chunk in (250, 350):
        gpu.step(chunk)
        s = m.run(s, chunk)
    fg, fo = gpu.fields(), m.fields(s)
    us = max(float(fo["ux"].abs().max()), float(fo["uy"].abs().max()))
    for key in ("ux", "uy"):
        assert float((fg[key].cpu() - fo[key]).abs().max()) / us < 1e-12, key
    for key in ("theta", "c", "p"):
        e = float((fg[key].cpu() - fo[key]).abs().max()) / float(fo[key].abs().max())
        print(f"buoyant {key}: rel err {e:.2e}", flush=True)
        assert e < 1e-12, key
    og, oo = gpu.observables(), m.observables(s)
    for key in ("current_density", "heat_rate", "o2_utilisation", "sum_c", "T_max"):
        ref = float(oo[key])
        e = abs(og[key] - ref) / abs(ref)
        print(f"buoyant obs {key}: gpu {og[key]:.12e} oracle {ref:.12e} rel {e:.1e}", flush=True)
        assert e < 1e-12, key
    # the buoyancy changed the flow: against the same run without it
    ref_w = dict(w)
    del ref_w["buoyancy"]
    plain = lbm.Cathode.from_workload(ref_w)
    plain.step(600)
    assert float((plain.fields()["uy"] - fg["uy"]).abs().max()) > 1e-3 * us


def test_buoyant_case_in_a_batch_equals_its_single_context():
    lbm = _lbm()
    cases = [dict(c) for c in W.batched_cases(3)]
    cases[0]["buoyancy"] = (1e-5, -4e-5)
    b = lbm.BatchedSweep(cases)
    b.set_schedule(256, 1, 0)
    b.step(120)
    for i, w in enumerate(cases):
        s = lbm.Cathode.from_workload(w)
        s.step(120)
        assert torch.equal(b.populations(i), s.populations()), w["name"]
