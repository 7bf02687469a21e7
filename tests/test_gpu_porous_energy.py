"""Porous energy equation with the heat-capacity ratio (LBM_SIGMA_ENERGY)
and the physically signed reaction heat (LBM_PHYSICAL_HEAT) on the GPU
against the FP64 oracle: one step of arbitrary states in every material
mode, an FP64 cathode run with its observables, the 3D heat sign and
the batched solver.  The adjoint with these options is tested with the other
adjoint parity cases."""
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
@pytest.mark.parametrize("heat_physical", [False, True])
def test_one_step_sigma_energy(mode, precision, heat_physical):
    lbm = _lbm()
    nx, ny, layers = 170, 31, (14, 13, 4)
    w = dict(W.cathode2d_200x40(), nx=nx, ny=ny, ny_channel=layers[0], ny_gdl=layers[1], ny_cl=layers[2],
             precision=precision, Re=4.0, V_op=0.45, sigma_energy=True, heat_physical=heat_physical)
    rng = np.random.default_rng(1200 + precision)
    phi = inv_k = d_eff = None
    if mode != "layered":
        phi = np.ones((ny, nx))
        phi[layers[0]:] = rng.uniform(0.4, 0.8, size=(ny - layers[0], nx))
        w["dp_over_hgdl"] = 0.3325
    if mode == "full":
        inv_k = np.zeros((ny, nx))
        inv_k[layers[0]:] = rng.uniform(0.0, 2.0, size=(ny - layers[0], nx))
        d_eff = rng.uniform(0.001, 0.02, size=(ny, nx))
    pops = W.random_populations(ny, nx, 1210 + precision)
    if precision == 32:
        phi, inv_k, d_eff, pops = _r32(phi), _r32(inv_k), _r32(d_eff), _r32(pops)
    gpu = lbm.Cathode.from_workload(w, phi=phi, inv_k=inv_k, d_eff=d_eff)
    t = lambda a: None if a is None else torch.as_tensor(a, dtype=DT)
    m = L.Model(L.geometry_from_workload(w), L.Params.from_workload(w), phi=t(phi), inv_k=t(inv_k), d_eff=t(d_eff))
    assert m.p.sigma_energy and m.p.heat_physical == heat_physical and float(m.sigma.max()) > 100
    pops = torch.from_numpy(pops)
    gpu.set_populations(pops)
    gpu.step(1)
    out = gpu.populations().double().cpu()
    ref = m.step(pops)
    err = float((out - ref).abs().max())
    print(f"sigma energy one step {mode} fp{precision} physical heat {heat_physical}: max |df| = {err:.2e}",
          flush=True)
    # sigma T reaches a few hundred here: relative to the largest population
    assert err < (1e-13 if precision == 64 else 1e-5) * float(ref.abs().max())


@pytest.mark.parametrize("thin", [False, True])
def test_fp64_sigma_energy_cathode_run_and_observables(thin):
    lbm = _lbm()
    w = dict(W.cathode2d_200x40(), nx=60, ny=20, ny_channel=10, ny_gdl=8, ny_cl=2, precision=64, Re=3.0,
             V_op=0.4, sigma_energy=True, heat_physical=True)
    if thin:
        w.update(thin_cl=True, ny_gdl=10, ny_cl=0)
    gpu = lbm.Cathode.from_workload(w)
    m = L.Model(L.geometry_from_workload(w), L.Params.from_workload(w))
    s = m.initial_state()
    for chunk in (250, 350):
        gpu.step(chunk)
        s = m.run(s, chunk)
    fg, fo = gpu.fields(), m.fields(s)
    for key in ("ux", "uy", "theta", "c"):
        scale = float(fo[key].abs().max())
        assert float((fg[key].cpu() - fo[key]).abs().max()) / scale < 1e-12, key
    og, oo = gpu.observables(), m.observables(s)
    for key in ("current_density", "heat_rate", "consumed_c", "heat_added", "sum_theta", "T_max"):
        ref = float(oo[key])
        e = abs(og[key] - ref) / abs(ref)
        print(f"sigma obs {key}: gpu {og[key]:.12e} oracle {ref:.12e} rel {e:.1e}", flush=True)
        assert e < 1e-12, key
    assert og["heat_rate"] > 0 and np.abs(og["T_profile"] - oo["T_profile"].numpy()).max() < 1e-9


def test_physical_heat_3d_one_step():
    from test_gpu_3d import _case
    gpu, m, pops = _case(13, 5, 8, (3, 3, 2), "phi", 64, seed=1250, heat_physical=True, V_op=0.2)
    assert m.p.heat_physical
    gpu.set_populations(pops)
    gpu.step(1)
    err = float((gpu.populations().double().cpu() - m.step(pops)).abs().max())
    print(f"physical heat 3d one step: max |df| = {err:.2e}", flush=True)
    assert err < 1e-13


def test_sigma_case_in_a_batch_equals_its_single_context():
    lbm = _lbm()
    cases = [dict(c) for c in W.batched_cases(3)]
    cases[1].update(sigma_energy=True, heat_physical=True)
    b = lbm.BatchedSweep(cases)
    b.set_schedule(256, 1, 0)
    b.step(120)
    for i, w in enumerate(cases):
        s = lbm.Cathode.from_workload(w)
        s.step(120)
        assert torch.equal(b.populations(i), s.populations()), w["name"]
