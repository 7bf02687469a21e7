"""Thin-film catalyst layer (LBM_THIN_CL: a reactive wall under the GDL, the
paper's CL of negligible thickness) on the GPU against the FP64 oracle:
one step of arbitrary states in every material mode, FP64 runs with every
observable and the CL profiles, and the batched solver.  The adjoint with
the film is tested with the other adjoint parity cases."""
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


def _thin(w, **over):
    """A workload with its CL rows turned into GDL rows and a film below."""
    w = dict(w, thin_cl=True, **over)
    w["ny_gdl"] += w["ny_cl"]
    w["ny_cl"] = 0
    return w


@pytest.mark.parametrize("mode", ["layered", "phi", "full"])
@pytest.mark.parametrize("precision", [64, 32])
def test_one_step_thin_cl(mode, precision):
    lbm = _lbm()
    nx, ny, layers = 203, 37, (18, 19, 0)
    w = _thin(dict(W.cathode2d_200x40(), nx=nx, ny=ny, ny_channel=layers[0], ny_gdl=layers[1], ny_cl=layers[2],
                   precision=precision, Re=4.0, V_op=0.45), thin_cl_cm=3e-4)
    rng = np.random.default_rng(1000 + precision)
    phi = inv_k = d_eff = None
    if mode != "layered":
        phi = np.ones((ny, nx))
        phi[layers[0]:] = rng.uniform(0.4, 0.8, size=(ny - layers[0], nx))
        w["dp_over_hgdl"] = 0.3325
    if mode == "full":
        inv_k = np.zeros((ny, nx))
        inv_k[layers[0]:] = rng.uniform(0.0, 2.0, size=(ny - layers[0], nx))
        d_eff = rng.uniform(0.001, 0.02, size=(ny, nx))
    pops = W.random_populations(ny, nx, 1010 + precision)
    if precision == 32:
        phi, inv_k, d_eff, pops = _r32(phi), _r32(inv_k), _r32(d_eff), _r32(pops)
    gpu = lbm.Cathode.from_workload(w, phi=phi, inv_k=inv_k, d_eff=d_eff)
    t = lambda a: None if a is None else torch.as_tensor(a, dtype=DT)
    m = L.Model(L.geometry_from_workload(w), L.Params.from_workload(w), phi=t(phi), inv_k=t(inv_k), d_eff=t(d_eff))
    assert m.p.thin_cl and m.thin == 3e-4
    pops = torch.from_numpy(pops)
    d_c, *_ = m.surface_reaction(pops)
    assert float(d_c.min()) > 1e-3  # the film takes a visible share of the crossing O2
    gpu.set_populations(pops)
    gpu.step(1)
    out = gpu.populations().double().cpu()
    ref = m.step(pops)
    err = float((out - ref).abs().max())
    print(f"thin CL one step {mode} fp{precision}: max |df| = {err:.2e}", flush=True)
    assert err < (1e-13 if precision == 64 else 1e-5 * float(ref.abs().max()))


@pytest.mark.parametrize("butler_volmer", [False, True])
def test_fp64_thin_cl_run_observables_and_profiles(butler_volmer):
    lbm = _lbm()
    over = dict(butler_volmer=True, alpha_a=0.5, V_op=1.1, aj0_ref=1e5) if butler_volmer else dict(V_op=0.5)
    w = _thin(dict(W.cathode2d_200x40(), nx=60, ny=20, ny_channel=10, ny_gdl=8, ny_cl=2, precision=64, Re=3.0),
              **over)
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
    for key in ("current_density", "heat_rate", "o2_utilisation", "consumed_c", "heat_added", "sum_c", "T_max"):
        ref = float(oo[key])
        e = abs(og[key] - ref) / abs(ref)
        print(f"thin CL obs {key}: gpu {og[key]:.12e} oracle {ref:.12e} rel {e:.1e}", flush=True)
        assert e < 1e-12, key
    for g, o in (("i_profile", "i_profile"), ("c_profile", "c_profile"), ("T_profile", "T_profile")):
        ref = oo[o].numpy()
        assert np.abs(og[g] - ref).max() / np.abs(ref).max() < 1e-12, g
    assert og["i_profile"][1] > og["i_profile"][-2] > 0  # O2 is used up along the film


def test_thin_cl_case_in_a_batch_equals_its_single_context():
    lbm = _lbm()
    cases = [dict(c) for c in W.batched_cases(3)]
    cases[2] = _thin(cases[2])
    b = lbm.BatchedSweep(cases)
    b.set_schedule(256, 1, 0)
    b.step(120)
    obs = b.observables()
    for i, w in enumerate(cases):
        s = lbm.Cathode.from_workload(w)
        s.step(120)
        assert torch.equal(b.populations(i), s.populations()), w["name"]
        assert s.observables()["current_density"] == obs[i]["current_density"]
