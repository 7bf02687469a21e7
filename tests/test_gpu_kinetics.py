"""Butler-Volmer kinetics (lbm_params.kinetics = LBM_KINETICS_BUTLER_VOLMER,
Eq. 13 with its anodic branch) on the GPU against the FP64 oracle: one
step of arbitrary states (2D and 3D, every material mode), FP64 runs with
their observables near the equilibrium potential where the anodic branch
matters, and the batched solver.  The adjoint with these kinetics is
tested with the other adjoint parity cases."""
import numpy as np
import pytest
import torch

import workloads as W
from oracle import lbm2d as L

pytestmark = pytest.mark.gpu
DT = torch.float64
# Near the equilibrium potential (U0 = 1.115 V at 353 K) both branches are
# of the same size (c_eq = 0.47 at 1.1 V); alpha_a 0.5 differs from the
# default, and a j0 raised 1e9-fold makes the reaction move c by a few
# percent per step so that a wrong term shows in one step.
BV = dict(butler_volmer=True, alpha_a=0.5, V_op=1.1, aj0_ref=1e5)


def _lbm():
    from paper_2103_01444_amd import lbm
    return lbm


def _r32(a):
    return None if a is None else a.astype(np.float32).astype(np.float64)


@pytest.mark.parametrize("mode", ["layered", "phi", "full"])
@pytest.mark.parametrize("precision", [64, 32])
def test_one_step_butler_volmer_2d(mode, precision):
    lbm = _lbm()
    nx, ny, layers = 131, 23, (10, 9, 4)
    w = dict(W.cathode2d_200x40(), nx=nx, ny=ny, ny_channel=layers[0], ny_gdl=layers[1], ny_cl=layers[2],
             precision=precision, Re=4.0, **BV)
    rng = np.random.default_rng(900 + precision)
    phi = inv_k = d_eff = None
    if mode != "layered":
        phi = np.ones((ny, nx))
        phi[layers[0]:] = rng.uniform(0.4, 0.8, size=(ny - layers[0], nx))
        w["dp_over_hgdl"] = 0.3325
    if mode == "full":
        inv_k = np.zeros((ny, nx))
        inv_k[layers[0]:] = rng.uniform(0.0, 2.0, size=(ny - layers[0], nx))
        d_eff = rng.uniform(0.001, 0.02, size=(ny, nx))
    pops = W.random_populations(ny, nx, 910 + precision)
    if precision == 32:
        phi, inv_k, d_eff, pops = _r32(phi), _r32(inv_k), _r32(d_eff), _r32(pops)
    gpu = lbm.Cathode.from_workload(w, phi=phi, inv_k=inv_k, d_eff=d_eff)
    t = lambda a: None if a is None else torch.as_tensor(a, dtype=DT)
    m = L.Model(L.geometry_from_workload(w), L.Params.from_workload(w), phi=t(phi), inv_k=t(inv_k), d_eff=t(d_eff))
    assert m.p.butler_volmer and m.p.alpha_a == 0.5
    pops = torch.from_numpy(pops)
    gpu.set_populations(pops)
    gpu.step(1)
    out = gpu.populations().double().cpu()
    ref = m.step(pops)
    err = float((out - ref).abs().max())
    print(f"Butler-Volmer one step {mode} fp{precision}: max |df| = {err:.2e}", flush=True)
    assert err < (1e-13 if precision == 64 else 1e-5 * float(ref.abs().max()))


def test_fp64_butler_volmer_run_and_observables():
    """60x20 FP64 cathode at 1.1 V over 600 steps: O2 is produced where the
    anodic branch wins and consumed elsewhere; fields and observables
    against the oracle."""
    lbm = _lbm()
    w = dict(W.cathode2d_200x40(), nx=60, ny=20, ny_channel=10, ny_gdl=8, ny_cl=2, precision=64, Re=3.0, **BV)
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
    for key in ("current_density", "heat_rate", "consumed_c", "heat_added", "sum_c"):
        ref = float(oo[key])
        e = abs(og[key] - ref) / abs(ref)
        print(f"BV obs {key}: gpu {og[key]:.12e} oracle {ref:.12e} rel {e:.1e}", flush=True)
        assert e < 1e-12, key


def test_one_step_butler_volmer_3d():
    from test_gpu_3d import _case
    gpu, m, pops = _case(13, 5, 8, (3, 3, 2), "phi", 64, seed=950, **BV)
    assert m.p.butler_volmer
    gpu.set_populations(pops)
    gpu.step(1)
    err = float((gpu.populations().double().cpu() - m.step(pops)).abs().max())
    print(f"Butler-Volmer 3d one step: max |df| = {err:.2e}", flush=True)
    assert err < 1e-13


def test_butler_volmer_case_in_a_batch_equals_its_single_context():
    lbm = _lbm()
    cases = [dict(c) for c in W.batched_cases(3)]
    cases[1].update(BV)
    b = lbm.BatchedSweep(cases)
    b.set_schedule(256, 1, 0)
    b.step(120)
    for i, w in enumerate(cases):
        s = lbm.Cathode.from_workload(w)
        s.step(120)
        assert torch.equal(b.populations(i), s.populations()), w["name"]
