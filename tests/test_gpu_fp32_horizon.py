"""FP32 parity over the benchmark workloads' full run lengths: the FP32 HIP
path against the FP64 oracle's fields at the end of 10^4 steps (the
4096x1024 recipe at 512x128), 5000 steps (a case of the 64-case sweep, run
in the batched kernel) and 5000 steps (the 3D recipe at 64x32x16).  The
oracle's results are stored by ``tests/golden/make_fp32_horizon.py`` (which
calls only the oracle); the GPU runs here.  Bar: 1e-4 relative on velocity
(against the largest speed), temperature, temperature rise and O2, and on
the current density."""
import json
import os

import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu
GOLD = os.path.join(os.path.dirname(__file__), "golden")
TOL = 1e-4


def _lbm():
    from paper_2103_01444_amd import lbm
    return lbm


def _golden(name):
    d = np.load(os.path.join(GOLD, f"fp32_horizon_{name}.npz"))
    w = json.loads(str(d["workload"]))
    return w, d


def _compare(fg, d, vel, label):
    us = max(float(np.abs(d[k]).max()) for k in vel)
    errs = {"u": max(float(np.abs(fg[k].double().cpu().numpy() - d[k]).max()) for k in vel) / us}
    for key in ("T", "theta", "c"):
        ref = d[key].astype(np.float64)
        errs[key] = float(np.abs(fg[key].double().cpu().numpy() - ref).max()) / float(np.abs(ref).max())
    print(label + " rel err: " + ", ".join(f"{k} {v:.2e}" for k, v in errs.items()), flush=True)
    for k, v in errs.items():
        assert v < TOL, (label, k, v)


def _obs(og, d, label):
    for key in ("current_density", "heat_rate", "T_max"):
        ref = float(d[f"obs_{key}"])
        e = abs(og[key] / ref - 1)
        print(f"{label} {key}: gpu {og[key]:.8e} oracle {ref:.8e} rel {e:.2e}", flush=True)
        assert e < TOL, (label, key)


def test_fp32_cathode2d_512x128_over_10000_steps():
    lbm = _lbm()
    import workloads as W
    w, d = _golden("cathode2d_512x128")
    phi = W.porosity_field(w).astype(np.float32).astype(np.float64)
    print(f"fp32 horizon: {w['nx']}x{w['ny']}, {w['steps']} steps", flush=True)
    gpu = lbm.Cathode.from_workload(w, phi=phi)
    gpu.step(int(w["steps"]))
    _compare(gpu.fields(), d, ("ux", "uy"), "2d 512x128 fp32 10^4 steps")
    _obs(gpu.observables(), d, "2d 512x128 fp32 10^4 steps")


def test_fp32_batched_case_over_5000_steps():
    lbm = _lbm()
    w, d = _golden("batch_case09_256x64")
    steps = int(w["steps"])
    print(f"fp32 horizon: batched {w['name']}, {steps} steps", flush=True)
    b = lbm.BatchedSweep([w])
    b.step(steps)
    ob = b.observables()[0]
    single = lbm.Cathode.from_workload(w)  # computes the fields of the batch's populations
    single.set_populations(b.populations(0), steps)
    _compare(single.fields(), d, ("ux", "uy"), f"batched {w['name']} fp32 {steps} steps")
    _obs(ob, d, f"batched {w['name']} fp32 {steps} steps")


def test_fp32_cathode3d_64x32x16_over_5000_steps():
    lbm = _lbm()
    import workloads as W
    w, d = _golden("cathode3d_64x32x16")
    phi = W.sphere_pack_porosity(w).astype(np.float32).astype(np.float64)
    steps = int(w["steps"])
    print(f"fp32 horizon: 3D {w['nx']}x{w['ny']}x{w['nz']}, {steps} steps", flush=True)
    gpu = lbm.Cathode3D.from_workload(w, phi=phi)
    gpu.step(steps)
    _compare(gpu.fields(), d, ("ux", "uy", "uz"), f"3d {w['nx']}x{w['ny']}x{w['nz']} fp32 {steps} steps")
    _obs(gpu.observables(), d, "3d fp32")
    del gpu
    torch.cuda.empty_cache()
