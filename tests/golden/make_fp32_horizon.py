"""Write the FP64 oracle's fields and observables at the end of the
configured run lengths, for the FP32 long-horizon GPU parity tests
(``tests/test_gpu_fp32_horizon.py``).  Calls only ``oracle/`` and the seeded
inputs of ``workloads``; run from the repository root:

    python tests/golden/make_fp32_horizon.py            # all cases
    python tests/golden/make_fp32_horizon.py cathode2d  # one case

Cases (each the recipe of a benchmark workload at a size the oracle finishes
in minutes, for the benchmark's full number of steps):

* ``cathode2d_512x128``: the 4096x1024 recipe (per-cell porosity U[0.4,
  0.8], Kozeny-Carman permeability, Re 50, 0.5 V, 343 K) at 512x128, 10^4
  steps.
* ``batch_case09_256x64``: case 9 of the 64-case sweep (256x64, Re 70,
  0.42 V, 352 K; the sweep's fastest flow), 5000 steps.
* ``cathode3d_64x32x16``: the 3D recipe (sphere-pack GDL, Kozeny-Carman
  permeability, 0.55 V, 353 K) at 64x32x16 with the spheres, the filter box
  and the particle diameter scaled down (radius 2, box 5, d_p 4) and Re 5,
  which keeps the full-size lattice velocities (mean inlet speed Re nu / H
  = 0.031), 5000 steps.

The porosity fields are rounded to float32 first, the precision in which
the FP32 solver holds them, so that both sides start from the same inputs.
The fields are stored in float32 (their rounding, 6e-8 relative, is far
below the 1e-4 the tests check), the observables in float64.
"""
import json
import os
import sys
import time

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import workloads as W  # noqa: E402
from oracle import lbm2d as L  # noqa: E402
from oracle import lbm3d as L3  # noqa: E402

OBS = ("current_density", "heat_rate", "o2_utilisation", "T_max", "sum_c", "sum_theta")


def cases() -> dict:
    w2 = W.cathode2d_scaled(512, 128, precision=32)
    w2.update(steps=10000)
    wb = dict(W.batched_cases()[9])
    w3 = W.cathode3d_scaled(64, 32, 16, precision=32, sphere_radius=2.0, filter_box=5, dp_lat=4.0, Re=5.0)
    w3.update(steps=5000)
    return {"cathode2d_512x128": w2, "batch_case09_256x64": wb, "cathode3d_64x32x16": w3}


def path_of(name: str) -> str:
    return os.path.join(HERE, f"fp32_horizon_{name}.npz")


def run(name: str, w: dict) -> None:
    t0 = time.time()
    steps = int(w["steps"])
    if "nz" in w:
        phi = W.sphere_pack_porosity(w).astype(np.float32).astype(np.float64)
        m = L3.Model3D(L3.geometry_from_workload(w), L3.params_from_workload(w), phi=torch.as_tensor(phi))
        keys = ("ux", "uy", "uz", "T", "theta", "c")
    else:
        phi = (torch.as_tensor(W.porosity_field(w).astype(np.float32).astype(np.float64))
               if "phi_seed" in w else None)
        m = L.Model(L.geometry_from_workload(w), L.Params.from_workload(w), phi=phi)
        keys = ("ux", "uy", "T", "theta", "c")
    s = m.initial_state()
    done = 0
    while done < steps:
        n = min(1000, steps - done)
        s = m.run(s, n)
        done += n
        print(f"{name}: {done}/{steps} steps, {time.time() - t0:.0f} s", flush=True)
    f = m.fields(s)
    o = m.observables(s)
    out = {k: f[k].numpy().astype(np.float32) for k in keys}
    out.update({f"obs_{k}": np.float64(float(o[k])) for k in OBS})
    out["workload"] = np.array(json.dumps({k: v for k, v in w.items()}, sort_keys=True, default=str))
    np.savez_compressed(path_of(name), **out)
    print(f"{name}: wrote {path_of(name)} ({time.time() - t0:.0f} s)", flush=True)


if __name__ == "__main__":
    torch.set_num_threads(int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1)))
    want = sys.argv[1:]
    for name, w in cases().items():
        if not want or any(name.startswith(p) for p in want):
            run(name, w)
