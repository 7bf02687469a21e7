"""Benchmark of the fused coupled-LBM cathode step on one MI355X.

Workload: the 4096x1024 FP32 cathode (per-cell porosity U[0.4, 0.8],
Kozeny-Carman permeability, Re 50, 0.5 V, 343 K).  A step is one time step
of the whole coupled update (stream, boundary columns, macros, MRT flow
collision with porous drag, CL reaction, two scalar collisions) over the
whole lattice.  Prints one JSON line; besides the headline it carries the
model-option variants on the same lattice, the 64-case batched sweep, the
2D adjoint, the 39-case polarisation sweep, the 3D cathode and its adjoint,
and the FP64 oracle timed on the host (each can be skipped, see --help).

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, published
BYTES_PER_LU_POPS = 19 * 4 * 2  # 19 FP32 populations read and written per lattice update
BYTES_PER_LU_PHI = 4            # per-cell porosity read
# The library advances lattices of at least this many nodes (with walls and
# inlet / outlet columns: no periodic axis) two steps per launch (k_step2).
TWO_STEP_MIN_CELLS = 1 << 19
# Committed rocprofv3 counter summaries (HBM bytes per launch) and the
# sources of the kernel each one measured.
COUNTERS = {
    "step2d": (os.path.join(ROOT, "profiles", "step2d_4096x1024_fp32_counters.json"),
               ("lbm_device.hpp", "lbm_kernels2d.hpp", "lbm_host.hpp", "lbm_api.hip")),
    "step3d": (os.path.join(ROOT, "profiles", "step3d_256x128x64_fp32_counters.json"),
               ("lbm_device.hpp", "lbm_kernels2d.hpp", "lbm_host.hpp", "lbm3d_device.hpp", "lbm3d_kernels.hpp",
                "lbm3d_api.hip")),
}


def kernel_source_hash(which: str = "step2d") -> str:
    h = hashlib.sha256()
    for fn in COUNTERS[which][1]:
        with open(os.path.join(ROOT, "paper_2103_01444_amd", "csrc", fn), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic(per_launch_cells: int, which: str = "step2d"):
    """HBM bytes per launch from committed rocprofv3 counter runs, or None
    if the kernel source changed since they were taken."""
    path = COUNTERS[which][0]
    if not os.path.exists(path):
        return None
    with open(path) as f:
        c = json.load(f)
    if c.get("kernel_source_hash") != kernel_source_hash(which) or c.get("cells") != per_launch_cells:
        return None
    return c.get("hbm_bytes_per_launch")


def _oracle_sample(w, phi, target_s: float):
    """Steps per second of the FP64 oracle on lattice w: one untimed step,
    then as many as fit in about target_s seconds (at least one)."""
    import torch

    from oracle import lbm2d as L
    m = L.Model(L.geometry_from_workload(w), L.Params.from_workload(w),
                phi=None if phi is None else torch.as_tensor(phi))
    s = m.initial_state()
    t0 = time.perf_counter()
    s = m.step(s)
    first = time.perf_counter() - t0
    n = max(1, min(2000, int(target_s / max(first, 1e-4)) - 1))
    t0 = time.perf_counter()
    for _ in range(n):
        s = m.step(s)
    return n, time.perf_counter() - t0


def cpu_baseline(w, phi, target_s: float = 10.0):
    """The FP64 oracle on the host cores, timed on bounded samples: the
    whole 4096x1024 lattice with all the threads torch uses and with one,
    and the 200x40 FP64 cathode (all threads) for up to its 2000 steps."""
    import torch

    import workloads as W
    cells = w["nx"] * w["ny"]
    threads = torch.get_num_threads()
    n, dt = _oracle_sample(w, phi, target_s)
    out = {"value": round(cells * n / dt / 1e6, 3), "unit": "MLUPS", "cores": threads, "kind": "oracle",
           "sample": f"FP64 oracle, full {w['nx']}x{w['ny']} lattice, {n} steps after 1 untimed ({dt:.1f} s), "
                     f"{threads} threads (os.cpu_count() {os.cpu_count()})"}
    torch.set_num_threads(1)
    try:
        n1, dt1 = _oracle_sample(w, phi, target_s)
    finally:
        torch.set_num_threads(threads)
    out["single_thread"] = {"value": round(cells * n1 / dt1 / 1e6, 3), "unit": "MLUPS", "cores": 1,
                            "sample": f"same lattice, {n1} steps after 1 untimed ({dt1:.1f} s)"}
    w1 = W.cathode2d_200x40()
    n2, dt2 = _oracle_sample(w1, None, target_s)
    out["cathode2d_200x40"] = {"value": round(w1["nx"] * w1["ny"] * n2 / dt2 / 1e6, 3), "unit": "MLUPS",
                               "cores": threads, "sample": f"FP64 oracle, {n2} of its {w1['steps']} steps "
                                                           f"after 1 untimed ({dt2:.1f} s)"}
    return out


def _timed(stream, fn):
    """Run fn() between two events on ``stream``; returns (wall s, event s)."""
    import torch
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    t0 = time.perf_counter()
    fn()
    e1.record(stream)
    torch.cuda.synchronize()
    return time.perf_counter() - t0, e0.elapsed_time(e1) / 1e3


def bench_batched(steps: int, seq_steps: int) -> dict:
    """The 64-case sweep in one batch (autotuned schedule) against the plain
    single-case solver run on the same cases one after the other."""
    import numpy as np

    import workloads as W
    from paper_2103_01444_amd import BatchedSweep, Cathode

    cases = W.batched_cases()
    cells = sum(w["nx"] * w["ny"] for w in cases)
    b = BatchedSweep(cases)
    tune = b.autotune(trial_steps=10, cache_path=os.environ.get(
        "LBMPEM_TUNE_CACHE", os.path.join(os.path.expanduser("~"), ".cache", "lbmpem_batch_schedules.json")))
    b.step(20)
    wall, ev = _timed(b.stream, lambda: b.step(steps))
    obs = b.observables()
    b.close()
    del b
    sims = [Cathode.from_workload(w) for w in cases]
    for s in sims:
        s.step(5)

    def seq():
        for s in sims:
            s.step(seq_steps)

    wall_seq, _ = _timed(sims[0].stream, seq)
    for s in sims:
        s.close()
    del sims
    mlups = cells * steps / wall / 1e6
    mlups_seq = cells * seq_steps / wall_seq / 1e6
    achieved = cells * BYTES_PER_LU_POPS * steps / ev / 1e9
    return {"workload": "batched_sweep_64", "cases": len(cases), "cells": cells, "steps": steps,
            "value": round(mlups, 1), "unit": "MLUPS", "ms_per_step": round(wall * 1e3 / steps, 4),
            "schedule": {k: tune.get(k, 0) for k in ("tile_x", "tile_y", "persistent", "block")},
            "steps_per_launch": 2 if tune.get("block", 0) == 960 else 1,
            "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": round(achieved / HBM_PEAK_GBS, 4), "bytes_per_lattice_update": BYTES_PER_LU_POPS},
            "plain_sequential": {"value": round(mlups_seq, 1), "unit": "MLUPS", "steps_per_case": seq_steps},
            "speedup_vs_plain_sequential": round(mlups / mlups_seq, 3),
            "mean_current_density_A_cm2": float(np.mean([o["current_density"] for o in obs]))}


BYTES_PER_LU_FP64 = 19 * 8 * 2  # 19 FP64 populations read and written per lattice update


def bench_fp64(steps_large: int) -> dict:
    """FP64 mode: the 200x40 cathode over its 2000 steps (8000 nodes: the
    launch latency bounds it), and the 4096x1024 recipe in FP64 against the
    304 B/LU (+8 for the porosity) roofline."""
    import workloads as W
    from paper_2103_01444_amd import Cathode

    w1 = W.cathode2d_200x40()
    with Cathode.from_workload(w1) as sim:
        sim.step(20)
        wall1, ev1 = _timed(sim.stream, lambda: sim.step(w1["steps"]))
    c1 = w1["nx"] * w1["ny"]
    out = {"cathode2d_200x40": {"cells": c1, "steps": w1["steps"], "value": round(c1 * w1["steps"] / wall1 / 1e6, 1),
                                "unit": "MLUPS", "avg_launch_us": round(ev1 / w1["steps"] * 1e6, 3)}}
    w = W.cathode2d_4096x1024()
    w = dict(w, precision=64)
    with Cathode.from_workload(w, phi=W.porosity_field(w)) as sim:
        sim.step(20)
        wall, ev = _timed(sim.stream, lambda: sim.step(steps_large))
    cells = w["nx"] * w["ny"]
    spl = 2 if cells >= TWO_STEP_MIN_CELLS else 1
    launches = steps_large // spl + steps_large % spl
    launch_s = ev / launches
    bpl = BYTES_PER_LU_FP64 + 8
    achieved = cells * bpl * steps_large / ev / 1e9
    out["cathode2d_4096x1024"] = {
        "cells": cells, "steps": steps_large, "value": round(cells * steps_large / wall / 1e6, 1), "unit": "MLUPS",
        "kernel": {"name": "k_step2<double, MAT_PHI>" if spl == 2 else "k_step<double, MAT_PHI>",
                   "steps_per_launch": spl, "launches": launches, "avg_launch_us": round(launch_s * 1e6, 3),
                   "us_per_step": round(ev / steps_large * 1e6, 3), "bytes_per_lattice_update": bpl},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4)}}
    return out


ADJ_BYTES_PER_LU = 19 * 4 * 3 + 3 * 4 + 3 * 4 * 2  # reverse step: pull S, read lambda, push lambda', 3 fields, gradient RMW
FWD_FULL_BYTES_PER_LU = 19 * 4 * 2 + 3 * 4          # replayed forward step with three per-cell fields


def bench_adjoint(nsteps: int = 4000, every: int = 200) -> dict:
    """1024x256 FP32 cathode with per-cell (porosity, 1/K, D_eff): plain
    forward, checkpointed forward and the hand-written adjoint."""
    import workloads as W
    from paper_2103_01444_amd import Cathode

    w = W.adjoint2d()
    phi = W.porosity_field(w)
    sim = Cathode.from_workload(w, phi=phi, independent_fields=1)
    cells = w["nx"] * w["ny"]
    sim.step(50)
    wall_f, _ = _timed(sim.stream, lambda: sim.step(nsteps))
    res = {}
    wall_cf, _ = _timed(sim.stream, lambda: res.update(J=sim.forward_checkpointed(nsteps, every)))
    wall_b, _ = _timed(sim.stream, lambda: res.update(g=sim.backward(1.0, permeability=False)))
    g = res["g"]
    mlups_f = cells * nsteps / wall_f / 1e6
    mlups_b = cells * nsteps / wall_b / 1e6
    # backward = replay (one forward per step) + reverse step
    achieved = cells * nsteps * (ADJ_BYTES_PER_LU + FWD_FULL_BYTES_PER_LU) / wall_b / 1e9
    sim.close()
    return {"workload": w["name"], "cells": cells, "steps": nsteps, "checkpoint_every": every,
            "forward": {"value": round(mlups_f, 1), "unit": "MLUPS"},
            "forward_checkpointed": {"value": round(cells * nsteps / wall_cf / 1e6, 1), "unit": "MLUPS"},
            "adjoint": {"value": round(mlups_b, 1), "unit": "MLUPS", "seconds": round(wall_b, 4)},
            "adjoint_over_forward_time": round(wall_b / wall_f, 3),
            "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": round(achieved / HBM_PEAK_GBS, 4),
                         "bytes_per_lattice_update": ADJ_BYTES_PER_LU + FWD_FULL_BYTES_PER_LU},
            "J_A_cm2": res["J"],
            "max_abs_grad": {k: float(v.abs().max()) for k, v in g.items()}}


BYTES_PER_LU_3D = 33 * 4 * 2 + 4  # 33 FP32 populations read and written, porosity read


def bench_3d(steps: int, warmup: int = 50) -> dict:
    """The 256x128x64 FP32 3D cathode (D3Q19 + 2 x D3Q7, sphere-pack GDL)."""
    import workloads as W
    from paper_2103_01444_amd import Cathode3D

    w = W.cathode3d_256x128x64()
    phi = W.sphere_pack_porosity(w)
    sim = Cathode3D.from_workload(w, phi=phi)
    sim.step(warmup)
    wall, ev = _timed(sim.stream, lambda: sim.step(steps))
    obs = sim.observables()
    sim.close()
    del sim
    cells = w["nx"] * w["ny"] * w["nz"]
    launch_s = ev / steps
    achieved = cells * BYTES_PER_LU_3D / launch_s / 1e9
    return {"workload": w["name"], "cells": cells, "steps": steps, "value": round(cells * steps / wall / 1e6, 1),
            "unit": "MLUPS", "ms_per_step": round(wall * 1e3 / steps, 5),
            "kernel": {"name": "k3_step<float, MAT_PHI>", "avg_launch_us": round(launch_s * 1e6, 3),
                       "algorithmic_bytes_per_launch": cells * BYTES_PER_LU_3D,
                       "bytes_per_lattice_update": BYTES_PER_LU_3D},
            "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": measured_traffic(cells, "step3d")},
            "observables": {"current_density_A_cm2": obs["current_density"], "T_max_K": obs["T_max"],
                            "o2_utilisation": obs["o2_utilisation"]}}


def bench_polarisation(steps: int, block: int = 500000, tol: float = 1e-4) -> dict:
    """Polarisation / power / heat curves of the pressure-driven 200x40
    cathode (3 outlet pressures x 13 voltages = 39 cases in one batch), run
    to steady state: blocks of ``block`` steps until the current density of
    every case changes by less than ``tol`` (relative) over a block, or
    ``steps`` steps.  The slowest mode is heat conduction along the channel
    in the solid of the GDL (a few 10^6 steps at this lattice's time step,
    which the gas thermal diffusivity bounds).  The throughput is timed over
    the first block."""
    import numpy as np

    import workloads as W
    from paper_2103_01444_amd import BatchedSweep

    cases = W.polarisation_sweep(steps)
    cells = sum(w["nx"] * w["ny"] for w in cases)
    b = BatchedSweep(cases)
    tune = b.autotune(trial_steps=10, cache_path=os.environ.get(
        "LBMPEM_TUNE_CACHE", os.path.join(os.path.expanduser("~"), ".cache", "lbmpem_batch_schedules.json")))
    first = min(block, steps)
    wall, ev = _timed(b.stream, lambda: b.step(first))
    done, drift = first, float("inf")
    prev = [o["current_density"] for o in b.observables()]
    while done < steps and drift >= tol:
        n = min(block, steps - done)
        b.step(n)
        done += n
        obs = b.observables()
        drift = max(abs(o["current_density"] - p) / abs(o["current_density"]) for o, p in zip(obs, prev))
        prev = [o["current_density"] for o in obs]
    obs = b.observables()
    b.close()
    del b
    nu = (cases[0]["tau_f"] - 0.5) / 3.0
    nv = len(W.POLARISATION_V)
    v = np.array(W.POLARISATION_V)
    I = np.array([o["current_density"] for o in obs]).reshape(-1, nv)
    curves = []
    for j, p_out in enumerate(W.POLARISATION_P_OUT):
        o = obs[j * nv:(j + 1) * nv]
        curves.append({"p_in": W.POLARISATION_P_IN, "p_out": p_out, "Re": round(o[-1]["inlet_flux"] / nu, 3),
                       "V": list(W.POLARISATION_V),
                       "I_A_cm2": [round(x["current_density"], 4) for x in o],
                       "P_W_cm2": [round(x["power_density"], 4) for x in o],
                       "heat_W_cm2": [round(x["heat_rate"], 4) for x in o],
                       "T_max_K": [round(x["T_max"], 3) for x in o]})
    kinetic, plateau = v >= 0.599, v <= 0.551
    trends = {  # Section 5 (Figs. 9, 12): on the steady curves
        "I_falls_with_V_above_0.6V": bool(np.all(np.diff(I[:, kinetic], axis=1) < 0)),
        "I_rises_with_flow_rate_up_to_0.55V": bool(np.all(np.diff(I[:, plateau], axis=0) > 0)),
        "power_peaks_inside_the_range": bool(all(0 < int(np.argmax(c["P_W_cm2"])) < nv - 1 for c in curves)),
    }
    achieved = cells * BYTES_PER_LU_POPS * first / ev / 1e9
    return {"workload": "polarisation_sweep_39", "cases": len(cases), "cells": cells, "steps_timed": first,
            "value": round(cells * first / wall / 1e6, 1), "unit": "MLUPS", "ms_per_step": round(wall * 1e3 / first, 4),
            "schedule": {k: tune.get(k, 0) for k in ("tile_x", "tile_y", "persistent", "block")},
            "steps_per_launch": 2 if tune.get("block", 0) == 960 else 1,
            "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": round(achieved / HBM_PEAK_GBS, 4), "bytes_per_lattice_update": BYTES_PER_LU_POPS},
            "curves_after_steps": done, "steady_block_steps": block,
            "max_rel_change_I_last_block": round(drift, 8), "steady": bool(drift < tol), "trends": trends,
            "curves": curves}


def bench_variants(steps: int) -> dict:
    """The 4096x1024 FP32 benchmark lattice under the model options, same
    porosity field: pressure-driven inlet and outlet pressure, Butler-Volmer
    kinetics, thin-film CL (CL rows merged into the GDL, film below),
    buoyancy, heat-capacity-ratio energy equation with the physical heat sign."""
    import workloads as W
    from paper_2103_01444_amd import Cathode

    base = W.cathode2d_4096x1024()
    phi = W.porosity_field(base)
    thin = dict(base, thin_cl=True, ny_gdl=base["ny_gdl"] + base["ny_cl"], ny_cl=0)
    variants = {"pressure_inlet": dict(base, pressure_inlet=True, p_in=2e-4, p_out=5e-5),
                "butler_volmer": dict(base, butler_volmer=True),
                "thin_cl": thin,
                "buoyancy": dict(base, buoyancy=(0.0, -1e-6)),
                "sigma_energy_physical_heat": dict(base, sigma_energy=True, heat_physical=True)}
    cells = base["nx"] * base["ny"]
    out = {}
    for name, w in variants.items():
        sim = Cathode.from_workload(w, phi=phi)
        sim.step(50)
        wall, ev = _timed(sim.stream, lambda: sim.step(steps))
        o = sim.observables()
        sim.close()
        del sim
        achieved = cells * (BYTES_PER_LU_POPS + BYTES_PER_LU_PHI) * steps / ev / 1e9
        out[name] = {"value": round(cells * steps / wall / 1e6, 1), "unit": "MLUPS", "steps": steps,
                     "roofline_frac": round(achieved / HBM_PEAK_GBS, 4),
                     "current_density_A_cm2": o["current_density"]}
    return out


ADJ3_BYTES_PER_LU = 33 * 4 * 3 + 3 * 4 + 3 * 4 * 2  # 3D reverse step, same streams as in 2D
FWD3_FULL_BYTES_PER_LU = 33 * 4 * 2 + 3 * 4         # replayed 3D forward step with three per-cell fields


def bench_adjoint3d(nsteps: int = 5000, every: int = 70) -> dict:
    """256x128x64 FP32 sphere pack with per-cell (porosity, 1/K, D_eff):
    plain forward, checkpointed forward and the hand-written 3D adjoint."""
    import workloads as W
    from paper_2103_01444_amd import Cathode3D

    w = W.cathode3d_256x128x64()
    sim = Cathode3D.from_workload(w, phi=W.sphere_pack_porosity(w), independent_fields=1)
    cells = w["nx"] * w["ny"] * w["nz"]
    sim.step(20)
    wall_f, _ = _timed(sim.stream, lambda: sim.step(nsteps))
    res = {}
    wall_cf, _ = _timed(sim.stream, lambda: res.update(J=sim.forward_checkpointed(nsteps, every)))
    wall_b, _ = _timed(sim.stream, lambda: res.update(g=sim.backward(1.0, permeability=False)))
    g = res["g"]
    achieved = cells * nsteps * (ADJ3_BYTES_PER_LU + FWD3_FULL_BYTES_PER_LU) / wall_b / 1e9
    out = {"workload": w["name"], "cells": cells, "steps": nsteps, "checkpoint_every": every,
           "workspace_GB": round(sim.adj_ws.numel() / 1e9, 2),
           "forward": {"value": round(cells * nsteps / wall_f / 1e6, 1), "unit": "MLUPS"},
           "forward_checkpointed": {"value": round(cells * nsteps / wall_cf / 1e6, 1), "unit": "MLUPS"},
           "adjoint": {"value": round(cells * nsteps / wall_b / 1e6, 1), "unit": "MLUPS", "seconds": round(wall_b, 4)},
           "adjoint_over_forward_time": round(wall_b / wall_f, 3),
           "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": round(achieved / HBM_PEAK_GBS, 4),
                        "bytes_per_lattice_update": ADJ3_BYTES_PER_LU + FWD3_FULL_BYTES_PER_LU},
           "J_A_cm2": res["J"],
           "max_abs_grad_inv_k": float(g["inv_k"].abs().max())}
    sim.close()
    del sim, g, res
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10000)
    ap.add_argument("--warmup", type=int, default=500)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--batched-steps", type=int, default=500, help="0 skips the batched sweep")
    ap.add_argument("--adjoint-steps", type=int, default=4000, help="0 skips the adjoint")
    ap.add_argument("--steps3d", type=int, default=5000, help="0 skips the 3D cathode")
    ap.add_argument("--adjoint3d-steps", type=int, default=5000, help="0 skips the 3D adjoint")
    ap.add_argument("--polarisation-steps", type=int, default=8000000,
                    help="most steps of the polarisation sweep (it stops at steady state); 0 skips it")
    ap.add_argument("--variant-steps", type=int, default=2000, help="0 skips the model-option variants")
    ap.add_argument("--fp64-steps", type=int, default=1000, help="0 skips the FP64 rows")
    ap.add_argument("--sustained-s", type=float, default=8.0,
                    help="seconds of continued stepping before the sustained k_step figure (0 skips it)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a plain 1 GiB read + 1 GiB write copy kernel 5 times (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build measures one GPU only; run with --gpus 1"}))
        sys.exit(2)

    import numpy as np
    import torch

    if args.calibrate_copy:
        x = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        y = torch.empty_like(x)
        for _ in range(5):
            torch.mul(x, 1.0, out=y)
        torch.cuda.synchronize()
        print(json.dumps({"copy_kernel_bytes_read": x.numel() * 4, "copy_kernel_bytes_written": y.numel() * 4}))
        return

    import workloads as W
    from paper_2103_01444_amd import Cathode

    w = W.cathode2d_4096x1024()
    phi = W.porosity_field(w)
    print(f"bench: {w['name']} fp32, warmup {args.warmup}, steps {args.steps}", file=sys.stderr, flush=True)
    sim = Cathode.from_workload(w, phi=phi)
    sim.step(args.warmup)
    sim.synchronize()
    torch.cuda.synchronize()
    stream = sim.stream
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    t0 = time.perf_counter()
    sim.step(args.steps)
    e1.record(stream)
    sim.synchronize()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ev_ms = e0.elapsed_time(e1)
    obs = sim.observables()
    cells = w["nx"] * w["ny"]
    mlups = cells * args.steps / (wall) / 1e6
    spl = 2 if cells >= TWO_STEP_MIN_CELLS else 1  # steps per launch
    launches = args.steps // spl + args.steps % spl  # an odd count ends with one single step
    launch_s = ev_ms / 1e3 / launches
    bpu = BYTES_PER_LU_POPS + BYTES_PER_LU_PHI
    bytes_per_launch = spl * cells * bpu  # algorithmic: the per-update figure times the updates of a launch
    achieved = cells * bpu * args.steps / (ev_ms / 1e3) / 1e9
    traffic = measured_traffic(cells)
    print(f"bench: {mlups:.1f} MLUPS, kernel avg {launch_s * 1e6:.2f} us per launch of {spl} steps, "
          f"{achieved:.0f} GB/s, I = {obs['current_density']:.4e} A/cm2", file=sys.stderr, flush=True)
    if not np.isfinite(obs["current_density"]):
        raise SystemExit("non-finite result")

    line = {
        "metric": "coupled-LBM MLUPS, % of HBM BW peak; batched sweep and adjoint vs plain, 1 GPU",
        "value": round(mlups, 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(wall * 1e3 / args.steps, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded porosity field)",
        "config": {"workload": w["name"], "nx": w["nx"], "ny": w["ny"],
                   "layers": [w["ny_channel"], w["ny_gdl"], w["ny_cl"]], "Re": w["Re"], "V_op": w["V_op"],
                   "T_in_K": w["T_in"], "porosity": "per-cell U[0.4,0.8], seed 21030144"},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": traffic,
                     "traffic_frac": None if traffic is None else round(traffic / launch_s / 1e9 / HBM_PEAK_GBS, 4),
                     "note": ("achieved prices each lattice update at the single-step pull scheme's "
                              f"{bpu} B; the kernel advances {spl} step(s) per launch and moves `traffic` "
                              "bytes per launch (counters)")},
        "kernel": {"name": "k_step2<float, MAT_PHI>" if spl == 2 else "k_step<float, MAT_PHI>",
                   "steps_per_launch": spl, "launches": launches, "avg_launch_us": round(launch_s * 1e6, 3),
                   "us_per_step": round(ev_ms * 1e3 / args.steps, 3),
                   "algorithmic_bytes_per_launch": bytes_per_launch,
                   "bytes_per_lattice_update": bpu},
        "observables": {"current_density_A_cm2": obs["current_density"], "T_max_K": obs["T_max"],
                        "o2_utilisation": obs["o2_utilisation"]},
    }
    if args.sustained_s > 0:
        # the same kernel after args.sustained_s seconds of continuous load
        # (the first seconds of a process run faster than the steady state)
        n_load = max(2, int(args.sustained_s / launch_s) * spl)
        sim.step(n_load)
        n_meas = 2000
        _, ev_s = _timed(stream, lambda: sim.step(n_meas))
        ls = ev_s / n_meas  # per step
        line["sustained"] = {"after_steps": n_load + args.steps + args.warmup, "steps": n_meas,
                             "avg_launch_us": round(ls * spl * 1e6, 3), "us_per_step": round(ls * 1e6, 3),
                             "frac": round(cells * bpu / ls / 1e9 / HBM_PEAK_GBS, 4)}
        print(f"bench: sustained kernel avg {ls * spl * 1e6:.2f} us per launch after {n_load} more steps",
              file=sys.stderr, flush=True)
    sim.close()
    del sim
    if args.fp64_steps > 0:
        print("bench: FP64 rows", file=sys.stderr, flush=True)
        line["fp64"] = bench_fp64(args.fp64_steps)
        print(f"bench: fp64 4096x1024 {line['fp64']['cathode2d_4096x1024']['value']} MLUPS, "
              f"200x40 {line['fp64']['cathode2d_200x40']['value']} MLUPS", file=sys.stderr, flush=True)
    if args.variant_steps > 0:
        print("bench: model-option variants", file=sys.stderr, flush=True)
        line["variants"] = bench_variants(args.variant_steps)
        print("bench: variants " + ", ".join(f"{k} {v['value']} MLUPS" for k, v in line["variants"].items()),
              file=sys.stderr, flush=True)
    if args.batched_steps > 0:
        print("bench: batched sweep", file=sys.stderr, flush=True)
        line["batched"] = bench_batched(args.batched_steps, max(1, args.batched_steps // 2))
        print(f"bench: batched {line['batched']['value']} MLUPS, "
              f"{line['batched']['speedup_vs_plain_sequential']}x plain sequential", file=sys.stderr, flush=True)
    if args.adjoint_steps > 0:
        print("bench: adjoint", file=sys.stderr, flush=True)
        line["adjoint"] = bench_adjoint(args.adjoint_steps)
        print(f"bench: adjoint {line['adjoint']['adjoint']['value']} MLUPS, "
              f"{line['adjoint']['adjoint_over_forward_time']}x forward time", file=sys.stderr, flush=True)
    if args.polarisation_steps > 0:
        print("bench: polarisation sweep", file=sys.stderr, flush=True)
        line["polarisation"] = bench_polarisation(args.polarisation_steps)
        print(f"bench: polarisation {line['polarisation']['value']} MLUPS", file=sys.stderr, flush=True)
    if args.steps3d > 0:
        print("bench: 3D cathode", file=sys.stderr, flush=True)
        line["cathode3d"] = bench_3d(args.steps3d)
        print(f"bench: 3D {line['cathode3d']['value']} MLUPS, {line['cathode3d']['roofline']['achieved']} GB/s",
              file=sys.stderr, flush=True)
    if args.adjoint3d_steps > 0:
        print("bench: 3D adjoint", file=sys.stderr, flush=True)
        line["adjoint3d"] = bench_adjoint3d(args.adjoint3d_steps)
        print(f"bench: 3D adjoint {line['adjoint3d']['adjoint']['value']} MLUPS, "
              f"{line['adjoint3d']['adjoint_over_forward_time']}x forward time", file=sys.stderr, flush=True)
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(w, phi)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
