"""Seeded synthetic workloads for the coupled lattice-Boltzmann cathode model.

This module is the only code shared by the FP64 oracle side (tests) and the
HIP side (binding, bench).  It holds plain numbers and seeded random draws:
lattice sizes, layer thicknesses, operating points, porosity fields, batched
case draws and arbitrary population states.  It contains none of the
method's arithmetic (no equilibria, no permeability or diffusivity laws, no
unit conversions); every quantity derived from these inputs is computed
separately by each side.

Workload recipe (the paper measures on no public dataset; these synthetic
inputs stand in for its parametric sweeps over voltage, temperature, flow
rate, permeability, porosity and effective diffusivity, Section 5):

* ``cathode2d_200x40``: 200x40 lattice, channel rows 0-19, GDL rows 20-37
  (porosity 0.6, Darcy number 1e-3), CL rows 38-39; Re 10, 353 K, 0.6 V;
  FP64; 2000 steps.  No randomness.
* ``cathode2d_4096x1024``: 4096x1024 lattice, layers scaled from the
  200x40 case (channel = round(NY/2), CL = max(1, round(NY/20)), GDL = rest);
  porosity i.i.d. U[0.4, 0.8] over GDL and CL cells (seed 21030144);
  Kozeny-Carman permeability with particle diameter 0.3325 x GDL thickness;
  Re 50, 0.5 V, 343 K; FP32; 10^4 steps.
* ``batched_sweep_64``: 64 cases (seed 21030145), per case in this order
  nx in {256,512,1024}, ny in {64,128,256}, V ~ U[0.3,0.9], T ~ U[333,363],
  Re ~ U[5,100], porosity ~ U[0.4,0.8], log10 Da ~ U[-4,-2],
  diffusivity ratio ~ U[0.1,1.0]; FP32; 5000 steps.
* ``adjoint2d_1024x256``: 1024x256, porosity field U[0.4,0.8] (seed
  21030146), 4000 steps, checkpoint every 200; 32 finite-difference cells
  drawn from the GDL (seed 21030147); a 64x16 copy for the oracle.
"""
from __future__ import annotations

import numpy as np

SEED_ROOFLINE_PHI = 21030144
SEED_BATCH = 21030145
SEED_ADJOINT_PHI = 21030146
SEED_ADJOINT_FD = 21030147


def scaled_layers(ny: int) -> tuple[int, int, int]:
    """Channel / GDL / CL row counts for a lattice of ``ny`` rows.

    The 200x40 case has 20/18/2 rows; other heights keep the same
    proportions: channel = round(ny/2), CL = max(1, round(ny/20)).
    """
    ch = int(0.5 * ny + 0.5)
    cl = max(1, int(0.05 * ny + 0.5))
    return ch, ny - ch - cl, cl


def base_case() -> dict:
    """Operating point and lattice shared by every 2D workload.

    Values that the paper leaves open (relaxation time, lattice diffusivity,
    heat capacities) are the builder's defaults.
    """
    return dict(
        tau_f=0.65,          # flow relaxation time (lattice)
        D_f_lat=0.0125,      # O2 diffusivity in clear gas (lattice units)
        c_in=1.0,            # inlet O2 relative to the reference concentration
        deff_ratio_gdl=0.0,  # 0: Bruggeman law in the porous layers
        dp_over_hgdl=0.0,    # 0: permeability from the Darcy number
    )


def cathode2d_200x40() -> dict:
    w = base_case()
    w.update(name="cathode2d_200x40", nx=200, ny=40, ny_channel=20, ny_gdl=18,
             ny_cl=2, precision=64, steps=2000, Re=10.0, T_in=353.0,
             V_op=0.6, phi_gdl=0.6, Da_gdl=1e-3)
    return w


def cathode2d_4096x1024() -> dict:
    w = base_case()
    ch, gdl, cl = scaled_layers(1024)
    w.update(name="cathode2d_4096x1024", nx=4096, ny=1024, ny_channel=ch,
             ny_gdl=gdl, ny_cl=cl, precision=32, steps=10000, Re=50.0,
             T_in=343.0, V_op=0.5, phi_gdl=0.6, Da_gdl=1e-3,
             dp_over_hgdl=0.3325, phi_seed=SEED_ROOFLINE_PHI,
             phi_range=(0.4, 0.8))
    return w


def cathode2d_scaled(nx: int, ny: int, precision: int = 32, **over) -> dict:
    """The 4096x1024 recipe at another lattice size (parity-test sizes)."""
    w = cathode2d_4096x1024()
    ch, gdl, cl = scaled_layers(ny)
    w.update(name=f"cathode2d_{nx}x{ny}", nx=nx, ny=ny, ny_channel=ch,
             ny_gdl=gdl, ny_cl=cl, precision=precision)
    w.update(over)
    return w


def adjoint2d(nx: int = 1024, ny: int = 256) -> dict:
    w = base_case()
    ch, gdl, cl = scaled_layers(ny)
    w.update(name=f"adjoint2d_{nx}x{ny}", nx=nx, ny=ny, ny_channel=ch,
             ny_gdl=gdl, ny_cl=cl, precision=32, steps=4000, every=200,
             Re=10.0, T_in=353.0, V_op=0.6, phi_gdl=0.6, Da_gdl=1e-3,
             dp_over_hgdl=0.3325, phi_seed=SEED_ADJOINT_PHI,
             phi_range=(0.4, 0.8))
    return w


def porosity_field(w: dict) -> np.ndarray:
    """Per-cell porosity [ny, nx] (float64): 1 in channel rows, i.i.d.
    uniform on ``w['phi_range']`` over GDL and CL rows, seeded."""
    rng = np.random.default_rng(w["phi_seed"])
    lo, hi = w["phi_range"]
    phi = np.ones((w["ny"], w["nx"]), dtype=np.float64)
    ch = w["ny_channel"]
    phi[ch:, :] = rng.uniform(lo, hi, size=(w["ny"] - ch, w["nx"]))
    return phi


def batched_cases(n: int = 64, seed: int = SEED_BATCH) -> list[dict]:
    """Draw ``n`` independent cathode cases (order of draws is fixed)."""
    rng = np.random.default_rng(seed)
    cases = []
    for k in range(n):
        nx = int(rng.choice([256, 512, 1024]))
        ny = int(rng.choice([64, 128, 256]))
        V = float(rng.uniform(0.3, 0.9))
        T = float(rng.uniform(333.0, 363.0))
        Re = float(rng.uniform(5.0, 100.0))
        phi = float(rng.uniform(0.4, 0.8))
        log_da = float(rng.uniform(-4.0, -2.0))
        ratio = float(rng.uniform(0.1, 1.0))
        w = base_case()
        ch, gdl, cl = scaled_layers(ny)
        # Lattice viscosity per case: at most 0.05, and small enough that
        # the mean inlet speed Re nu / H stays at or below 0.04; a clear-gas
        # O2 lattice diffusivity of 0.025 keeps the D2Q5 equilibria
        # non-negative at that speed.
        nu = min(0.05, 0.04 * ch / Re)
        w.update(name=f"case{k:02d}_{nx}x{ny}", nx=nx, ny=ny, ny_channel=ch,
                 ny_gdl=gdl, ny_cl=cl, precision=32, steps=5000, Re=Re,
                 T_in=T, V_op=V, phi_gdl=phi, Da_gdl=10.0 ** log_da,
                 deff_ratio_gdl=ratio, tau_f=3.0 * nu + 0.5, D_f_lat=0.025)
        cases.append(w)
    return cases


def fd_cells(w: dict, n: int = 32, seed: int = SEED_ADJOINT_FD, depth: int = 12) -> list[tuple[int, int]]:
    """``n`` distinct porous cells (y, x), seeded, for finite-difference
    checks, drawn from the ``depth`` GDL rows next to the CL and the CL rows
    (the cells a few thousand steps of diffusion from the CL can reach)."""
    rng = np.random.default_rng(seed)
    y0 = max(w["ny_channel"], w["ny"] - w["ny_cl"] - depth)
    rows = w["ny"] - y0
    flat = rng.choice(rows * w["nx"], size=n, replace=False)
    return [(int(y0 + i // w["nx"]), int(i % w["nx"])) for i in flat]


def random_populations(ny: int, nx: int, seed: int) -> np.ndarray:
    """An arbitrary, positive population state [19, ny, nx] (float64).

    Planes 0-8 are the flow populations (rest population near 1, moving ones
    near 0.02), planes 9-13 the temperature-rise populations, planes 14-18
    the O2 populations.  Any state is a valid input to one update; these
    ranges keep velocities, temperature rises and concentrations in the
    magnitudes of the cathode workloads.
    """
    rng = np.random.default_rng(seed)
    s = np.empty((19, ny, nx), dtype=np.float64)
    s[0] = rng.uniform(0.97, 1.0, size=(ny, nx))
    s[1:9] = rng.uniform(0.0, 0.02, size=(8, ny, nx))
    s[9:14] = rng.uniform(0.0, 0.4, size=(5, ny, nx))
    s[14:19] = rng.uniform(0.15, 0.25, size=(5, ny, nx))
    return s
