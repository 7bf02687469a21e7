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
* ``polarisation_sweep``: the paper's own flow driving (Section 4: a
  pressure difference between inlet and outlet) on the 200x40 cathode with
  GDL porosity 0.4 and permeability 0.176e-6 cm^2 (Darcy number 2.73e-4 on
  the 254 um GDL; the Fig. 5 base case), 353 K: 3 inlet pressures x 13
  voltages 0.30..0.90 V = 39 cases in one batch, FP32, O2 lattice
  diffusivity 0.025 (so that the GDL approaches steady state within a few
  10^4 steps), 20000 steps.  No randomness.
* ``cathode3d_256x128x64``: 256 (x, along the channel) x 128 (y, across)
  x 64 (z, through the layers): channel 32 layers, GDL 29, CL 3.  GDL
  porosity from a seeded sphere pack (seed 21030148): spheres of radius 4
  lattice units with centres uniform in the GDL box are added until the
  solid fraction reaches 0.3; the solid indicator is averaged over a 9^3
  box (truncated at the GDL faces) and porosity = 1 - that average (mean
  0.7).  The CL is a planar layer of uniform porosity 0.7.  Kozeny-Carman
  permeability with particle diameter 8 lattice units; Bruggeman
  diffusivity; Re 20, 0.55 V, 353 K; FP32; 5000 steps.
"""
from __future__ import annotations

import numpy as np

SEED_ROOFLINE_PHI = 21030144
SEED_BATCH = 21030145
SEED_ADJOINT_PHI = 21030146
SEED_ADJOINT_FD = 21030147
SEED_SPHERE_PACK = 21030148
SEED_ADJOINT3D_FD = 21030149

# Polarisation sweep: fixed inlet pressure, three outlet pressures (lattice
# units); the pressure drops 2e-3, 4e-3 and 8e-3 give plane-Poiseuille
# channel peak velocities of about 0.01, 0.02 and 0.04 on the 200x40 lattice.
POLARISATION_P_IN = 8e-3                   # fixed inlet pressure (lattice units)
POLARISATION_P_OUT = (6e-3, 4e-3, 0.0)     # outlet pressures: rising flow rate
POLARISATION_V = tuple(round(0.30 + 0.05 * i, 2) for i in range(13))


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


# --------------------------------------------------------------------- 3D
def scaled_layers3d(nz: int) -> tuple[int, int, int]:
    """Channel / GDL / CL layer counts for ``nz`` layers, in the proportions
    of the 64-layer case (32 / 29 / 3)."""
    ch = int(0.5 * nz + 0.5)
    cl = max(1, int(3.0 * nz / 64.0 + 0.5))
    return ch, nz - ch - cl, cl


def cathode3d_256x128x64() -> dict:
    w = base_case()
    w.update(name="cathode3d_256x128x64", nx=256, ny=128, nz=64, nz_channel=32, nz_gdl=29, nz_cl=3,
             precision=32, steps=5000, Re=20.0, T_in=353.0, V_op=0.55, phi_gdl=0.7, dp_lat=8.0,
             sphere_radius=4.0, solid_fraction=0.3, filter_box=9, phi_cl=0.7, phi_seed=SEED_SPHERE_PACK)
    return w


def cathode3d_scaled(nx: int, ny: int, nz: int, precision: int = 32, **over) -> dict:
    """The 256x128x64 recipe at another lattice size (parity-test sizes)."""
    w = cathode3d_256x128x64()
    ch, gdl, cl = scaled_layers3d(nz)
    w.update(name=f"cathode3d_{nx}x{ny}x{nz}", nx=nx, ny=ny, nz=nz, nz_channel=ch, nz_gdl=gdl, nz_cl=cl,
             precision=precision)
    w.update(over)
    return w


def _box_mean(a: np.ndarray, k: int) -> np.ndarray:
    """Mean over the k^d box centred on each cell, the box cut at the array
    faces (separable: the cut box is a product of intervals)."""
    h = k // 2
    out = a.astype(np.float64)
    for axis in range(a.ndim):
        n = out.shape[axis]
        c = np.concatenate([np.zeros_like(np.take(out, [0], axis=axis)), np.cumsum(out, axis=axis)], axis=axis)
        lo = np.clip(np.arange(n) - h, 0, n)
        hi = np.clip(np.arange(n) + h + 1, 0, n)
        shape = [1] * a.ndim
        shape[axis] = n
        out = (np.take(c, hi, axis=axis) - np.take(c, lo, axis=axis)) / (hi - lo).reshape(shape)
    return out


def sphere_pack_solid(nx: int, ny: int, nz: int, radius: float, solid_fraction: float,
                      seed: int) -> np.ndarray:
    """Solid indicator [nz, ny, nx] (bool) of a random sphere pack: spheres
    with centres uniform in the box are added (cells whose centres lie
    within ``radius`` of a sphere centre become solid) until the solid
    fraction reaches ``solid_fraction``."""
    rng = np.random.default_rng(seed)
    solid = np.zeros((nz, ny, nx), dtype=bool)
    R = int(np.ceil(radius))
    off = np.arange(-R, R + 1)
    target = solid_fraction * solid.size
    count = 0
    while count < target:
        cz, cy, cx = rng.uniform((0.0, 0.0, 0.0), (nz, ny, nx))
        idx = []
        for c, n in ((cz, nz), (cy, ny), (cx, nx)):
            i = int(np.floor(c)) + off
            idx.append(i[(i >= 0) & (i < n)])
        dz, dy, dx = (idx[0] + 0.5 - cz), (idx[1] + 0.5 - cy), (idx[2] + 0.5 - cx)
        inside = dz[:, None, None] ** 2 + dy[None, :, None] ** 2 + dx[None, None, :] ** 2 <= radius * radius
        sub = solid[idx[0][0]:idx[0][-1] + 1, idx[1][0]:idx[1][-1] + 1, idx[2][0]:idx[2][-1] + 1]
        count += int((inside & ~sub).sum())
        sub |= inside
    return solid


def sphere_pack_porosity(w: dict) -> np.ndarray:
    """Per-cell porosity [nz, ny, nx] (float64) of a 3D workload: 1 in the
    channel, the box-filtered sphere pack in the GDL, ``phi_cl`` in the CL."""
    nx, ny, nz = w["nx"], w["ny"], w["nz"]
    ch, gdl = w["nz_channel"], w["nz_gdl"]
    phi = np.ones((nz, ny, nx), dtype=np.float64)
    if gdl > 0:
        solid = sphere_pack_solid(nx, ny, gdl, w["sphere_radius"], w["solid_fraction"], w["phi_seed"])
        phi[ch:ch + gdl] = 1.0 - _box_mean(solid, w["filter_box"])
    phi[ch + gdl:] = w["phi_cl"]
    return phi


def random_populations3d(nz: int, ny: int, nx: int, seed: int) -> np.ndarray:
    """An arbitrary, positive population state [33, nz, ny, nx] (float64):
    planes 0-18 flow (rest near 1, moving near 0.01), 19-25 temperature
    rise, 26-32 O2, in the magnitudes of the 3D workload."""
    rng = np.random.default_rng(seed)
    s = np.empty((33, nz, ny, nx), dtype=np.float64)
    s[0] = rng.uniform(0.97, 1.0, size=(nz, ny, nx))
    s[1:19] = rng.uniform(0.0, 0.01, size=(18, nz, ny, nx))
    s[19:26] = rng.uniform(0.0, 0.3, size=(7, nz, ny, nx))
    s[26:33] = rng.uniform(0.1, 0.2, size=(7, nz, ny, nx))
    return s


def fd_cells3d(w: dict, n: int = 8, seed: int = SEED_ADJOINT3D_FD, depth: int = 6) -> list[tuple[int, int, int]]:
    """``n`` distinct porous cells (z, y, x), seeded, for finite-difference
    checks of the 3D adjoint: drawn from the ``depth`` GDL layers next to
    the CL and the CL layers, away from the x ends."""
    rng = np.random.default_rng(seed)
    z0 = max(w["nz_channel"], w["nz"] - w["nz_cl"] - depth)
    layers = w["nz"] - z0
    nx_in = w["nx"] - 4
    flat = rng.choice(layers * w["ny"] * nx_in, size=n, replace=False)
    out = []
    for i in flat:
        z, r = divmod(int(i), w["ny"] * nx_in)
        y, x = divmod(r, nx_in)
        out.append((z0 + z, y, x + 2))
    return out


def polarisation_sweep(steps: int = 20000) -> list[dict]:
    """Cases of the polarisation / power / heat curves: the flow rate is set
    by the outlet pressure at a fixed inlet pressure (order: outlet pressure,
    then voltage)."""
    cases = []
    for p_out in POLARISATION_P_OUT:
        for v in POLARISATION_V:
            w = base_case()
            w.update(name=f"pol_pout{p_out:g}_V{v:.2f}", nx=200, ny=40, ny_channel=20, ny_gdl=18, ny_cl=2,
                     precision=32, steps=steps, T_in=353.0, V_op=v, phi_gdl=0.4, Da_gdl=2.73e-4,
                     D_f_lat=0.025, pressure_inlet=True, p_in=POLARISATION_P_IN, p_out=p_out)
            cases.append(w)
    return cases
