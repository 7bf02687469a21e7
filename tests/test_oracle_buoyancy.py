"""Pins of the oracle's Boussinesq buoyancy (the thermal-to-flow coupling of
the paper's Section 3 cavity validations): the closed-form buoyant shear
wave of a periodic box, clear and porous, and uniform heating acting as
a plain body force (exact Poiseuille flow).  CPU only."""
import math

import torch

from oracle import lbm2d as L

DT = torch.float64


def _shear_wave(nx, porous, b, ny=3, frac=0.25):
    """theta = sin(k x) at t = 0, fluid at rest, buoyancy b along y, every
    direction periodic.  u_y(x) is divergence-free and advects nothing, so
    theta diffuses, theta = sin(kx) e^{-alpha k^2 t}, and u_y = A(t) sin(kx)
    with dA/dt = -gamma A + phi b theta-amplitude, gamma = nu k^2 + phi nu / K
    (Brinkman-Darcy momentum of the Guo-Zhao model; the Forchheimer term is
    quadratic in the tiny amplitude):
    A = phi b (e^{-alpha k^2 t} - e^{-gamma t}) / (gamma - alpha k^2)."""
    if porous:
        g = L.Geometry(nx, ny, 0, ny, 0, periodic_x=True, periodic_y=True)
        pr = L.Params(reaction=False, buoyancy=(0.0, b), phi_gdl=0.5, Da_gdl=1.0, dx_cm=1e-3, deff_ratio_gdl=1.0)
    else:
        g = L.Geometry(nx, ny, ny, 0, 0, periodic_x=True, periodic_y=True)
        pr = L.Params(reaction=False, buoyancy=(0.0, b), dx_cm=1e-3)
    m = L.Model(g, pr)
    k = 2 * math.pi / nx
    x = torch.arange(nx, dtype=DT).view(1, nx).expand(ny, nx)
    z = torch.zeros(ny, nx, dtype=DT)
    s = m.equilibrium_state(z, z, z, torch.sin(k * x), torch.ones(ny, nx, dtype=DT))
    alpha, phi, inv_k = float(m.alpha[0, 0]), float(m.phi[0, 0]), float(m.inv_k[0, 0])
    gam, a = m.nu * k * k + phi * m.nu * inv_k, alpha * k * k
    n = int(frac / (m.nu * k * k))
    s = m.run(s, n)
    uy = m.fields(s)["uy"].mean(0)
    A = float((uy * torch.sin(k * x[0])).sum() * 2 / nx)
    exact = phi * b * (math.exp(-a * n) - math.exp(-gam * n)) / (gam - a)
    return A / exact - 1


def test_buoyant_shear_wave_clear_fluid_second_order():
    e16, e32 = _shear_wave(16, False, 1e-6), _shear_wave(32, False, 1e-6)
    print(f"clear: rel err {e16:.3e} (nx 16), {e32:.3e} (nx 32)")
    assert abs(e16) < 2e-2
    assert 3.5 < e16 / e32 < 4.5


def test_buoyant_shear_wave_porous_medium_converges():
    errs = [_shear_wave(nx, True, 1e-9) for nx in (16, 32, 64)]
    print("porous: rel err", errs)
    assert abs(errs[0]) < 5e-3 and abs(errs[2]) < 1e-4
    assert abs(errs[0]) > 3 * abs(errs[1]) > 9 * abs(errs[2])


def test_uniform_heating_is_a_body_force():
    # theta = theta0 everywhere (adiabatic walls, no reaction) and buoyancy
    # along x: the force is b theta0, and the flow is plane Poiseuille flow
    # to round-off (half-way walls, magic relaxation rates).  The D2Q5
    # scheme's O(u^2) error lets the sheared flow perturb theta by a
    # relative ~1e-12 at this amplitude (~1e-8 at a 100 times larger b).
    nx, H, b, theta0 = 5, 9, 2e-8, 3.0
    m = L.Model(L.Geometry(nx, H, H, 0, 0, periodic_x=True),
                L.Params(tau_f=1.0, reaction=False, buoyancy=(b, 0.0), dx_cm=1e-3))
    z = torch.zeros(H, nx, dtype=DT)
    s = m.equilibrium_state(z, z, z, torch.full((H, nx), theta0, dtype=DT), torch.ones(H, nx, dtype=DT))
    f = m.fields(m.run(s, 6000))
    assert float((f["theta"] - theta0).abs().max()) < 1e-10
    y = torch.arange(H, dtype=DT)
    exact = b * theta0 / (2 * m.nu) * (y + 0.5) * (H - 0.5 - y)
    assert float((f["ux"] - exact.view(H, 1)).abs().max() / exact.max()) < 1e-11
    assert float(f["uy"].abs().max()) < 1e-7 * float(exact.max())
