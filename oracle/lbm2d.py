"""Plain FP64 oracle of one coupled lattice-Boltzmann time step (2D).

TEST INFRASTRUCTURE ONLY (see the package docstring).  Float64 PyTorch CPU
tensors shaped [plane, ny, nx]; x runs from the inlet (column 0) to the
outlet (column nx-1), y from the channel-side wall (row 0) through the gas
diffusion layer (GDL) to the catalyst layer (CL, last rows).

State convention: a *state* is the set of post-collision populations
(9 flow planes, 5 temperature-rise planes, 5 O2 planes) ready to stream.
One step is: stream (pull) with half-way bounce-back -> open-boundary
columns -> macroscopic fields -> D2Q9 MRT collision with porous drag ->
CL reaction -> two D2Q5 MRT collisions -> new state.  Fields and
observables "of a state" are evaluated on the pre-collision populations
obtained by streaming that state and applying the boundary columns.

Readings taken where the paper is silent or garbled are stated at the
place they are used, each tagged [R#].
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import torch

DT = torch.float64
RHO0 = 1.0  # mean fluid density in lattice units (Section 2.1, Eq. 5)


# --------------------------------------------------------------------------
# Lattices
# --------------------------------------------------------------------------
def d2q9_velocities() -> list[tuple[int, int]]:
    """Eq. 2 with c = 1: e_0 = 0; e_1..4 = [cos((i-1)pi/2), sin((i-1)pi/2)];
    e_5..8 = sqrt(2)[cos((i-5)pi/2 + pi/4), sin((i-5)pi/2 + pi/4)]."""
    e = [(0, 0)]
    for i in range(1, 5):
        a = (i - 1) * math.pi / 2
        e.append((round(math.cos(a)), round(math.sin(a))))
    for i in range(5, 9):
        a = (i - 5) * math.pi / 2 + math.pi / 4
        e.append((round(math.sqrt(2) * math.cos(a)), round(math.sqrt(2) * math.sin(a))))
    return e


def d2q5_velocities() -> list[tuple[int, int]]:
    """Eq. 9: the rest vector and the four axis vectors of Eq. 2."""
    return d2q9_velocities()[:5]


def opposite(e: list[tuple[int, int]]) -> list[int]:
    return [e.index((-ex, -ey)) for (ex, ey) in e]


E9 = d2q9_velocities()
E5 = d2q5_velocities()
OPP9 = opposite(E9)
OPP5 = opposite(E5)

# Eq. 3: D2Q9 transformation matrix, moments (rho, e, zeta, jx, qx, jy, qy, pxx, pxy).
M9 = torch.tensor([
    [1, 1, 1, 1, 1, 1, 1, 1, 1],
    [-4, -1, -1, -1, -1, 2, 2, 2, 2],
    [4, -2, -2, -2, -2, 1, 1, 1, 1],
    [0, 1, 0, -1, 0, 1, -1, -1, 1],
    [0, -2, 0, 2, 0, 1, -1, -1, 1],
    [0, 0, 1, 0, -1, 1, 1, -1, -1],
    [0, 0, -2, 0, 2, 1, 1, -1, -1],
    [0, 1, -1, 1, -1, 0, 0, 0, 0],
    [0, 0, 0, 0, 0, 1, -1, 1, -1],
], dtype=DT)
# The rows of M are orthogonal: M M^T = diag(9, 36, 36, 6, 12, 6, 12, 4, 4),
# so M^-1 = M^T diag(M M^T)^-1.
M9_INV = M9.T / (M9 * M9).sum(1)

# Eq. 10: D2Q5 transformation matrix and relaxation rates.
N5 = torch.tensor([
    [1, 1, 1, 1, 1],
    [0, 1, 0, -1, 0],
    [0, 0, 1, 0, -1],
    [-4, 1, 1, 1, 1],
    [0, 1, -1, 1, -1],
], dtype=DT)
# N N^T = diag(5, 2, 2, 20, 4), so N^-1 = N^T diag(N N^T)^-1.
N5_INV = N5.T / (N5 * N5).sum(1)
_S3 = math.sqrt(3.0)
Q5 = torch.tensor([0.0, 6 / (3 + _S3), 6 / (3 + _S3), 6 / (3 + 2 * _S3), 6 / (3 + 2 * _S3)], dtype=DT)


def relaxation_d2q9(tau: float) -> torch.Tensor:
    """Diagonal of S (Section 2.1): (s_0, 1/tau, 1/tau, 0, s_q, 0, s_q, 1/tau,
    1/tau) with s_q = 8(2 - 1/tau)/(8 - 1/tau).

    [R0] The paper prints s_0 = 0.  With its equilibrium density moment
    fixed at rho0 (Eq. 5) and the pressure taken from the moving populations,
    s_0 = 0 leaves the density moment as a second conserved field coupled to
    the pressure, and the scheme is linearly unstable (von Neumann growth
    factor about 1.4 per step at tau = 0.65).  The density moment is relaxed
    at the rate of the other two scalar moments, s_0 = 1/tau, which makes the
    (rho, e, zeta) block that of the incompressible BGK model the equilibrium
    comes from, conserves the moving-population sum exactly in clear fluid,
    and is stable.
    """
    s = 1.0 / tau
    sq = 8.0 * (2.0 - s) / (8.0 - s)
    return torch.tensor([s, s, s, 0.0, sq, 0.0, sq, s, s], dtype=DT)


# --------------------------------------------------------------------------
# Problem description
# --------------------------------------------------------------------------
@dataclass
class Geometry:
    nx: int
    ny: int
    ny_channel: int
    ny_gdl: int
    ny_cl: int
    periodic_x: bool = False
    periodic_y: bool = False

    def __post_init__(self):
        if self.ny_channel + self.ny_gdl + self.ny_cl != self.ny:
            raise ValueError("layer rows must sum to ny")
        if self.nx < 3 or self.ny < 1:
            raise ValueError("lattice too small")


@dataclass
class Params:
    """Inputs of the model.  Physical constants default to the paper's
    Nomenclature; lattice choices (tau_f, D_f_lat) and the heat capacities
    are defaults the paper does not fix [R1]."""
    tau_f: float = 0.65          # flow relaxation time; 3 nu = tau - 1/2 (Section 2.1)
    D_f_lat: float = 0.0125      # clear-gas O2 diffusivity in lattice units [R1]
    Re: float = 10.0             # inlet Reynolds number U_avg H_channel / nu [R2]
    T_in: float = 353.0          # inlet / operating temperature, K
    c_in: float = 1.0            # inlet O2 concentration / C_ref [R3]
    V_op: float = 0.6            # operating voltage, V
    phi_gdl: float = 0.4         # porosity of GDL and CL (layered inputs)
    Da_gdl: float = 1e-3         # Darcy number K / h_gdl^2 (layered inputs) [R4]
    deff_ratio_gdl: float = 0.0  # D_eff / D_f in GDL and CL; 0 selects Eq. 18
    dp_lat: float = 0.0          # Kozeny-Carman particle diameter (lattice); >0 derives K from porosity
    gdl_thickness_cm: float = 0.0254  # [R4]
    dx_cm: float = 0.0           # >0 overrides gdl_thickness_cm / ny_gdl
    D_O2: float = 5.2197e-2      # cm^2/s (Nomenclature)
    aj0_ref: float = 1.0e-4      # A/cm^3 (Nomenclature)
    C_ref: float = 17.808e-6     # mol/cm^3 [R3]
    alpha_c: float = 1.0
    faraday: float = 96487.0
    R_gas: float = 8.314
    E_over_R: float = 16456.0    # Eq. 17
    T_arrh: float = 353.15       # Eq. 17
    U0_slope: float = 0.0025     # Eq. 16
    U0_icept: float = 0.2329     # Eq. 16
    k_f: float = 0.026           # W/(m K) (Nomenclature)
    k_s: float = 1.5             # W/(m K) (Nomenclature)
    rhocp_f: float = 1.0e-3      # J/(cm^3 K) [R1]
    rhocp_s: float = 1.6         # J/(cm^3 K) [R1]
    body_force: tuple = (0.0, 0.0)  # test mode only: acceleration in lattice units [R5]
    buoyancy: tuple = (0.0, 0.0)    # Boussinesq acceleration per kelvin of T - T_in, lattice units [R20]
    sigma_energy: bool = False   # porous energy equation with the heat-capacity ratio sigma [R21]
    heat_physical: bool = False  # reaction heat with the irreversible part counted positive [R22]
    reaction: bool = True
    pressure_inlet: bool = False  # Section 4's pressure-driven flow: inlet pressure p_in, outlet p_out [R17]
    p_in: float = 0.0            # lattice inlet pressure when pressure_inlet (Re is then an output)
    p_out: float = 0.0           # lattice outlet pressure (Section 5 varies it to set the flow rate) [R17]
    butler_volmer: bool = False  # Eq. 13 with its anodic branch [R18]; False: the printed Tafel form
    alpha_a: float = 1.0         # anodic transfer coefficient (not given by the paper) [R18]
    thin_cl: bool = False        # CL of negligible thickness: a reactive wall under the GDL [R19]
    thin_cl_cm: float = 0.0      # thickness whose volumetric a j0 the film carries; <= 0: one lattice spacing

    @staticmethod
    def from_workload(w: dict) -> "Params":
        p = Params()
        for k in ("tau_f", "D_f_lat", "Re", "T_in", "c_in", "V_op", "phi_gdl",
                  "Da_gdl", "deff_ratio_gdl", "p_in", "p_out", "alpha_a", "aj0_ref", "thin_cl_cm"):
            if k in w:
                setattr(p, k, float(w[k]))
        if "buoyancy" in w:
            p.buoyancy = tuple(float(v) for v in w["buoyancy"])
        p.pressure_inlet = bool(w.get("pressure_inlet", False))
        p.butler_volmer = bool(w.get("butler_volmer", False))
        p.thin_cl = bool(w.get("thin_cl", False))
        p.sigma_energy = bool(w.get("sigma_energy", False))
        p.heat_physical = bool(w.get("heat_physical", False))
        if w.get("dp_over_hgdl", 0.0) > 0:
            p.dp_lat = w["dp_over_hgdl"] * w["ny_gdl"]
        return p


def geometry_from_workload(w: dict) -> Geometry:
    return Geometry(w["nx"], w["ny"], w["ny_channel"], w["ny_gdl"], w["ny_cl"])


# --------------------------------------------------------------------------
# Small helpers
# --------------------------------------------------------------------------
def _safe_sqrt(a: torch.Tensor) -> torch.Tensor:
    """sqrt with derivative 0 at a = 0 (the model's composite maps are C^1
    there, see the velocity recovery).  A complex argument (complex-step
    differentiation in the tests) is tested on its real part."""
    pos = (a.real if a.is_complex() else a) > 0
    return torch.where(pos, torch.sqrt(torch.where(pos, a, torch.ones_like(a))), torch.zeros_like(a))


def catalyst_reaction(pr: "Params", dt: float, theta, c, rhocp):
    """Catalyst-layer oxygen reduction over one step of length dt (s); see
    Model.reaction for the definitions (Eqs. 12-17, [R11], [R12]).

    [R18] Butler-Volmer option: Eq. 13 with the anodic branch,
    j = -a j0 [ c exp(-alpha_c F eta / (R T)) - exp(alpha_a F eta / (R T)) ],
    concentration dependence on the cathodic branch only.  The O2 balance
    4 F C_ref dc/dt = -(k c - k_a) is again integrated exactly over the
    step: c relaxes toward c_eq = k_a / k = exp((alpha_a + alpha_c) F eta
    / (R T)) at the rate kappa, s_c = (c - c_eq)(1 - exp(-kappa)).
    """
    T = pr.T_in + theta
    U0 = pr.U0_slope * T + pr.U0_icept
    eta = pr.V_op - U0
    aj0 = pr.aj0_ref * torch.exp(-pr.E_over_R * (1.0 / T - 1.0 / pr.T_arrh))
    k = aj0 * torch.exp(-pr.alpha_c * pr.faraday * eta / (pr.R_gas * T))
    four_f_cref = 4.0 * pr.faraday * pr.C_ref
    kappa = k * dt / four_f_cref
    if pr.butler_volmer:
        c_eq = torch.exp((pr.alpha_a + pr.alpha_c) * pr.faraday * eta / (pr.R_gas * T))
        s_c = -(c - c_eq) * torch.expm1(-kappa)
    else:
        s_c = -c * torch.expm1(-kappa)
    j_eff = -four_f_cref * s_c / dt
    if pr.heat_physical:
        # [R22] with dU0/dT > 0 and eta < 0 the printed -j eta is negative;
        # the irreversible heat is |j| |eta|, the entropic part stays -j T dU0/dT
        Q = -j_eff * (T * pr.U0_slope - eta)
    else:
        Q = -j_eff * (eta + T * pr.U0_slope)
    S_T = Q * dt / rhocp
    return s_c, S_T, j_eff, Q, k


def _mv(mat: torch.Tensor, planes: torch.Tensor) -> torch.Tensor:
    """Matrix times a stack of planes: out[i] = sum_j mat[i, j] planes[j]
    (the real matrix is taken in the planes' type, complex in the tests'
    complex-step differentiation)."""
    return torch.einsum("ij,j...->i...", mat.to(planes.dtype), planes)


# --------------------------------------------------------------------------
# The model
# --------------------------------------------------------------------------
class Model:
    """Coupled D2Q9 / 2 x D2Q5 MRT model on one lattice.

    ``phi``, ``inv_k`` and ``d_eff`` are optional per-cell float64 tensors
    [ny, nx] (porosity, inverse permeability and O2 diffusivity, both in
    lattice units); a missing one is built from the layered inputs in
    ``Params``.  They may require grad (see ``adjoint2d``).
    """

    def __init__(self, geom: Geometry, prm: Params, phi=None, inv_k=None, d_eff=None):
        self.g, self.p = geom, prm
        ny, nx = geom.ny, geom.nx
        self.nu = (prm.tau_f - 0.5) / 3.0            # 3 nu / dt = tau - 0.5 (Section 2.1)
        self.S9 = relaxation_d2q9(prm.tau_f)
        # Lattice <-> physical scales [R4]: dx from the GDL thickness, dt from
        # the O2 diffusivity, D_lat = D_phys dt / dx^2.
        if prm.dx_cm > 0:
            self.dx = prm.dx_cm
        else:
            self.dx = prm.gdl_thickness_cm / geom.ny_gdl
        self.dt = prm.D_f_lat * self.dx ** 2 / prm.D_O2
        self.u_avg = (prm.Re * self.nu / geom.ny_channel
                      if geom.ny_channel > 0 and not prm.pressure_inlet else 0.0)
        if prm.thin_cl and (geom.ny_cl != 0 or geom.ny_gdl < 1 or geom.periodic_y):
            raise ValueError("the thin-film CL lies under the GDL: ny_cl = 0, ny_gdl >= 1, walls in y")
        self.thin = prm.thin_cl * (prm.thin_cl_cm if prm.thin_cl_cm > 0 else self.dx)

        rows = torch.arange(ny).view(ny, 1).expand(ny, nx)
        self.is_channel = rows < geom.ny_channel
        self.is_cl = rows >= geom.ny_channel + geom.ny_gdl
        porous = ~self.is_channel

        # Porosity: 1 in the clear channel, phi_gdl in GDL and CL (Section 4) [R6].
        if phi is None:
            phi = torch.where(porous, torch.full((ny, nx), prm.phi_gdl, dtype=DT),
                              torch.ones((ny, nx), dtype=DT))
        self.phi = phi
        # Inverse permeability: channel K = infinity [R6]; porous layers
        # K = Da h^2 with h the GDL thickness [R4], or the Kozeny-Carman law
        # of Eq. 7 on the porosity when a particle diameter is given.
        if inv_k is None:
            if prm.dp_lat > 0:
                inv_k = (1.0 - phi) ** 2 / (0.0067 * phi ** 3 * prm.dp_lat ** 2)
            else:
                k_lat = prm.Da_gdl * geom.ny_gdl ** 2
                inv_k_gdl = 1.0 / k_lat if k_lat > 0 else 0.0
                inv_k = torch.where(porous, torch.full((ny, nx), inv_k_gdl, dtype=DT),
                                    torch.zeros((ny, nx), dtype=DT))
        self.inv_k = inv_k
        # O2 diffusivity: Bruggeman, Eq. 18, or a given ratio in the porous layers.
        if d_eff is None:
            if prm.deff_ratio_gdl > 0:
                d_eff = torch.where(porous, torch.full((ny, nx), prm.deff_ratio_gdl * prm.D_f_lat, dtype=DT),
                                    torch.full((ny, nx), prm.D_f_lat, dtype=DT))
            else:
                d_eff = phi ** 1.5 * prm.D_f_lat
        self.d_eff = d_eff
        # Eq. 19: effective thermal diffusivity, then to lattice units
        # (conductivities W/(m K) -> W/(cm K)).
        self.rhocp = phi * prm.rhocp_f + (1.0 - phi) * prm.rhocp_s
        k_eff = (prm.k_f * phi + prm.k_s * (1.0 - phi)) / 100.0
        if prm.sigma_energy:
            # [R21] sigma dT/dt + u.grad T = div(alpha_m grad T) + Q / (rho c_p)_f,
            # sigma = (rho c_p)_eff / (rho c_p)_f, alpha_m = k_eff / (rho c_p)_f:
            # the temperature lattice conserves sigma T.
            self.sigma = self.rhocp / prm.rhocp_f
            self.alpha = k_eff / prm.rhocp_f * self.dt / self.dx ** 2
        else:
            self.sigma = torch.ones_like(self.rhocp)
            self.alpha = k_eff / self.rhocp * self.dt / self.dx ** 2
        # Eq. 10: b = 20 sqrt(3) alpha - 4 for each scalar lattice.
        self.b_T = 20.0 * _S3 * self.alpha - 4.0
        self.b_C = 20.0 * _S3 * self.d_eff - 4.0
        # [R10] Scalar material of the outlet column: its nodes collide the
        # copied scalar populations with the b and (rho c_p) of column nx-2,
        # so the last two columns act as one medium for temperature and O2
        # ("fully developed", Section 4).  With the node's own b the
        # equilibrium fluxes (4 + b) X / 20 of the two columns differ and the
        # outlet becomes a source or sink proportional to X (unstable for
        # porosity fields); for layers uniform in x both choices coincide.
        self.b_T_coll, self.b_C_coll, self.rhocp_coll = self.b_T, self.b_C, self.rhocp
        self.sigma_coll = self.sigma
        if not geom.periodic_x:
            last = lambda a: torch.cat([a[:, :-1], a[:, -2:-1]], dim=1)
            self.b_T_coll, self.b_C_coll, self.rhocp_coll = last(self.b_T), last(self.b_C), last(self.rhocp)
            self.sigma_coll = last(self.sigma)
        # Eq. 7 and Eq. 8 coefficients (dt = 1).
        self.F_phi = 0.143 * phi ** (-1.5)
        self.sqrt_inv_k = _safe_sqrt(inv_k)
        self.l0 = 0.5 + phi * self.nu * inv_k / 4.0
        self.l1 = phi * self.F_phi * self.sqrt_inv_k / 2.0
        # Link masks for streaming: inside[q][y, x] is True when the source
        # node x - e_q lies in the lattice (no wall crossed).
        self._inside9 = [self._link_inside(ex, ey) for (ex, ey) in E9]
        self._inside5 = self._inside9[:5]

    # ---------------------------------------------------------------- geometry
    def _link_inside(self, ex: int, ey: int) -> torch.Tensor:
        ny, nx = self.g.ny, self.g.nx
        ys = torch.arange(ny).view(ny, 1).expand(ny, nx) - ey
        xs = torch.arange(nx).view(1, nx).expand(ny, nx) - ex
        ok = torch.ones((ny, nx), dtype=torch.bool)
        if not self.g.periodic_y:
            ok &= (ys >= 0) & (ys < ny)
        if not self.g.periodic_x:
            ok &= (xs >= 0) & (xs < nx)
        return ok

    def inlet_velocity(self) -> torch.Tensor:
        """Parabolic inlet profile over the channel rows [R7]: zero at the
        wall y = -1/2 and at the channel/GDL interface y = H - 1/2, mean
        U_avg = Re nu / H over the continuous cross-section."""
        H = self.g.ny_channel
        y = torch.arange(H, dtype=DT)
        return 6.0 * self.u_avg * (y + 0.5) * (H - 0.5 - y) / H ** 2

    # ------------------------------------------------------------- equilibria
    def meq(self, p, ux, uy, phi):
        """Eq. 5: porous equilibrium moments (rho0 = 1)."""
        u2 = ux * ux + uy * uy
        return torch.stack([
            torch.full_like(p, RHO0),
            -4.0 * RHO0 + 6.0 * phi * p + 3.0 * RHO0 * u2 / phi,
            4.0 * RHO0 - 9.0 * phi * p - 3.0 * RHO0 * u2 / phi,
            RHO0 * ux, -RHO0 * ux, RHO0 * uy, -RHO0 * uy,
            RHO0 * (ux * ux - uy * uy) / phi,
            RHO0 * ux * uy / phi,
        ])

    def feq(self, p, ux, uy, phi):
        return _mv(M9_INV, self.meq(p, ux, uy, phi))

    @staticmethod
    def neq(X, ux, uy, b, sigma=None):
        """Eq. 10: scalar equilibrium moments (X, u_x X, u_y X, b X, 0) [R8].
        [R21] With the heat-capacity ratio: (sigma X, u_x X, u_y X,
        (b + 4 (1 - sigma)) X, 0), which keeps the second moments of the
        moving populations, (4 + b) X / 10, and so the diffusivity."""
        if sigma is None:
            return torch.stack([X, ux * X, uy * X, b * X, torch.zeros_like(X)])
        return torch.stack([sigma * X, ux * X, uy * X, (b + 4.0 * (1.0 - sigma)) * X, torch.zeros_like(X)])

    def geq(self, X, ux, uy, b, sigma=None):
        return _mv(N5_INV, self.neq(X, ux, uy, b, sigma))

    @staticmethod
    def forcing_moments(ux, uy, Fx, Fy, phi):
        """Eq. 6: porous forcing in moment space.  G0..G6 as printed; G7 and
        G8 are read as the velocity derivative of Eq. 5's p_xx and p_xy along
        F, 2 rho0 (u_x F_x - u_y F_y)/phi and rho0 (u_x F_y + u_y F_x)/phi,
        which is what the printed G1..G6 are for e and zeta [R13]."""
        uF = ux * Fx + uy * Fy
        return torch.stack([
            torch.zeros_like(uF),
            6.0 * RHO0 * uF / phi, -6.0 * RHO0 * uF / phi,
            RHO0 * Fx, -RHO0 * Fx, RHO0 * Fy, -RHO0 * Fy,
            2.0 * RHO0 * (ux * Fx - uy * Fy) / phi,
            RHO0 * (ux * Fy + uy * Fx) / phi,
        ])

    # ---------------------------------------------------------------- macros
    def flow_macros(self, f, phi, l0, l1, inv_k, sqrt_inv_k, F_phi, theta=None):
        """Eq. 8 and the pressure relation of Section 2.1.

        v = sum e_i f_i / rho0 (+ dt phi a / 2 in body-force test mode [R5]);
        u = v / (l0 + sqrt(l0^2 + l1 |v|));
        F = -phi nu K^-1 u - phi F_phi K^-1/2 |u| u (+ phi a)   (Eq. 7);
        p = (0.6/phi) sum_{i=1..8} f_i - 6 rho0 |u|^2 / (15 phi^2).
        [R20] Buoyancy: a = body force + b theta, theta = T - T_in of the same
        node's temperature populations (the Boussinesq force -beta g (T - T_in)
        of the cavity validations in Section 3, b = -beta g).
        """
        vx = sum(E9[q][0] * f[q] for q in range(9)) / RHO0
        vy = sum(E9[q][1] * f[q] for q in range(9)) / RHO0
        ax, ay = self.p.body_force
        bx, by = self.p.buoyancy
        if bx != 0.0 or by != 0.0:
            ax = ax + bx * theta
            ay = ay + by * theta
        vx = vx + 0.5 * phi * ax
        vy = vy + 0.5 * phi * ay
        vmag = _safe_sqrt(vx * vx + vy * vy)
        den = l0 + torch.sqrt(l0 * l0 + l1 * vmag)
        ux, uy = vx / den, vy / den
        umag = _safe_sqrt(ux * ux + uy * uy)
        drag = phi * self.nu * inv_k + phi * F_phi * sqrt_inv_k * umag
        Fx = phi * ax - drag * ux
        Fy = phi * ay - drag * uy
        p = (0.6 / phi) * sum(f[q] for q in range(1, 9)) - 6.0 * RHO0 * (ux * ux + uy * uy) / (15.0 * phi * phi)
        return ux, uy, p, Fx, Fy

    # ------------------------------------------------------------- streaming
    def stream(self, post: torch.Tensor) -> torch.Tensor:
        """LHS of Eq. 1 and of the scalar LBE of Eq. 10, pulled:
        f_q(x) = f*_q(x - e_q); where the link crosses a wall, half-way
        bounce-back f_q(x) = f*_{opp q}(x) (no slip for the flow, zero flux
        for temperature and O2, Section 4) [R9]."""
        out = torch.empty_like(post)
        blocks = ((0, E9, OPP9, self._inside9), (9, E5, OPP5, self._inside5), (14, E5, OPP5, self._inside5))
        for base, E, OPP, inside in blocks:
            for q, (ex, ey) in enumerate(E):
                src = torch.roll(post[base + q], shifts=(ey, ex), dims=(0, 1))
                out[base + q] = torch.where(inside[q], src, post[base + OPP[q]])
        if self.p.thin_cl and self.p.reaction:
            d_c, d_t, _, _ = self.surface_reaction(post)
            y = self.g.ny - 1
            out[9 + 4, y] = out[9 + 4, y] + d_t * self.sigma[y]  # reflected temperature population (-y) [R21]
            out[14 + 4, y] = out[14 + 4, y] - d_c    # reflected O2 population (-y)
        return out

    def surface_reaction(self, post: torch.Tensor):
        """[R19] Thin-film CL (the paper's CL of negligible thickness): the
        wall half a cell below the last GDL row reacts.  Each bottom node's
        populations that cross that wall (index 2 of Eq. 9, moving +y) are
        reflected minus the O2 the film consumes and plus the heat it
        releases.  The film carries the volumetric rate of Eq. 13 over a
        thickness delta: k_s = a j0(T) delta exp(-alpha_c F eta / (R T))
        [A/cm^2 per unit c].  Wall values: c_w = g_in / a and theta_w =
        g_T,in / a_T with a = (4 + b)/20 the equilibrium weight of a moving
        population (zero wall-normal velocity).  Over one step, exactly in
        time for the incident population: kappa_s = k_s dt / (4 F C_ref dx),
        d_c = (g_in - a c_eq)(1 - exp(-kappa_s / a)) (c_eq = 0 for Tafel, the
        Butler-Volmer value [R18] otherwise); heat d_T = 4 F C_ref d_c
        (eta + T dU0/dT) / (rho c_p) (Eq. 15).  Returns per column (d_c, d_T,
        i_s [A/cm^2], Q_s [W/cm^2])."""
        pr, y = self.p, self.g.ny - 1
        a_t = (4.0 + self.b_T[y]) / 20.0
        a_c = (4.0 + self.b_C[y]) / 20.0
        g_t, g_c = post[9 + 2, y], post[14 + 2, y]
        T = pr.T_in + g_t / a_t
        eta = pr.V_op - (pr.U0_slope * T + pr.U0_icept)
        aj0 = pr.aj0_ref * torch.exp(-pr.E_over_R * (1.0 / T - 1.0 / pr.T_arrh))
        k_s = aj0 * self.thin * torch.exp(-pr.alpha_c * pr.faraday * eta / (pr.R_gas * T))
        four_f_cref = 4.0 * pr.faraday * pr.C_ref
        kappa_s = k_s * self.dt / (four_f_cref * self.dx)
        if pr.butler_volmer:
            c_eq = torch.exp((pr.alpha_a + pr.alpha_c) * pr.faraday * eta / (pr.R_gas * T))
        else:
            c_eq = torch.zeros_like(T)
        d_c = -(g_c - a_c * c_eq) * torch.expm1(-kappa_s / a_c)
        ehs = (T * pr.U0_slope - eta) if pr.heat_physical else (eta + T * pr.U0_slope)
        d_t = four_f_cref * d_c * ehs / self.rhocp[y]
        i_s = four_f_cref * self.dx * d_c / self.dt
        return d_c, d_t, i_s, i_s * ehs

    def open_boundaries(self, pre: torch.Tensor) -> torch.Tensor:
        """Inlet and outlet columns by non-equilibrium extrapolation [R7].

        Inlet (x = 0, channel rows): f = f_eq(p_1, u_in) + (f_1 - f_eq(p_1, u_1));
        scalars g = g_eq(X_in, u_in) + (g_1 - g_eq(X_1, u_1)), X_in = 0 for the
        temperature rise and c_in for O2 (Dirichlet, Section 4).
        Outlet (x = nx-1, all rows): f = f_eq(p_out, u_2) + (f_2 - f_eq(p_2, u_2)),
        with column 2 = nx-2; scalars copied from column nx-2 (fully
        developed, Section 4), and collided with column nx-2's scalar
        material [R10].
        """
        if self.g.periodic_x:
            return pre
        out = pre.clone()
        nx, H = self.g.nx, self.g.ny_channel
        if H > 0:
            f1 = pre[0:9, :H, 1]
            ux1, uy1, p1, _, _ = self.flow_macros(
                f1, self.phi[:H, 1], self.l0[:H, 1], self.l1[:H, 1], self.inv_k[:H, 1],
                self.sqrt_inv_k[:H, 1], self.F_phi[:H, 1], pre[9:14, :H, 1].sum(0) / self.sigma[:H, 1])
            # [R17] Section 4 drives the flow by a pressure difference between
            # inlet and outlet: the inlet nodes get the pressure p_in with the
            # velocity of column 1 (non-equilibrium extrapolation, as the
            # outlet), the outlet has p_out; the scalars stay Dirichlet.
            if self.p.pressure_inlet:
                ubx, uby, pb = ux1, uy1, torch.full_like(p1, self.p.p_in)
            else:  # [R7]: parabolic velocity, pressure of column 1
                ubx, uby, pb = self.inlet_velocity(), torch.zeros_like(p1), p1
            zero = torch.zeros_like(p1)
            out[0:9, :H, 0] = self.feq(pb, ubx, uby, self.phi[:H, 0]) + f1 - self.feq(p1, ux1, uy1, self.phi[:H, 1])
            gT1, gC1 = pre[9:14, :H, 1], pre[14:19, :H, 1]
            th1, c1 = gT1.sum(0) / self.sigma[:H, 1], gC1.sum(0)
            out[9:14, :H, 0] = (self.geq(zero, ubx, uby, self.b_T[:H, 0], self.sigma[:H, 0]) + gT1
                                - self.geq(th1, ux1, uy1, self.b_T[:H, 1], self.sigma[:H, 1]))
            cin = torch.full_like(p1, self.p.c_in)
            out[14:19, :H, 0] = (self.geq(cin, ubx, uby, self.b_C[:H, 0]) + gC1
                                 - self.geq(c1, ux1, uy1, self.b_C[:H, 1]))
        c2 = nx - 2
        f2 = pre[0:9, :, c2]
        ux2, uy2, p2, _, _ = self.flow_macros(
            f2, self.phi[:, c2], self.l0[:, c2], self.l1[:, c2], self.inv_k[:, c2],
            self.sqrt_inv_k[:, c2], self.F_phi[:, c2], pre[9:14, :, c2].sum(0) / self.sigma[:, c2])
        out[0:9, :, nx - 1] = (self.feq(torch.full_like(p2, self.p.p_out), ux2, uy2, self.phi[:, nx - 1]) + f2
                               - self.feq(p2, ux2, uy2, self.phi[:, c2]))
        out[9:19, :, nx - 1] = pre[9:19, :, c2]
        return out

    def pre_collision(self, post: torch.Tensor) -> torch.Tensor:
        return self.open_boundaries(self.stream(post))

    # ------------------------------------------------------------- reaction
    def reaction(self, theta, c, rhocp):
        """Catalyst-layer oxygen reduction over one time step (Eqs. 12-17).

        Returns (s_c, S_T, j_eff, Q, k):
          k     = a j0(T) exp(-alpha_c F eta / (R T))       [A/cm^3 per unit c]
                  with eta = V - U0(T) (Eqs. 13, 14, 16) and a j0(T) of Eq. 17;
          s_c   = c (1 - exp(-kappa)), kappa = k dt / (4 F C_ref): O2 (relative
                  to C_ref) consumed in the step by the 4-electron reaction of
                  Eq. 12, integrated exactly over the step [R11];
          j_eff = -4 F C_ref s_c / dt                         [A/cm^3];
          Q     = -j_eff (eta + T dU0/dT)                      [W/cm^3] (Eq. 15);
          S_T   = Q dt / (rho c_p)_eff                         [K] per step [R12].
        """
        return catalyst_reaction(self.p, self.dt, theta, c, rhocp)

    # ------------------------------------------------------------- one step
    def collide(self, pre: torch.Tensor) -> torch.Tensor:
        """Collision of every node (Eq. 1 RHS, Eq. 10 RHS) plus the CL source."""
        f, gT, gC = pre[0:9], pre[9:14], pre[14:19]
        ux, uy, p, Fx, Fy = self.flow_macros(f, self.phi, self.l0, self.l1, self.inv_k,
                                             self.sqrt_inv_k, self.F_phi, gT.sum(0) / self.sigma_coll)
        phi = self.phi
        # Eq. 1 in moment space: m* = m - S (m - m_eq) + (I - S/2) G.
        m = _mv(M9, f)
        meq = self.meq(p, ux, uy, phi)
        G = self.forcing_moments(ux, uy, Fx, Fy, phi)
        S = self.S9.view(9, 1, 1)
        m_post = m - S * (m - meq) + (1.0 - S / 2.0) * G
        f_post = _mv(M9_INV, m_post)

        theta, c = gT.sum(0) / self.sigma_coll, gC.sum(0)
        if self.p.reaction:
            s_c, S_T, _, _, _ = self.reaction(theta, c, self.rhocp_coll)
            zero = torch.zeros_like(theta)
            src_C = torch.where(self.is_cl, -s_c, zero)
            src_T = torch.where(self.is_cl, S_T, zero)
        else:
            src_C = src_T = torch.zeros_like(theta)
        gT_post = self._collide_scalar(gT, theta, ux, uy, self.b_T_coll, src_T, self.sigma_coll)
        gC_post = self._collide_scalar(gC, c, ux, uy, self.b_C_coll, src_C)
        return torch.cat([f_post, gT_post, gC_post])

    def _collide_scalar(self, g, X, ux, uy, b, src, sigma=None):
        """Eq. 10 RHS in moment space, n* = n - Q (n - n_eq), plus the source
        injected with the rest-equilibrium moments src (1, 0, 0, b, 0) [R14]
        (with sigma [R21]: src (sigma, 0, 0, b + 4 (1 - sigma), 0))."""
        n = _mv(N5, g)
        n_post = n - Q5.view(5, 1, 1) * (n - self.neq(X, ux, uy, b, sigma))
        n_post = n_post + self.neq(src, torch.zeros_like(src), torch.zeros_like(src), b, sigma)
        return _mv(N5_INV, n_post)

    def step(self, post: torch.Tensor) -> torch.Tensor:
        return self.collide(self.pre_collision(post))

    def run(self, post: torch.Tensor, nsteps: int) -> torch.Tensor:
        for _ in range(nsteps):
            post = self.step(post)
        return post

    # ---------------------------------------------------------- initial state
    def equilibrium_state(self, p, ux, uy, theta, c) -> torch.Tensor:
        """Post-collision state equal to the equilibria of given fields."""
        return torch.cat([self.feq(p, ux, uy, self.phi),
                          self.geq(theta, ux, uy, self.b_T, self.sigma),
                          self.geq(c, ux, uy, self.b_C)])

    def initial_state(self) -> torch.Tensor:
        """Fluid at rest at zero pressure, temperature rise 0, O2 at the inlet
        value everywhere [R15]."""
        ny, nx = self.g.ny, self.g.nx
        z = torch.zeros((ny, nx), dtype=DT)
        return self.equilibrium_state(z, z, z, z, torch.full((ny, nx), self.p.c_in, dtype=DT))

    # ----------------------------------------------------------- read-outs
    def fields(self, post: torch.Tensor) -> dict:
        """u_x, u_y, p (lattice), T (K), c (relative) of the pre-collision
        populations of a state."""
        pre = self.pre_collision(post)
        theta = pre[9:14].sum(0) / self.sigma_coll
        ux, uy, p, _, _ = self.flow_macros(pre[0:9], self.phi, self.l0, self.l1, self.inv_k,
                                           self.sqrt_inv_k, self.F_phi, theta)
        return dict(ux=ux, uy=uy, p=p, T=self.p.T_in + theta, theta=theta, c=pre[14:19].sum(0))

    def observables(self, post: torch.Tensor) -> dict:
        """Cell observables of Section 5 on the pre-collision populations [R16].

        i(x) = sum over CL rows of (-j_eff) dx [A/cm^2]; I = mean_x i(x);
        P = V I; H = mean_x sum_CL Q dx [W/cm^2];
        O2 utilisation = sum_CL s_c / sum_inlet u_in c_in (per step; with the
        pressure inlet [R17] the inlet velocities are those of the state);
        inlet flux = sum over the inlet nodes of u_x (lattice units);
        T_max; CL profiles of c and T on the CL row next to the GDL;
        population sums and the per-step consumption / heating.  With the
        thin-film CL [R19], i(x) and the heat are the film's, taken in the
        streaming that produced the pre-collision populations, and the
        profiles are those of the row above the film.
        """
        pre = self.pre_collision(post)
        theta, c = pre[9:14].sum(0) / self.sigma_coll, pre[14:19].sum(0)
        s_c, S_T, j_eff, Q, _ = self.reaction(theta, c, self.rhocp_coll)
        zero = torch.zeros_like(theta)
        cl = self.is_cl if self.p.reaction else torch.zeros_like(self.is_cl)
        s_c, S_T = torch.where(cl, s_c, zero), torch.where(cl, S_T, zero)
        j_eff, Q = torch.where(cl, j_eff, zero), torch.where(cl, Q, zero)
        i_x = (-j_eff).sum(0) * self.dx
        q_x = Q.sum(0) * self.dx
        if self.p.thin_cl and self.p.reaction:
            # [R19] the film's consumption and heat in the streaming that
            # produced these pre-collision populations; the outlet column
            # carries the copy of column nx-2 [R10].
            d_c, d_t, i_x, q_x = self.surface_reaction(post)
            if not self.g.periodic_x:
                last = lambda a: torch.cat([a[:-1], a[-2:-1]])
                d_c, d_t, i_x, q_x = last(d_c), last(d_t), last(i_x), last(q_x)
            s_c = torch.zeros_like(theta)
            S_T = torch.zeros_like(theta)
            s_c[-1], S_T[-1] = d_c, d_t
        I = i_x.mean()
        H = q_x.mean()
        hc = self.g.ny_channel
        if hc > 0 and not self.g.periodic_x:
            u_in, _, _, _, _ = self.flow_macros(pre[0:9, :hc, 0], self.phi[:hc, 0], self.l0[:hc, 0],
                                                self.l1[:hc, 0], self.inv_k[:hc, 0], self.sqrt_inv_k[:hc, 0],
                                                self.F_phi[:hc, 0], theta[:hc, 0])
            flux = u_in.sum()
        else:
            flux = torch.zeros((), dtype=DT)
        if self.p.pressure_inlet:
            inflow = flux * self.p.c_in
        else:
            inflow = (self.inlet_velocity() * self.p.c_in).sum() if hc > 0 else torch.zeros((), dtype=DT)
        util = s_c.sum() / inflow if float(inflow.real) > 0 else torch.zeros((), dtype=DT)
        ycl = self.g.ny - self.g.ny_cl
        if self.p.thin_cl:  # [R19] the row above the film
            c_prof, T_prof = c[-1], self.p.T_in + theta[-1]
        elif self.g.ny_cl > 0:
            c_prof, T_prof = c[ycl], self.p.T_in + theta[ycl]
        else:  # no CL row: the profiles are defined as zeros
            c_prof = T_prof = torch.zeros(self.g.nx, dtype=DT)
        return dict(
            current_density=I, power_density=self.p.V_op * I, heat_rate=H, o2_utilisation=util,
            T_max=(self.p.T_in + theta).real.max(), sum_f=pre[0:9].sum(), sum_theta=theta.sum(),
            sum_c=c.sum(), consumed_c=s_c.sum(), heat_added=S_T.sum(),
            i_profile=i_x, c_profile=c_prof, T_profile=T_prof, inlet_flux=flux,
        )
