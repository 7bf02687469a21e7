"""Thin ctypes binding of ``liblbmpem.so`` (C ABI in ``include/lbm_pem.h``).

Argument marshalling only: every step of the solver runs in the HIP
kernels of the library.  PyTorch provides device memory (the workspace and
per-cell arrays are CUDA tensors) and the stream.  There is no CPU fallback:
if the library is not built, or no GPU is present, constructing a solver
raises.
"""
from __future__ import annotations

import ctypes
import os
import sys

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblbmpem.so")

LBM_PERIODIC_X = 1
LBM_PERIODIC_Y = 2
LBM_BODY_FORCE = 4
LBM_NO_REACTION = 8
LBM_PERIODIC_Z = 16
LBM_PRESSURE_INLET = 32
LBM_THIN_CL = 64
LBM_BUOYANCY = 128
LBM_SIGMA_ENERGY = 256
LBM_PHYSICAL_HEAT = 512
LBM_CELL_FIELDS = 1024
LBM_KINETICS_TAFEL = 0
LBM_KINETICS_BUTLER_VOLMER = 1

STATUS = {0: "ok", 1: "invalid argument", 2: "parameters outside the stable range", 3: "device error",
          4: "non-finite result", 5: "call out of order"}


class Geometry(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("ny_channel", ctypes.c_int32),
                ("ny_gdl", ctypes.c_int32), ("ny_cl", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("flags", ctypes.c_uint32)]


_PARAM_NAMES = ["tau_f", "D_f_lat", "Re", "T_in_K", "c_in", "V_op", "phi_gdl", "Da_gdl", "deff_ratio_gdl",
                "dp_lat", "gdl_thickness_cm", "dx_cm", "D_O2_cm2s", "aj0_ref", "C_ref", "alpha_c", "faraday",
                "R_gas", "E_over_R", "T_arrh", "U0_slope", "U0_icept", "k_f", "k_s", "rhocp_f", "rhocp_s",
                "body_force_x", "body_force_y"]


class Geometry3D(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("nz_channel", ctypes.c_int32), ("nz_gdl", ctypes.c_int32), ("nz_cl", ctypes.c_int32),
                ("precision", ctypes.c_int32), ("flags", ctypes.c_uint32)]


class Params(ctypes.Structure):
    _fields_ = [(n, ctypes.c_double) for n in _PARAM_NAMES] + [
        ("independent_fields", ctypes.c_int32), ("kinetics", ctypes.c_int32), ("p_inlet", ctypes.c_double),
        ("p_outlet", ctypes.c_double), ("alpha_a", ctypes.c_double), ("thin_cl_cm", ctypes.c_double),
        ("buoyancy_x", ctypes.c_double), ("buoyancy_y", ctypes.c_double)]


class Obs(ctypes.Structure):
    _fields_ = [("step", ctypes.c_int64)] + [(n, ctypes.c_double) for n in (
        "current_density", "power_density", "heat_rate", "o2_utilisation", "T_max", "sum_f", "sum_theta",
        "sum_c", "consumed_c", "heat_added", "inlet_flux")]


class Schedule(ctypes.Structure):
    _fields_ = [("tile_x", ctypes.c_int32), ("tile_y", ctypes.c_int32), ("persistent", ctypes.c_int32),
                ("block", ctypes.c_int32)]


_lib = None

EXPORTED = ["lbm_default_params", "lbm_workspace_bytes", "lbm_create", "lbm_set_params", "lbm_init_equilibrium",
            "lbm_step", "lbm_observables", "lbm_observables_noalloc", "lbm_get_fields", "lbm_get_material", "lbm_get_populations",
            "lbm_set_populations",
            "lbm_state_bytes", "lbm_save_state", "lbm_load_state", "lbm_step_count", "lbm_synchronize",
            "lbm_destroy", "lbm_status_string", "lbm_last_error",
            "lbm_batch_workspace_bytes", "lbm_batch_create", "lbm_batch_init_equilibrium", "lbm_batch_set_fields",
            "lbm_batch_set_schedule",
            "lbm_batch_get_schedule", "lbm_batch_autotune", "lbm_batch_autotune_cached", "lbm_batch_set_barrier_timeout",
            "lbm_batch_step",
            "lbm_batch_observables",
            "lbm_batch_get_populations", "lbm_batch_step_count", "lbm_batch_synchronize", "lbm_batch_destroy",
            "lbm_batch_last_error", "lbm_adjoint_workspace_bytes", "lbm_forward_checkpointed", "lbm_backward",
            "lbm3d_workspace_bytes", "lbm3d_create", "lbm3d_set_params", "lbm3d_init_equilibrium", "lbm3d_step",
            "lbm3d_observables", "lbm3d_get_fields", "lbm3d_get_material", "lbm3d_get_populations",
            "lbm3d_set_populations", "lbm3d_step_count", "lbm3d_synchronize", "lbm3d_destroy", "lbm3d_last_error",
            "lbm3d_adjoint_workspace_bytes", "lbm3d_forward_checkpointed", "lbm3d_backward"]


def load_library(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load the HIP library (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is not built; run `python -m paper_2103_01444_amd.build`")
    lib = ctypes.CDLL(path)
    vp, sz, i64 = ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int64
    P = ctypes.POINTER
    sig = {
        "lbm_default_params": (None, [P(Params)]),
        "lbm_workspace_bytes": (sz, [P(Geometry)]),
        "lbm_create": (ctypes.c_int, [P(Geometry), vp, sz, vp, P(vp)]),
        "lbm_set_params": (ctypes.c_int, [vp, P(Params), vp, vp, vp]),
        "lbm_init_equilibrium": (ctypes.c_int, [vp]),
        "lbm_step": (ctypes.c_int, [vp, i64]),
        "lbm_observables": (ctypes.c_int, [vp, P(Obs), vp, vp, vp]),
        "lbm_observables_noalloc": (ctypes.c_int, [vp, P(Obs), vp, vp, vp]),
        "lbm_get_fields": (ctypes.c_int, [vp, vp, vp, vp, vp, vp, vp]),
        "lbm_get_populations": (ctypes.c_int, [vp, vp]),
        "lbm_get_material": (ctypes.c_int, [vp, vp, vp, vp]),
        "lbm_set_populations": (ctypes.c_int, [vp, vp, i64]),
        "lbm_state_bytes": (sz, [vp]),
        "lbm_save_state": (ctypes.c_int, [vp, vp, P(i64)]),
        "lbm_load_state": (ctypes.c_int, [vp, vp, i64]),
        "lbm_step_count": (i64, [vp]),
        "lbm_synchronize": (ctypes.c_int, [vp]),
        "lbm_destroy": (None, [vp]),
        "lbm_status_string": (ctypes.c_char_p, [ctypes.c_int]),
        "lbm_last_error": (ctypes.c_char_p, [vp]),
        "lbm_batch_workspace_bytes": (sz, [P(Geometry), ctypes.c_int32]),
        "lbm_batch_create": (ctypes.c_int, [P(Geometry), P(Params), ctypes.c_int32, vp, sz, vp, P(vp)]),
        "lbm_batch_init_equilibrium": (ctypes.c_int, [vp]),
        "lbm_batch_set_fields": (ctypes.c_int, [vp, ctypes.c_int32, vp, vp, vp]),
        "lbm_batch_set_schedule": (ctypes.c_int, [vp, P(Schedule)]),
        "lbm_batch_get_schedule": (ctypes.c_int, [vp, P(Schedule)]),
        "lbm_batch_autotune": (ctypes.c_int, [vp, ctypes.c_int32, P(Schedule), P(ctypes.c_double)]),
        "lbm_batch_autotune_cached": (ctypes.c_int, [vp, ctypes.c_int32, ctypes.c_char_p, P(Schedule),
                                                     P(ctypes.c_double), P(ctypes.c_int32)]),
        "lbm_batch_set_barrier_timeout": (ctypes.c_int, [vp, ctypes.c_double]),
        "lbm_batch_step": (ctypes.c_int, [vp, i64]),
        "lbm_batch_observables": (ctypes.c_int, [vp, P(Obs)]),
        "lbm_batch_get_populations": (ctypes.c_int, [vp, ctypes.c_int32, vp]),
        "lbm_batch_step_count": (i64, [vp]),
        "lbm_batch_synchronize": (ctypes.c_int, [vp]),
        "lbm_batch_destroy": (None, [vp]),
        "lbm_batch_last_error": (ctypes.c_char_p, [vp]),
        "lbm_adjoint_workspace_bytes": (sz, [vp, i64, ctypes.c_int32]),
        "lbm_forward_checkpointed": (ctypes.c_int, [vp, i64, ctypes.c_int32, vp, sz, P(ctypes.c_double)]),
        "lbm_backward": (ctypes.c_int, [vp, ctypes.c_double, vp, vp, vp]),
        "lbm3d_workspace_bytes": (sz, [P(Geometry3D)]),
        "lbm3d_create": (ctypes.c_int, [P(Geometry3D), vp, sz, vp, P(vp)]),
        "lbm3d_set_params": (ctypes.c_int, [vp, P(Params), vp, vp, vp]),
        "lbm3d_init_equilibrium": (ctypes.c_int, [vp]),
        "lbm3d_step": (ctypes.c_int, [vp, i64]),
        "lbm3d_observables": (ctypes.c_int, [vp, P(Obs)]),
        "lbm3d_get_fields": (ctypes.c_int, [vp, vp, vp, vp, vp, vp, vp, vp]),
        "lbm3d_get_material": (ctypes.c_int, [vp, vp, vp, vp]),
        "lbm3d_get_populations": (ctypes.c_int, [vp, vp]),
        "lbm3d_set_populations": (ctypes.c_int, [vp, vp, i64]),
        "lbm3d_step_count": (i64, [vp]),
        "lbm3d_synchronize": (ctypes.c_int, [vp]),
        "lbm3d_destroy": (None, [vp]),
        "lbm3d_last_error": (ctypes.c_char_p, [vp]),
        "lbm3d_adjoint_workspace_bytes": (sz, [vp, i64, ctypes.c_int32]),
        "lbm3d_forward_checkpointed": (ctypes.c_int, [vp, i64, ctypes.c_int32, vp, sz, P(ctypes.c_double)]),
        "lbm3d_backward": (ctypes.c_int, [vp, ctypes.c_double, vp, vp, vp]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


class LbmError(RuntimeError):
    pass


def default_params() -> Params:
    p = Params()
    load_library().lbm_default_params(ctypes.byref(p))
    return p


def params_from_workload(w: dict, **over) -> Params:
    """lbm_params for a workload dictionary (see ``workloads``)."""
    p = default_params()
    keymap = {"T_in": "T_in_K"}
    for k in ("tau_f", "D_f_lat", "Re", "T_in", "c_in", "V_op", "phi_gdl", "Da_gdl", "deff_ratio_gdl"):
        if k in w:
            setattr(p, keymap.get(k, k), float(w[k]))
    if w.get("dp_over_hgdl", 0.0) > 0:
        p.dp_lat = float(w["dp_over_hgdl"] * w.get("ny_gdl", w.get("nz_gdl")))
    if w.get("dp_lat", 0.0) > 0:
        p.dp_lat = float(w["dp_lat"])
    if "p_in" in w:
        p.p_inlet = float(w["p_in"])
    if "p_out" in w:
        p.p_outlet = float(w["p_out"])
    if w.get("butler_volmer", False):
        p.kinetics = LBM_KINETICS_BUTLER_VOLMER
    if "alpha_a" in w:
        p.alpha_a = float(w["alpha_a"])
    if "aj0_ref" in w:
        p.aj0_ref = float(w["aj0_ref"])
    if "thin_cl_cm" in w:
        p.thin_cl_cm = float(w["thin_cl_cm"])
    if "buoyancy" in w:
        p.buoyancy_x, p.buoyancy_y = (float(v) for v in w["buoyancy"])
    for k, v in over.items():
        setattr(p, k, v)
    return p


def workload_flags(w: dict) -> int:
    """Geometry flags a workload dictionary asks for (pressure-driven inlet)."""
    return ((LBM_PRESSURE_INLET if w.get("pressure_inlet", False) else 0)
            | (LBM_THIN_CL if w.get("thin_cl", False) else 0)
            | (LBM_BUOYANCY if "buoyancy" in w else 0)
            | (LBM_SIGMA_ENERGY if w.get("sigma_energy", False) else 0)
            | (LBM_PHYSICAL_HEAT if w.get("heat_physical", False) else 0))


def _ptr(t):
    if t is None:
        return None
    if not isinstance(t, torch.Tensor) or not t.is_cuda or not t.is_contiguous():
        raise ValueError("expected a contiguous CUDA tensor")
    return ctypes.c_void_p(t.data_ptr())


class Cathode:
    """One 2D cathode lattice on the current GPU.

    ``phi``, ``inv_k``, ``d_eff``: optional per-cell [ny, nx] tensors (any
    device; copied to the GPU in the context precision).
    """

    def __init__(self, nx, ny, ny_channel, ny_gdl, ny_cl, params: Params, precision=32, flags=0,
                 phi=None, inv_k=None, d_eff=None, device=None):
        if not torch.cuda.is_available():
            raise LbmError("no GPU: the solver runs only on the HIP device")
        self.lib = load_library()
        self.device = torch.device(device or "cuda")
        self.dtype = torch.float64 if precision == 64 else torch.float32
        self.geom = Geometry(nx, ny, ny_channel, ny_gdl, ny_cl, precision, flags)
        self.nx, self.ny = nx, ny
        nbytes = self.lib.lbm_workspace_bytes(ctypes.byref(self.geom))
        if nbytes == 0:
            raise LbmError("invalid geometry")
        with torch.cuda.device(self.device):
            self.ws = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
            self.stream = torch.cuda.current_stream(self.device)
        self.ctx = ctypes.c_void_p()
        self._check(self.lib.lbm_create(ctypes.byref(self.geom), ctypes.c_void_p(self.ws.data_ptr()), nbytes,
                                        ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(self.ctx)))
        self.params = params
        self.set_params(params, phi, inv_k, d_eff)
        self.init_equilibrium()

    @classmethod
    def from_workload(cls, w: dict, phi=None, inv_k=None, d_eff=None, flags=0, **over):
        flags |= workload_flags(w)
        return cls(w["nx"], w["ny"], w["ny_channel"], w["ny_gdl"], w["ny_cl"], params_from_workload(w, **over),
                   precision=w.get("precision", 32), flags=flags, phi=phi, inv_k=inv_k, d_eff=d_eff)

    # ------------------------------------------------------------------ util
    def _check(self, st):
        if st != 0:
            msg = ""
            if self.ctx:
                msg = self.lib.lbm_last_error(self.ctx).decode()
            raise LbmError(f"{STATUS.get(st, st)}: {msg}")

    def _dev(self, a):
        if a is None:
            return None
        t = torch.as_tensor(a).to(device=self.device, dtype=self.dtype).contiguous()
        if tuple(t.shape) != (self.ny, self.nx):
            raise ValueError(f"per-cell array must be [{self.ny}, {self.nx}]")
        return t

    # --------------------------------------------------------------- the ABI
    def set_params(self, params: Params, phi=None, inv_k=None, d_eff=None):
        arrs = [self._dev(a) for a in (phi, inv_k, d_eff)]
        self._check(self.lib.lbm_set_params(self.ctx, ctypes.byref(params), *[_ptr(a) for a in arrs]))
        self.params = params

    def init_equilibrium(self):
        self._check(self.lib.lbm_init_equilibrium(self.ctx))

    def step(self, n: int = 1):
        self._check(self.lib.lbm_step(self.ctx, int(n)))

    @property
    def step_count(self) -> int:
        return int(self.lib.lbm_step_count(self.ctx))

    def synchronize(self):
        self._check(self.lib.lbm_synchronize(self.ctx))

    def observables(self, noalloc: bool = False) -> dict:
        """Observables of the current state (lbm_observables, or with
        ``noalloc`` lbm_observables_noalloc)."""
        o = Obs()
        pi = np.zeros(self.nx)
        pc = np.zeros(self.nx)
        pT = np.zeros(self.nx)
        fn = self.lib.lbm_observables_noalloc if noalloc else self.lib.lbm_observables
        st = fn(self.ctx, ctypes.byref(o), pi.ctypes.data_as(ctypes.c_void_p), pc.ctypes.data_as(ctypes.c_void_p),
                pT.ctypes.data_as(ctypes.c_void_p))
        self._check(st)
        d = {name: getattr(o, name) for name, _ in Obs._fields_}
        d.update(i_profile=pi, c_profile=pc, T_profile=pT)
        return d

    def fields(self) -> dict:
        out = {k: torch.empty((self.ny, self.nx), dtype=self.dtype, device=self.device)
               for k in ("ux", "uy", "p", "T", "theta", "c")}
        self._check(self.lib.lbm_get_fields(self.ctx, *[_ptr(out[k]) for k in ("ux", "uy", "p", "T", "theta", "c")]))
        return out

    def material(self) -> dict:
        out = {k: torch.empty((self.ny, self.nx), dtype=self.dtype, device=self.device)
               for k in ("phi", "inv_k", "d_eff")}
        self._check(self.lib.lbm_get_material(self.ctx, _ptr(out["phi"]), _ptr(out["inv_k"]), _ptr(out["d_eff"])))
        return out

    def populations(self) -> torch.Tensor:
        out = torch.empty((19, self.ny, self.nx), dtype=self.dtype, device=self.device)
        self._check(self.lib.lbm_get_populations(self.ctx, _ptr(out)))
        return out

    def set_populations(self, pops, step: int = 0):
        t = torch.as_tensor(pops).to(device=self.device, dtype=self.dtype).contiguous()
        if tuple(t.shape) != (19, self.ny, self.nx):
            raise ValueError("populations must be [19, ny, nx]")
        self._check(self.lib.lbm_set_populations(self.ctx, _ptr(t), int(step)))
        self.synchronize()  # t may be freed after return

    def save_state(self):
        n = self.lib.lbm_state_bytes(self.ctx)
        buf = torch.empty(n, dtype=torch.uint8, device=self.device)
        step = ctypes.c_int64()
        self._check(self.lib.lbm_save_state(self.ctx, _ptr(buf), ctypes.byref(step)))
        return buf, step.value

    def load_state(self, buf, step: int):
        self._check(self.lib.lbm_load_state(self.ctx, _ptr(buf), int(step)))

    # ------------------------------------------------------------ adjoint
    def forward_checkpointed(self, nsteps: int, every: int = 200) -> float:
        """Run nsteps steps from the equilibrium state keeping a checkpoint
        every ``every`` steps; returns the mean current density J (A/cm^2)."""
        n = self.lib.lbm_adjoint_workspace_bytes(self.ctx, int(nsteps), int(every))
        if n == 0:
            raise LbmError("invalid adjoint run length")
        self.adj_ws = torch.empty(n, dtype=torch.uint8, device=self.device)
        J = ctypes.c_double()
        self._check(self.lib.lbm_forward_checkpointed(self.ctx, int(nsteps), int(every), _ptr(self.adj_ws), n,
                                                      ctypes.byref(J)))
        return J.value

    def backward(self, dJ: float = 1.0, permeability: bool = True) -> dict:
        """dJ times the gradient of J with respect to the per-cell 1/K
        (``inv_k``), porosity (``phi``) and D_eff (``d_eff``), and with
        ``permeability`` with respect to the permeability K itself (``K``:
        -(1/K)^2 dJ/d(1/K), zero in the clear channel where 1/K = 0), as
        [ny, nx] tensors."""
        out = {k: torch.empty((self.ny, self.nx), dtype=self.dtype, device=self.device)
               for k in ("inv_k", "phi", "d_eff")}
        self._check(self.lib.lbm_backward(self.ctx, float(dJ), _ptr(out["inv_k"]), _ptr(out["phi"]),
                                          _ptr(out["d_eff"])))
        if permeability:
            out["K"] = grad_wrt_permeability(self.material()["inv_k"], out["inv_k"])
        return out

    def close(self):
        """Wait for the stream and destroy the library context (idempotent).
        Call it, or use the object as a context manager, before the process
        ends: at interpreter shutdown the HIP runtime may already be gone, so
        the destructor then leaves the context alone."""
        h = getattr(self, "ctx", None)
        if h:
            self.ctx = None
            self.lib.lbm_synchronize(h)
            self.lib.lbm_destroy(h)

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self, _finalizing=sys.is_finalizing):
        # bound at definition: at interpreter exit the module's globals may already be None
        if _finalizing():
            return
        try:
            self.close()
        except Exception:
            pass


class Cathode3D:
    """One 3D cathode lattice (D3Q19 + 2 x D3Q7, C ABI lbm3d_*) on the
    current GPU.  ``phi``, ``inv_k``, ``d_eff``: optional per-cell
    [nz, ny, nx] tensors."""

    FIELDS = ("ux", "uy", "uz", "p", "T", "theta", "c")

    def __init__(self, nx, ny, nz, nz_channel, nz_gdl, nz_cl, params: Params, precision=32, flags=0,
                 phi=None, inv_k=None, d_eff=None, device=None):
        if not torch.cuda.is_available():
            raise LbmError("no GPU: the solver runs only on the HIP device")
        self.lib = load_library()
        self.device = torch.device(device or "cuda")
        self.dtype = torch.float64 if precision == 64 else torch.float32
        self.geom = Geometry3D(nx, ny, nz, nz_channel, nz_gdl, nz_cl, precision, flags)
        self.shape = (nz, ny, nx)
        nbytes = self.lib.lbm3d_workspace_bytes(ctypes.byref(self.geom))
        if nbytes == 0:
            raise LbmError("invalid 3D geometry")
        with torch.cuda.device(self.device):
            self.ws = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
            self.stream = torch.cuda.current_stream(self.device)
        self.ctx = ctypes.c_void_p()
        self._check(self.lib.lbm3d_create(ctypes.byref(self.geom), ctypes.c_void_p(self.ws.data_ptr()), nbytes,
                                          ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(self.ctx)))
        self.set_params(params, phi, inv_k, d_eff)
        self.init_equilibrium()

    @classmethod
    def from_workload(cls, w: dict, phi=None, inv_k=None, d_eff=None, flags=0, **over):
        flags |= workload_flags(w)
        return cls(w["nx"], w["ny"], w["nz"], w["nz_channel"], w["nz_gdl"], w["nz_cl"],
                   params_from_workload(w, **over), precision=w.get("precision", 32), flags=flags, phi=phi,
                   inv_k=inv_k, d_eff=d_eff)

    def _check(self, st):
        if st != 0:
            msg = self.lib.lbm3d_last_error(self.ctx).decode() if self.ctx else ""
            raise LbmError(f"{STATUS.get(st, st)}: {msg}")

    def _dev(self, a):
        if a is None:
            return None
        t = torch.as_tensor(a).to(device=self.device, dtype=self.dtype).contiguous()
        if tuple(t.shape) != self.shape:
            raise ValueError(f"per-cell array must be {list(self.shape)}")
        return t

    def set_params(self, params: Params, phi=None, inv_k=None, d_eff=None):
        arrs = [self._dev(a) for a in (phi, inv_k, d_eff)]
        self._check(self.lib.lbm3d_set_params(self.ctx, ctypes.byref(params), *[_ptr(a) for a in arrs]))
        self.params = params

    def init_equilibrium(self):
        self._check(self.lib.lbm3d_init_equilibrium(self.ctx))

    def step(self, n: int = 1):
        self._check(self.lib.lbm3d_step(self.ctx, int(n)))

    @property
    def step_count(self) -> int:
        return int(self.lib.lbm3d_step_count(self.ctx))

    def synchronize(self):
        self._check(self.lib.lbm3d_synchronize(self.ctx))

    def observables(self) -> dict:
        o = Obs()
        self._check(self.lib.lbm3d_observables(self.ctx, ctypes.byref(o)))
        return {name: getattr(o, name) for name, _ in Obs._fields_}

    def fields(self) -> dict:
        out = {k: torch.empty(self.shape, dtype=self.dtype, device=self.device) for k in self.FIELDS}
        self._check(self.lib.lbm3d_get_fields(self.ctx, *[_ptr(out[k]) for k in self.FIELDS]))
        return out

    def material(self) -> dict:
        out = {k: torch.empty(self.shape, dtype=self.dtype, device=self.device) for k in ("phi", "inv_k", "d_eff")}
        self._check(self.lib.lbm3d_get_material(self.ctx, _ptr(out["phi"]), _ptr(out["inv_k"]), _ptr(out["d_eff"])))
        return out

    def populations(self) -> torch.Tensor:
        out = torch.empty((33,) + self.shape, dtype=self.dtype, device=self.device)
        self._check(self.lib.lbm3d_get_populations(self.ctx, _ptr(out)))
        return out

    def set_populations(self, pops, step: int = 0):
        t = torch.as_tensor(pops).to(device=self.device, dtype=self.dtype).contiguous()
        if tuple(t.shape) != (33,) + self.shape:
            raise ValueError("populations must be [33, nz, ny, nx]")
        self._check(self.lib.lbm3d_set_populations(self.ctx, _ptr(t), int(step)))
        self.synchronize()

    def forward_checkpointed(self, nsteps: int, every: int = 100) -> float:
        """Run nsteps steps from equilibrium keeping a checkpoint every
        ``every`` steps; returns the mean current density J (A/cm^2)."""
        n = self.lib.lbm3d_adjoint_workspace_bytes(self.ctx, int(nsteps), int(every))
        if n == 0:
            raise LbmError("invalid adjoint run length")
        self.adj_ws = torch.empty(n, dtype=torch.uint8, device=self.device)
        J = ctypes.c_double()
        self._check(self.lib.lbm3d_forward_checkpointed(self.ctx, int(nsteps), int(every), _ptr(self.adj_ws), n,
                                                        ctypes.byref(J)))
        return J.value

    def backward(self, dJ: float = 1.0, permeability: bool = True) -> dict:
        """dJ times the gradient of J with respect to the per-cell 1/K,
        porosity and D_eff, and with ``permeability`` K (-(1/K)^2
        dJ/d(1/K)), as [nz, ny, nx] tensors."""
        out = {k: torch.empty(self.shape, dtype=self.dtype, device=self.device) for k in ("inv_k", "phi", "d_eff")}
        self._check(self.lib.lbm3d_backward(self.ctx, float(dJ), _ptr(out["inv_k"]), _ptr(out["phi"]),
                                            _ptr(out["d_eff"])))
        if permeability:
            out["K"] = grad_wrt_permeability(self.material()["inv_k"], out["inv_k"])
        return out

    def close(self):
        """Wait for the stream and destroy the library context (idempotent).
        Call it, or use the object as a context manager, before the process
        ends: at interpreter shutdown the HIP runtime may already be gone, so
        the destructor then leaves the context alone."""
        h = getattr(self, "ctx", None)
        if h:
            self.ctx = None
            self.lib.lbm3d_synchronize(h)
            self.lib.lbm3d_destroy(h)

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self, _finalizing=sys.is_finalizing):
        # bound at definition: at interpreter exit the module's globals may already be None
        if _finalizing():
            return
        try:
            self.close()
        except Exception:
            pass


class BatchedSweep:
    """Many independent cathode cases advanced together (C ABI
    lbm_batch_*).  ``cases``: workload dictionaries (see ``workloads``), all
    of one precision.  The schedule (tile shape, per-step or persistent
    launch) is picked by ``autotune``, which the library caches in a JSON
    file keyed by GPU architecture, precision and the case lattice sizes.  ``fields``: None
    (layered cases), or one entry per case, None or a dict with any of
    ``phi``, ``inv_k``, ``d_eff`` ([ny, nx] arrays): the cases then carry
    per-cell fields (missing ones derived from the layers) and each steps
    as a single ``Cathode`` with ``independent_fields=1``."""

    def __init__(self, cases: list, device=None, fields=None):
        if not torch.cuda.is_available():
            raise LbmError("no GPU: the solver runs only on the HIP device")
        self.lib = load_library()
        self.device = torch.device(device or "cuda")
        n = len(cases)
        if n == 0:
            raise LbmError("a batch needs at least one case")
        prec = cases[0].get("precision", 32)
        self.dtype = torch.float64 if prec == 64 else torch.float32
        self.shapes = [(w["nx"], w["ny"]) for w in cases]
        if fields is not None and len(fields) != n:
            raise ValueError("fields needs one entry (None or a dict) per case")
        cell = LBM_CELL_FIELDS if fields is not None else 0
        self.geoms = (Geometry * n)(*[Geometry(w["nx"], w["ny"], w["ny_channel"], w["ny_gdl"], w["ny_cl"],
                                               w.get("precision", 32), workload_flags(w) | cell) for w in cases])
        self.params = (Params * n)(*[params_from_workload(w) for w in cases])
        self.n = n
        nbytes = self.lib.lbm_batch_workspace_bytes(self.geoms, n)
        if nbytes == 0:
            raise LbmError("invalid batch geometry")
        with torch.cuda.device(self.device):
            self.ws = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
            self.stream = torch.cuda.current_stream(self.device)
        self.h = ctypes.c_void_p()
        st = self.lib.lbm_batch_create(self.geoms, self.params, n, ctypes.c_void_p(self.ws.data_ptr()), nbytes,
                                       ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(self.h))
        self._check(st)
        for i, f in enumerate(fields or []):
            if f:
                self.set_fields(i, **f)
        self._check(self.lib.lbm_batch_init_equilibrium(self.h))

    def set_fields(self, i: int, phi=None, inv_k=None, d_eff=None):
        """Per-cell fields of case i (lbm_batch_set_fields); call
        ``init_equilibrium`` afterwards to start from their equilibrium."""
        nx, ny = self.shapes[i]
        arrs = []
        for a in (phi, inv_k, d_eff):
            if a is None:
                arrs.append(None)
                continue
            t = torch.as_tensor(a).to(device=self.device, dtype=self.dtype).contiguous()
            if tuple(t.shape) != (ny, nx):
                raise ValueError(f"per-cell array of case {i} must be [{ny}, {nx}]")
            arrs.append(t)
        self._check(self.lib.lbm_batch_set_fields(self.h, int(i), *[_ptr(a) for a in arrs]))

    def _check(self, st):
        if st != 0:
            msg = self.lib.lbm_batch_last_error(self.h).decode() if self.h else ""
            raise LbmError(f"{STATUS.get(st, st)}: {msg}")

    @property
    def schedule(self) -> dict:
        s = Schedule()
        self._check(self.lib.lbm_batch_get_schedule(self.h, ctypes.byref(s)))
        return dict(tile_x=s.tile_x, tile_y=s.tile_y, persistent=s.persistent, block=s.block)

    def set_schedule(self, tile_x: int, tile_y: int, persistent: int, block: int = 0):
        """Tiles of tile_x x tile_y nodes, one launch per step (persistent
        = 0) or one cooperative launch (1); block: workgroup size of the
        per-step form (0 or 256; 64 / 128 for tiles of that many cells; 960
        with 64 x 12 tiles: two steps per launch)."""
        s = Schedule(tile_x, tile_y, persistent, block)
        self._check(self.lib.lbm_batch_set_schedule(self.h, ctypes.byref(s)))

    def autotune(self, trial_steps: int = 20, cache_path: str | None = None) -> dict:
        """Pick the fastest schedule (lbm_batch_autotune_cached: from the
        library's tuner cache file at ``cache_path`` when it holds one for
        this GPU, precision and set of lattice sizes)."""
        best = Schedule()
        ms = ctypes.c_double()
        hit = ctypes.c_int32()
        path = None
        if cache_path:
            os.makedirs(os.path.dirname(os.path.abspath(cache_path)), exist_ok=True)
            path = os.fsencode(cache_path)
        self._check(self.lib.lbm_batch_autotune_cached(self.h, int(trial_steps), path, ctypes.byref(best),
                                                       ctypes.byref(ms), ctypes.byref(hit)))
        return dict(tile_x=best.tile_x, tile_y=best.tile_y, persistent=best.persistent, block=best.block,
                    ms_per_step=ms.value, cached=bool(hit.value))

    def step(self, n: int = 1):
        self._check(self.lib.lbm_batch_step(self.h, int(n)))

    def init_equilibrium(self):
        """Every case back to its initial state (step 0)."""
        self._check(self.lib.lbm_batch_init_equilibrium(self.h))

    def set_barrier_timeout(self, seconds: float):
        """Bound on each grid-barrier wait of a persistent launch (4 s by default)."""
        self._check(self.lib.lbm_batch_set_barrier_timeout(self.h, float(seconds)))

    @property
    def step_count(self) -> int:
        return int(self.lib.lbm_batch_step_count(self.h))

    def synchronize(self):
        self._check(self.lib.lbm_batch_synchronize(self.h))

    def observables(self) -> list:
        out = (Obs * self.n)()
        self._check(self.lib.lbm_batch_observables(self.h, out))
        return [{name: getattr(o, name) for name, _ in Obs._fields_} for o in out]

    def populations(self, i: int) -> torch.Tensor:
        nx, ny = self.shapes[i]
        t = torch.empty((19, ny, nx), dtype=self.dtype, device=self.device)
        self._check(self.lib.lbm_batch_get_populations(self.h, int(i), _ptr(t)))
        return t

    def close(self):
        """Wait for the stream and destroy the library context (idempotent).
        Call it, or use the object as a context manager, before the process
        ends: at interpreter shutdown the HIP runtime may already be gone, so
        the destructor then leaves the context alone."""
        h = getattr(self, "h", None)
        if h:
            self.h = None
            self.lib.lbm_batch_synchronize(h)
            self.lib.lbm_batch_destroy(h)

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self, _finalizing=sys.is_finalizing):
        # bound at definition: at interpreter exit the module's globals may already be None
        if _finalizing():
            return
        try:
            self.close()
        except Exception:
            pass


def grad_wrt_permeability(inv_k: torch.Tensor, grad_inv_k: torch.Tensor) -> torch.Tensor:
    """dJ/dK from dJ/d(1/K): the chain rule through K = 1/(1/K),
    dJ/dK = -(1/K)^2 dJ/d(1/K); zero where 1/K = 0 (the clear channel,
    K infinite)."""
    return -(inv_k * inv_k) * grad_inv_k


class CurrentDensity(torch.autograd.Function):
    """J = mean current density after ``nsteps`` steps of a cathode whose
    porous layers are given cell by cell: 1/K (``inv_k``), porosity
    (``phi``) and O2 diffusivity (``d_eff``), all [ny, nx] (2D workload) or
    [nz, ny, nx] (3D workload, one with ``nz``) CUDA tensors in lattice
    units.  ``backward`` runs the library's hand-written discrete adjoint
    (checkpointed recomputation every ``every`` steps).

        J = CurrentDensity.apply(inv_k, phi, d_eff, workload, nsteps, every)

    The gradients are those of 1/K, porosity and D_eff.  For the gradient
    with respect to the permeability K, pass ``inv_k = 1.0 / K`` computed in
    torch (autograd applies dJ/dK = -(1/K)^2 dJ/d(1/K)), or convert with
    ``grad_wrt_permeability``.
    """

    @staticmethod
    def forward(ctx, inv_k, phi, d_eff, workload: dict, nsteps: int, every: int = 200):
        cls = Cathode3D if "nz" in workload else Cathode
        sim = cls.from_workload(workload, phi=phi.detach(), inv_k=inv_k.detach(), d_eff=d_eff.detach(),
                                independent_fields=1)
        J = sim.forward_checkpointed(nsteps, every)
        ctx.sim = sim
        return torch.tensor(J, dtype=torch.float64, device=phi.device)

    @staticmethod
    def backward(ctx, gJ):
        g = ctx.sim.backward(float(gJ))
        ctx.sim = None
        return g["inv_k"], g["phi"], g["d_eff"], None, None, None
