"""The C-ABI library loads and exports every entry point its header
declares; host-side argument checks.  CPU only (no kernel launches)."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2103_01444_amd", "liblbmpem.so")


def _declared():
    names = set()
    inc = os.path.join(ROOT, "include")
    for fn in os.listdir(inc):
        if fn.endswith(".h"):
            txt = open(os.path.join(inc, fn)).read()
            txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
            names |= set(re.findall(r"\b(lbm(?:3d)?_[a-z0-9_]+)\s*\(", txt))
    return names


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.fail("liblbmpem.so is not built (python -m paper_2103_01444_amd.build)")
    from paper_2103_01444_amd import lbm
    return lbm.load_library(LIB)


def test_every_declared_symbol_is_exported(lib):
    declared = _declared()
    assert len(declared) >= 18
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True, check=True).stdout
    exported = set(re.findall(r"\b(lbm(?:3d)?_[a-z0-9_]+)\b", out))
    missing = declared - exported
    assert not missing, missing
    for name in declared:
        assert hasattr(lib, name)


def test_binding_names_match_header():
    from paper_2103_01444_amd import lbm
    assert set(lbm.EXPORTED) <= _declared()


def test_struct_layouts_match_header(tmp_path):
    """Every binding struct has the size and field offsets that a C compiler
    gives the header's struct of the same name."""
    from paper_2103_01444_amd import lbm
    pairs = [(lbm.Geometry, "lbm_geometry"), (lbm.Params, "lbm_params"), (lbm.Obs, "lbm_obs"),
             (lbm.Geometry3D, "lbm3d_geometry"), (lbm.Schedule, "lbm_schedule")]
    lines = ["#include <stddef.h>", "#include <stdio.h>", '#include "lbm_pem.h"', "int main(void) {"]
    expect = []
    for cls, cname in pairs:
        lines.append(f'  printf("%zu\\n", sizeof({cname}));')
        expect.append(ctypes.sizeof(cls))
        for name, _ in cls._fields_:
            lines.append(f'  printf("%zu\\n", offsetof({cname}, {name}));')
            expect.append(getattr(cls, name).offset)
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = [int(v) for v in subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split()]
    assert got == expect


def test_defaults_are_the_paper_constants(lib):
    from paper_2103_01444_amd import lbm
    p = lbm.default_params()
    assert (p.aj0_ref, p.C_ref, p.alpha_c, p.faraday, p.R_gas) == (1e-4, 17.808e-6, 1.0, 96487.0, 8.314)
    assert (p.D_O2_cm2s, p.k_f, p.k_s, p.U0_slope, p.U0_icept) == (5.2197e-2, 0.026, 1.5, 0.0025, 0.2329)
    assert (p.E_over_R, p.T_arrh) == (16456.0, 353.15)
    assert (p.kinetics, p.alpha_a, p.p_inlet, p.p_outlet) == (lbm.LBM_KINETICS_TAFEL, 1.0, 0.0, 0.0)


def test_workspace_size_and_geometry_checks(lib):
    from paper_2103_01444_amd import lbm
    g = lbm.Geometry(200, 40, 20, 18, 2, 64, 0)
    n64 = lib.lbm_workspace_bytes(ctypes.byref(g))
    # two states of 19 planes of 256 x 40 doubles (pitch padded to 64)
    assert n64 >= 2 * 19 * 256 * 40 * 8
    g32 = lbm.Geometry(200, 40, 20, 18, 2, 32, 0)
    assert lib.lbm_workspace_bytes(ctypes.byref(g32)) < n64
    for bad in (lbm.Geometry(2, 40, 20, 18, 2, 64, 0),      # nx < 3
                lbm.Geometry(200, 40, 20, 18, 3, 64, 0),    # layers do not sum to ny
                lbm.Geometry(200, 40, 20, 18, 2, 16, 0),    # precision
                lbm.Geometry(200, 40, 20, 18, 2, 32, 2048),  # unknown flag
                lbm.Geometry(200, 40, 20, 18, 2, 32, 64),   # thin-film CL with CL rows
                lbm.Geometry(200, 40, 40, 0, 0, 32, 64),    # thin-film CL without a GDL
                lbm.Geometry(200, 40, 20, 20, 0, 32, 64 | 2),  # thin-film CL with periodic y
                lbm.Geometry(1 << 16, 1 << 12, 1 << 11, 1 << 11, 0, 32, 0)):  # 32-bit offsets
        assert lib.lbm_workspace_bytes(ctypes.byref(bad)) == 0
    assert lib.lbm_workspace_bytes(ctypes.byref(lbm.Geometry(200, 40, 20, 20, 0, 32, 64))) > 0
    # batches: per-cell field rows (LBM_CELL_FIELDS) widen every case's state rows from 19 to 22; the cases
    # of one batch must agree on the flag
    two = (lbm.Geometry * 2)(lbm.Geometry(256, 64, 32, 29, 3, 32, 0), lbm.Geometry(512, 64, 32, 29, 3, 32, 0))
    two_f = (lbm.Geometry * 2)(lbm.Geometry(256, 64, 32, 29, 3, 32, lbm.LBM_CELL_FIELDS),
                               lbm.Geometry(512, 64, 32, 29, 3, 32, lbm.LBM_CELL_FIELDS))
    mixed = (lbm.Geometry * 2)(lbm.Geometry(256, 64, 32, 29, 3, 32, lbm.LBM_CELL_FIELDS),
                               lbm.Geometry(512, 64, 32, 29, 3, 32, 0))
    n, n_f = lib.lbm_batch_workspace_bytes(two, 2), lib.lbm_batch_workspace_bytes(two_f, 2)
    assert n > 0 and n_f - n >= 3 * 2 * (256 + 512) * 64 * 4 * 3 // 2
    assert lib.lbm_batch_workspace_bytes(mixed, 2) == 0
    ctx = ctypes.c_void_p()
    assert lib.lbm_create(ctypes.byref(lbm.Geometry(2, 40, 20, 18, 2, 64, 0)), ctypes.c_void_p(256), 1 << 30,
                          None, ctypes.byref(ctx)) == 1
    assert lib.lbm_create(ctypes.byref(g), None, 1 << 30, None, ctypes.byref(ctx)) == 1
    assert lib.lbm_create(ctypes.byref(g), ctypes.c_void_p(256), 16, None, ctypes.byref(ctx)) == 1
    assert lib.lbm_status_string(2) == b"parameters outside the stable range"
    # an empty batch (or a negative case count) has no workspace
    gs = (lbm.Geometry * 2)(g32, g32)
    assert lib.lbm_batch_workspace_bytes(gs, 2) > 0
    assert lib.lbm_batch_workspace_bytes(gs, 0) == 0
    assert lib.lbm_batch_workspace_bytes(gs, -1) == 0


def test_workspace_size_and_geometry_checks_3d(lib):
    from paper_2103_01444_amd import lbm
    g = lbm.Geometry3D(256, 128, 64, 32, 29, 3, 32, 0)
    n = lib.lbm3d_workspace_bytes(ctypes.byref(g))
    assert n >= 2 * 33 * 256 * 128 * 64 * 4 + 3 * 256 * 128 * 64 * 4
    assert any(x in lbm.EXPORTED for x in ("lbm3d_step",))
    for bad in (lbm.Geometry3D(2, 8, 8, 4, 3, 1, 32, 0),          # nx < 3
                lbm.Geometry3D(16, 8, 8, 4, 3, 2, 32, 0),         # layers do not sum to nz
                lbm.Geometry3D(16, 8, 8, 4, 3, 1, 16, 0),         # precision
                lbm.Geometry3D(16, 8, 8, 4, 3, 1, 32, lbm.LBM_PRESSURE_INLET),  # 2D-only options
                lbm.Geometry3D(16, 8, 8, 4, 3, 1, 32, lbm.LBM_THIN_CL),
                lbm.Geometry3D(16, 8, 8, 4, 3, 1, 32, lbm.LBM_BUOYANCY),
                lbm.Geometry3D(16, 8, 8, 4, 3, 1, 32, lbm.LBM_SIGMA_ENERGY),
                lbm.Geometry3D(16, 8, 8, 4, 3, 1, 32, 1024),      # unknown flag
                lbm.Geometry3D(16, 0, 8, 4, 3, 1, 32, 0),         # empty y
                lbm.Geometry3D(1024, 1024, 64, 32, 29, 3, 32, 0)):  # 32-bit offsets
        assert lib.lbm3d_workspace_bytes(ctypes.byref(bad)) == 0
    # the heat sign and the test-mode flags are 3D options too
    for ok in (lbm.LBM_PHYSICAL_HEAT, lbm.LBM_PERIODIC_Z | lbm.LBM_BODY_FORCE | lbm.LBM_NO_REACTION):
        assert lib.lbm3d_workspace_bytes(ctypes.byref(lbm.Geometry3D(16, 8, 8, 4, 3, 1, 32, ok))) > 0
    ctx = ctypes.c_void_p()
    assert lib.lbm3d_create(ctypes.byref(g), None, n, None, ctypes.byref(ctx)) == 1
    assert lib.lbm3d_create(ctypes.byref(g), ctypes.c_void_p(256), 16, None, ctypes.byref(ctx)) == 1
    assert lib.lbm3d_create(ctypes.byref(g), ctypes.c_void_p(300), n, None, ctypes.byref(ctx)) == 1  # misaligned


def test_binding_constants_match_header_defines():
    from paper_2103_01444_amd import lbm
    txt = open(os.path.join(ROOT, "include", "lbm_pem.h")).read()
    defines = {name: int(val) for name, val in re.findall(r"#define\s+(LBM_[A-Z0-9_]+)\s+(\d+)u?\b", txt)}
    assert len(defines) >= 12
    for name, val in defines.items():
        assert getattr(lbm, name) == val, name


def test_null_handles_are_refused_without_touching_the_gpu(lib):
    """Every entry point given a null context / batch returns
    LBM_ERR_INVALID_ARG (or 0 / -1 / a message) and launches nothing;
    destroying a null handle is a no-op."""
    assert lib.lbm_step(None, 1) == 1 and lib.lbm3d_step(None, 1) == 1 and lib.lbm_batch_step(None, 1) == 1
    assert lib.lbm_init_equilibrium(None) == 1 and lib.lbm_synchronize(None) == 1
    assert lib.lbm_observables(None, None, None, None, None) == 1 and lib.lbm_batch_observables(None, None) == 1
    assert lib.lbm_backward(None, 1.0, None, None, None) == 1 and lib.lbm3d_backward(None, 1.0, None, None, None) == 1
    assert lib.lbm_adjoint_workspace_bytes(None, 10, 5) == 0 and lib.lbm3d_adjoint_workspace_bytes(None, 10, 5) == 0
    assert lib.lbm_step_count(None) == -1 and lib.lbm3d_step_count(None) == -1 and lib.lbm_batch_step_count(None) == -1
    assert lib.lbm_last_error(None) == b"null context" and lib.lbm3d_last_error(None) == b"null context"
    assert lib.lbm_batch_last_error(None) == b"null batch"
    lib.lbm_destroy(None)
    lib.lbm3d_destroy(None)
    lib.lbm_batch_destroy(None)


def test_destructors_survive_interpreter_teardown(monkeypatch):
    """At interpreter exit a module's globals may already be None when a
    context is collected: the destructors must neither raise nor make HIP
    calls while the interpreter is finalising, and must close otherwise."""
    from paper_2103_01444_amd import lbm
    for cls in (lbm.Cathode, lbm.Cathode3D, lbm.BatchedSweep):
        closed = []
        monkeypatch.setattr(cls, "close", lambda self, closed=closed: closed.append(1))
        obj = cls.__new__(cls)
        with monkeypatch.context() as m:
            m.setattr(lbm, "sys", None)
            obj.__del__()
        assert closed == [1], cls.__name__
        obj.__del__(lambda: True)  # finalising: no call at all
        assert closed == [1], cls.__name__
