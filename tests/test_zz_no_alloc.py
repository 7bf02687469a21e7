"""lbm_observables_noalloc (the observables with the reduction's scratch in
the library's static device array, for callers that cannot allocate) gives
exactly what lbm_observables gives, called through the C ABI: on two calls
in a row, the second on a smaller lattice (the static array keeps the first
call's contents), in FP64 and FP32, and it refuses lattices whose scratch
exceeds the static array."""
import ctypes

import numpy as np
import pytest
import torch

import workloads as W

pytestmark = pytest.mark.gpu


def _lbm():
    from paper_2103_01444_amd import lbm
    return lbm


def _call(lbm, cat, name):
    o = lbm.Obs()
    prof = [np.full(cat.nx, np.nan) for _ in range(3)]
    fn = getattr(cat.lib, name)
    st = fn(cat.ctx, ctypes.byref(o), *[p.ctypes.data_as(ctypes.c_void_p) for p in prof])
    assert st == 0, (name, cat.lib.lbm_last_error(cat.ctx).decode())
    return {n: getattr(o, n) for n, _ in lbm.Obs._fields_}, prof


def _same(lbm, cat, label):
    ref, ref_prof = _call(lbm, cat, "lbm_observables")
    got, got_prof = _call(lbm, cat, "lbm_observables_noalloc")
    print(f"{label}: I = {got['current_density']:.12e} (lbm_observables {ref['current_density']:.12e})", flush=True)
    for key, v in ref.items():
        assert got[key] == v, (label, key, got[key], v)
    for a, b in zip(got_prof, ref_prof):
        assert np.array_equal(a, b), label
    assert ref["current_density"] > 0


@pytest.mark.parametrize("precision", [64, 32])
def test_noalloc_observables_equal_the_workspace_ones(precision):
    lbm = _lbm()
    big = W.cathode2d_scaled(700, 90, precision=precision)
    phi = W.porosity_field(big)
    cat = lbm.Cathode.from_workload(big, phi=phi)
    cat.step(120)
    print(f"noalloc first call: {big['nx']}x{big['ny']} fp{precision}", flush=True)
    _same(lbm, cat, f"{big['nx']}x{big['ny']} fp{precision}")
    small = W.cathode2d_200x40()
    small.update(nx=37, ny=11, ny_channel=5, ny_gdl=5, ny_cl=1, precision=precision, Re=2.0)
    cat2 = lbm.Cathode.from_workload(small)
    cat2.step(60)
    print(f"noalloc second call: {small['nx']}x{small['ny']} fp{precision}", flush=True)
    _same(lbm, cat2, f"{small['nx']}x{small['ny']} fp{precision}")
    # and the first lattice again, after the smaller one overwrote part of the array
    cat.step(5)
    _same(lbm, cat, f"{big['nx']}x{big['ny']} fp{precision} again")


def test_noalloc_refuses_lattices_beyond_the_static_array():
    lbm = _lbm()
    w = W.cathode2d_scaled(4096, 3700, precision=32)  # (16 x 3700 + 1) x 9 + 3 x 4096 doubles > 4 MiB
    cat = lbm.Cathode.from_workload(w)
    o = lbm.Obs()
    print("noalloc refusal: 4096x3700 fp32", flush=True)
    st = cat.lib.lbm_observables_noalloc(cat.ctx, ctypes.byref(o), None, None, None)
    assert st == 1  # LBM_ERR_INVALID_ARG, before any launch
    assert b"static observable scratch" in cat.lib.lbm_last_error(cat.ctx)
    del cat
    torch.cuda.empty_cache()
