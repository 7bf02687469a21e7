"""Hand-written discrete adjoint on the GPU (lbm_forward_checkpointed /
lbm_backward) against the oracle's exact discrete gradient and against
central finite differences of the GPU forward map in FP64."""
import numpy as np
import pytest
import torch

import workloads as W
from oracle import adjoint2d as A
from oracle import lbm2d as L

pytestmark = pytest.mark.gpu
DT = torch.float64


def _lbm():
    from paper_2103_01444_amd import lbm
    return lbm


def _oracle_fields(w, phi):
    """The oracle's own porosity-derived 1/K (Kozeny-Carman) and D_eff
    (Bruggeman), as independent leaves."""
    m = L.Model(L.geometry_from_workload(w), L.Params.from_workload(w), phi=torch.as_tensor(phi, dtype=DT))
    return [torch.as_tensor(phi, dtype=DT), m.inv_k.detach().clone(), m.d_eff.detach().clone()]


def _compare(gpu_g, ora, ny_channel, tol, label):
    """Relative max error over the porous rows (GDL and CL)."""
    names = ("phi", "inv_k", "d_eff")
    for i, name in enumerate(names):
        g = gpu_g[name].double().cpu()
        ref = ora[i]
        porous = torch.zeros_like(ref, dtype=torch.bool)
        porous[ny_channel:] = True
        scale = float(ref[porous].abs().max())
        err = float((g - ref)[porous].abs().max()) / scale
        print(f"{label} d/d{name}: max |g| {scale:.3e}, rel err {err:.2e}", flush=True)
        assert err < tol, (name, err)


@pytest.mark.parametrize("size,nsteps,every", [((14, 10, (5, 4, 1)), 40, 15), ((64, 16, None), 4000, 200)])
def test_fp64_adjoint_matches_oracle_gradient(size, nsteps, every):
    lbm = _lbm()
    nx, ny, layers = size
    w = W.adjoint2d(nx, ny)
    if layers:
        w.update(ny_channel=layers[0], ny_gdl=layers[1], ny_cl=layers[2], Re=2.0, V_op=0.45)
    w["precision"] = 64
    phi = W.porosity_field(w)
    sim = lbm.Cathode.from_workload(w, phi=phi, independent_fields=1)
    J = sim.forward_checkpointed(nsteps, every)
    g = sim.backward(1.0)
    fields = _oracle_fields(w, phi)
    Jo, gphi, gk, gd = A.gradient(L.geometry_from_workload(w), L.Params.from_workload(w), *fields, nsteps=nsteps,
                                  every=every)
    print(f"{nx}x{ny} J gpu {J:.15e} oracle {float(Jo):.15e}", flush=True)
    assert abs(J / float(Jo) - 1) < 1e-12
    _compare(g, (gphi, gk, gd), w["ny_channel"], 1e-9, f"{nx}x{ny} fp64")


def test_fp64_adjoint_with_outlet_pressure_matches_oracle_gradient():
    # a nonzero outlet pressure enters the outlet column's equilibrium through its porosity
    lbm = _lbm()
    w = W.adjoint2d(14, 10)
    w.update(ny_channel=5, ny_gdl=4, ny_cl=1, Re=2.0, V_op=0.45, precision=64, p_out=3e-3)
    phi = W.porosity_field(w)
    sim = lbm.Cathode.from_workload(w, phi=phi, independent_fields=1)
    J = sim.forward_checkpointed(40, 15)
    g = sim.backward(1.0)
    fields = _oracle_fields(w, phi)
    Jo, gphi, gk, gd = A.gradient(L.geometry_from_workload(w), L.Params.from_workload(w), *fields, nsteps=40,
                                  every=15)
    assert abs(J / float(Jo) - 1) < 1e-12
    _compare(g, (gphi, gk, gd), w["ny_channel"], 1e-9, "14x10 fp64 p_out")


@pytest.mark.parametrize("nx", [14, 130])
def test_fp64_periodic_adjoint_matches_oracle_gradient(nx):
    """Periodic in x with a body force along x (no boundary columns: the
    reverse sweep runs the interior kernel alone), at a width inside one
    workgroup and one spanning a ragged second workgroup."""
    lbm = _lbm()
    w = W.adjoint2d(nx, 10)
    w.update(ny_channel=5, ny_gdl=4, ny_cl=1, Re=0.0, V_op=0.45, precision=64)
    phi = W.porosity_field(w)
    bf = 2e-5
    sim = lbm.Cathode.from_workload(w, phi=phi, independent_fields=1, flags=lbm.LBM_PERIODIC_X | lbm.LBM_BODY_FORCE,
                                    body_force_x=bf)
    J = sim.forward_checkpointed(40, 15)
    g = sim.backward(1.0)
    fields = _oracle_fields(w, phi)
    p = L.Params.from_workload(w)
    p.body_force = (bf, 0.0)
    geo = L.Geometry(nx, 10, 5, 4, 1, periodic_x=True)
    Jo, gphi, gk, gd = A.gradient(geo, p, *fields, nsteps=40, every=15)
    print(f"periodic {nx}x10 J gpu {J:.15e} oracle {float(Jo):.15e}", flush=True)
    assert abs(J / float(Jo) - 1) < 1e-12
    _compare(g, (gphi, gk, gd), w["ny_channel"], 1e-9, f"periodic {nx}x10 fp64")


def test_fp64_gradient_along_a_dense_direction_equals_forward_mode_derivative():
    """<grad J, d> of the GPU's reverse sweep, over every porous cell at
    once, against the oracle's forward-mode derivative of J along d (no
    reverse pass on either side of the comparison)."""
    from test_oracle_adjoint import _dense_direction, forward_mode_derivative
    lbm = _lbm()
    w = W.adjoint2d(14, 10)
    w.update(ny_channel=5, ny_gdl=4, ny_cl=1, Re=2.0, V_op=0.45, precision=64)
    phi = W.porosity_field(w)
    sim = lbm.Cathode.from_workload(w, phi=phi, independent_fields=1)
    sim.forward_checkpointed(40, 15)
    g = sim.backward(1.0)
    fields = _oracle_fields(w, phi)
    dirs = _dense_direction(fields, w["ny_channel"])
    dot = sum(float((g[name].double().cpu() * d).sum()) for name, d in zip(("phi", "inv_k", "d_eff"), dirs))
    jvp = forward_mode_derivative(L.geometry_from_workload(w), L.Params.from_workload(w), fields, dirs, 40)
    print(f"gpu <grad, d> {dot:.15e}, oracle forward mode {jvp:.15e}", flush=True)
    assert abs(dot / jvp - 1) < 1e-10


# Relative finite-difference steps: J is about 1e3 times less sensitive to
# 1/K than to porosity, so a 1e-5 step for 1/K would leave the difference
# quotient dominated by the ~1e-14 relative rounding of J.
FD_REL_H = {"phi": 1e-5, "inv_k": 1e-3, "d_eff": 1e-5}


def _fd_gradient(lbm, w, fields, cells, nsteps):
    """Central differences of J in FP64 on the GPU, one cell and field at a time."""
    base = lbm.Cathode.from_workload(dict(w, precision=64), phi=fields["phi"], inv_k=fields["inv_k"],
                                     d_eff=fields["d_eff"])
    out = {k: [] for k in fields}
    for name in ("phi", "inv_k", "d_eff"):
        for (y, x) in cells:
            v0 = float(fields[name][y, x])
            h = FD_REL_H[name] * abs(v0)
            js = []
            for sgn in (1.0, -1.0):
                f = {k: t.clone() for k, t in fields.items()}
                f[name][y, x] = v0 + sgn * h
                base.set_params(base.params, f["phi"], f["inv_k"], f["d_eff"])
                base.init_equilibrium()
                base.step(nsteps)
                js.append(base.observables()["current_density"])
            out[name].append((js[0] - js[1]) / (2 * h))
    return {k: np.array(v) for k, v in out.items()}


def test_adjoint_1024x256_against_central_differences():
    """The 1024x256 adjoint workload (4000 steps, checkpoint every 200):
    FP32 and FP64 adjoints against FP64 central differences on 32 seeded
    porous cells."""
    lbm = _lbm()
    w = W.adjoint2d()
    nsteps, every = w["steps"], w["every"]
    phi = W.porosity_field(w)
    cells = W.fd_cells(w)
    probe = lbm.Cathode.from_workload(dict(w, precision=64), phi=phi, independent_fields=1)
    fields = {k: v.clone() for k, v in probe.material().items()}  # the library's own derived fields (FP64)
    del probe
    fd = _fd_gradient(lbm, w, fields, cells, nsteps)
    for prec, tol in ((64, 1e-5), (32, 1e-4)):  # FP64: the differences' own truncation error
        sim = lbm.Cathode.from_workload(dict(w, precision=prec), phi=fields["phi"], inv_k=fields["inv_k"],
                                        d_eff=fields["d_eff"])
        J = sim.forward_checkpointed(nsteps, every)
        g = sim.backward(1.0)
        for name in ("phi", "inv_k", "d_eff"):
            ad = np.array([float(g[name][y, x]) for (y, x) in cells])
            scale = np.abs(fd[name]).max()
            err = np.abs(ad - fd[name]).max() / scale
            print(f"fp{prec} J={J:.6e} d/d{name}: max |fd| {scale:.3e}, rel err {err:.2e}", flush=True)
            assert err < tol, (prec, name, err)


def test_autograd_function_matches_library_backward():
    lbm = _lbm()
    w = W.adjoint2d(64, 16)
    phi = W.porosity_field(w)
    probe = lbm.Cathode.from_workload(w, phi=phi, independent_fields=1)
    mat = probe.material()
    inv_k = mat["inv_k"].clone().requires_grad_(True)
    ph = mat["phi"].clone().requires_grad_(True)
    d = mat["d_eff"].clone().requires_grad_(True)
    J = lbm.CurrentDensity.apply(inv_k, ph, d, w, 400, 100)
    (2.0 * J).backward()
    sim = lbm.Cathode.from_workload(w, phi=mat["phi"], inv_k=mat["inv_k"], d_eff=mat["d_eff"])
    J2 = sim.forward_checkpointed(400, 100)
    g = sim.backward(2.0)
    assert float(J) == J2
    assert torch.equal(inv_k.grad, g["inv_k"]) and torch.equal(ph.grad, g["phi"]) and torch.equal(d.grad, g["d_eff"])


def test_checkpoint_interval_does_not_change_the_gradient():
    """Replays reproduce the forward states bit for bit, so the gradient is
    the same for every checkpoint interval: one step per segment, a partial
    last segment, one segment of the whole run, and an interval longer
    than the run (the replay buffers are sized for the shorter of the two)."""
    lbm = _lbm()
    w = W.adjoint2d(40, 10)
    w.update(ny_channel=5, ny_gdl=4, ny_cl=1, Re=2.0, V_op=0.45)
    phi = W.porosity_field(w)
    sim = lbm.Cathode.from_workload(w, phi=phi, independent_fields=1)
    ref_J, ref_g = None, None
    for every in (7, 1, 40, 100):
        J = sim.forward_checkpointed(40, every)
        g = sim.backward(1.0)
        if ref_g is None:
            ref_J, ref_g = J, {k: v.clone() for k, v in g.items()}
            continue
        assert J == ref_J, every
        for name in ("phi", "inv_k", "d_eff"):
            assert torch.equal(g[name], ref_g[name]), (every, name)


def test_second_backward_replays_the_last_segment():
    """The checkpointed forward run leaves its last segment's states in the
    replay buffer, where the first backward reads them; a second backward
    after the same forward run replays that segment from its checkpoint and
    gives the same gradient, bit for bit (last segments of 5, 10 and 1
    steps, and one segment of the whole run)."""
    lbm = _lbm()
    w = W.adjoint2d(40, 10)
    w.update(ny_channel=5, ny_gdl=4, ny_cl=1, Re=2.0, V_op=0.45)
    sim = lbm.Cathode.from_workload(w, phi=W.porosity_field(w), independent_fields=1)
    for every in (7, 10, 1, 100):
        sim.forward_checkpointed(40, every)
        first = {k: v.clone() for k, v in sim.backward(1.0).items()}
        second = sim.backward(1.0)
        for name in ("phi", "inv_k", "d_eff"):
            assert torch.equal(first[name], second[name]), (every, name)


def test_backward_needs_a_checkpointed_forward():
    lbm = _lbm()
    w = W.adjoint2d(64, 16)
    sim = lbm.Cathode.from_workload(w, phi=W.porosity_field(w), independent_fields=1)
    with pytest.raises(lbm.LbmError, match="order"):
        sim.backward(1.0)
    layered = lbm.Cathode.from_workload(w)
    with pytest.raises(lbm.LbmError, match="order"):
        layered.forward_checkpointed(10, 5)


def test_permeability_gradient_is_the_chain_rule_of_the_inverse():
    """dJ/dK from the binding (-(1/K)^2 dJ/d(1/K)) equals torch's autograd
    through inv_k = 1/K, and a central difference in K at GDL cells (FP64)."""
    lbm = _lbm()
    w = W.adjoint2d(24, 10)
    w.update(ny_channel=5, ny_gdl=4, ny_cl=1, Re=2.0, V_op=0.45, precision=64)
    phi = W.porosity_field(w)
    probe = lbm.Cathode.from_workload(w, phi=phi, independent_fields=1)
    mat = probe.material()
    K = torch.where(mat["inv_k"] > 0, 1.0 / mat["inv_k"], torch.zeros_like(mat["inv_k"]))
    porous = mat["inv_k"] > 0
    Kv = K.clone().requires_grad_(True)
    inv_k = torch.where(porous, 1.0 / torch.where(porous, Kv, torch.ones_like(Kv)), torch.zeros_like(Kv))
    J = lbm.CurrentDensity.apply(inv_k, mat["phi"], mat["d_eff"], w, 60, 20)
    J.backward()
    sim = lbm.Cathode.from_workload(w, phi=mat["phi"], inv_k=mat["inv_k"], d_eff=mat["d_eff"])
    sim.forward_checkpointed(60, 20)
    g = sim.backward(1.0)
    gK = g["K"].double().cpu()
    err = float((Kv.grad.cpu() - gK).abs().max()) / float(gK.abs().max())
    print(f"dJ/dK: binding vs autograd rel err {err:.1e}", flush=True)
    assert err < 1e-12
    assert float(gK[~porous.cpu()].abs().max()) == 0.0
    for (y, x) in [(6, 3), (7, 12), (9, 11)]:
        h = 1e-4 * float(K[y, x])
        Js = []
        for sgn in (1, -1):
            ik = mat["inv_k"].clone()
            ik[y, x] = 1.0 / (float(K[y, x]) + sgn * h)
            fd = lbm.Cathode.from_workload(w, phi=mat["phi"], inv_k=ik, d_eff=mat["d_eff"])
            Js.append(fd.forward_checkpointed(60, 20))
        d = (Js[0] - Js[1]) / (2 * h)
        e = abs(d - float(gK[y, x])) / abs(float(gK[y, x]))
        print(f"dJ/dK at ({y}, {x}): adjoint {float(gK[y, x]):.6e}, central difference {d:.6e}, rel {e:.1e}",
              flush=True)
        assert e < 1e-4


@pytest.mark.parametrize("nx", [14, 130])
def test_fp64_periodic_y_adjoint_matches_oracle_gradient(nx):
    """Open x (inlet, outlet and the columns feeding them) with periodic y:
    the pushes and the transposed boundary columns wrap across the y ends.
    FP64 gradient against the oracle's exact discrete gradient."""
    lbm = _lbm()
    w = W.adjoint2d(nx, 10)
    w.update(ny_channel=5, ny_gdl=4, ny_cl=1, Re=0.8, V_op=0.45, precision=64)
    phi = W.porosity_field(w)
    sim = lbm.Cathode.from_workload(w, phi=phi, independent_fields=1, flags=lbm.LBM_PERIODIC_Y)
    J = sim.forward_checkpointed(40, 15)
    g = sim.backward(1.0)
    fields = _oracle_fields(w, phi)
    geo = L.Geometry(nx, 10, 5, 4, 1, periodic_y=True)
    Jo, gphi, gk, gd = A.gradient(geo, L.Params.from_workload(w), *fields, nsteps=40, every=15)
    print(f"periodic-y {nx}x10 J gpu {J:.15e} oracle {float(Jo):.15e}", flush=True)
    assert abs(J / float(Jo) - 1) < 1e-12
    _compare(g, (gphi, gk, gd), w["ny_channel"], 1e-9, f"periodic-y {nx}x10 fp64")


# option -> (workload keys, keys whose removal gives the case without it)
OPTIONS = {
    "butler_volmer": (dict(butler_volmer=True, alpha_a=0.5, V_op=1.1, aj0_ref=1e5), ("butler_volmer",)),
    "heat_physical": (dict(heat_physical=True), ("heat_physical",)),
    "buoyancy": (dict(buoyancy=(3e-3, -5e-3)), ("buoyancy",)),
    "sigma_energy": (dict(sigma_energy=True, heat_physical=True), ("sigma_energy",)),
    "pressure_inlet": (dict(pressure_inlet=True, p_in=4e-3), ("pressure_inlet", "p_in")),
    "all": (dict(butler_volmer=True, alpha_a=0.5, V_op=1.1, aj0_ref=1e5, heat_physical=True, buoyancy=(3e-3, -5e-3),
                 sigma_energy=True, pressure_inlet=True, p_in=4e-3),
            ("butler_volmer", "heat_physical", "buoyancy", "sigma_energy", "pressure_inlet", "p_in")),
    "thin_cl": (dict(thin_cl=True, ny_gdl=5, ny_cl=0), ("thin_cl",)),
    "thin_cl_all": (dict(thin_cl=True, ny_gdl=5, ny_cl=0, butler_volmer=True, alpha_a=0.5, V_op=1.1, aj0_ref=1e5,
                         heat_physical=True, buoyancy=(3e-3, -5e-3), sigma_energy=True, pressure_inlet=True, p_in=4e-3),
                    ("butler_volmer", "heat_physical", "buoyancy", "sigma_energy", "pressure_inlet", "p_in")),
}


@pytest.mark.parametrize("option", list(OPTIONS))
def test_fp64_adjoint_with_model_option_matches_oracle_gradient(option):
    """Butler-Volmer kinetics (Eq. 13 with its anodic branch, near the
    equilibrium potential where that branch is as large as the cathodic
    one), the physically signed reaction heat, Boussinesq buoyancy, the
    energy equation with the heat-capacity ratio, the pressure-driven inlet,
    the thin-film CL (the film's update transposed in the bottom row, the
    seed of J on the film's consumption), and all of them at once with the
    volumetric and with the thin-film CL: FP64 gradient against the oracle's exact
    discrete gradient.  The oracle's gradient without the option differs
    from it by more than 1e-5 of its maximum in every field, so the option's
    own reverse terms are what the 1e-9 bar tests."""
    lbm = _lbm()
    extra, drop = OPTIONS[option]
    w = W.adjoint2d(14, 10)
    w.update(ny_channel=5, ny_gdl=4, ny_cl=1, Re=2.0, V_op=0.45, precision=64)
    w.update(extra)
    phi = W.porosity_field(w)
    sim = lbm.Cathode.from_workload(w, phi=phi, independent_fields=1)
    J = sim.forward_checkpointed(40, 15)
    g = sim.backward(1.0)
    fields = _oracle_fields(w, phi)
    Jo, gphi, gk, gd = A.gradient(L.geometry_from_workload(w), L.Params.from_workload(w), *fields, nsteps=40,
                                  every=15)
    print(f"{option} 14x10 J gpu {J:.15e} oracle {float(Jo):.15e}", flush=True)
    assert abs(J / float(Jo) - 1) < 1e-12
    _compare(g, (gphi, gk, gd), w["ny_channel"], 1e-9, f"{option} 14x10 fp64")
    base = {k: v for k, v in w.items() if k not in drop}
    _, *g0 = A.gradient(L.geometry_from_workload(base), L.Params.from_workload(base), *fields, nsteps=40, every=15)
    for ref, other in zip((gphi, gk, gd), g0):
        assert float((ref - other)[w["ny_channel"]:].abs().max()) > 1e-5 * float(ref[w["ny_channel"]:].abs().max())


@pytest.mark.parametrize("option", ["all", "thin_cl_all"])
def test_fp32_adjoint_with_every_option_follows_fp64(option):
    """The FP32 instances of the reverse step that carry the model options
    (buoyancy, sigma, the pressure-driven inlet, the thin-film CL, with
    Butler-Volmer kinetics and the physical heat) against the FP64 GPU
    gradient of the same case: 40 steps of FP32 rounding stay within 1e-3 of
    each field's maximum."""
    lbm = _lbm()
    extra, _ = OPTIONS[option]
    grads = {}
    for precision in (32, 64):
        w = W.adjoint2d(14, 10)
        w.update(ny_channel=5, ny_gdl=4, ny_cl=1, Re=2.0, V_op=0.45, precision=precision)
        w.update(extra)
        sim = lbm.Cathode.from_workload(w, phi=W.porosity_field(w), independent_fields=1)
        sim.forward_checkpointed(40, 15)
        grads[precision] = {k: v.double().cpu() for k, v in sim.backward(1.0).items()}
        sim.close()
    for name in ("phi", "inv_k", "d_eff"):
        ref, got = grads[64][name], grads[32][name]
        err = float((got - ref).abs().max()) / float(ref.abs().max())
        print(f"{option} fp32 d/d{name}: rel err {err:.2e}", flush=True)
        assert torch.isfinite(got).all()
        assert err < 1e-3, (name, err)


@pytest.mark.parametrize("precision", [32, 64])
def test_option_instances_give_the_same_bits_every_run(precision):
    """Repeated backward passes after one forward run (three segments, each
    replayed on the second stream) with every model option and the
    thin-film CL return the same gradient bit for bit, also from a second
    context of the same case."""
    lbm = _lbm()
    extra, _ = OPTIONS["thin_cl_all"]
    runs = []
    for _ in range(2):
        w = W.adjoint2d(14, 10)
        w.update(ny_channel=5, ny_gdl=4, ny_cl=1, Re=2.0, V_op=0.45, precision=precision)
        w.update(extra)
        sim = lbm.Cathode.from_workload(w, phi=W.porosity_field(w), independent_fields=1)
        sim.forward_checkpointed(40, 15)
        for _ in range(3):
            g = sim.backward(1.0, permeability=False)
            runs.append({k: v.clone() for k, v in g.items()})
        sim.close()
    for r in runs[1:]:
        for name in ("phi", "inv_k", "d_eff"):
            assert torch.isfinite(r[name]).all(), name
            assert torch.equal(r[name], runs[0][name]), name


@pytest.mark.parametrize("case", ["periodic_x", "periodic_y"])
def test_fp64_adjoint_with_options_on_periodic_lattices_matches_oracle_gradient(case):
    """The option terms on periodic lattices: periodic in x with a body force
    (no boundary columns), the thin-film CL, buoyancy, sigma and the
    physical heat; periodic in y with the pressure-driven inlet, sigma and
    Butler-Volmer kinetics.  FP64 gradient against the oracle's exact
    discrete gradient."""
    lbm = _lbm()
    w = W.adjoint2d(14, 10)
    if case == "periodic_x":
        w.update(ny_channel=5, ny_gdl=5, ny_cl=0, Re=0.0, V_op=0.45, precision=64, thin_cl=True,
                 buoyancy=(3e-3, -5e-3), sigma_energy=True, heat_physical=True)
        flags, geo = lbm.LBM_PERIODIC_X | lbm.LBM_BODY_FORCE, dict(periodic_x=True)
    else:
        w.update(ny_channel=5, ny_gdl=4, ny_cl=1, Re=0.8, V_op=1.1, precision=64, pressure_inlet=True, p_in=4e-3,
                 sigma_energy=True, butler_volmer=True, alpha_a=0.5, aj0_ref=1e5)
        flags, geo = lbm.LBM_PERIODIC_Y, dict(periodic_y=True)
    phi = W.porosity_field(w)
    bf = 2e-5 if case == "periodic_x" else 0.0
    sim = lbm.Cathode.from_workload(w, phi=phi, independent_fields=1, flags=flags, body_force_x=bf)
    J = sim.forward_checkpointed(40, 15)
    g = sim.backward(1.0)
    fields = _oracle_fields(w, phi)
    p = L.Params.from_workload(w)
    p.body_force = (bf, 0.0)
    g_oracle = L.Geometry(14, 10, w["ny_channel"], w["ny_gdl"], w["ny_cl"], **geo)
    Jo, gphi, gk, gd = A.gradient(g_oracle, p, *fields, nsteps=40, every=15)
    print(f"{case} options J gpu {J:.15e} oracle {float(Jo):.15e}", flush=True)
    assert abs(J / float(Jo) - 1) < 1e-12
    _compare(g, (gphi, gk, gd), w["ny_channel"], 1e-9, f"{case} options fp64")
