"""FP64 CPU oracle of the coupled MRT lattice-Boltzmann PEM-cathode model.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports, links or
runs this package; only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` use it, as the reference against which
the HIP kernels are checked.  It shares no code with the HIP path.

``lbm2d`` follows the paper (Jithin, Siddharth, Das, De, "Simulation of
coupled heat and mass transport with reaction in PEM fuel cell cathode using
lattice Boltzmann method"): Section 2.1 (Eqs. 1-8, D2Q9 MRT flow with
Darcy-Forchheimer drag), Section 2.2 (Eqs. 9-11, D2Q5 MRT scalars), Section 4
(Eqs. 12-19, catalyst-layer Tafel kinetics, reaction heat, effective
properties, boundary conditions), written plainly in float64 with no
blocking or fusion.  ``adjoint2d`` obtains the exact discrete gradient of
the mean current density by reverse-mode differentiation of ``lbm2d``.
"""
