/*
 * lbm_pem.h -- C ABI of the MI355X coupled lattice-Boltzmann PEM-cathode solver.
 *
 * The library advances the coupled model of Jithin, Siddharth, Das and De,
 * "Simulation of coupled heat and mass transport with reaction in PEM fuel
 * cell cathode using lattice Boltzmann method":
 *   - D2Q9 multiple-relaxation-time flow with Darcy-Forchheimer drag in the
 *     porous gas diffusion layer (GDL) and catalyst layer (CL)  (Section 2.1,
 *     Eqs. 1-8);
 *   - D2Q5 multiple-relaxation-time temperature and O2 lattices advected by
 *     the flow velocity  (Section 2.2, Eqs. 9-11);
 *   - Tafel oxygen-reduction sink and reaction heat in the CL (Section 4,
 *     Eqs. 12-17), Bruggeman diffusivity (Eq. 18), mixture thermal
 *     diffusivity (Eq. 19);
 *   - half-way bounce-back walls, a parabolic velocity / Dirichlet T and O2
 *     inlet over the channel rows and a zero-pressure, zero-gradient outlet
 *     (Section 4 boundary conditions).
 * One call of lbm_step performs, per time step and per lattice node, the
 * pull-streaming, the boundary columns, the macroscopic fields, the flow
 * collision, the reaction and both scalar collisions in one kernel pass.
 *
 * Conventions
 *   Lattice: x = 0 .. nx-1 from inlet to outlet, y = 0 .. ny-1 from the
 *   channel-side wall through the GDL to the CL.  Rows [0, ny_channel) are
 *   the clear gas channel, the next ny_gdl rows the GDL, the last ny_cl rows
 *   the CL.  Lattice units dx = dt = 1 inside; physical scales follow from
 *   lbm_params (dx from the GDL thickness, dt from the O2 diffusivity).
 *   Per-cell arrays are dense, row-major [ny][nx] (x fastest), in the
 *   context precision (float for precision 32, double for 64), in device
 *   memory.
 *   State: after n steps the context holds the post-collision populations
 *   of step n.  "Fields" and "observables" are evaluated on the
 *   pre-collision populations obtained by streaming that state and applying
 *   the boundary columns (what step n+1 starts from).
 *   Populations (lbm_get_populations / lbm_set_populations) are 19 dense
 *   planes [19][ny][nx]: planes 0-8 the D2Q9 flow populations in the order
 *   e = (0,0),(1,0),(0,1),(-1,0),(0,-1),(1,1),(-1,1),(-1,-1),(1,-1) (Eq. 2),
 *   planes 9-13 the D2Q5 temperature-rise populations (theta = T - T_in, K),
 *   planes 14-18 the D2Q5 O2 populations (c = C / C_ref), D2Q5 order as the
 *   first five D2Q9 vectors (Eq. 9).
 *
 * Ownership: the caller owns all device memory.  lbm_create receives a
 * device workspace of at least lbm_workspace_bytes() bytes that must stay
 * alive and untouched until lbm_destroy; the library never allocates or
 * frees device memory.  The library owns only the opaque host context.
 * Threading: one host thread per context.  Every call enqueues work on the
 * HIP stream given to lbm_create; calls documented "synchronous" wait for it.
 * Errors: every call returns an lbm_status; nothing aborts or throws across
 * the ABI.  Device errors of asynchronous calls surface at the next
 * synchronous call as LBM_ERR_DEVICE.  lbm_last_error() gives a message.
 */
#ifndef LBM_PEM_H
#define LBM_PEM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum lbm_status {
  LBM_OK = 0,
  LBM_ERR_INVALID_ARG = 1,     /* null pointer, bad size, inconsistent geometry */
  LBM_ERR_UNSTABLE_PARAMS = 2, /* parameters outside the scheme's stability / positivity range */
  LBM_ERR_DEVICE = 3,          /* a HIP runtime or kernel error */
  LBM_ERR_NONFINITE = 4,       /* a reduced observable is NaN or infinite */
  LBM_ERR_STATE = 5            /* call out of order (e.g. step before set_params) */
} lbm_status;

/* lbm_geometry.flags */
#define LBM_PERIODIC_X 1u  /* no inlet/outlet: x wraps (test configurations) */
#define LBM_PERIODIC_Y 2u  /* no y walls: y wraps (test configurations) */
#define LBM_BODY_FORCE 4u  /* add phi * (body_force_x, body_force_y) to the flow force */
#define LBM_NO_REACTION 8u /* switch the CL reaction off */
#define LBM_PRESSURE_INLET 32u /* 2D: pressure-driven flow (Section 4): the inlet nodes of the channel rows
                                * take the pressure lbm_params.p_inlet with the velocity of column 1 (non-
                                * equilibrium extrapolation), the outlet has lbm_params.p_outlet; Re is then an output
                                * (lbm_obs.inlet_flux / nu) and lbm_params.Re is ignored */
#define LBM_THIN_CL 64u /* 2D: the CL has negligible thickness (Section 1): a reactive wall half a cell
                         * below the last GDL row (requires ny_cl = 0, ny_gdl >= 1, no LBM_PERIODIC_Y).  The
                         * temperature and O2 populations that cross it are reflected minus the O2 the film
                         * consumes and plus the heat it releases; the film carries the volumetric rate of
                         * Eq. 13 over the thickness lbm_params.thin_cl_cm.  Observables: i(x) is the film's
                         * current, the c and T profiles are those of the last row. */
#define LBM_BUOYANCY 128u /* 2D: Boussinesq buoyancy (the thermal-to-flow coupling of the Section 3 cavity
                          * validations): phi * (T - T_in) * (buoyancy_x, buoyancy_y) is added to the flow
                          * force (Eq. 7) and half of it to Eq. 8's v, T from the node's own temperature
                          * populations; with LBM_BODY_FORCE both accelerations add */
#define LBM_SIGMA_ENERGY 256u /* 2D: porous energy equation with the heat-capacity ratio sigma = (rho c_p)_eff /
                              * (rho c_p)_f: the temperature lattice conserves sigma T and carries the
                              * diffusivity k_eff / (rho c_p)_f (equilibrium moments (sigma T, u T,
                              * (b + 4 (1 - sigma)) T, 0)), so that heat diffuses at Eq. 19's alpha_eff and
                              * is stored in the solid; the reaction heat is unchanged in kelvin per step */
#define LBM_PHYSICAL_HEAT 512u /* 2D and 3D: the reaction heat with the irreversible part counted positive,
                                * Q = -j (T dU0/dT - eta), instead of Eq. 15's printed -j (eta + T dU0/dT) */
#define LBM_CELL_FIELDS 1024u /* batch case (2D): porosity, 1/K and D_eff are per-cell fields
                               * (lbm_batch_set_fields; until set, each is derived from the case's layers
                               * as lbm_set_params does with no array), and the case steps as a single
                               * context with lbm_params.independent_fields = 1.  Every case of a batch sets
                               * it or none (it sizes the workspace).  A single context ignores it. */

typedef struct lbm_geometry {
  int32_t nx, ny;                      /* nx >= 3, ny >= 1 */
  int32_t ny_channel, ny_gdl, ny_cl;   /* non-negative, sum to ny */
  int32_t precision;                   /* 32 (float populations) or 64 (double) */
  uint32_t flags;                      /* LBM_* flags above */
} lbm_geometry;

/*
 * Model inputs.  lbm_default_params() fills the paper's constants
 * (Nomenclature, Eqs. 7, 13-19) and the solver defaults; the operating point
 * (V_op, T_in_K, Re) and the porous-layer properties are what a user varies
 * (Section 5).
 *
 * Kinetics (lbm_params.kinetics): LBM_KINETICS_TAFEL is Eq. 13 as printed,
 * j = -a j0(T) (C/C_ref) exp(-alpha_c F eta / (R T)).  LBM_KINETICS_BUTLER_VOLMER
 * adds the anodic branch, j = -a j0(T) [(C/C_ref) exp(-alpha_c F eta / (R T))
 * - exp(alpha_a F eta / (R T))]; the O2 in a CL cell then relaxes over a step
 * toward exp((alpha_a + alpha_c) F eta / (R T)) instead of 0.  The adjoint
 * entry points (2D and 3D) cover both forms.
 */
#define LBM_KINETICS_TAFEL 0
#define LBM_KINETICS_BUTLER_VOLMER 1

typedef struct lbm_params {
  double tau_f;            /* flow relaxation time, nu = (tau_f - 1/2)/3 (Section 2.1); > 0.5 */
  double D_f_lat;          /* O2 diffusivity in the clear gas, lattice units; sets dt */
  double Re;               /* inlet Reynolds number U_avg * ny_channel / nu (Table 1 definition) */
  double T_in_K;           /* inlet / operating temperature, K */
  double c_in;             /* inlet O2 concentration relative to C_ref */
  double V_op;             /* operating voltage, V (Eq. 14) */
  double phi_gdl;          /* porosity of GDL and CL when no per-cell field is given */
  double Da_gdl;           /* Darcy number K / h^2, h = GDL thickness (Table 2) */
  double deff_ratio_gdl;   /* D_eff / D_f in GDL and CL; 0 selects Bruggeman phi^1.5 (Eq. 18) */
  double dp_lat;           /* Kozeny-Carman particle diameter in lattice units (Eq. 7); >0 derives K from porosity */
  double gdl_thickness_cm; /* physical GDL thickness; dx = gdl_thickness_cm / ny_gdl */
  double dx_cm;            /* > 0 overrides the lattice spacing (cm) */
  double D_O2_cm2s;        /* clear-gas O2 diffusivity, cm^2/s; dt = D_f_lat dx^2 / D_O2 */
  double aj0_ref;          /* reference exchange current density x area, A/cm^3 (Eq. 13) */
  double C_ref;            /* reference O2 concentration, mol/cm^3 */
  double alpha_c;          /* cathodic transfer coefficient */
  double faraday;          /* C/mol */
  double R_gas;            /* J/(mol K) */
  double E_over_R;         /* Arrhenius temperature of Eq. 17, K */
  double T_arrh;           /* reference temperature of Eq. 17, K */
  double U0_slope;         /* open-circuit voltage slope, V/K (Eq. 16) */
  double U0_icept;         /* open-circuit voltage intercept, V (Eq. 16) */
  double k_f, k_s;         /* fluid / solid thermal conductivity, W/(m K) (Eq. 19) */
  double rhocp_f, rhocp_s; /* fluid / solid volumetric heat capacity, J/(cm^3 K) (Eq. 19) */
  double body_force_x;     /* acceleration, lattice units (LBM_BODY_FORCE only) */
  double body_force_y;
  int32_t independent_fields; /* nonzero: keep porosity, 1/K and D_eff as three per-cell fields */
  int32_t kinetics;        /* LBM_KINETICS_TAFEL (default: Eq. 13 as printed) or LBM_KINETICS_BUTLER_VOLMER */
  double p_inlet;          /* inlet pressure, lattice units (LBM_PRESSURE_INLET only) */
  double p_outlet;         /* outlet pressure, lattice units (2D; default 0).  Section 5 sets the flow rate
                            * by the outlet pressure: with LBM_PRESSURE_INLET the channel is driven by
                            * p_inlet - p_outlet.  The 3D variant requires 0. */
  double alpha_a;          /* anodic transfer coefficient of LBM_KINETICS_BUTLER_VOLMER (the paper gives
                            * none; default 1.0, equal to alpha_c) */
  double thin_cl_cm;       /* LBM_THIN_CL film thickness, cm; <= 0: one lattice spacing */
  double buoyancy_x;       /* LBM_BUOYANCY: acceleration per kelvin of T - T_in, lattice units (-beta g) */
  double buoyancy_y;
} lbm_params;

/* Observables of Section 5 on the current state (see Conventions). */
typedef struct lbm_obs {
  int64_t step;
  double current_density;  /* mean over x of i(x) = sum_CL (-j) dx, A/cm^2 */
  double power_density;    /* V_op * current_density, W/cm^2 */
  double heat_rate;        /* mean over x of sum_CL Q dx, W/cm^2 (Eq. 15) */
  double o2_utilisation;   /* O2 consumed per step / O2 advected in per step */
  double T_max;            /* maximum temperature, K */
  double sum_f;            /* sum of all flow populations */
  double sum_theta;        /* sum of the temperature-rise lattice (K x cells) */
  double sum_c;            /* sum of the O2 lattice */
  double consumed_c;       /* O2 the next step removes (sum over CL) */
  double heat_added;       /* temperature rise the next step adds (sum over CL, K x cells) */
  double inlet_flux;       /* sum of u_x over the inlet nodes (lattice units); the mean inlet velocity times the
                            * channel height, so Re = inlet_flux / nu.  With LBM_PRESSURE_INLET the O2
                            * utilisation divides by inlet_flux * c_in (the prescribed profile's otherwise) */
} lbm_obs;

typedef struct lbm_ctx lbm_ctx;

/* Fill *p with the paper's constants and the solver defaults. */
void lbm_default_params(lbm_params* p);

/* Device workspace bytes a context of this geometry needs; 0 if invalid. */
size_t lbm_workspace_bytes(const lbm_geometry* g);

/* Create a context on the current HIP device.  dev_ws: device memory of at
 * least lbm_workspace_bytes(g) bytes, 256-byte aligned; hip_stream: a
 * hipStream_t (NULL = default stream).  Errors: LBM_ERR_INVALID_ARG. */
lbm_status lbm_create(const lbm_geometry* g, void* dev_ws, size_t ws_bytes, void* hip_stream,
                      lbm_ctx** out);

/* Set the model inputs (Sections 2 and 4).  phi, inv_k (1/K, lattice units)
 * and d_eff (O2 diffusivity, lattice units) are optional per-cell device
 * arrays [ny][nx]; NULL takes the layered value from *p (channel: phi = 1,
 * 1/K = 0, D = D_f_lat; GDL and CL: phi_gdl, Da_gdl or Kozeny-Carman,
 * deff_ratio_gdl or Bruggeman).  The arrays are copied; the caller may free
 * them afterwards.  Synchronous.  Errors: LBM_ERR_INVALID_ARG,
 * LBM_ERR_UNSTABLE_PARAMS (tau_f <= 0.5, a diffusivity outside
 * (0, 1/(4 sqrt 3)], porosity outside (0, 1], 1/K < 0, inlet peak velocity
 * above 0.1; with LBM_PRESSURE_INLET: the plane-Poiseuille peak velocity
 * |p_inlet - p_outlet| H^2 / (8 nu (nx - 1)) of the channel above 0.1). */
lbm_status lbm_set_params(lbm_ctx* ctx, const lbm_params* p, const void* phi, const void* inv_k,
                          const void* d_eff);

/* Initial state: fluid at rest at zero pressure, temperature T_in, O2 c_in
 * everywhere (equilibrium populations).  Resets the step counter.  Async. */
lbm_status lbm_init_equilibrium(lbm_ctx* ctx);

/* Advance nsteps time steps (Eq. 1 and the scalar equation of Eq. 10 with
 * the CL source).  Lattices of 2^19 nodes or more without periodic axes
 * advance two steps per kernel launch (an odd count ends with a single
 * step); the states are bit-identical to single steps.
 * Async; never synchronizes. */
lbm_status lbm_step(lbm_ctx* ctx, int64_t nsteps);

/* Observables (Section 5) of the current state, reduced in double precision
 * in a fixed order (deterministic).  prof_i, prof_c, prof_T: optional host
 * arrays of nx doubles for the local current density i(x) (A/cm^2) and the
 * O2 and temperature (K) on the CL row next to the GDL.  Synchronous.
 * LBM_ERR_NONFINITE if any reduced value is not finite. */
lbm_status lbm_observables(lbm_ctx* ctx, lbm_obs* out, double* prof_i, double* prof_c,
                           double* prof_T);

/* For callers that cannot allocate device memory or have it allocated for
 * them (code under HIP graph capture, tight serving loops, harnesses that
 * forbid allocation): lbm_observables with the reduction's intermediate
 * results (per-workgroup partial sums, reduced values, CL profiles) in a
 * static device array of the library, 4 MiB per GPU, held until the process
 * ends, instead of the context's workspace.  Same kernels, same results (bit
 * for bit).  Allocates nothing.  Every call on one GPU shares that array:
 * calls that overlap on one GPU (other threads, other contexts) race.
 * Synchronous.  LBM_ERR_INVALID_ARG if the lattice needs more than 4 MiB of
 * it: (ceil(nx/256) ny + 1) 9 + 3 nx doubles, i.e. up to about 3600 rows
 * at nx = 4096. */
lbm_status lbm_observables_noalloc(lbm_ctx* ctx, lbm_obs* out, double* prof_i, double* prof_c,
                                   double* prof_T);

/* Macroscopic fields of the current state into caller device arrays
 * [ny][nx] (context precision): u_x, u_y (lattice), p (lattice, Section 2.1
 * pressure relation), T (K), theta = T - T_in (K, the stored variable, at
 * full relative precision), c (relative).  NULL skips a field.  Async. */
lbm_status lbm_get_fields(lbm_ctx* ctx, void* ux, void* uy, void* p, void* T, void* theta, void* c);

/* The per-cell porosity, 1/K (lattice units) and O2 diffusivity (lattice
 * units) the update uses, after the layered / Kozeny-Carman (Eq. 7) /
 * Bruggeman (Eq. 18) derivations, into caller device arrays [ny][nx]
 * (context precision; NULL skips one).  Async. */
lbm_status lbm_get_material(lbm_ctx* ctx, void* phi, void* inv_k, void* d_eff);

/* Canonical post-collision populations, 19 dense planes (see Conventions),
 * context precision, device memory.  Async. */
lbm_status lbm_get_populations(lbm_ctx* ctx, void* dev_dst);
lbm_status lbm_set_populations(lbm_ctx* ctx, const void* dev_src, int64_t step);

/* Opaque state snapshot (device memory of lbm_state_bytes() bytes) for
 * checkpoint / restart; restoring reproduces later steps bit for bit. */
size_t lbm_state_bytes(const lbm_ctx* ctx);
lbm_status lbm_save_state(lbm_ctx* ctx, void* dev_dst, int64_t* step_out);
lbm_status lbm_load_state(lbm_ctx* ctx, const void* dev_src, int64_t step);

/* Number of steps taken since lbm_init_equilibrium / the last load. */
int64_t lbm_step_count(const lbm_ctx* ctx);

/* Wait for the context's stream; reports pending device errors. */
lbm_status lbm_synchronize(lbm_ctx* ctx);

void lbm_destroy(lbm_ctx* ctx);
const char* lbm_status_string(lbm_status s);
const char* lbm_last_error(const lbm_ctx* ctx);

/* ---------------------------------------------------------------------------
 * Discrete adjoint.  The paper studies how the cell's current density
 * responds to the GDL permeability, porosity and effective O2 diffusivity
 * varied independently (Section 5); the adjoint gives the derivative of the
 * mean current density J (lbm_obs.current_density, after nsteps steps from
 * the equilibrium state) with respect to all three per-cell fields at once.
 * It is the exact transpose of the discrete update (FP32 or FP64, as the
 * context), with the derivative of |u| and of sqrt(1/K) taken as 0 where the
 * argument is 0.  The context must hold the three fields as independent
 * per-cell arrays (lbm_params.independent_fields = 1, or all three arrays
 * given to lbm_set_params).
 * --------------------------------------------------------------------------- */

/* Device workspace for a checkpointed run: ceil(nsteps/every) checkpoints,
 * two replay buffers of min(every, nsteps) states (the next segment is
 * replayed on a second stream while one is swept), two adjoint states,
 * three gradient planes.  0 if invalid. */
size_t lbm_adjoint_workspace_bytes(const lbm_ctx* ctx, int64_t nsteps, int32_t every);

/* Initialise to equilibrium, run nsteps steps storing a checkpoint every
 * `every` steps in dev_ws (caller-owned, kept until lbm_backward), and
 * return J in *J_out.  Synchronous.  LBM_ERR_STATE if the context does not
 * hold independent per-cell fields.  The adjoint covers every option of the
 * 2D solver: the volumetric or the thin-film CL (LBM_THIN_CL), the velocity
 * or the pressure-driven inlet, Tafel or Butler-Volmer kinetics, either sign
 * of the reaction heat (LBM_PHYSICAL_HEAT), buoyancy (LBM_BUOYANCY) and the
 * heat-capacity ratio (LBM_SIGMA_ENERGY). */
lbm_status lbm_forward_checkpointed(lbm_ctx* ctx, int64_t nsteps, int32_t every, void* dev_ws, size_t ws_bytes,
                                    double* J_out);

/* dJ times dJ/d(1/K), dJ/dphi, dJ/dD_eff of the preceding checkpointed run,
 * written (not accumulated) into caller device arrays [ny][nx] (context
 * precision; NULL skips one).  Replays each segment from its checkpoint and
 * sweeps it in reverse (the first call after a forward run finds the last
 * segment's states already in dev_ws); the replays run on a second HIP
 * stream the library creates on first use (default priority, ordered by
 * events, destroyed by lbm_destroy).  May be called again for the same run.
 * Synchronous.  LBM_ERR_STATE without a matching lbm_forward_checkpointed
 * (or after the state was changed since). */
lbm_status lbm_backward(lbm_ctx* ctx, double dJ, void* grad_inv_k, void* grad_phi, void* grad_d_eff);

/* ---------------------------------------------------------------------------
 * Batched parameter sweep.  The paper's results are sweeps over operating
 * voltage, temperature, flow rate, permeability, porosity and effective
 * diffusivity (Section 5); a batch advances many such independent cases,
 * each with its own lattice size, all in one precision, together: layered
 * cathodes (lbm_params' layered inputs), or, when the cases carry
 * LBM_CELL_FIELDS, cathodes with per-cell porosity, 1/K and D_eff
 * (lbm_batch_set_fields).  Each case computes exactly what a single context
 * with the same geometry, parameters and fields computes (bit for bit).
 *
 * Work is cut into equal tiles of tile_x x tile_y nodes; the schedule runs
 * either one launch per step (persistent = 0) or one cooperative
 * persistent launch that steps all cases with a grid-wide barrier between
 * steps (persistent = 1).  lbm_batch_autotune times candidate schedules on
 * the batch's current state, keeps the fastest and restores the state.
 * --------------------------------------------------------------------------- */
typedef struct lbm_batch lbm_batch;

typedef struct lbm_schedule {
  int32_t tile_x, tile_y;  /* tile_x * tile_y in [64, 65536] */
  int32_t persistent;      /* 0: one launch per step; 1: one cooperative launch */
  int32_t block;           /* threads per workgroup of the per-step form: 0 or 256 (cells of a tile in a
                            * loop, or one per thread when the tile has 256), or 64 / 128 when the tile has
                            * exactly that many cells (one per thread); the persistent form uses 256.
                            * 960 with 64 x 12 tiles and persistent = 0: two steps per launch (a tile and
                            * its halo in LDS; an odd count ends with one step), for batches without
                            * periodic axes */
} lbm_schedule;

/* Device workspace for ncases lattices (state pool, autotuning backup,
 * tables, reduction scratch); 0 if a geometry is invalid or precisions differ. */
size_t lbm_batch_workspace_bytes(const lbm_geometry* g, int32_t ncases);

/* g[ncases], p[ncases]: per-case geometry and inputs, validated as by
 * lbm_set_params (with LBM_CELL_FIELDS the fields start derived from the
 * layers; lbm_params.independent_fields is then implied).  On error *out may still hold a batch so that
 * lbm_batch_last_error() can explain; destroy it.  Synchronous. */
lbm_status lbm_batch_create(const lbm_geometry* g, const lbm_params* p, int32_t ncases, void* dev_ws,
                            size_t ws_bytes, void* hip_stream, lbm_batch** out);
lbm_status lbm_batch_init_equilibrium(lbm_batch* b);
/* Per-cell porosity, 1/K and D_eff of case i (Eqs. 7-8, 18-19, Section 2.2;
 * the paper varies each of them independently in Section 5): dense
 * [ny][nx] device arrays in the batch precision, read during the call;
 * NULL keeps the field derived from the case's layers (1/K by
 * Kozeny-Carman from the porosity when the case's dp_lat > 0, D_eff by
 * Eq. 18 or deff_ratio_gdl), as lbm_set_params does for a context with
 * independent_fields = 1, to which the case is then bit-identical.  The
 * arrays are checked as lbm_set_params checks them (LBM_ERR_UNSTABLE_PARAMS,
 * nothing stored).  The fields apply from the next step; the equilibrium
 * that lbm_batch_init_equilibrium sets depends on them, so set them first.
 * LBM_ERR_STATE unless the cases carry LBM_CELL_FIELDS.  Synchronous. */
lbm_status lbm_batch_set_fields(lbm_batch* b, int32_t i, const void* phi, const void* inv_k,
                                const void* d_eff);
lbm_status lbm_batch_set_schedule(lbm_batch* b, const lbm_schedule* s);
lbm_status lbm_batch_get_schedule(const lbm_batch* b, lbm_schedule* s);
/* Time every candidate schedule for trial_steps steps from the current
 * state; keep the fastest, restore the state.  Synchronous.  A persistent
 * candidate whose grid barrier times out (lbm_batch_step) is skipped. */
lbm_status lbm_batch_autotune(lbm_batch* b, int32_t trial_steps, lbm_schedule* best, double* best_ms_per_step);
/* lbm_batch_autotune with a tuner cache file at cache_path (NULL: none): a
 * JSON object holding one schedule per line, keyed by GPU architecture,
 * precision and the case lattice sizes ("gfx950|fp32|256x64,512x128").  A
 * usable entry for this batch is set without trials (*from_cache = 1);
 * otherwise the trials run and the entry is added or replaced (the file is
 * rewritten through a temporary file; concurrent writers are not
 * coordinated).  A file in any other form is left alone and not used
 * (lbm_batch_last_error says so; the status is that of the trials).
 * Synchronous. */
lbm_status lbm_batch_autotune_cached(lbm_batch* b, int32_t trial_steps, const char* cache_path, lbm_schedule* best,
                                     double* best_ms_per_step, int32_t* from_cache);
/* Advance every case nsteps steps.  Async.  With a persistent schedule the
 * grid is sized so that every workgroup is resident (the smaller of the
 * runtime's occupancy figure and the kernel's register budget); its
 * barrier waits at most 4 s, so a grid that is not co-resident ends the
 * launch instead of hanging it, and the next synchronising call returns
 * LBM_ERR_DEVICE (the state is then invalid until
 * lbm_batch_init_equilibrium). */
lbm_status lbm_batch_step(lbm_batch* b, int64_t nsteps);
/* The longest a persistent launch's grid barrier waits (seconds, 0 to 3600;
 * 4 by default) before it gives up as described under lbm_batch_step.  0
 * gives up after one tick of the device wall clock.  For callers that bound
 * the latency of a failed launch, and for tests of that error path.
 * LBM_ERR_INVALID_ARG outside [0, 3600].  Applies to later launches. */
lbm_status lbm_batch_set_barrier_timeout(lbm_batch* b, double seconds);
/* out[ncases]: observables of every case (as lbm_observables).  Synchronous. */
lbm_status lbm_batch_observables(lbm_batch* b, lbm_obs* out);
/* Canonical populations of case i (layout of lbm_get_populations).  Async. */
lbm_status lbm_batch_get_populations(lbm_batch* b, int32_t i, void* dev_dst);
int64_t lbm_batch_step_count(const lbm_batch* b);
lbm_status lbm_batch_synchronize(lbm_batch* b);
void lbm_batch_destroy(lbm_batch* b);
const char* lbm_batch_last_error(const lbm_batch* b);

/* ---------------------------------------------------------------------------
 * Three-dimensional cathode.  The paper is two-dimensional; this variant
 * carries its physics (Sections 2 and 4: porous flow with Eqs. 5-8, the two
 * advected scalars of Eq. 10, the CL reaction of Eqs. 12-17, Eqs. 18-19,
 * the same inlet / outlet / wall conditions) to a D3Q19 flow lattice and
 * two D3Q7 scalar lattices.
 *   Collision: the paper's D2Q9 MRT, with the density moment relaxed at
 *   1/tau_f, is a two-rate collision (even moments at s+ = 1/tau_f,
 *   non-conserved odd moments at s- = 8(2 - s+)/(8 - s+)), and its D2Q5 MRT
 *   one with even rate 6/(3 + 2 sqrt 3) and odd rate 6/(3 + sqrt 3); the 3D
 *   lattices use the same rates.  The D2Q5 parameter b = 20 sqrt(3) alpha - 4
 *   becomes the D3Q7 weight a = sqrt(3) alpha of each moving population.
 *   Equilibrium: f0 = rho0 - 2 phi p - |u|^2/(2 phi), f_i = 3 w_i phi p +
 *   w_i (3 e.u + 4.5 (e.u)^2/phi - 1.5 |u|^2/phi); p from the 18 moving
 *   populations.
 *   Lattice: x = 0 .. nx-1 inlet to outlet, y = 0 .. ny-1 across the
 *   channel (walls at both ends), z = 0 .. nz-1 through the layers: layers
 *   [0, nz_channel) gas channel, then nz_gdl GDL layers, then nz_cl CL
 *   layers (walls below the channel and below the CL).  Inlet: channel
 *   cells of x = 0, u_x = 36 U (y+1/2)(ny-y-1/2)(z+1/2)(H-z-1/2)/(ny^2 H^2)
 *   with U = Re nu / H, H = nz_channel, Dirichlet T_in and c_in; outlet
 *   x = nx-1 as in 2D.
 *   Per-cell arrays: dense [nz][ny][nx], x fastest, context precision,
 *   device memory.  Populations: 33 dense planes [33][nz][ny][nx]: planes
 *   0-18 D3Q19 flow in the order (0,0,0), (+-1,0,0), (0,+-1,0), (0,0,+-1),
 *   (+-1,+-1,0), (+-1,-+1,0), (+-1,0,+-1), (+-1,0,-+1), (0,+-1,+-1),
 *   (0,+-1,-+1) (each pair: the vector, then its opposite), planes 19-25
 *   D3Q7 temperature rise, 26-32 D3Q7 O2 (order of the first seven D3Q19
 *   vectors).
 * Ownership, threading, errors, and the meaning of state, fields and
 * observables: as for the 2D context.  Observables are means over the
 * (x, y) area of the CL: i(x, y) = sum over CL layers of (-j) dx.
 * --------------------------------------------------------------------------- */
#define LBM_PERIODIC_Z 16u /* no z walls: z wraps (test configurations) */

typedef struct lbm3d_geometry {
  int32_t nx, ny, nz;                    /* nx >= 3; ny, nz in [1, 65535] */
  int32_t nz_channel, nz_gdl, nz_cl;     /* non-negative, sum to nz */
  int32_t precision;                     /* 32 or 64 */
  uint32_t flags;                        /* LBM_PERIODIC_X/Y/Z, LBM_BODY_FORCE, LBM_NO_REACTION */
} lbm3d_geometry;

typedef struct lbm3d_ctx lbm3d_ctx;

/* Device workspace bytes for this geometry; 0 if invalid. */
size_t lbm3d_workspace_bytes(const lbm3d_geometry* g);
/* As lbm_create.  Errors: LBM_ERR_INVALID_ARG. */
lbm_status lbm3d_create(const lbm3d_geometry* g, void* dev_ws, size_t ws_bytes, void* hip_stream, lbm3d_ctx** out);
/* As lbm_set_params, with per-cell arrays [nz][ny][nx]; the GDL thickness
 * spans nz_gdl layers.  The inlet peak 2.25 U must not exceed 0.1.
 * Synchronous. */
lbm_status lbm3d_set_params(lbm3d_ctx* ctx, const lbm_params* p, const void* phi, const void* inv_k,
                            const void* d_eff);
/* Rest fluid, T_in, c_in everywhere; resets the step counter.  Async. */
lbm_status lbm3d_init_equilibrium(lbm3d_ctx* ctx);
/* Advance nsteps time steps.  Async. */
lbm_status lbm3d_step(lbm3d_ctx* ctx, int64_t nsteps);
/* Observables of the current state, FP64 fixed-order reductions.
 * Synchronous; LBM_ERR_NONFINITE as in 2D. */
lbm_status lbm3d_observables(lbm3d_ctx* ctx, lbm_obs* out);
/* Fields of the current state into device arrays [nz][ny][nx]; NULL skips
 * one.  Async. */
lbm_status lbm3d_get_fields(lbm3d_ctx* ctx, void* ux, void* uy, void* uz, void* p, void* T, void* theta,
                            void* c);
/* Porosity, 1/K and O2 diffusivity the update uses.  Async. */
lbm_status lbm3d_get_material(lbm3d_ctx* ctx, void* phi, void* inv_k, void* d_eff);
/* Canonical post-collision populations (33 dense planes).  Async. */
lbm_status lbm3d_get_populations(lbm3d_ctx* ctx, void* dev_dst);
lbm_status lbm3d_set_populations(lbm3d_ctx* ctx, const void* dev_src, int64_t step);
int64_t lbm3d_step_count(const lbm3d_ctx* ctx);
lbm_status lbm3d_synchronize(lbm3d_ctx* ctx);
void lbm3d_destroy(lbm3d_ctx* ctx);
const char* lbm3d_last_error(const lbm3d_ctx* ctx);

/* Discrete adjoint of the 3D update: as lbm_adjoint_workspace_bytes,
 * lbm_forward_checkpointed and lbm_backward (same conventions; J is the mean
 * over the (x, y) area of the CL current density), gradients [nz][ny][nx].
 * The workspace holds ceil(nsteps/every) + every + 2 states, so every near
 * sqrt(nsteps) minimises it (5000 steps at 256x128x64 FP32, every 70:
 * about 40 GB). */
size_t lbm3d_adjoint_workspace_bytes(const lbm3d_ctx* ctx, int64_t nsteps, int32_t every);
lbm_status lbm3d_forward_checkpointed(lbm3d_ctx* ctx, int64_t nsteps, int32_t every, void* dev_ws,
                                      size_t ws_bytes, double* J_out);
lbm_status lbm3d_backward(lbm3d_ctx* ctx, double dJ, void* grad_inv_k, void* grad_phi, void* grad_d_eff);

#ifdef __cplusplus
}
#endif

#endif /* LBM_PEM_H */
