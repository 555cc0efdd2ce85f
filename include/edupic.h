/*
 * edupic.h -- C ABI of the MI355X (gfx950) PIC/MCC hot path.
 *
 * The library advances 1D3V electrostatic particle-in-cell / Monte Carlo
 * collision simulations of capacitively coupled RF discharges in argon, as
 * described in Donko et al., "eduPIC: an introductory particle based code for
 * radio-frequency plasma simulation" (arXiv:2103.09642).  One time step
 * (section 2.1, the six steps of the PIC/MCC cycle; Algorithms 2-6) is:
 *   1. charge assignment of electrons (every step) and ions (every N_SUB-th
 *      step) to the grid  [charge-assignment equations, Algorithm 2],
 *   2. rho = e (n_i - n_e), the discrete Poisson equation with phi_0 = V(t),
 *      phi_{N_g-1} = 0 (Thomas algorithm) and the grid field including the
 *      boundary forms  [Poisson and field equations, Algorithm 3],
 *   3-4. linear field interpolation and leapfrog push  [Algorithm 4],
 *   5. absorption at the electrodes  [Algorithm 5],
 *   6. Monte Carlo collisions: e-Ar elastic / excitation / ionization and
 *      Ar+-Ar isotropic / backward, probability 1 - exp(-n sigma_tot g dt)
 *      from tabulated cross sections  [collision equations, Algorithm 6].
 * Ions are subcycled (pushed and collided every N_SUB-th step with
 * dt_i = N_SUB dt_e).
 *
 * All particle state is FP64 structure-of-arrays in device memory.  Random
 * numbers come from Philox4x32-10 keyed by (particle id, step), so results do
 * not depend on particle order or launch shape.  Charge is deposited as int64
 * fixed point (2^32 units per particle), so densities are bit-reproducible.
 *
 * Conventions
 *  - Every function returns an int status: EDP_OK (0) or a negative EDP_E*
 *    code; edp_last_error() gives a message (thread-local).  Nothing throws.
 *  - "host" pointers point to CPU memory owned by the caller and are only
 *    read or written during the call.  "device" pointers point to GPU memory.
 *  - A context is bound to one device and one HIP stream; all GPU work it
 *    issues is asynchronous on that stream unless stated.  Use one context
 *    per host thread.
 *  - Arrays indexed by grid node have n_grid entries, node p at x = p dx,
 *    dx = gap / (n_grid - 1).
 */
#ifndef EDUPIC_H
#define EDUPIC_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Status codes. */
#define EDP_OK 0
#define EDP_EINVAL (-1)    /* invalid argument or descriptor                 */
#define EDP_ECAPACITY (-2) /* particle capacity exceeded; case marked failed */
#define EDP_EUNSTABLE (-3) /* a stability criterion of section 2.2 failed    */
#define EDP_EHIP (-4)      /* HIP runtime error                              */
#define EDP_EARENA (-5)    /* device arena too small or misaligned           */
#define EDP_ESTATE (-6)    /* state does not fit or case has failed          */

/* Case flags (measurement mode of section 3.5 and options). */
#define EDP_DIAG_DENSITY 1u         /* time-averaged n_e(x), n_i(x)            */
#define EDP_DIAG_EEPF 2u            /* EEPF in the central 10% of the gap      */
#define EDP_DIAG_CURRENT 4u         /* time-averaged j_e(x), j_i(x)            */
#define EDP_DIAG_MEANE 8u           /* time-averaged mean electron energy(x)   */
#define EDP_IONIZ_ANGLE_LITERAL 16u /* ionization: chi = sqrt(eps/(E-eps_ion)) taken
                                       as an angle instead of its cosine     */
#define EDP_ALLOW_UNSTABLE 32u      /* create even if a stability check fails  */
#define EDP_NULL_COLLISION 64u      /* select colliding particles by the
                                       null-collision method (section 2.1.6):
                                       candidates with P* = 1 - exp(-nu* dt),
                                       nu* = max n sigma_tot g over the table
                                       (bin upper edges, the last bin at four
                                       times the table range), processes with
                                       nu_k/nu*, the rest null; same random
                                       slots as the direct test            */
#define EDP_DIAG_XT 128u            /* spatio-temporal (xt) arrays of section
                                       3.5: N_t / n_xt_bin time bins per RF
                                       period, read by edp_read_xt          */
#define EDP_DIAG_IFED 256u          /* ion flux-energy distribution at each
                                       electrode (section 3.5, Algorithm 5) */

/* Quantities of edp_read_xt (the xt files of section 3.5). */
#define EDP_XT_POT 0      /* potential [V]                                     */
#define EDP_XT_EFIELD 1   /* electric field [V m^-1]                           */
#define EDP_XT_NE 2       /* electron density [m^-3]                           */
#define EDP_XT_NI 3       /* ion density [m^-3]                                */
#define EDP_XT_JE 4       /* electron current density [A m^-2]                 */
#define EDP_XT_JI 5       /* ion current density [A m^-2]                      */
#define EDP_XT_POWERE 6   /* electron power density j_e E [W m^-3]             */
#define EDP_XT_POWERI 7   /* ion power density j_i E [W m^-3]                  */
#define EDP_XT_MEANEE 8   /* mean electron energy [eV]                         */
#define EDP_XT_MEANEI 9   /* mean ion energy [eV]                              */
#define EDP_XT_IONIZ 10   /* ionization rate [m^-3 s^-1]                       */
#define EDP_XT_N 11

/* Slots of edp_read_info: the run report of section 3.5 with the accuracy
 * and stability criteria of section 2.2 on the measured state. */
#define EDP_INFO_MEAN_E 0     /* mean electron energy over the gap [eV]        */
#define EDP_INFO_NE_MAX 1     /* peak time-averaged electron density [m^-3]    */
#define EDP_INFO_DEBYE 2      /* Debye length, T_e = 2/3 <eps>, peak density   */
#define EDP_INFO_DX_DEBYE 3   /* dx / lambda_D (criterion 1: < 1)              */
#define EDP_INFO_WPE_DT 4     /* omega_pe dt_e (criterion 2: < 2)              */
#define EDP_INFO_PMAX_E 5     /* largest electron collision probability per
                                 step over the tables (criterion 3: < 0.05)   */
#define EDP_INFO_PMAX_I 6     /* same for ions per ion step                    */
#define EDP_INFO_CFL_EV 7     /* electron energy crossing one cell per step
                                 (criterion 4: the EEPF must be negligible
                                 above it) [eV]                                */
#define EDP_INFO_POWER_E 8    /* space-time mean of j_e E [W m^-3]             */
#define EDP_INFO_POWER_I 9    /* space-time mean of j_i E [W m^-3]             */
#define EDP_INFO_FLUX_I_POW 10 /* ion flux to the powered electrode [m^-2 s^-1] */
#define EDP_INFO_FLUX_I_GND 11 /* ion flux to the grounded electrode          */
#define EDP_INFO_EI_POW 12    /* mean ion impact energy, powered [eV]          */
#define EDP_INFO_EI_GND 13    /* mean ion impact energy, grounded [eV]         */
#define EDP_INFO_FAIL 14      /* failed criteria: 1 (bit 0), 2 (bit 1), 3 (bit 2) */
#define EDP_INFO_N 15

/* Species index. */
#define EDP_ELECTRONS 0
#define EDP_IONS 1

/* Execution options for edp_set_option. */
#define EDP_OPT_MODE 1        /* 0 plain launches, 1 step windows replayed as
                                 captured hipGraphs                           */
#define EDP_OPT_SORT_EVERY 2  /* steps between compaction + cell sort (>= 1;
                                 default 100); results do not depend on it,
                                 speed does: the Python autotuner (tune.py)
                                 picks it per batch                             */
#define EDP_OPT_PROFILE 5     /* 1: time every particle-kernel launch with events */
#define EDP_OPT_GRAPH_STEPS 6 /* steps captured per hipGraph (multiple of N_SUB)  */
#define EDP_OPT_POISSON 8     /* field solve: 0 parallel flux scans (default),
                                 1 sequential Thomas, bit-reproducible           */
#define EDP_OPT_GROUPS 11     /* lockstep groups of a multi-case advance, 1..4
                                 (default 2; at most one per case, so a
                                 single case runs alone): the cases are split
                                 by expected work (particles x steps), group 0
                                 runs on the context's stream and the others
                                 on streams the library creates (default
                                 priority), so that one group's launch ramp
                                 and tail overlap another's streaming; work
                                 enqueued later on the context's
                                 stream is ordered after every group.
                                 Results do not depend on it, speed does: the
                                 autotuner (tune.py) picks it */
#define EDP_OPT_SMALL_MAX 12   /* cases with at most this many particle slots
                                 per species (the library's estimate) run in
                                 the persistent small-case kernel: one
                                 workgroup advances one case through a whole
                                 window of steps in one launch, every case at
                                 its own pace, on a stream of the context's
                                 own forked from and joined back into its
                                 stream; 0 (default) none.  Results do not
                                 depend on it, speed does */
#define EDP_OPT_PART_WG_PER_CU 9 /* resident particle workgroups per CU a batch
                                 uses: 0 (default) all that fit, k >= 1 at
                                 most k; results do not depend on it, speed
                                 does: the autotuner (tune.py) picks it       */
#define EDP_OPT_PART_SKEW 13   /* per mille, 0..900, or -1 (default):
                                 a particle launch's workgroups are
                                 dispatched one per CU in turn, and each
                                 later layer streams its chunks more slowly;
                                 layer l of L then takes a share of its
                                 case's chunks weighted by
                                 1 - skew l / (L - 1).  -1: 200 (L - 1), at
                                 most 900, when the launch serves one case,
                                 else 0.  Results do not depend on it, speed
                                 does */
#define EDP_OPT_PRETEST 14     /* the collision pre-test's bound of P (section
                                 2.1.6, direct test): 0 (default) automatic,
                                 1 the bound over the whole table, 2 the
                                 bound by energy block (the tables' maximum
                                 up to the particle's energy).  Either is a
                                 bound, so decisions are those of the exact
                                 test; results do not depend on it, speed
                                 does */

typedef struct edp_ctx edp_ctx; /* opaque */
typedef int64_t edp_case;       /* case handle, > 0 */

/* One discharge case: the constants of Table 1 as runtime values. */
typedef struct {
  double gap_m;            /* L, electrode gap [m]                              */
  double pressure_pa;      /* argon pressure [Pa]                               */
  double gas_temp_k;       /* gas temperature T_g [K]                           */
  double area_m2;          /* electrode area unit A [m^2] (1e-4 in the paper)   */
  int32_t n_grid;          /* N_g, 2..2048 (2..1024 with measurement flags)     */
  int32_t steps_per_cycle; /* steps per RF cycle, the unit of edp_advance       */
  int32_t ion_subcycle;    /* N_SUB >= 1                                        */
  int32_t n_harm;          /* waveform harmonics used, 0..4                     */
  double dt_e;             /* electron time step [s]                            */
  double v_amp[4];         /* V(t) = sum_k v_amp[k] sin(2 pi freq_hz[k] t +     */
  double freq_hz[4];       /*        phase_rad[k]) at x = 0; x = L is grounded  */
  double phase_rad[4];
  double weight;           /* W, real particles per superparticle               */
  int64_t n_init_e;        /* superparticles seeded at creation                 */
  int64_t n_init_i;
  double te_init_ev;       /* seed electron temperature k T_e [eV]             */
  double ti_init_k;        /* seed ion temperature [K]                         */
  int64_t cap_e;           /* particle capacity; 0 = automatic                 */
  int64_t cap_i;
  uint64_t seed;           /* random-number key                                 */
  uint32_t flags;          /* EDP_DIAG_* and option flags                       */
  int32_t n_eepf;          /* EEPF bins (2000 in section 4.1)                  */
  double de_eepf_ev;       /* EEPF bin width [eV] (0.05 in section 4.1)         */
  int32_t n_xt_bin;        /* N_BIN: steps per xt time bin, divides steps_per_cycle */
  int32_t n_ifed;          /* IFEDF bins per electrode, 1..4096 (200)          */
  double de_ifed_ev;       /* IFEDF bin width [eV] (1)                         */
  /* Surface processes suggested in section 5, [0] the powered electrode
   * (x = 0), [1] the grounded one (x = L); 0 turns a process off.  An
   * electron leaving the gap is reflected specularly (x mirrored in the
   * electrode, v_x reversed) with probability eta_refl unless the mirror
   * image lies outside the gap; an absorbed ion emits an electron with
   * probability gamma_see, placed on the electrode with the velocity of a
   * thermal flux at see_te_ev (Rayleigh normal component into the gap,
   * normal tangential ones), taking part from the next step. */
  double gamma_see[2];     /* ion-induced secondary electron yield, 0..1       */
  double eta_refl[2];      /* elastic electron reflection probability, 0..1    */
  double see_te_ev;        /* temperature of the emitted electrons [eV], > 0
                              when a gamma_see is                            */
  double v_dc;             /* DC offset added to V(t) at x = 0 [V] (a self-bias) */
} edp_case_desc;

/* Cross sections tabulated at energies i * de_ev, i = 0..n_bins-1
 * (section 3.2): electron processes versus LAB energy, Ar+ versus COM
 * energy, all in m^2.  Host arrays, copied by the call. */
typedef struct {
  int32_t n_bins;
  double de_ev;
  const double *e_el, *e_exc, *e_ion; /* elastic, excitation, ionization      */
  const double *i_iso, *i_back;       /* Ar+ isotropic and backward parts      */
  double e_exc_thr_ev;                /* excitation energy loss [eV]           */
  double e_ion_thr_ev;                /* ionization energy [eV]                */
  double w_ioniz_ev;                  /* energy-sharing parameter w [eV]       */
} edp_xsec;

/* Counters since the case was created (or its state last set). */
typedef struct {
  int64_t n_e, n_i;          /* live superparticles                          */
  int64_t step;              /* global step index s (t = s dt_e)             */
  int64_t abs_e_pow, abs_e_gnd, abs_i_pow, abs_i_gnd; /* absorbed per wall    */
  int64_t coll_e, coll_i;    /* collisions                                   */
  int64_t ioniz;             /* ionizations = electrons born = ions born     */
  int64_t anomalies;         /* clamped negative post-collision energies     */
  int64_t dropped;           /* births lost to a full capacity               */
  int64_t psteps_e;          /* electron pushes done (sum over steps of n_e) */
  int64_t psteps_i;          /* ion pushes done (sum over ion steps of n_i)  */
  int64_t see_pow, see_gnd;  /* secondary electrons emitted by ion impact at
                                x = 0 and at x = L                           */
  int64_t refl;              /* electrons reflected at an electrode          */
} edp_counts;

/* Create a context on `device` issuing work on `hip_stream` (a hipStream_t,
 * NULL = the legacy default stream).  *out receives the context.  The
 * context also creates and owns three non-blocking streams of default
 * priority for lockstep groups 1-3 of a multi-case advance (EDP_OPT_GROUPS);
 * every advance joins them back into `hip_stream`, and edp_destroy destroys
 * them.  EDP_EHIP if they cannot be created. */
int edp_create(edp_ctx **out, int device, void *hip_stream);
/* Destroy a context; cases still alive are destroyed (arenas stay the
 * caller's). */
int edp_destroy(edp_ctx *ctx);
/* Set the cross-section tables used by cases created afterwards (section
 * 3.2; n sigma_tot is formed per case from its gas density). */
int edp_set_xsec(edp_ctx *ctx, const edp_xsec *xs);
/* Device bytes a case needs in its arena for the current tables, or a
 * negative status for an invalid descriptor. */
int64_t edp_case_bytes(const edp_ctx *ctx, const edp_case_desc *desc);
/* Create a case inside `dev_arena` (device memory of at least
 * edp_case_bytes bytes, 256-byte aligned, owned by the caller and kept alive
 * until edp_case_destroy).  Seeds n_init_e / n_init_i particles at uniform
 * random positions with Maxwellian velocities (Algorithm 1, init) and
 * deposits them.  Returns EDP_EUNSTABLE if the time step violates
 * omega_pe dt < 2 or P_coll < 0.05 at the seed density unless
 * EDP_ALLOW_UNSTABLE is set (section 2.2). */
int edp_case_create(edp_ctx *ctx, const edp_case_desc *desc, void *dev_arena,
                    int64_t arena_bytes, edp_case *out);
int edp_case_destroy(edp_ctx *ctx, edp_case c);
/* Move a case into a new arena with other particle capacities (0 keeps a
 * species' capacity): the paper's codes fix the largest particle count at
 * compile time (section 3.1); a long run whose plasma grows can instead be
 * given room at a cycle boundary.  dev_arena: device memory of at least
 * edp_case_bytes for the descriptor with the new capacities, 256-byte
 * aligned, caller-owned; the old arena returns to the caller when the call
 * returns.  Particles, counters, deposits, fields and every diagnostic carry
 * over unchanged, so the run continues bit for bit as it would have.
 * Synchronous.  EDP_ESTATE if the slots in use exceed a new capacity,
 * EDP_EARENA for a short or misaligned arena, EDP_EINVAL otherwise. */
int edp_case_resize(edp_ctx *ctx, edp_case c, int64_t cap_e, int64_t cap_i, void *dev_arena,
                    int64_t arena_bytes);
/* The cycle loop of Algorithm 1 (a run given arg1 > 0 cycles, each cycle
 * N_t repetitions of the six-step PIC/MCC cycle of section 2.1, ions every
 * N_SUB-th step): advance each listed case by n_cycles[k] RF cycles of
 * steps_per_cycle steps.  cases: host array of n_cases distinct handles of
 * this context; n_cycles: host array of n_cases counts >= 0 (both read during
 * the call only).  Asynchronous on the context's stream.  The cases advance
 * in lockstep groups: every kernel launch serves all cases of a group still
 * running, and a case's results do not depend on the others in the call.
 * EDP_EINVAL for a null, unknown, repeated or failed case or a negative count
 * (nothing is enqueued); EDP_EHIP if a launch fails.  A capacity overflow
 * during the advance is reported by edp_sync and edp_read_counts. */
int edp_advance(edp_ctx *ctx, const edp_case *cases, int32_t n_cases, const int32_t *n_cycles);
/* Same as edp_advance with a step count per case (n_steps: host array of
 * n_cases counts >= 0), for windows that are not whole RF cycles. */
int edp_advance_steps(edp_ctx *ctx, const edp_case *cases, int32_t n_cases,
                      const int64_t *n_steps);
/* For callers that cannot allocate device memory -- code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc: the same
 * advance as edp_advance_steps (same arguments, same results bit for bit),
 * but it allocates nothing.  The workgroup role table its launches read
 * (device memory beyond the cases' arenas; the first kernel of each window
 * writes the cases' steps into it) is a file-scope array of 16384 entries
 * (1 MiB) that each GPU the library runs on holds until the process ends;
 * the call makes no hipMalloc, hipFree, graph, stream or event and launches
 * plainly, as one lockstep group, on the context's stream.  Host
 * bookkeeping uses the C++ heap only.  Limit: a call whose cases need more
 * than 16384 workgroup roles (one per case plus its particle and sort
 * workgroups: about 100 cases of a few hundred particle workgroups each)
 * returns
 * EDP_EINVAL before enqueuing anything.  Every call on a GPU shares that
 * GPU's array and rewrites it at its start: calls that overlap on one GPU
 * (from two contexts, or two threads) race and must be serialised by the
 * caller. */
int edp_advance_steps_noalloc(edp_ctx *ctx, const edp_case *cases, int32_t n_cases,
                              const int64_t *n_steps);
/* Wait for the context's stream; returns EDP_ECAPACITY if any case overflowed. */
int edp_sync(edp_ctx *ctx);
/* The conv.dat quantities of section 3.5 (superparticle numbers) plus the
 * collision, absorption and birth counters of section 2.1's steps 5-6.
 * Synchronous (waits for the stream); *out: caller-owned.  EDP_EINVAL for
 * an unknown case; EDP_ECAPACITY (with *out still filled) if the case
 * overflowed its capacity, so its state is no longer physical. */
int edp_read_counts(edp_ctx *ctx, edp_case c, edp_counts *out);
/* The measurement mode's time-averaged densities of section 3.5 (the
 * density.dat file) [m^-3], needs EDP_DIAG_DENSITY.  ne, ni: caller-owned host
 * arrays of n >= n_grid doubles, node p at x = p dx.  reset != 0 restarts
 * every diagnostic of the case after the read.  Synchronous.  Without the
 * flag the arrays read zero.  EDP_EINVAL for an unknown case or a short
 * array; EDP_ECAPACITY if the case overflowed its capacity (the arrays are
 * still written, but the state is no longer physical). */
int edp_read_density(edp_ctx *ctx, edp_case c, double *ne, double *ni, int32_t n, int32_t reset);
/* The EEPF of section 3.5 (eepf.dat): f(eps) [eV^-3/2] with
 * sum f_i sqrt(eps_i) de = 1, eps_i = (i+1/2) de, over the electrons in
 * [0.45 L, 0.55 L] from their time-centred velocity (section 3.6); needs
 * EDP_DIAG_EEPF.  f: host array of n >= n_eepf doubles; counts (may be
 * NULL): the raw histogram.  Errors as edp_read_density. */
int edp_read_eepf(edp_ctx *ctx, edp_case c, double *f, int64_t *counts, int32_t n, int32_t reset);
/* Time-averaged electron and ion current densities [A m^-2] per node from
 * the time-centred velocity (sections 3.5-3.6); needs EDP_DIAG_CURRENT.
 * je, ji: host arrays of n >= n_grid doubles.  Errors as edp_read_density. */
int edp_read_currents(edp_ctx *ctx, edp_case c, double *je, double *ji, int32_t n, int32_t reset);
/* Time-averaged mean electron energy [eV] per node (section 3.5), needs
 * EDP_DIAG_MEANE.  mee_ev: host array of n >= n_grid doubles.  Errors as
 * edp_read_density. */
int edp_read_mean_energy(edp_ctx *ctx, edp_case c, double *mee_ev, int32_t n, int32_t reset);
/* xt array `quantity` (EDP_XT_*) as out[t * n_grid + p] for time bin
 * t = (s mod steps_per_cycle) / n_xt_bin: the mean over the steps s of the
 * bin since the last reset (ion quantities over its ion steps; the mean
 * energies as weight-averaged ratios).  n: capacity of out in doubles, at
 * least n_xt * n_grid with n_xt = steps_per_cycle / n_xt_bin.  EDP_EINVAL if
 * the case has no EDP_DIAG_XT.  Synchronous. */
int edp_read_xt(edp_ctx *ctx, edp_case c, int32_t quantity, double *out, int64_t n);
/* Steps and ion steps accumulated per xt bin (either pointer may be NULL). */
int edp_read_xt_steps(edp_ctx *ctx, edp_case c, int64_t *steps, int64_t *ion_steps, int32_t n);
/* IFEDF of the ions absorbed at the powered and grounded electrode, each
 * normalised to sum_k F_k de_ifed = 1 over its n_ifed bins (energy M v^2 / 2
 * of the half-step velocity that carried the ion out); counts (may be NULL)
 * receives [2][n_ifed + 1] impacts, the last bin of each side holding those
 * beyond the range.  n: length of f_pow and f_gnd (>= n_ifed). */
int edp_read_ifed(edp_ctx *ctx, edp_case c, double *f_pow, double *f_gnd, int64_t *counts, int32_t n);
/* Run report (EDP_INFO_* slots; n >= EDP_INFO_N): the criteria of section 2.2
 * from the time-averaged density and mean energy (EDP_DIAG_DENSITY and
 * EDP_DIAG_MEANE), the absorbed power (EDP_DIAG_XT) and the electrode ion
 * fluxes and impact energies (EDP_DIAG_IFED); slots whose diagnostics are off
 * read 0. */
int edp_read_info(edp_ctx *ctx, edp_case c, double *out, int32_t n);
/* Change the driving waveform from the next advance on: the n_harm harmonic
 * amplitudes (frequencies and phases stay) and the DC offset v_dc.  This is
 * the actuator of the outer control loops of section 5 (DC self-bias, power
 * target).  Host amplitudes are copied.  EDP_EINVAL if n_harm differs from
 * the case's or a value is not finite. */
int edp_set_voltage(edp_ctx *ctx, edp_case c, const double *v_amp, int32_t n_harm, double v_dc);
/* Restart every diagnostic of the case (time sums, xt arrays, EEPF, IFEDF). */
int edp_reset_diag(edp_ctx *ctx, edp_case c);
/* The charge assignment of Algorithm 2 (equations for delta n_p and
 * delta n_{p+1}) in fixed point: each superparticle adds 2^32 units split
 * between the two enclosing nodes, so the density is cnt * W/(A dx) / 2^32
 * (edge nodes doubled).  Returns the counts the next step will use:
 * electrons as they are now, ions as held since the last ion step.  cnt_e,
 * cnt_i: caller-owned host arrays of n >= n_grid int64.  Synchronous (applies
 * pending collisions first).  EDP_EINVAL for an unknown case or short
 * arrays.  Bit-exact: integer sums do not depend on particle order. */
int edp_read_deposit(edp_ctx *ctx, edp_case c, int64_t *cnt_e, int64_t *cnt_i, int32_t n);
/* rho [C m^-3], phi [V] and E [V m^-1] of the last completed step. */
int edp_read_fields(edp_ctx *ctx, edp_case c, double *rho, double *phi, double *efield, int32_t n);
/* The state save of Algorithm 1 (the particle coordinates written to
 * picdata.bin at the end of a run): copy out the live particles of a species
 * (EDP_ELECTRONS or EDP_IONS, any order) into caller-owned host arrays of
 * capacity `cap` (x [m], v [m/s] at the half step t - dt/2, uid); any array
 * may be NULL to skip it.  *n_out gets the live count even if it exceeds
 * cap.  Synchronous (applies pending collisions first).  EDP_EINVAL for an
 * unknown case or species. */
int edp_get_state(edp_ctx *ctx, edp_case c, int32_t species, double *x, double *vx, double *vy,
                  double *vz, uint64_t *uid, int64_t cap, int64_t *n_out);
/* The state load of Algorithm 1 (a run continuing from picdata.bin): replace
 * a species' particles from n entries of caller-owned host arrays (copied)
 * and set the step index; x must lie in [0, L], velocities are the
 * half-step ones v(t - dt/2) and finite, uids distinct.  Counters and
 * diagnostics restart; the species is redeposited, for ions the deposit also
 * stands until the next ion step.  Synchronous.  EDP_ESTATE if n exceeds the
 * capacity, EDP_EINVAL for a bad argument (nothing is changed then). */
int edp_set_state(edp_ctx *ctx, edp_case c, int32_t species, const double *x, const double *vx,
                  const double *vy, const double *vz, const uint64_t *uid, int64_t n,
                  int64_t step);
/* Execution options (EDP_OPT_*), per context. */
int edp_set_option(edp_ctx *ctx, int32_t key, int64_t value);
/* Launch timing when EDP_OPT_PROFILE is on: summed HIP-event milliseconds
 * and number of launches of the electron particle kernel in plain mode, since
 * the last call (then reset).  Synchronous. */
int edp_read_profile(edp_ctx *ctx, double *ms, int64_t *launches);
const char *edp_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
