/*
 * CPU oracle for the 1D3V electrostatic PIC/MCC time step of the eduPIC paper
 * (Donko et al., "eduPIC: an introductory particle based code for
 * radio-frequency plasma simulation", arXiv:2103.09642).
 *
 * TEST INFRASTRUCTURE ONLY.  This is the plain, slow, single-threaded
 * reference that the GPU library is checked against.  It shares no code with
 * the library: its own constants, its own Philox, its own Thomas solver, its
 * own descriptor structs.  Only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark may load it.
 *
 * Everything is FP64 (the paper's codes use C doubles) and is compiled with
 * -ffp-contract=off so that no multiply-add is ever fused.
 *
 * Parity status: every function is pinned by tests against closed forms,
 * invariants, brute force or the rocRAND library, except the absolute physics
 * of a whole discharge run, which is "parity unpinned" (the paper's
 * cross-section data and figures are not available).
 */
#ifndef EDUPIC_ORACLE_H
#define EDUPIC_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Diagnostic and option flags (measurement mode of section 3.5). */
#define ORC_DIAG_DENSITY 1u  /* time-averaged n_e(x), n_i(x)                 */
#define ORC_DIAG_EEPF 2u     /* EEPF in the central 10% of the gap           */
#define ORC_DIAG_CURRENT 4u  /* time-averaged j_e(x), j_i(x)                 */
#define ORC_DIAG_MEANE 8u    /* time-averaged mean electron energy <eps>(x)   */
#define ORC_IONIZ_ANGLE_LITERAL 16u /* ionization angles: chi = sqrt(..) as radians */
#define ORC_NULL_COLLISION 64u /* null-collision selection of colliding particles */
#define ORC_DIAG_XT 128u     /* spatio-temporal (xt) arrays of section 3.5    */
#define ORC_DIAG_IFED 256u   /* ion flux-energy distribution at each electrode */

/* Quantities of the xt arrays (section 3.5), read as [n_xt][n_grid]. */
enum {
  ORC_XT_POT = 0, ORC_XT_EFIELD, ORC_XT_NE, ORC_XT_NI, ORC_XT_JE, ORC_XT_JI,
  ORC_XT_POWERE, ORC_XT_POWERI, ORC_XT_MEANEE, ORC_XT_MEANEI, ORC_XT_IONIZ, ORC_XT_N
};

/* Slots of orc_info(): the run report of section 3.5 with the accuracy and
 * stability criteria of section 2.2. */
enum {
  ORC_INFO_MEAN_E = 0,   /* mean electron energy over the gap [eV]           */
  ORC_INFO_NE_MAX,       /* peak of the time-averaged electron density      */
  ORC_INFO_DEBYE,        /* Debye length with T_e = 2/3 <eps>, n = peak [m] */
  ORC_INFO_DX_DEBYE,     /* dx / lambda_D (criterion 1: < 1)                */
  ORC_INFO_WPE_DT,       /* omega_pe dt_e (criterion 2: < 2)                */
  ORC_INFO_PMAX_E,       /* largest electron collision probability per step */
  ORC_INFO_PMAX_I,       /* largest ion collision probability per ion step  */
  ORC_INFO_CFL_EV,       /* electron energy that crosses one cell per step  */
  ORC_INFO_POWER_E,      /* space-time mean of j_e E [W m^-3]               */
  ORC_INFO_POWER_I,      /* space-time mean of j_i E [W m^-3]               */
  ORC_INFO_FLUX_I_POW,   /* ion flux to the powered electrode [m^-2 s^-1]   */
  ORC_INFO_FLUX_I_GND,   /* ion flux to the grounded electrode              */
  ORC_INFO_EI_POW,       /* mean ion impact energy, powered electrode [eV]  */
  ORC_INFO_EI_GND,       /* mean ion impact energy, grounded electrode      */
  ORC_INFO_FAIL,         /* bits: 1 criterion 1, 2 criterion 2, 4 criterion 3 */
  ORC_INFO_N
};

/* Counter slots returned by orc_counts(). */
enum {
  ORC_C_ABS_E_POW = 0, ORC_C_ABS_E_GND, ORC_C_ABS_I_POW, ORC_C_ABS_I_GND,
  ORC_C_COLL_E, ORC_C_COLL_I, ORC_C_IONIZ, ORC_C_ANOMALY,
  ORC_C_SEE_POW, /* electrons emitted by ion impact at x = 0             */
  ORC_C_SEE_GND, /* ... at x = L                                         */
  ORC_C_REFL,    /* electrons reflected at an electrode                   */
  ORC_C_N
};

/* One discharge case (Table 1 constants, made runtime values). */
typedef struct {
  double gap_m;        /* L, electrode gap                                  */
  double pressure_pa;  /* gas pressure                                      */
  double gas_temp_k;   /* T_g                                               */
  double area_m2;      /* A, electrode area unit (1 cm^2 in the paper)      */
  int32_t n_grid;      /* N_g >= 2                                          */
  int32_t steps_per_cycle; /* N_t (used only to count RF cycles)           */
  int32_t ion_subcycle;    /* N_SUB >= 1                                    */
  int32_t n_harm;          /* number of waveform harmonics, 0..4           */
  double dt_e;         /* electron time step [s]                            */
  double v_amp[4], freq_hz[4], phase_rad[4]; /* V(t)=sum V_k sin(2 pi f_k t + phi_k) */
  double weight;       /* W, real particles per superparticle               */
  int64_t n_init_e, n_init_i; /* seeded superparticles                      */
  double te_init_ev;   /* seed electron temperature k T_e [eV]             */
  double ti_init_k;    /* seed ion temperature [K]                         */
  uint64_t seed;       /* Philox key                                        */
  uint32_t flags;      /* ORC_* flags                                       */
  int32_t n_eepf;      /* EEPF bins                                         */
  double de_eepf_ev;   /* EEPF bin width [eV]                              */
  int32_t n_xt_bin;    /* N_BIN: steps per xt time bin (divides N_t)       */
  int32_t n_ifed;      /* IFEDF bins                                        */
  double de_ifed_ev;   /* IFEDF bin width [eV]                             */
  /* Surface processes (section 5), index 0 the powered electrode (x = 0),
   * 1 the grounded one (x = L); zero turns a process off. */
  double gamma_see[2]; /* ion-induced secondary electron yield, 0..1        */
  double eta_refl[2];  /* elastic electron reflection probability, 0..1     */
  double see_te_ev;    /* temperature of the emitted electrons [eV]        */
  double v_dc;         /* DC offset of the powered electrode's voltage [V]   */
} orc_case;

/* Tabulated cross sections (section 3.2): bin i <-> energy i*de_ev. */
typedef struct {
  int32_t n_bins;
  double de_ev;
  const double *e_el, *e_exc, *e_ion; /* electron: LAB energy, m^2          */
  const double *i_iso, *i_back;       /* Ar+ : COM energy, m^2              */
  double e_exc_thr_ev, e_ion_thr_ev;  /* excitation / ionization thresholds */
  double w_ioniz_ev;                  /* energy-sharing parameter w         */
} orc_xsec;

typedef struct orc_sim orc_sim;

/* Whole-case API ---------------------------------------------------------- */
orc_sim *orc_new(const orc_case *c, const orc_xsec *xs); /* NULL on error   */
void orc_free(orc_sim *s);
const char *orc_error(void);
/* Seed n_init_e electrons and n_init_i ions (uid 0..N-1 each). */
int orc_seed(orc_sim *s);
/* Replace one species' particles; sets the step counter.  Returns 0. */
int orc_set_state(orc_sim *s, int species, const double *x, const double *vx,
                  const double *vy, const double *vz, const uint64_t *uid,
                  int64_t n, int64_t step);
/* Copy out up to cap particles; returns the count (may exceed cap). */
int64_t orc_get_state(const orc_sim *s, int species, double *x, double *vx,
                      double *vy, double *vz, uint64_t *uid, int64_t cap);
/* Advance n full PIC/MCC steps. */
int orc_step(orc_sim *s, int64_t n);
int64_t orc_count(const orc_sim *s, int species); /* live particles */
int64_t orc_step_index(const orc_sim *s);
void orc_counts(const orc_sim *s, int64_t out[ORC_C_N]);
/* Fixed-point densities the NEXT step will use (electrons; ions as held). */
void orc_deposit_state(const orc_sim *s, int64_t *cnt_e, int64_t *cnt_i);
/* rho, phi, E of the last completed step. */
void orc_fields(const orc_sim *s, double *rho, double *phi, double *efield);
/* Diagnostics (time averages since the last reset). */
void orc_read_density(const orc_sim *s, double *ne, double *ni);
void orc_read_eepf(const orc_sim *s, double *f, int64_t *counts);
void orc_read_currents(const orc_sim *s, double *je, double *ji);
void orc_read_mean_energy(const orc_sim *s, double *mee);
void orc_reset_diag(orc_sim *s);
/* xt arrays: time bin t holds the steps s with (s mod N_t) / N_BIN = t;
 * each cell is the mean over the steps of its bin since the last reset (ion
 * quantities over the ion steps).  out: [n_xt][n_grid], n_xt = N_t / N_BIN. */
int32_t orc_n_xt(const orc_sim *s);
void orc_read_xt(const orc_sim *s, int q, double *out);
void orc_xt_steps(const orc_sim *s, int64_t *steps, int64_t *ion_steps);
/* IFEDF per electrode, sum_k F_k de = 1 over the in-range bins; counts:
 * [2][n_ifed + 1] (powered, grounded; the last bin counts impacts beyond the
 * range).  Any output may be NULL. */
void orc_read_ifed(const orc_sim *s, double *f_pow, double *f_gnd, int64_t *counts);
void orc_info(const orc_sim *s, double out[ORC_INFO_N]);
/* Debye length [m] and electron plasma frequency [rad/s] for a density
 * [m^-3] and an electron temperature [eV]. */
void orc_plasma_params(double n_e, double te_ev, double out[2]);
/* Derived per-case constants (for tests): dx, dt_i, factor_w, factor_e,
 * factor_i, gas density, V at step 0. */
void orc_constants(const orc_sim *s, double out[8]);
double orc_voltage(const orc_sim *s, int64_t step);
/* Replace the harmonic amplitudes (n = n_harm of the case) and the DC offset
 * from the next step on (the outer control loops of section 5). */
int orc_set_voltage(orc_sim *s, const double *v_amp, int32_t n, double v_dc);
void orc_nsig_tot(const orc_sim *s, double *nsig_e, double *nsig_i);
/* Null-collision parameters: nu*_e, nu*_i, P*_e, P*_i. */
void orc_null_params(const orc_sim *s, double out[4]);
/* nu* = max n sigma_tot(E) g(E) over a table (upper bin edges; the last bin
 * at four times the table range); mass: electron or Ar+ + Ar reduced mass. */
double orc_nu_star(const double *nsig, int32_t nb, double de_ev, double mass);

/* Building blocks, exposed for the pin tests -------------------------------- */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
/* Two uniforms in [0,1) for (uid, step, species, purpose, call). */
void orc_uniform2(uint64_t seed, uint64_t uid, uint32_t step, uint32_t species,
                  uint32_t purpose, uint32_t call, double out[2]);
uint64_t orc_mix64(uint64_t z);
uint64_t orc_child_uid(uint64_t parent, int64_t step, uint64_t kind);
void orc_deposit(const double *x, int64_t n, int32_t ng, double inv_dx, int64_t *cnt);
/* Cross-section table row of a kinetic energy [eV]: the nearest tabulated
 * energy i * de, the last row for every energy beyond the table. */
int orc_energy_bin(const orc_sim *s, double energy_ev);
void orc_poisson(int32_t ng, double dx, const double *rho, double v_left, double *phi);
void orc_efield(int32_t ng, double dx, const double *phi, const double *rho, double *efield);
/* Scatter a projectile of relative velocity g about COM velocity w (eq. for v1'). */
void orc_scatter(const double g[3], double gmag, double gnew, double f2,
                 double cos_chi, double sin_chi, double eta, const double w[3],
                 double out[3]);
/* Electron-Ar collision for given uniforms.  proc_out: 0 el, 1 exc, 2 ion.
 * Writes the new velocity, and for ionization the ejected electron's. */
int orc_collide_electron(const orc_sim *s, const double v[3], int idx,
                         double r_proc, double r_chi, double r_eta, double r_share,
                         double vout[3], double vej[3], int *anomaly);
int orc_collide_ion(const orc_sim *s, const double v[3], const double va[3], int idx,
                    double r_proc, double r_chi, double r_eta, double vout[3]);

#ifdef __cplusplus
}
#endif
#endif
