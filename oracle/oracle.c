/*
 * CPU oracle for the eduPIC PIC/MCC time step (arXiv:2103.09642).
 * TEST INFRASTRUCTURE ONLY -- see oracle.h.
 *
 * Each step follows the six-step cycle of section 2.1 in the paper's order:
 *   1. densities   (eqs. for delta n_p, delta n_{p+1}; Algorithm 2)
 *   2. rho, Poisson, field (discrete Poisson equation, Thomas algorithm,
 *      field equations incl. the boundary forms; Algorithm 3)
 *   3-4. field interpolation and leapfrog push (Algorithm 4)
 *   5. absorbing walls (Algorithm 5)
 *   6. Monte Carlo collisions (eq. for P_coll, process selection, COM
 *      kinematics, Euler-angle rotation; Algorithm 6)
 * Ions are pushed, wall-checked and collided only on steps with
 * step % N_SUB == 0 (ion subcycling, section 2.1 and Algorithm 6); between
 * ion steps the last ion density is kept.
 *
 * Readings where the paper is silent or ambiguous are listed with the
 * code that takes them; they are the same readings the GPU library takes.
 */
#include "oracle.h"

#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

/* Physical constants: CODATA 2018 (the paper does not list its values). */
static const double E_CHARGE = 1.602176634e-19;   /* C    */
static const double M_ELECTRON = 9.1093837015e-31;    /* kg   */
static const double K_BOLTZMANN = 1.380649e-23;  /* J/K  */
static const double EPSILON0 = 8.8541878128e-12;  /* F/m  */
static const double AMU = 1.66053906660e-27;      /* kg   */
#define M_ARGON (39.948 * AMU)
#define MU_ION_ATOM (M_ARGON / 2.0)                  /* reduced mass Ar+ + Ar */
#define MU_ELECTRON_ATOM (M_ELECTRON * M_ARGON / (M_ELECTRON + M_ARGON)) /* reduced mass e + Ar */
#define J_PER_EV E_CHARGE
static const double PI_D = 3.14159265358979323846;
static const double TWO_PI_D = 6.28318530717958647692;
static const double TWO32 = 4294967296.0; /* fixed-point unit of one particle */

/* Fixed-point scales of the per-step diagnostic sums. */
static const double DIAG_JS = 1024.0;    /* c * vbar_x          [m/s]  */
static const double DIAG_WS = 1048576.0; /* c                          */
static const double DIAG_ES = 1048576.0; /* c * energy          [eV]   */
static const double DIAG_IZS = 4294967296.0; /* c * nu_ion dt_e        */

static char g_err[256];
const char *orc_error(void) { return g_err; }
static void set_err(const char *m) { snprintf(g_err, sizeof g_err, "%s", m); }

typedef struct {
  double *x, *vx, *vy, *vz;
  uint64_t *uid;
  int64_t n, cap;
} parts;

struct orc_sim {
  orc_case c;
  int32_t ng, nbins;
  double L, dx, inv_dx, dt_e, dt_i, dv, factor_w, factor_e, factor_i;
  double gas_n, sigma_a, de_cs, thr_exc, thr_ion, w_ion;
  double *sig_el, *sig_exc, *sig_ion, *sig_iso, *sig_back;
  double *nsig_e, *nsig_i; /* n * sigma_tot, per bin (section 3.2) */
  double nu_star_e, nu_star_i; /* null-collision maximum frequencies      */
  double p_null_e, p_null_i;   /* 1 - exp(-nu* dt) for each species      */
  parts e, i;
  int64_t step;
  int64_t *cnt_e, *cnt_i_cur; /* fixed-point densities of this step     */
  double *ne, *ni, *rho, *phi, *efield;
  int64_t counts[ORC_C_N];
  /* diagnostics */
  int64_t diag_steps, diag_ion_steps;
  double *sum_ne, *sum_ni;
  int64_t *eepf;
  int64_t *acc_je, *acc_ji, *acc_w, *acc_e; /* per step, fixed point    */
  double *sum_je, *sum_ji, *sum_w, *sum_e;  /* time sums                */
  /* xt arrays and IFEDF (section 3.5) */
  int32_t n_xt;
  int64_t *acc_wi, *acc_ei, *acc_iz; /* per step: ion weight and energy,
                                        electron ionization probability   */
  double *x_pot, *x_ef, *x_ne, *x_ni;       /* [n_xt][ng] sums of the grid values */
  double *x_je, *x_ji, *x_pe, *x_pi;        /* sums of acc, acc * E              */
  double *x_we, *x_ee, *x_wi, *x_ei, *x_iz; /* sums of acc                       */
  int64_t *x_steps, *x_ion_steps;           /* [n_xt] steps per bin              */
  int64_t *ifed;                            /* [2][n_ifed + 1]                   */
  parts see_new; /* electrons emitted in this step, added after step 6 */
};

/* ---------------------------------------------------------------------------
 * Random numbers.  Philox4x32-10 as defined by Salmon, Moraes, Dror & Shaw,
 * "Parallel random numbers: as easy as 1, 2, 3" (SC'11): ten rounds of two
 * 32x32->64 multiplies with the Weyl key schedule.  The paper uses a
 * sequential Mersenne Twister (section 3.3); a counter-based generator keyed
 * by (particle id, step) gives every particle its own reproducible stream,
 * which is what lets a parallel implementation draw the very same numbers.
 * ------------------------------------------------------------------------- */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
  uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
  uint32_t k0 = key[0], k1 = key[1];
  for (int round = 0; round < 10; ++round) {
    if (round > 0) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)x0;
    uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)x2;
    uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    uint32_t n0 = hi1 ^ x1 ^ k0;
    uint32_t n2 = hi0 ^ x3 ^ k1;
    x0 = n0;
    x1 = lo1;
    x2 = n2;
    x3 = lo0;
  }
  out[0] = x0;
  out[1] = x1;
  out[2] = x2;
  out[3] = x3;
}

/* Counter = (uid_lo, uid_hi, step, species<<24 | purpose<<8 | call);
 * key = (seed_lo, seed_hi).  Each pair of output words gives one uniform in
 * [0,1) with 53 random bits. */
void orc_uniform2(uint64_t seed, uint64_t uid, uint32_t step, uint32_t species,
                  uint32_t purpose, uint32_t call, double out[2]) {
  uint32_t ctr[4] = {(uint32_t)uid, (uint32_t)(uid >> 32), step,
                     (species << 24) | (purpose << 8) | call};
  uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
  uint32_t w[4];
  orc_philox4x32_10(ctr, key, w);
  uint64_t a = ((uint64_t)w[0] << 32) | w[1];
  uint64_t b = ((uint64_t)w[2] << 32) | w[3];
  out[0] = (double)(a >> 11) * (1.0 / 9007199254740992.0);
  out[1] = (double)(b >> 11) * (1.0 / 9007199254740992.0);
}

/* Two standard normal samples by the Box-Muller transform from two uniforms;
 * 1-u keeps the logarithm's argument in (0,1]. */
static void box_muller(const double u[2], double z[2]) {
  double r = sqrt(-2.0 * log(1.0 - u[0]));
  z[0] = r * cos(TWO_PI_D * u[1]);
  z[1] = r * sin(TWO_PI_D * u[1]);
}

/* Three normals for (uid, step, species, purpose) from calls 1 and 2. */
static void normals3(uint64_t seed, uint64_t uid, uint32_t step, uint32_t species,
                     uint32_t purpose, uint32_t first_call, double z[3]) {
  double u[2], a[2], b[2];
  orc_uniform2(seed, uid, step, species, purpose, first_call, u);
  box_muller(u, a);
  orc_uniform2(seed, uid, step, species, purpose, first_call + 1, u);
  box_muller(u, b);
  z[0] = a[0];
  z[1] = a[1];
  z[2] = b[0];
}

/* splitmix64 finaliser (Steele, Lea & Flood, OOPSLA 2014). */
uint64_t orc_mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

/* Identity of a particle born in an ionization at `step`: a hash of the
 * parent's identity, the step and the kind (1 = ejected electron, 2 = new
 * ion), so it does not depend on the order in which births happen. */
uint64_t orc_child_uid(uint64_t parent, int64_t step, uint64_t kind) {
  return orc_mix64(orc_mix64(parent) ^ ((uint64_t)step * 0x9E3779B97F4A7C15ull) ^ kind);
}

/* ---------------------------------------------------------------------------
 * Particle arrays
 * ------------------------------------------------------------------------- */
static int parts_reserve(parts *p, int64_t need) {
  if (need <= p->cap) return 0;
  int64_t cap = p->cap ? p->cap : 1024;
  while (cap < need) cap *= 2;
  double *nx = realloc(p->x, (size_t)cap * sizeof(double));
  if (!nx) return -1;
  p->x = nx;
  double *nvx = realloc(p->vx, (size_t)cap * sizeof(double));
  if (!nvx) return -1;
  p->vx = nvx;
  double *nvy = realloc(p->vy, (size_t)cap * sizeof(double));
  if (!nvy) return -1;
  p->vy = nvy;
  double *nvz = realloc(p->vz, (size_t)cap * sizeof(double));
  if (!nvz) return -1;
  p->vz = nvz;
  uint64_t *nu = realloc(p->uid, (size_t)cap * sizeof(uint64_t));
  if (!nu) return -1;
  p->uid = nu;
  p->cap = cap;
  return 0;
}

static void parts_free(parts *p) {
  free(p->x);
  free(p->vx);
  free(p->vy);
  free(p->vz);
  free(p->uid);
  memset(p, 0, sizeof *p);
}

static void parts_append(parts *p, double x, double vx, double vy, double vz, uint64_t uid) {
  if (parts_reserve(p, p->n + 1) != 0) {
    fprintf(stderr, "oracle: out of memory\n");
    abort();
  }
  p->x[p->n] = x;
  p->vx[p->n] = vx;
  p->vy[p->n] = vy;
  p->vz[p->n] = vz;
  p->uid[p->n] = uid;
  p->n++;
}

/* ---------------------------------------------------------------------------
 * Step 1: charge assignment (eqs. for delta n_p and delta n_{p+1}, Alg. 2).
 * Each particle carries 2^32 fixed-point units split linearly between the
 * two nodes that enclose it, so sums are exact integers and independent of
 * summation order.  p = int(x/dx), clamped to N_g-2 so that x = L puts its
 * whole weight on the last node.  The split truncates f*2^32 toward zero
 * (f >= 0) and is capped at 2^32.
 * ------------------------------------------------------------------------- */
void orc_deposit(const double *x, int64_t n, int32_t ng, double inv_dx, int64_t *cnt) {
  const int64_t unit = (int64_t)4294967296LL; /* one particle */
  for (int64_t k = 0; k < n; ++k) {
    const double xi = x[k] * inv_dx; /* position in cell units */
    int cell = (int)xi;
    if (cell > ng - 2) cell = ng - 2;
    const double frac = xi - (double)cell; /* share of node cell + 1 */
    int64_t upper = (int64_t)(frac * TWO32);
    if (upper > unit) upper = unit;
    cnt[cell] += unit - upper;
    cnt[cell + 1] += upper;
  }
}

/* Densities on the grid: counts times W/(A dx) / 2^32; the two edge nodes
 * own half cells, so they are doubled (Algorithm 2). */
static void density_from_counts(const orc_sim *s, const int64_t *cnt, double *n) {
  const double scale = s->factor_w / TWO32;
  for (int p = 0; p < s->ng; ++p) n[p] = (double)cnt[p] * scale;
  n[0] *= 2.0;
  n[s->ng - 1] *= 2.0;
}

/* ---------------------------------------------------------------------------
 * Step 2: the discrete Poisson equation (-phi_{p-1}+2phi_p-phi_{p+1})/dx^2 =
 * rho_p/eps0 with phi_0 = V(t), phi_{N_g-1} = 0, solved by the Thomas
 * algorithm for the constant tridiagonal matrix (Algorithm 3).  With
 * r_1 = 1/2 and r_p = 1/(2 - r_{p-1}) the forward sweep is
 * y_p = (d_p + y_{p-1}) r_p and the back substitution phi_p = y_p + r_p phi_{p+1}.
 * ------------------------------------------------------------------------- */
void orc_poisson(int32_t ng, double dx, const double *rho, double v_left, double *phi) {
  const int m = ng - 2; /* interior unknowns 1..m */
  phi[0] = v_left;
  phi[ng - 1] = 0.0;
  if (m <= 0) return;
  double *r = malloc((size_t)(m + 1) * sizeof(double));
  double *y = malloc((size_t)(m + 1) * sizeof(double));
  const double k = dx * dx / EPSILON0;
  r[1] = 0.5;
  for (int p = 2; p <= m; ++p) r[p] = 1.0 / (2.0 - r[p - 1]);
  double prev = 0.0;
  for (int p = 1; p <= m; ++p) {
    double d = rho[p] * k;
    if (p == 1) d = d + v_left;
    y[p] = (d + prev) * r[p];
    prev = y[p];
  }
  phi[m] = y[m];
  for (int p = m - 1; p >= 1; --p) phi[p] = y[p] + r[p] * phi[p + 1];
  free(r);
  free(y);
}

/* Field on the grid: centred difference inside, and the boundary forms that
 * add the half-cell charge (field equations of section 2.1.2). */
void orc_efield(int32_t ng, double dx, const double *phi, const double *rho, double *efield) {
  for (int p = 1; p < ng - 1; ++p) efield[p] = (phi[p - 1] - phi[p + 1]) / (2.0 * dx);
  efield[0] = (phi[0] - phi[1]) / dx - rho[0] * dx / (2.0 * EPSILON0);
  efield[ng - 1] = (phi[ng - 2] - phi[ng - 1]) / dx + rho[ng - 1] * dx / (2.0 * EPSILON0);
}

/* Driving voltage at the powered electrode at t_s = step*dt_e: a sum of
 * harmonics V_k sin(2 pi f_k t + phi_k) plus a DC offset (a self-bias, zero
 * unless set).  The paper's cosine is phi = pi/2. */
double orc_voltage(const orc_sim *s, int64_t step) {
  const double t = (double)step * s->dt_e;
  double v = 0.0;
  for (int k = 0; k < s->c.n_harm; ++k)
    v += s->c.v_amp[k] * sin(TWO_PI_D * s->c.freq_hz[k] * t + s->c.phase_rad[k]);
  return v + s->c.v_dc;
}

int orc_set_voltage(orc_sim *s, const double *v_amp, int32_t n, double v_dc) {
  if (n != s->c.n_harm) return set_err("amplitude count differs from n_harm"), -1;
  for (int k = 0; k < n; ++k) s->c.v_amp[k] = v_amp[k];
  s->c.v_dc = v_dc;
  return 0;
}

/* ---------------------------------------------------------------------------
 * Collisions (section 2.1.6).
 * ------------------------------------------------------------------------- */

/* Table row of a kinetic energy (section 3.2 tabulates the cross sections at
 * the energies i * de, i = 0..nbins-1): the row whose tabulation energy is
 * nearest, i.e. the integer part of energy/de + 1/2, with every energy past
 * the table's end taken by its last row (Algorithm 6). */
static int energy_bin(const orc_sim *s, double energy_ev) {
  const double rows = energy_ev / s->de_cs + 0.5;
  const int last = s->nbins - 1;
  return rows >= (double)last ? last : (int)rows;
}

int orc_energy_bin(const orc_sim *s, double energy_ev) { return energy_bin(s, energy_ev); }

/* v1' = w + m2/(m1+m2) g' R(theta,phi) (cos chi, sin chi cos eta, sin chi sin eta),
 * with the Euler angles of g taken from its components: cos theta = g_x/g,
 * sin theta = sqrt(g_y^2+g_z^2)/g, cos phi = g_y/g_yz, sin phi = g_z/g_yz,
 * and phi = 0 when g points along x.  The three components are written out
 * as in the final post-collision velocity equation. */
void orc_scatter(const double g[3], double gmag, double gnew, double f2,
                 double cos_chi, double sin_chi, double eta, const double w[3],
                 double out[3]) {
  double cos_theta, sin_theta, cos_phi, sin_phi;
  if (gmag > 0.0) {
    double gyz = sqrt(g[1] * g[1] + g[2] * g[2]);
    cos_theta = g[0] / gmag;
    sin_theta = gyz / gmag;
    if (gyz > 0.0) {
      cos_phi = g[1] / gyz;
      sin_phi = g[2] / gyz;
    } else {
      cos_phi = 1.0;
      sin_phi = 0.0;
    }
  } else {
    cos_theta = 1.0;
    sin_theta = 0.0;
    cos_phi = 1.0;
    sin_phi = 0.0;
  }
  const double cos_eta = cos(eta), sin_eta = sin(eta);
  const double a = f2 * gnew;
  out[0] = w[0] + a * (cos_theta * cos_chi - sin_theta * sin_chi * cos_eta);
  out[1] = w[1] + a * (sin_theta * cos_phi * cos_chi + cos_theta * cos_phi * sin_chi * cos_eta -
                       sin_phi * sin_chi * sin_eta);
  out[2] = w[2] + a * (sin_theta * sin_phi * cos_chi + cos_theta * sin_phi * sin_chi * cos_eta +
                       cos_phi * sin_chi * sin_eta);
}

/* e- + Ar with the atom at rest (cold gas): g = v, w = m_e/(m_e+M) v.
 * Process by partitioning [0,1) as elastic | excitation | ionization.
 * Elastic: g' = g, cos chi = 1 - 2R, eta = 2 pi R (isotropic).
 * Excitation: mu g'^2/2 = mu g^2/2 - eps_exc.
 * Ionization: E' = mu g^2/2 - eps_ion (COM energy), eps_e = w tan[R atan(E'/2w)],
 * eps_s = E' - eps_e; cos chi_{s,e} = sqrt(eps_{s,e}/E') and eta_e = eta_s + pi;
 * the ejected electron is scattered like the projectile about the same w.
 * A negative remaining energy (cannot happen with tables that are zero at
 * and below threshold) is clamped to zero and reported as an anomaly. */
static int electron_kinematics(const orc_sim *s, const double v[3], int proc, double r_chi,
                               double r_eta, double r_share, double vout[3], double vej[3],
                               int *anomaly);

int orc_collide_electron(const orc_sim *s, const double v[3], int idx,
                         double r_proc, double r_chi, double r_eta, double r_share,
                         double vout[3], double vej[3], int *anomaly) {
  const double s_el = s->sig_el[idx], s_exc = s->sig_exc[idx], s_ion = s->sig_ion[idx];
  const double st = s_el + s_exc + s_ion;
  int proc;
  if (!(st > 0.0) || r_proc < s_el / st)
    proc = 0;
  else if (r_proc < (s_el + s_exc) / st)
    proc = 1;
  else
    proc = 2;
  return electron_kinematics(s, v, proc, r_chi, r_eta, r_share, vout, vej, anomaly);
}

/* The new velocities of an electron collision whose process is chosen. */
static int electron_kinematics(const orc_sim *s, const double v[3], int proc, double r_chi,
                               double r_eta, double r_share, double vout[3], double vej[3],
                               int *anomaly) {
  const double f1 = M_ELECTRON / (M_ELECTRON + M_ARGON);
  const double f2 = M_ARGON / (M_ELECTRON + M_ARGON);
  /* squared speed, the three squares summed from x to z (Algorithm 6) */
  const double v2 = v[0] * v[0] + v[1] * v[1] + v[2] * v[2];
  const double g = sqrt(v2);
  const double w[3] = {f1 * v[0], f1 * v[1], f1 * v[2]};
  *anomaly = 0;
  const double eta = TWO_PI_D * r_eta;
  if (proc == 0 || proc == 1) {
    double gnew = g;
    if (proc == 1) {
      double ec = 0.5 * MU_ELECTRON_ATOM * v2 - s->thr_exc * J_PER_EV;
      if (ec < 0.0) {
        ec = 0.0;
        *anomaly = 1;
      }
      gnew = sqrt(2.0 * ec / MU_ELECTRON_ATOM);
    }
    const double cos_chi = 1.0 - 2.0 * r_chi;
    const double sin_chi = sqrt(1.0 - cos_chi * cos_chi);
    orc_scatter(v, g, gnew, f2, cos_chi, sin_chi, eta, w, vout);
    return proc;
  }
  double e_ev = 0.5 * MU_ELECTRON_ATOM * v2 / J_PER_EV - s->thr_ion;
  if (e_ev < 0.0) {
    e_ev = 0.0;
    *anomaly = 1;
  }
  const double e_ej = s->w_ion * tan(r_share * atan(e_ev / (2.0 * s->w_ion)));
  const double e_sc = e_ev - e_ej;
  const double g_sc = sqrt(2.0 * e_sc * J_PER_EV / MU_ELECTRON_ATOM);
  const double g_ej = sqrt(2.0 * e_ej * J_PER_EV / MU_ELECTRON_ATOM);
  double cs_sc, sn_sc, cs_ej, sn_ej;
  if (s->c.flags & ORC_IONIZ_ANGLE_LITERAL) {
    const double chi_sc = e_ev > 0.0 ? sqrt(e_sc / e_ev) : 0.0;
    const double chi_ej = e_ev > 0.0 ? sqrt(e_ej / e_ev) : 0.0;
    cs_sc = cos(chi_sc);
    sn_sc = sin(chi_sc);
    cs_ej = cos(chi_ej);
    sn_ej = sin(chi_ej);
  } else {
    cs_sc = e_ev > 0.0 ? sqrt(e_sc / e_ev) : 1.0;
    cs_ej = e_ev > 0.0 ? sqrt(e_ej / e_ev) : 1.0;
    sn_sc = sqrt(1.0 - cs_sc * cs_sc);
    sn_ej = sqrt(1.0 - cs_ej * cs_ej);
  }
  orc_scatter(v, g, g_sc, f2, cs_sc, sn_sc, eta, w, vout);
  orc_scatter(v, g, g_ej, f2, cs_ej, sn_ej, eta + PI_D, w, vej);
  return 2;
}

/* Ar+ + Ar with a thermal target va: g = v - va, w = (v + va)/2 (equal masses),
 * isotropic (cos chi = 1 - 2R) or backward (chi = pi) by partitioning [0,1)
 * as iso | back; |g'| = |g| (elastic). */
/* The new velocity of an ion collision whose process is chosen. */
static void ion_kinematics(const double v[3], const double va[3], int proc, double r_chi,
                           double r_eta, double vout[3]) {
  const double g3[3] = {v[0] - va[0], v[1] - va[1], v[2] - va[2]};
  const double g2 = g3[0] * g3[0] + g3[1] * g3[1] + g3[2] * g3[2];
  const double g = sqrt(g2);
  const double w[3] = {0.5 * (v[0] + va[0]), 0.5 * (v[1] + va[1]), 0.5 * (v[2] + va[2])};
  double cos_chi, sin_chi;
  if (proc == 0) {
    cos_chi = 1.0 - 2.0 * r_chi;
    sin_chi = sqrt(1.0 - cos_chi * cos_chi);
  } else {
    cos_chi = -1.0;
    sin_chi = 0.0;
  }
  orc_scatter(g3, g, g, 0.5, cos_chi, sin_chi, TWO_PI_D * r_eta, w, vout);
}

int orc_collide_ion(const orc_sim *s, const double v[3], const double va[3], int idx,
                    double r_proc, double r_chi, double r_eta, double vout[3]) {
  const double s_iso = s->sig_iso[idx], s_back = s->sig_back[idx];
  const int proc = (!(s_iso + s_back > 0.0) || r_proc < s_iso / (s_iso + s_back)) ? 0 : 1;
  ion_kinematics(v, va, proc, r_chi, r_eta, vout);
  return proc;
}

/* ---------------------------------------------------------------------------
 * Case set-up
 * ------------------------------------------------------------------------- */
/* Null-collision maximum frequency (section 2.1.6, the null-collision
 * method): nu* = max over the table of n sigma_tot(E) g(E), with g taken at
 * the upper end of every bin's energy range (bin i holds the energies that
 * round to i de) and, for the last bin, which also holds every energy beyond
 * the table, at four times the table's range.  mass is the electron mass
 * (LAB energy) or the Ar+ + Ar reduced mass (COM energy). */
double orc_nu_star(const double *nsig, int32_t nb, double de_ev, double mass) {
  double m = 0.0;
  for (int32_t i = 0; i < nb; ++i) {
    const double e_hi = (i == nb - 1) ? 4.0 * (double)nb * de_ev : ((double)i + 0.5) * de_ev;
    const double g = sqrt(2.0 * e_hi * J_PER_EV / mass);
    const double nu = nsig[i] * g;
    if (nu > m) m = nu;
  }
  return m;
}

static double *dup_table(const double *src, int n) {
  double *d = malloc((size_t)n * sizeof(double));
  if (d && src) memcpy(d, src, (size_t)n * sizeof(double));
  if (d && !src) memset(d, 0, (size_t)n * sizeof(double));
  return d;
}

orc_sim *orc_new(const orc_case *c, const orc_xsec *xs) {
  if (!c || !xs) return set_err("null argument"), NULL;
  if (c->n_grid < 2) return set_err("n_grid must be >= 2"), NULL;
  if (c->ion_subcycle < 1) return set_err("ion_subcycle must be >= 1"), NULL;
  if (!(c->dt_e > 0.0)) return set_err("dt_e must be > 0"), NULL;
  if (!(c->gap_m > 0.0)) return set_err("gap must be > 0"), NULL;
  if (!(c->area_m2 > 0.0)) return set_err("area must be > 0"), NULL;
  if (c->n_harm < 0 || c->n_harm > 4) return set_err("n_harm must be 0..4"), NULL;
  if (xs->n_bins < 1 || !(xs->de_ev > 0.0)) return set_err("bad cross-section table"), NULL;
  if ((c->flags & ORC_DIAG_EEPF) && (c->n_eepf < 1 || !(c->de_eepf_ev > 0.0)))
    return set_err("bad EEPF binning"), NULL;
  if ((c->flags & ORC_DIAG_XT) &&
      (c->n_xt_bin < 1 || c->steps_per_cycle < 1 || c->steps_per_cycle % c->n_xt_bin != 0))
    return set_err("N_BIN must divide the steps per cycle"), NULL;
  if ((c->flags & ORC_DIAG_IFED) && (c->n_ifed < 1 || !(c->de_ifed_ev > 0.0)))
    return set_err("bad IFEDF binning"), NULL;
  for (int k = 0; k < 2; ++k)
    if (!(c->gamma_see[k] >= 0.0 && c->gamma_see[k] <= 1.0) ||
        !(c->eta_refl[k] >= 0.0 && c->eta_refl[k] <= 1.0))
      return set_err("surface probabilities must be in [0, 1]"), NULL;
  if ((c->gamma_see[0] > 0.0 || c->gamma_see[1] > 0.0) && !(c->see_te_ev > 0.0))
    return set_err("secondary electron temperature must be > 0"), NULL;
  orc_sim *s = calloc(1, sizeof *s);
  if (!s) return set_err("out of memory"), NULL;
  s->c = *c;
  s->ng = c->n_grid;
  s->nbins = xs->n_bins;
  s->L = c->gap_m;
  s->dx = s->L / (double)(s->ng - 1);
  s->inv_dx = 1.0 / s->dx;
  s->dt_e = c->dt_e;
  s->dt_i = (double)c->ion_subcycle * c->dt_e;
  s->dv = c->area_m2 * s->dx;
  s->factor_w = c->weight / s->dv;
  s->factor_e = s->dt_e / M_ELECTRON * E_CHARGE;
  s->factor_i = s->dt_i / M_ARGON * E_CHARGE;
  s->gas_n = c->pressure_pa / (K_BOLTZMANN * c->gas_temp_k);
  s->sigma_a = sqrt(K_BOLTZMANN * c->gas_temp_k / M_ARGON);
  s->de_cs = xs->de_ev;
  s->thr_exc = xs->e_exc_thr_ev;
  s->thr_ion = xs->e_ion_thr_ev;
  s->w_ion = xs->w_ioniz_ev;
  const int nb = s->nbins, ng = s->ng;
  s->sig_el = dup_table(xs->e_el, nb);
  s->sig_exc = dup_table(xs->e_exc, nb);
  s->sig_ion = dup_table(xs->e_ion, nb);
  s->sig_iso = dup_table(xs->i_iso, nb);
  s->sig_back = dup_table(xs->i_back, nb);
  s->nsig_e = malloc((size_t)nb * sizeof(double));
  s->nsig_i = malloc((size_t)nb * sizeof(double));
  /* n sigma_tot per bin (calc_total_cross_sections, section 3.2). */
  for (int k = 0; k < nb; ++k) {
    s->nsig_e[k] = s->gas_n * (s->sig_el[k] + s->sig_exc[k] + s->sig_ion[k]);
    s->nsig_i[k] = s->gas_n * (s->sig_iso[k] + s->sig_back[k]);
  }
  s->nu_star_e = orc_nu_star(s->nsig_e, nb, s->de_cs, M_ELECTRON);
  s->nu_star_i = orc_nu_star(s->nsig_i, nb, s->de_cs, MU_ION_ATOM);
  s->p_null_e = 1.0 - exp(-s->nu_star_e * s->dt_e);
  s->p_null_i = 1.0 - exp(-s->nu_star_i * s->dt_i);
  s->cnt_e = calloc((size_t)ng, sizeof(int64_t));
  s->cnt_i_cur = calloc((size_t)ng, sizeof(int64_t));
  s->ne = calloc((size_t)ng, sizeof(double));
  s->ni = calloc((size_t)ng, sizeof(double));
  s->rho = calloc((size_t)ng, sizeof(double));
  s->phi = calloc((size_t)ng, sizeof(double));
  s->efield = calloc((size_t)ng, sizeof(double));
  s->sum_ne = calloc((size_t)ng, sizeof(double));
  s->sum_ni = calloc((size_t)ng, sizeof(double));
  s->acc_je = calloc((size_t)ng, sizeof(int64_t));
  s->acc_ji = calloc((size_t)ng, sizeof(int64_t));
  s->acc_w = calloc((size_t)ng, sizeof(int64_t));
  s->acc_e = calloc((size_t)ng, sizeof(int64_t));
  s->sum_je = calloc((size_t)ng, sizeof(double));
  s->sum_ji = calloc((size_t)ng, sizeof(double));
  s->sum_w = calloc((size_t)ng, sizeof(double));
  s->sum_e = calloc((size_t)ng, sizeof(double));
  s->eepf = calloc((size_t)(c->n_eepf > 0 ? c->n_eepf : 1), sizeof(int64_t));
  s->acc_wi = calloc((size_t)ng, sizeof(int64_t));
  s->acc_ei = calloc((size_t)ng, sizeof(int64_t));
  s->acc_iz = calloc((size_t)ng, sizeof(int64_t));
  s->n_xt = (c->flags & ORC_DIAG_XT) ? c->steps_per_cycle / c->n_xt_bin : 1;
  const size_t nx = (size_t)s->n_xt * (size_t)ng;
  double **xt[] = {&s->x_pot, &s->x_ef, &s->x_ne, &s->x_ni, &s->x_je, &s->x_ji, &s->x_pe,
                   &s->x_pi, &s->x_we, &s->x_ee, &s->x_wi, &s->x_ei, &s->x_iz};
  for (size_t k = 0; k < sizeof xt / sizeof xt[0]; ++k) *xt[k] = calloc(nx, sizeof(double));
  s->x_steps = calloc((size_t)s->n_xt, sizeof(int64_t));
  s->x_ion_steps = calloc((size_t)s->n_xt, sizeof(int64_t));
  s->ifed = calloc(2 * (size_t)((c->flags & ORC_DIAG_IFED) ? c->n_ifed + 1 : 1), sizeof(int64_t));
  return s;
}

void orc_free(orc_sim *s) {
  if (!s) return;
  parts_free(&s->e);
  parts_free(&s->i);
  parts_free(&s->see_new);
  double *dbl[] = {s->sig_el, s->sig_exc, s->sig_ion, s->sig_iso, s->sig_back, s->nsig_e,
                   s->nsig_i, s->ne, s->ni, s->rho, s->phi, s->efield, s->sum_ne, s->sum_ni,
                   s->sum_je, s->sum_ji, s->sum_w, s->sum_e, s->x_pot, s->x_ef, s->x_ne,
                   s->x_ni, s->x_je, s->x_ji, s->x_pe, s->x_pi, s->x_we, s->x_ee,
                   s->x_wi, s->x_ei, s->x_iz};
  for (size_t k = 0; k < sizeof dbl / sizeof dbl[0]; ++k) free(dbl[k]);
  free(s->cnt_e);
  free(s->cnt_i_cur);
  free(s->acc_je);
  free(s->acc_ji);
  free(s->acc_w);
  free(s->acc_e);
  free(s->eepf);
  free(s->acc_wi);
  free(s->acc_ei);
  free(s->acc_iz);
  free(s->x_steps);
  free(s->x_ion_steps);
  free(s->ifed);
  free(s);
}

static void redeposit_ions(orc_sim *s) {
  memset(s->cnt_i_cur, 0, (size_t)s->ng * sizeof(int64_t));
  orc_deposit(s->i.x, s->i.n, s->ng, s->inv_dx, s->cnt_i_cur);
}

/* Initial particles (Algorithm 1, init): uniform random positions in [0,L)
 * and, as the workloads ask, Maxwellian velocities (k T_e for electrons, the
 * ion temperature for Ar+), taken as the half-step velocities v(-dt/2). */
int orc_seed(orc_sim *s) {
  const double sig_e = sqrt(s->c.te_init_ev * J_PER_EV / M_ELECTRON);
  const double sig_i = sqrt(K_BOLTZMANN * s->c.ti_init_k / M_ARGON);
  parts *sp[2] = {&s->e, &s->i};
  const int64_t nn[2] = {s->c.n_init_e, s->c.n_init_i};
  const double sg[2] = {sig_e, sig_i};
  for (int sp_i = 0; sp_i < 2; ++sp_i) {
    parts *p = sp[sp_i];
    p->n = 0;
    if (parts_reserve(p, nn[sp_i] > 0 ? nn[sp_i] : 1) != 0) return set_err("out of memory"), -1;
    for (int64_t k = 0; k < nn[sp_i]; ++k) {
      double u[2], z[3];
      orc_uniform2(s->c.seed, (uint64_t)k, 0u, (uint32_t)sp_i, 1u, 0u, u);
      normals3(s->c.seed, (uint64_t)k, 0u, (uint32_t)sp_i, 1u, 1u, z);
      parts_append(p, s->L * u[0], sg[sp_i] * z[0], sg[sp_i] * z[1], sg[sp_i] * z[2],
                   (uint64_t)k);
    }
  }
  s->step = 0;
  redeposit_ions(s);
  return 0;
}

int orc_set_state(orc_sim *s, int species, const double *x, const double *vx,
                  const double *vy, const double *vz, const uint64_t *uid, int64_t n,
                  int64_t step) {
  parts *p = species == 0 ? &s->e : &s->i;
  if (parts_reserve(p, n > 0 ? n : 1) != 0) return set_err("out of memory"), -1;
  for (int64_t k = 0; k < n; ++k) {
    p->x[k] = x[k];
    p->vx[k] = vx[k];
    p->vy[k] = vy[k];
    p->vz[k] = vz[k];
    p->uid[k] = uid[k];
  }
  p->n = n;
  s->step = step;
  /* Reading: the ion density held until the next ion step is the one of the
   * ions as given. */
  if (species == 1) redeposit_ions(s);
  return 0;
}

int64_t orc_get_state(const orc_sim *s, int species, double *x, double *vx, double *vy,
                      double *vz, uint64_t *uid, int64_t cap) {
  const parts *p = species == 0 ? &s->e : &s->i;
  int64_t m = p->n < cap ? p->n : cap;
  for (int64_t k = 0; k < m; ++k) {
    if (x) x[k] = p->x[k];
    if (vx) vx[k] = p->vx[k];
    if (vy) vy[k] = p->vy[k];
    if (vz) vz[k] = p->vz[k];
    if (uid) uid[k] = p->uid[k];
  }
  return p->n;
}

/* ---------------------------------------------------------------------------
 * Steps 3-4: interpolate E to the particle (eq. for E_j) and leapfrog
 * (eqs. for v(t+dt/2) and x(t+dt)), Algorithm 4.  In measurement mode the
 * velocity at integer time, the mean of the old and new half-step velocities,
 * is used with the old position (section 3.6).  With the xt arrays the
 * ionization rate is measured there too, as the expected rate
 * n sigma_ion(eps) |v| of each electron at that velocity (reading: the paper
 * measures it where the particles move, with the time-centred velocities).
 * ------------------------------------------------------------------------- */
/* Linear field interpolation of section 2.1.3: in cell units xi = x / dx
 * (evaluated as x times the stored 1/dx), the particle lies between node
 * `cell` = floor(xi) (at most N_g - 2, so x = L sits in the last cell) and the
 * next one, whose weights are (cell + 1) - xi and xi - cell. */
typedef struct {
  int cell;
  double w_lo, w_hi; /* weights of node `cell` and node `cell + 1` */
} cic;

static cic cic_weights(const orc_sim *s, double x) {
  cic w;
  const double xi = x * s->inv_dx;
  w.cell = (int)xi;
  if (w.cell > s->ng - 2) w.cell = s->ng - 2;
  w.w_lo = (double)(w.cell + 1) - xi;
  w.w_hi = xi - (double)w.cell;
  return w;
}

static void push(orc_sim *s, parts *p, int is_ion) {
  const double *E = s->efield;
  const double dt = is_ion ? s->dt_i : s->dt_e;
  /* e dt / m per unit field: the velocity equation's kick is E_j times it,
   * added for an ion and subtracted for an electron (charge -e) */
  const double kick = is_ion ? s->factor_i : s->factor_e;
  const uint32_t fl = s->c.flags;
  const double x_lo = 0.45 * s->L, x_hi = 0.55 * s->L;
  for (int64_t k = 0; k < p->n; ++k) {
    const double x = p->x[k];
    const cic w = cic_weights(s, x);
    const int q = w.cell;
    const double e_here = E[q] * w.w_lo + E[q + 1] * w.w_hi;
    const double vx_old = p->vx[k];
    /* v(t + dt/2) = v(t - dt/2) + (q/m) E dt */
    const double vx_new = is_ion ? vx_old + e_here * kick : vx_old - e_here * kick;
    p->vx[k] = vx_new;
    /* x(t + dt) = x(t) + v(t + dt/2) dt */
    p->x[k] = x + vx_new * dt;
    if (!(fl & (ORC_DIAG_CURRENT | ORC_DIAG_MEANE | ORC_DIAG_EEPF | ORC_DIAG_XT))) continue;
    const double vbar = 0.5 * (vx_old + vx_new);
    const int xt = (fl & ORC_DIAG_XT) != 0;
    if (fl & (ORC_DIAG_CURRENT | ORC_DIAG_XT)) {
      int64_t *acc = is_ion ? s->acc_ji : s->acc_je;
      acc[q] += (int64_t)(w.w_lo * vbar * DIAG_JS);
      acc[q + 1] += (int64_t)(w.w_hi * vbar * DIAG_JS);
    }
    const double vy = p->vy[k], vz = p->vz[k];
    if (is_ion) {
      if (xt) {
        const double en_i = 0.5 * M_ARGON * (vbar * vbar + vy * vy + vz * vz) / J_PER_EV;
        s->acc_wi[q] += (int64_t)(w.w_lo * DIAG_WS);
        s->acc_wi[q + 1] += (int64_t)(w.w_hi * DIAG_WS);
        s->acc_ei[q] += (int64_t)(w.w_lo * en_i * DIAG_ES);
        s->acc_ei[q + 1] += (int64_t)(w.w_hi * en_i * DIAG_ES);
      }
      continue;
    }
    if (!(fl & (ORC_DIAG_MEANE | ORC_DIAG_EEPF | ORC_DIAG_XT))) continue;
    const double en = 0.5 * M_ELECTRON * (vbar * vbar + vy * vy + vz * vz) / J_PER_EV;
    if (xt) {
      const double vmag = sqrt(vbar * vbar + vy * vy + vz * vz);
      const double pdt = (s->gas_n * s->sig_ion[energy_bin(s, en)]) * vmag * s->dt_e;
      s->acc_iz[q] += (int64_t)(w.w_lo * pdt * DIAG_IZS);
      s->acc_iz[q + 1] += (int64_t)(w.w_hi * pdt * DIAG_IZS);
    }
    if (fl & (ORC_DIAG_MEANE | ORC_DIAG_XT)) {
      s->acc_w[q] += (int64_t)(w.w_lo * DIAG_WS);
      s->acc_w[q + 1] += (int64_t)(w.w_hi * DIAG_WS);
      s->acc_e[q] += (int64_t)(w.w_lo * en * DIAG_ES);
      s->acc_e[q + 1] += (int64_t)(w.w_hi * en * DIAG_ES);
    }
    if ((fl & ORC_DIAG_EEPF) && x >= x_lo && x <= x_hi) {
      const double t = en / s->c.de_eepf_ev;
      if (t < (double)s->c.n_eepf) s->eepf[(int)t]++;
    }
  }
}

/* Surface processes of section 5, drawn from purpose 3 of the particle's
 * counter at this step.  Electron reflection: with probability eta of the
 * electrode (R < eta, call 0), the electron is reflected specularly: the
 * position is mirrored in the electrode and v_x reversed, so the energy is
 * kept (reading: elastic means specular).  A mirror image outside the gap
 * (a flight longer than the gap) is absorbed.  Returns 1 if reflected. */
static int reflect_electron(orc_sim *s, parts *p, int64_t k, int side) {
  const double eta = s->c.eta_refl[side];
  if (!(eta > 0.0)) return 0;
  double r[2];
  orc_uniform2(s->c.seed, p->uid[k], (uint32_t)s->step, 0u, 3u, 0u, r);
  if (!(r[0] < eta)) return 0;
  const double xm = side == 0 ? -p->x[k] : 2.0 * s->L - p->x[k];
  if (!(xm >= 0.0 && xm <= s->L)) return 0;
  p->x[k] = xm;
  p->vx[k] = -p->vx[k];
  s->counts[ORC_C_REFL]++;
  return 1;
}

/* Ion-induced secondary emission: an ion absorbed at electrode `side` emits
 * an electron if R < gamma (call 0).  Reading: the electron starts on the
 * electrode surface with the velocity of a thermal flux leaving it at
 * temperature T_see: the normal component is Rayleigh distributed,
 * sigma sqrt(-2 ln(1 - u_a)) into the gap, the two tangential ones normal
 * (Box-Muller of u_b, u_c), sigma = sqrt(k T_see / m); calls 1 -> (u_a, u_b),
 * 2 -> u_c.  Its identity is the child of the ion with kind 3.  It is added
 * after the collisions of this step, like the other newborns. */
static void emit_secondary(orc_sim *s, const parts *p, int64_t k, int side) {
  const double gamma = s->c.gamma_see[side];
  if (!(gamma > 0.0)) return;
  const uint64_t uid = p->uid[k];
  const uint32_t st = (uint32_t)s->step;
  double r[2];
  orc_uniform2(s->c.seed, uid, st, 1u, 3u, 0u, r);
  if (!(r[0] < gamma)) return;
  double a[2], b[2];
  orc_uniform2(s->c.seed, uid, st, 1u, 3u, 1u, a);
  orc_uniform2(s->c.seed, uid, st, 1u, 3u, 2u, b);
  const double sig = sqrt(s->c.see_te_ev * J_PER_EV / M_ELECTRON);
  const double vn = sig * sqrt(-2.0 * log(1.0 - a[0]));
  const double vt = sig * sqrt(-2.0 * log(1.0 - a[1]));
  const double vy = vt * cos(TWO_PI_D * b[0]);
  const double vz = vt * sin(TWO_PI_D * b[0]);
  if (side == 0)
    parts_append(&s->see_new, 0.0, vn, vy, vz, orc_child_uid(uid, s->step, 3));
  else
    parts_append(&s->see_new, s->L, -vn, vy, vz, orc_child_uid(uid, s->step, 3));
  s->counts[side == 0 ? ORC_C_SEE_POW : ORC_C_SEE_GND]++;
}

/* Step 5: absorbing electrodes; removal by moving the last particle into the
 * hole (Algorithm 5).  x < 0: powered electrode, x > L: grounded.  An
 * absorbed ion adds its impact energy M v^2 / 2, from the half-step velocity
 * that carried it out, to its electrode's IFEDF (Algorithm 5, ions), and may
 * emit a secondary electron; an electron may be reflected instead. */
static void walls(orc_sim *s, parts *p, int is_ion) {
  const int ifed = is_ion && (s->c.flags & ORC_DIAG_IFED);
  int64_t k = 0;
  while (k < p->n) {
    const double x = p->x[k];
    if (!is_ion && (x < 0.0 || x > s->L) && reflect_electron(s, p, k, x < 0.0 ? 0 : 1)) {
      ++k;
      continue;
    }
    int out = 0;
    if (x < 0.0) {
      s->counts[is_ion ? ORC_C_ABS_I_POW : ORC_C_ABS_E_POW]++;
      out = 1;
    }
    if (x > s->L) {
      s->counts[is_ion ? ORC_C_ABS_I_GND : ORC_C_ABS_E_GND]++;
      out = 2;
    }
    if (out && is_ion) emit_secondary(s, p, k, out - 1);
    if (out && ifed) {
      const double vx = p->vx[k], vy = p->vy[k], vz = p->vz[k];
      const double en = 0.5 * M_ARGON * (vx * vx + vy * vy + vz * vz) / J_PER_EV;
      const double t = en / s->c.de_ifed_ev;
      const int nb = s->c.n_ifed;
      const int b = t < (double)nb ? (int)t : nb;
      s->ifed[(out - 1) * (nb + 1) + b]++;
    }
    if (out) {
      const int64_t last = p->n - 1;
      p->x[k] = p->x[last];
      p->vx[k] = p->vx[last];
      p->vy[k] = p->vy[last];
      p->vz[k] = p->vz[last];
      p->uid[k] = p->uid[last];
      p->n--;
    } else {
      ++k;
    }
  }
}

/* Kinetic energy [eV] of mass `mass` moving at squared speed g2: the LAB
 * energy of an electron hitting a gas atom at rest, or with the reduced mass
 * the COM energy of an ion-atom pair (section 2.1.6). */
static double kinetic_ev(double mass, double g2) { return 0.5 * mass * g2 / J_PER_EV; }

/* Probability of a collision within dt at relative speed g (the P_coll
 * equation of section 2.1.6): 1 - exp(-nu dt) with the total collision
 * frequency nu = n sigma_T(eps) g, n sigma_T being tabulated per table row. */
static double collision_probability(const double *nsig_tot, int row, double g, double dt) {
  const double nu = nsig_tot[row] * g;
  return 1.0 - exp(-nu * dt);
}

/* Step 6 for one electron: the gas atom is at rest, so g = |v| and the
 * energy is the LAB one; a collision happens iff R < P_coll (Algorithm 6). */
static void electron_mcc(orc_sim *s, int64_t k) {
  parts *p = &s->e;
  const double vx = p->vx[k], vy = p->vy[k], vz = p->vz[k];
  const double g2 = vx * vx + vy * vy + vz * vz;
  const double g = sqrt(g2);
  const int idx = energy_bin(s, kinetic_ev(M_ELECTRON, g2));
  const double p_coll = collision_probability(s->nsig_e, idx, g, s->dt_e);
  const uint64_t uid = p->uid[k];
  const uint32_t st = (uint32_t)s->step;
  double r0[2];
  orc_uniform2(s->c.seed, uid, st, 0u, 0u, 0u, r0);
  if (!(r0[0] < p_coll)) return;
  double r1[2], r2[2];
  orc_uniform2(s->c.seed, uid, st, 0u, 0u, 1u, r1);
  orc_uniform2(s->c.seed, uid, st, 0u, 0u, 2u, r2);
  const double vin[3] = {vx, vy, vz};
  double vout[3], vej[3];
  int anomaly = 0;
  const int proc = orc_collide_electron(s, vin, idx, r0[1], r1[0], r1[1], r2[0], vout, vej, &anomaly);
  p->vx[k] = vout[0];
  p->vy[k] = vout[1];
  p->vz[k] = vout[2];
  s->counts[ORC_C_COLL_E]++;
  s->counts[ORC_C_ANOMALY] += anomaly;
  if (proc == 2) {
    const double x = p->x[k];
    const uint64_t uid_e = orc_child_uid(uid, s->step, 1);
    const uint64_t uid_i = orc_child_uid(uid, s->step, 2);
    parts_append(&s->e, x, vej[0], vej[1], vej[2], uid_e);
    /* Reading: the new ion takes a thermal velocity of the gas. */
    double z[3];
    normals3(s->c.seed, uid_i, st, 1u, 2u, 1u, z);
    parts_append(&s->i, x, s->sigma_a * z[0], s->sigma_a * z[1], s->sigma_a * z[2], uid_i);
    s->counts[ORC_C_IONIZ]++;
  }
}

/* Step 6 for one electron with null-collision selection (section 2.1.6 and
 * the suggested extension of section 5): a candidate with probability
 * P* = 1 - exp(-nu* dt) (R_coll < P*), then process k with probability
 * nu_k(E)/nu* from R_proc nu* against the cumulative nu_el, nu_exc, nu_ion
 * (nu_k = (n sigma_k) v); the remainder is the null process, which leaves
 * the particle unchanged.  nu_tot > nu* (an energy beyond the bound) is an
 * anomaly; the candidate then always collides. */
static void electron_mcc_null(orc_sim *s, int64_t k) {
  parts *p = &s->e;
  const uint64_t uid = p->uid[k];
  const uint32_t st = (uint32_t)s->step;
  double r0[2];
  orc_uniform2(s->c.seed, uid, st, 0u, 0u, 0u, r0);
  if (!(r0[0] < s->p_null_e)) return;
  const double vx = p->vx[k], vy = p->vy[k], vz = p->vz[k];
  const double v2 = vx * vx + vy * vy + vz * vz;
  const double v = sqrt(v2);
  const int idx = energy_bin(s, kinetic_ev(M_ELECTRON, v2));
  const double nu_el = (s->gas_n * s->sig_el[idx]) * v;
  const double nu_exc = (s->gas_n * s->sig_exc[idx]) * v;
  const double nu_ion = (s->gas_n * s->sig_ion[idx]) * v;
  const double c1 = nu_el, c2 = c1 + nu_exc, c3 = c2 + nu_ion;
  if (c3 > s->nu_star_e) s->counts[ORC_C_ANOMALY]++;
  const double t = r0[1] * s->nu_star_e;
  const int proc = t < c1 ? 0 : (t < c2 ? 1 : (t < c3 ? 2 : -1));
  if (proc < 0) return; /* null collision */
  double r1[2], r2[2];
  orc_uniform2(s->c.seed, uid, st, 0u, 0u, 1u, r1);
  orc_uniform2(s->c.seed, uid, st, 0u, 0u, 2u, r2);
  const double vin[3] = {vx, vy, vz};
  double vout[3], vej[3];
  int anomaly = 0;
  electron_kinematics(s, vin, proc, r1[0], r1[1], r2[0], vout, vej, &anomaly);
  p->vx[k] = vout[0];
  p->vy[k] = vout[1];
  p->vz[k] = vout[2];
  s->counts[ORC_C_COLL_E]++;
  s->counts[ORC_C_ANOMALY] += anomaly;
  if (proc == 2) {
    const double x = p->x[k];
    const uint64_t uid_e = orc_child_uid(uid, s->step, 1);
    const uint64_t uid_i = orc_child_uid(uid, s->step, 2);
    parts_append(&s->e, x, vej[0], vej[1], vej[2], uid_e);
    double z[3];
    normals3(s->c.seed, uid_i, st, 1u, 2u, 1u, z);
    parts_append(&s->i, x, s->sigma_a * z[0], s->sigma_a * z[1], s->sigma_a * z[2], uid_i);
    s->counts[ORC_C_IONIZ]++;
  }
}

/* Step 6 for one ion with null-collision selection: candidate with
 * probability P* (R_coll < P*); the target atom is drawn for candidates
 * only (the same counter as in the direct method, so the same atom), then
 * isotropic / backward / null from R_proc nu* against nu_iso, nu_iso +
 * nu_back with nu_k = (n sigma_k) g. */
static void ion_mcc_null(orc_sim *s, int64_t k) {
  parts *p = &s->i;
  const uint64_t uid = p->uid[k];
  const uint32_t st = (uint32_t)s->step;
  double r2[2];
  orc_uniform2(s->c.seed, uid, st, 1u, 0u, 2u, r2);
  if (!(r2[0] < s->p_null_i)) return;
  double z[3];
  normals3(s->c.seed, uid, st, 1u, 0u, 0u, z);
  const double va[3] = {s->sigma_a * z[0], s->sigma_a * z[1], s->sigma_a * z[2]};
  const double vx = p->vx[k], vy = p->vy[k], vz = p->vz[k];
  const double gx = vx - va[0], gy = vy - va[1], gz = vz - va[2];
  const double g2 = gx * gx + gy * gy + gz * gz;
  const double g = sqrt(g2);
  const int idx = energy_bin(s, kinetic_ev(MU_ION_ATOM, g2));
  const double nu_iso = (s->gas_n * s->sig_iso[idx]) * g;
  const double nu_back = (s->gas_n * s->sig_back[idx]) * g;
  const double c1 = nu_iso, c2 = c1 + nu_back;
  if (c2 > s->nu_star_i) s->counts[ORC_C_ANOMALY]++;
  const double t = r2[1] * s->nu_star_i;
  const int proc = t < c1 ? 0 : (t < c2 ? 1 : -1);
  if (proc < 0) return;
  double r3[2];
  orc_uniform2(s->c.seed, uid, st, 1u, 0u, 3u, r3);
  const double vin[3] = {vx, vy, vz};
  double vout[3];
  ion_kinematics(vin, va, proc, r3[0], r3[1], vout);
  p->vx[k] = vout[0];
  p->vy[k] = vout[1];
  p->vz[k] = vout[2];
  s->counts[ORC_C_COLL_I]++;
}

/* Step 6 for one ion on an ion step: draw the target from the gas Maxwellian
 * first, then P from the COM energy mu g^2/2 (Algorithm 6). */
static void ion_mcc(orc_sim *s, int64_t k) {
  parts *p = &s->i;
  const uint64_t uid = p->uid[k];
  const uint32_t st = (uint32_t)s->step;
  double z[3];
  normals3(s->c.seed, uid, st, 1u, 0u, 0u, z);
  const double va[3] = {s->sigma_a * z[0], s->sigma_a * z[1], s->sigma_a * z[2]};
  const double vx = p->vx[k], vy = p->vy[k], vz = p->vz[k];
  const double gx = vx - va[0], gy = vy - va[1], gz = vz - va[2];
  const double g2 = gx * gx + gy * gy + gz * gz;
  const double g = sqrt(g2);
  const int idx = energy_bin(s, kinetic_ev(MU_ION_ATOM, g2));
  const double p_coll = collision_probability(s->nsig_i, idx, g, s->dt_i);
  double r2[2];
  orc_uniform2(s->c.seed, uid, st, 1u, 0u, 2u, r2);
  if (!(r2[0] < p_coll)) return;
  double r3[2];
  orc_uniform2(s->c.seed, uid, st, 1u, 0u, 3u, r3);
  const double vin[3] = {vx, vy, vz};
  double vout[3];
  orc_collide_ion(s, vin, va, idx, r2[1], r3[0], r3[1], vout);
  p->vx[k] = vout[0];
  p->vy[k] = vout[1];
  p->vz[k] = vout[2];
  s->counts[ORC_C_COLL_I]++;
}

static void one_step(orc_sim *s) {
  const int ng = s->ng;
  const int ion_step = (s->step % s->c.ion_subcycle) == 0;
  const uint32_t fl = s->c.flags;
  const int xt = (fl & ORC_DIAG_XT) != 0;
  /* xt time bin of this step: N_BIN consecutive steps of the RF period */
  const size_t row =
      xt ? (size_t)((s->step % s->c.steps_per_cycle) / s->c.n_xt_bin) * (size_t)ng : 0;
  /* 1. densities */
  memset(s->cnt_e, 0, (size_t)ng * sizeof(int64_t));
  orc_deposit(s->e.x, s->e.n, ng, s->inv_dx, s->cnt_e);
  if (ion_step) redeposit_ions(s);
  density_from_counts(s, s->cnt_e, s->ne);
  density_from_counts(s, s->cnt_i_cur, s->ni);
  /* 2. charge, potential, field */
  for (int p = 0; p < ng; ++p) s->rho[p] = E_CHARGE * (s->ni[p] - s->ne[p]);
  orc_poisson(ng, s->dx, s->rho, orc_voltage(s, s->step), s->phi);
  orc_efield(ng, s->dx, s->phi, s->rho, s->efield);
  if (fl & ORC_DIAG_DENSITY)
    for (int p = 0; p < ng; ++p) {
      s->sum_ne[p] += s->ne[p];
      s->sum_ni[p] += s->ni[p];
    }
  if (xt) {
    for (int p = 0; p < ng; ++p) {
      s->x_pot[row + p] += s->phi[p];
      s->x_ef[row + p] += s->efield[p];
      s->x_ne[row + p] += s->ne[p];
      s->x_ni[row + p] += s->ni[p];
    }
    s->x_steps[row / (size_t)ng]++;
    if (ion_step) s->x_ion_steps[row / (size_t)ng]++;
  }
  /* 3-4. push */
  push(s, &s->e, 0);
  if (ion_step) push(s, &s->i, 1);
  /* 5. walls */
  walls(s, &s->e, 0);
  if (ion_step) walls(s, &s->i, 1);
  /* 6. collisions, for the particles present when the loops start (reading:
   * particles born in this step act from the next step on). */
  const int64_t ne_loop = s->e.n, ni_loop = s->i.n;
  const int null_coll = (s->c.flags & ORC_NULL_COLLISION) != 0;
  for (int64_t k = 0; k < ne_loop; ++k) {
    if (null_coll)
      electron_mcc_null(s, k);
    else
      electron_mcc(s, k);
  }
  if (ion_step)
    for (int64_t k = 0; k < ni_loop; ++k) {
      if (null_coll)
        ion_mcc_null(s, k);
      else
        ion_mcc(s, k);
    }
  /* secondary electrons of this step's ion impacts join from the next step */
  for (int64_t k = 0; k < s->see_new.n; ++k)
    parts_append(&s->e, s->see_new.x[k], s->see_new.vx[k], s->see_new.vy[k], s->see_new.vz[k],
                 s->see_new.uid[k]);
  s->see_new.n = 0;
  /* fold this step's fixed-point diagnostic sums into the time sums and
   * the xt arrays; the power density is j E at the nodes with the field of
   * this step (section 3.5) */
  if (xt)
    for (int p = 0; p < ng; ++p) {
      const double je = (double)s->acc_je[p];
      s->x_je[row + p] += je;
      s->x_pe[row + p] += je * s->efield[p];
      s->x_we[row + p] += (double)s->acc_w[p];
      s->x_ee[row + p] += (double)s->acc_e[p];
      s->x_iz[row + p] += (double)s->acc_iz[p];
      if (ion_step) {
        const double ji = (double)s->acc_ji[p];
        s->x_ji[row + p] += ji;
        s->x_pi[row + p] += ji * s->efield[p];
        s->x_wi[row + p] += (double)s->acc_wi[p];
        s->x_ei[row + p] += (double)s->acc_ei[p];
      }
    }
  if (fl & ORC_DIAG_CURRENT) {
    for (int p = 0; p < ng; ++p) s->sum_je[p] += (double)s->acc_je[p];
    if (ion_step)
      for (int p = 0; p < ng; ++p) s->sum_ji[p] += (double)s->acc_ji[p];
  }
  if (fl & ORC_DIAG_MEANE)
    for (int p = 0; p < ng; ++p) {
      s->sum_w[p] += (double)s->acc_w[p];
      s->sum_e[p] += (double)s->acc_e[p];
    }
  int64_t *accs[] = {s->acc_je, s->acc_w, s->acc_e, s->acc_iz};
  for (size_t a = 0; a < sizeof accs / sizeof accs[0]; ++a)
    memset(accs[a], 0, (size_t)ng * sizeof(int64_t));
  if (ion_step) {
    int64_t *acci[] = {s->acc_ji, s->acc_wi, s->acc_ei};
    for (size_t a = 0; a < sizeof acci / sizeof acci[0]; ++a)
      memset(acci[a], 0, (size_t)ng * sizeof(int64_t));
  }
  s->diag_steps++;
  if (ion_step) s->diag_ion_steps++;
  s->step++;
}

int orc_step(orc_sim *s, int64_t n) {
  for (int64_t k = 0; k < n; ++k) one_step(s);
  return 0;
}

int64_t orc_step_index(const orc_sim *s) { return s->step; }

int64_t orc_count(const orc_sim *s, int species) { return species == 0 ? s->e.n : s->i.n; }

void orc_counts(const orc_sim *s, int64_t out[ORC_C_N]) {
  for (int k = 0; k < ORC_C_N; ++k) out[k] = s->counts[k];
}

void orc_deposit_state(const orc_sim *s, int64_t *cnt_e, int64_t *cnt_i) {
  memset(cnt_e, 0, (size_t)s->ng * sizeof(int64_t));
  orc_deposit(s->e.x, s->e.n, s->ng, s->inv_dx, cnt_e);
  if (s->step % s->c.ion_subcycle == 0) {
    memset(cnt_i, 0, (size_t)s->ng * sizeof(int64_t));
    orc_deposit(s->i.x, s->i.n, s->ng, s->inv_dx, cnt_i);
  } else {
    memcpy(cnt_i, s->cnt_i_cur, (size_t)s->ng * sizeof(int64_t));
  }
}

void orc_fields(const orc_sim *s, double *rho, double *phi, double *efield) {
  for (int p = 0; p < s->ng; ++p) {
    if (rho) rho[p] = s->rho[p];
    if (phi) phi[p] = s->phi[p];
    if (efield) efield[p] = s->efield[p];
  }
}

void orc_read_density(const orc_sim *s, double *ne, double *ni) {
  const double n = s->diag_steps > 0 ? (double)s->diag_steps : 1.0;
  for (int p = 0; p < s->ng; ++p) {
    ne[p] = s->sum_ne[p] / n;
    ni[p] = s->sum_ni[p] / n;
  }
}

/* EEPF normalised so that sum_i f_i sqrt(eps_i) de = 1, eps_i = (i+1/2) de. */
void orc_read_eepf(const orc_sim *s, double *f, int64_t *counts) {
  const int nb = s->c.n_eepf;
  const double de = s->c.de_eepf_ev;
  double tot = 0.0;
  for (int k = 0; k < nb; ++k) tot += (double)s->eepf[k];
  for (int k = 0; k < nb; ++k) {
    if (counts) counts[k] = s->eepf[k];
    if (f) f[k] = tot > 0.0 ? (double)s->eepf[k] / (tot * de * sqrt(((double)k + 0.5) * de)) : 0.0;
  }
}

/* Current densities j = q n vbar [A/m^2], time averaged (ions over ion steps). */
void orc_read_currents(const orc_sim *s, double *je, double *ji) {
  const double ns = s->diag_steps > 0 ? (double)s->diag_steps : 1.0;
  const double ni = s->diag_ion_steps > 0 ? (double)s->diag_ion_steps : 1.0;
  for (int p = 0; p < s->ng; ++p) {
    const double edge = (p == 0 || p == s->ng - 1) ? 2.0 : 1.0;
    je[p] = edge * (-E_CHARGE * s->factor_w) * (s->sum_je[p] / DIAG_JS) / ns;
    ji[p] = edge * (E_CHARGE * s->factor_w) * (s->sum_ji[p] / DIAG_JS) / ni;
  }
}

void orc_read_mean_energy(const orc_sim *s, double *mee) {
  for (int p = 0; p < s->ng; ++p)
    mee[p] = s->sum_w[p] > 0.0 ? (s->sum_e[p] / DIAG_ES) / (s->sum_w[p] / DIAG_WS) : 0.0;
}

void orc_reset_diag(orc_sim *s) {
  const size_t ng = (size_t)s->ng;
  s->diag_steps = 0;
  s->diag_ion_steps = 0;
  memset(s->sum_ne, 0, ng * sizeof(double));
  memset(s->sum_ni, 0, ng * sizeof(double));
  memset(s->sum_je, 0, ng * sizeof(double));
  memset(s->sum_ji, 0, ng * sizeof(double));
  memset(s->sum_w, 0, ng * sizeof(double));
  memset(s->sum_e, 0, ng * sizeof(double));
  memset(s->eepf, 0, (size_t)(s->c.n_eepf > 0 ? s->c.n_eepf : 1) * sizeof(int64_t));
  const size_t nx = (size_t)s->n_xt * ng;
  double *xt[] = {s->x_pot, s->x_ef, s->x_ne, s->x_ni, s->x_je, s->x_ji, s->x_pe,
                  s->x_pi, s->x_we, s->x_ee, s->x_wi, s->x_ei, s->x_iz};
  for (size_t k = 0; k < sizeof xt / sizeof xt[0]; ++k) memset(xt[k], 0, nx * sizeof(double));
  memset(s->x_steps, 0, (size_t)s->n_xt * sizeof(int64_t));
  memset(s->x_ion_steps, 0, (size_t)s->n_xt * sizeof(int64_t));
  memset(s->ifed, 0,
         2 * (size_t)((s->c.flags & ORC_DIAG_IFED) ? s->c.n_ifed + 1 : 1) * sizeof(int64_t));
}

int32_t orc_n_xt(const orc_sim *s) { return (s->c.flags & ORC_DIAG_XT) ? s->n_xt : 0; }

void orc_xt_steps(const orc_sim *s, int64_t *steps, int64_t *ion_steps) {
  for (int t = 0; t < s->n_xt; ++t) {
    if (steps) steps[t] = s->x_steps[t];
    if (ion_steps) ion_steps[t] = s->x_ion_steps[t];
  }
}

/* Cell means of the xt sums in SI units (eV for the mean energies):
 * current density j = q n vbar and power density j E from the time-centred
 * velocities, ionization rate n_e-weighted n sigma_ion |v| [m^-3 s^-1].
 * Edge nodes carry half a cell, so their particle sums count double (as in
 * the densities). */
void orc_read_xt(const orc_sim *s, int q, double *out) {
  const int ng = s->ng;
  const double fw = s->factor_w;
  for (int t = 0; t < s->n_xt; ++t) {
    const double ns = (double)s->x_steps[t], ni = (double)s->x_ion_steps[t];
    for (int p = 0; p < ng; ++p) {
      const size_t k = (size_t)t * ng + p;
      const double edge = (p == 0 || p == ng - 1) ? 2.0 : 1.0;
      double v = 0.0;
      switch (q) {
        case ORC_XT_POT: v = ns > 0 ? s->x_pot[k] / ns : 0.0; break;
        case ORC_XT_EFIELD: v = ns > 0 ? s->x_ef[k] / ns : 0.0; break;
        case ORC_XT_NE: v = ns > 0 ? s->x_ne[k] / ns : 0.0; break;
        case ORC_XT_NI: v = ns > 0 ? s->x_ni[k] / ns : 0.0; break;
        case ORC_XT_JE:
          v = ns > 0 ? edge * (-E_CHARGE * fw) * (s->x_je[k] / DIAG_JS) / ns : 0.0;
          break;
        case ORC_XT_JI:
          v = ni > 0 ? edge * (E_CHARGE * fw) * (s->x_ji[k] / DIAG_JS) / ni : 0.0;
          break;
        case ORC_XT_POWERE:
          v = ns > 0 ? edge * (-E_CHARGE * fw) * (s->x_pe[k] / DIAG_JS) / ns : 0.0;
          break;
        case ORC_XT_POWERI:
          v = ni > 0 ? edge * (E_CHARGE * fw) * (s->x_pi[k] / DIAG_JS) / ni : 0.0;
          break;
        case ORC_XT_MEANEE:
          v = s->x_we[k] > 0 ? (s->x_ee[k] / DIAG_ES) / (s->x_we[k] / DIAG_WS) : 0.0;
          break;
        case ORC_XT_MEANEI:
          v = s->x_wi[k] > 0 ? (s->x_ei[k] / DIAG_ES) / (s->x_wi[k] / DIAG_WS) : 0.0;
          break;
        case ORC_XT_IONIZ:
          v = ns > 0 ? edge * fw * (s->x_iz[k] / DIAG_IZS) / s->dt_e / ns : 0.0;
          break;
        default: break;
      }
      out[k] = v;
    }
  }
}

void orc_read_ifed(const orc_sim *s, double *f_pow, double *f_gnd, int64_t *counts) {
  const int nb = s->c.n_ifed;
  if (!(s->c.flags & ORC_DIAG_IFED) || nb < 1) return;
  double *f[2] = {f_pow, f_gnd};
  for (int side = 0; side < 2; ++side) {
    const int64_t *h = s->ifed + (size_t)side * (nb + 1);
    double tot = 0.0;
    for (int k = 0; k < nb; ++k) tot += (double)h[k];
    for (int k = 0; k <= nb; ++k)
      if (counts) counts[(size_t)side * (nb + 1) + k] = h[k];
    if (f[side])
      for (int k = 0; k < nb; ++k)
        f[side][k] = tot > 0.0 ? (double)h[k] / (tot * s->c.de_ifed_ev) : 0.0;
  }
}

void orc_plasma_params(double n_e, double te_ev, double out[2]) {
  out[0] = sqrt(EPSILON0 * te_ev * J_PER_EV / (n_e * E_CHARGE * E_CHARGE));
  out[1] = sqrt(n_e * E_CHARGE * E_CHARGE / (EPSILON0 * M_ELECTRON));
}

/* Run report (section 3.5): the accuracy and stability criteria 1-4 of
 * section 2.2 evaluated on the measured state, the power absorbed by each
 * species and the ion fluxes and mean impact energies at the electrodes.
 * Readings: lambda_D and omega_pe take the peak of the time-averaged
 * electron density and T_e = (2/3) of the mean electron energy over the
 * gap; the largest collision probabilities are the null-collision bounds
 * P* (the maximum of n sigma_tot g over the tables); the CFL energy is the
 * electron energy that moves one cell per step; the power is the space
 * (trapezoid) and time mean of the xt power density.  Quantities whose
 * diagnostics are off read 0. */
void orc_info(const orc_sim *s, double out[ORC_INFO_N]) {
  const int ng = s->ng;
  for (int k = 0; k < ORC_INFO_N; ++k) out[k] = 0.0;
  const double nst = s->diag_steps > 0 ? (double)s->diag_steps : 1.0;
  double ne_max = 0.0, sw = 0.0, se = 0.0;
  for (int p = 0; p < ng; ++p) {
    const double ne = s->sum_ne[p] / nst;
    if (ne > ne_max) ne_max = ne;
    sw += s->sum_w[p];
    se += s->sum_e[p];
  }
  const double mean_e = sw > 0.0 ? (se / DIAG_ES) / (sw / DIAG_WS) : 0.0;
  out[ORC_INFO_MEAN_E] = mean_e;
  out[ORC_INFO_NE_MAX] = ne_max;
  int fail = 0;
  if (ne_max > 0.0 && mean_e > 0.0) {
    double pp[2];
    orc_plasma_params(ne_max, 2.0 / 3.0 * mean_e, pp);
    out[ORC_INFO_DEBYE] = pp[0];
    out[ORC_INFO_DX_DEBYE] = s->dx / pp[0];
    out[ORC_INFO_WPE_DT] = pp[1] * s->dt_e;
    if (!(out[ORC_INFO_DX_DEBYE] < 1.0)) fail |= 1;
    if (!(out[ORC_INFO_WPE_DT] < 2.0)) fail |= 2;
  }
  out[ORC_INFO_PMAX_E] = s->p_null_e;
  out[ORC_INFO_PMAX_I] = s->p_null_i;
  if (!(s->p_null_e < 0.05) || !(s->p_null_i < 0.05)) fail |= 4;
  const double vc = s->dx / s->dt_e;
  out[ORC_INFO_CFL_EV] = 0.5 * M_ELECTRON * vc * vc / J_PER_EV;
  if (s->c.flags & ORC_DIAG_XT) {
    /* trapezoid weight 1/2 at the edges cancels their doubling */
    double pe = 0.0, pi = 0.0, ns = 0.0, ni = 0.0;
    for (int t = 0; t < s->n_xt; ++t) {
      ns += (double)s->x_steps[t];
      ni += (double)s->x_ion_steps[t];
      for (int p = 0; p < ng; ++p) {
        pe += s->x_pe[(size_t)t * ng + p];
        pi += s->x_pi[(size_t)t * ng + p];
      }
    }
    const double fw = s->factor_w;
    if (ns > 0) out[ORC_INFO_POWER_E] = (-E_CHARGE * fw) * (pe / DIAG_JS) / ((double)(ng - 1) * ns);
    if (ni > 0) out[ORC_INFO_POWER_I] = (E_CHARGE * fw) * (pi / DIAG_JS) / ((double)(ng - 1) * ni);
  }
  if (s->c.flags & ORC_DIAG_IFED) {
    const int nb = s->c.n_ifed;
    const double tspan = (double)s->diag_steps * s->dt_e;
    for (int side = 0; side < 2; ++side) {
      const int64_t *h = s->ifed + (size_t)side * (nb + 1);
      double all = 0.0, in = 0.0, en = 0.0;
      for (int k = 0; k <= nb; ++k) all += (double)h[k];
      for (int k = 0; k < nb; ++k) {
        in += (double)h[k];
        en += (double)h[k] * ((double)k + 0.5) * s->c.de_ifed_ev;
      }
      if (tspan > 0) out[side ? ORC_INFO_FLUX_I_GND : ORC_INFO_FLUX_I_POW] =
          all * s->c.weight / (s->c.area_m2 * tspan);
      if (in > 0) out[side ? ORC_INFO_EI_GND : ORC_INFO_EI_POW] = en / in;
    }
  }
  out[ORC_INFO_FAIL] = (double)fail;
}

void orc_constants(const orc_sim *s, double out[8]) {
  out[0] = s->dx;
  out[1] = s->dt_i;
  out[2] = s->factor_w;
  out[3] = s->factor_e;
  out[4] = s->factor_i;
  out[5] = s->gas_n;
  out[6] = s->sigma_a;
  out[7] = orc_voltage(s, 0);
}

void orc_nsig_tot(const orc_sim *s, double *nsig_e, double *nsig_i) {
  for (int k = 0; k < s->nbins; ++k) {
    if (nsig_e) nsig_e[k] = s->nsig_e[k];
    if (nsig_i) nsig_i[k] = s->nsig_i[k];
  }
}

void orc_null_params(const orc_sim *s, double out[4]) {
  out[0] = s->nu_star_e;
  out[1] = s->nu_star_i;
  out[2] = s->p_null_e;
  out[3] = s->p_null_i;
}
