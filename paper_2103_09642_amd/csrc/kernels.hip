// HIP kernels of the PIC/MCC time step for gfx950.
//
// One step s of a case (section 2.1; Algorithms 2-6):
//   k_field      one workgroup: fixed-point densities -> rho -> Thomas solve of
//                the discrete Poisson equation -> grid field E (LDS resident).
//   k_particles  every particle of a species: gather E, leapfrog push, wall
//                absorption, Monte Carlo collision with births, and the
//                deposit of the new position for step s+1 -- fused, so each
//                particle's state is streamed from HBM once per step.
// Ions run k_particles only on steps with s % N_SUB == 0 (ion subcycling).
//
// Deposits are int64 fixed point (2^32 units per particle), privatised in
// LDS per workgroup and flushed with one global atomic per touched node;
// integer addition makes the result independent of the order of particles,
// workgroups and atomics.  Densities use three rotating buffers so that a
// buffer is read at step s, cleared during step s+1 and refilled during step
// s+2 without any extra synchronisation.
//
// Every FP64 expression of the push and the collision kinematics is written
// in the same operation order as its definition, and the library is built
// with -ffp-contract=off, so no multiply-add is fused.
#include "impl.hpp"

namespace edp {

// ---------------------------------------------------------------------------
// Random numbers: Philox4x32-10 (Salmon et al., SC'11), counter
// (uid_lo, uid_hi, step, species<<24 | purpose<<8 | call), key (seed_lo,
// seed_hi); each pair of output words gives a uniform in [0,1) with 53 bits.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint4 philox(uint4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r > 0) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    const uint32_t lo0 = 0xD2511F53u * c.x, hi0 = __umulhi(0xD2511F53u, c.x);
    const uint32_t lo1 = 0xCD9E8D57u * c.z, hi1 = __umulhi(0xCD9E8D57u, c.z);
    c = make_uint4(hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0);
  }
  return c;
}

__device__ __forceinline__ uint32_t tag(uint32_t species, uint32_t purpose, uint32_t call) {
  return (species << 24) | (purpose << 8) | call;
}

__device__ __forceinline__ void uniform2(uint64_t seed, uint64_t uid, uint32_t step, uint32_t t,
                                         double& u0, double& u1) {
  const uint4 w = philox(make_uint4((uint32_t)uid, (uint32_t)(uid >> 32), step, t),
                         (uint32_t)seed, (uint32_t)(seed >> 32));
  const uint64_t a = ((uint64_t)w.x << 32) | w.y;
  const uint64_t b = ((uint64_t)w.z << 32) | w.w;
  u0 = (double)(a >> 11) * (1.0 / 9007199254740992.0);
  u1 = (double)(b >> 11) * (1.0 / 9007199254740992.0);
}

// Box-Muller: two standard normals from two uniforms (log argument in (0,1]).
__device__ __forceinline__ void box_muller(double u0, double u1, double& z0, double& z1) {
  const double r = sqrt(-2.0 * log(1.0 - u0));
  z0 = r * cos(kTwoPi * u1);
  z1 = r * sin(kTwoPi * u1);
}

// Three normals from calls first_call and first_call+1.
__device__ __forceinline__ void normals3(uint64_t seed, uint64_t uid, uint32_t step,
                                         uint32_t species, uint32_t purpose, uint32_t first_call,
                                         double& z0, double& z1, double& z2) {
  double u0, u1, z3;
  uniform2(seed, uid, step, tag(species, purpose, first_call), u0, u1);
  box_muller(u0, u1, z0, z1);
  uniform2(seed, uid, step, tag(species, purpose, first_call + 1), u0, u1);
  box_muller(u0, u1, z2, z3);
}

// splitmix64 finaliser (Steele, Lea & Flood, OOPSLA 2014).
__device__ __forceinline__ uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// Identity of a particle born in an ionization: hash of (parent, step, kind),
// kind 1 = ejected electron, 2 = new ion; independent of the order of births.
__device__ __forceinline__ uint64_t child_uid(uint64_t parent, int64_t step, uint64_t kind) {
  return mix64(mix64(parent) ^ ((uint64_t)step * 0x9E3779B97F4A7C15ull) ^ kind);
}

// Energy bin min(int(E/DE_CS + 0.5), CS_RANGES-1) (Algorithm 6).
__device__ __forceinline__ int energy_bin(double e_ev, double de, int nbins) {
  const double t = e_ev / de + 0.5;
  return t >= (double)(nbins - 1) ? nbins - 1 : (int)t;
}

// Post-collision velocity w + f2 g' R(theta,phi)(cos chi, sin chi cos eta,
// sin chi sin eta) with the Euler angles of g from its components (phi = 0
// when g is along x); the components follow the final velocity equation of
// section 2.1.6 term by term.
__device__ __forceinline__ void scatter(double gx, double gy, double gz, double gmag, double gnew,
                                        double f2, double cos_chi, double sin_chi, double eta,
                                        double wx, double wy, double wz, double& ox, double& oy,
                                        double& oz) {
  double cos_theta, sin_theta, cos_phi, sin_phi;
  if (gmag > 0.0) {
    const double gyz = sqrt(gy * gy + gz * gz);
    cos_theta = gx / gmag;
    sin_theta = gyz / gmag;
    if (gyz > 0.0) {
      cos_phi = gy / gyz;
      sin_phi = gz / gyz;
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
  ox = wx + a * (cos_theta * cos_chi - sin_theta * sin_chi * cos_eta);
  oy = wy + a * (sin_theta * cos_phi * cos_chi + cos_theta * cos_phi * sin_chi * cos_eta -
                 sin_phi * sin_chi * sin_eta);
  oz = wz + a * (sin_theta * sin_phi * cos_chi + cos_theta * sin_phi * sin_chi * cos_eta +
                 cos_phi * sin_chi * sin_eta);
}

// Fixed-point split of one particle between nodes p and p+1 (charge
// assignment equations): p = int(x/dx) clamped to N_g-2, f*2^32 truncated,
// capped at 2^32.
__device__ __forceinline__ int deposit_split(double x, double inv_dx, int ng, long long& r) {
  const double c0 = x * inv_dx;
  int p = (int)c0;
  p = p > ng - 2 ? ng - 2 : (p < 0 ? 0 : p);
  const double f = c0 - (double)p;
  long long q = (long long)(f * kTwo32);
  r = q > 4294967296LL ? 4294967296LL : q;
  return p;
}

// Slots in use, never beyond the capacity (alloc may pass it on overflow).
__device__ __forceinline__ int64_t slots(const CaseDev* C, int sp) {
  const int64_t a = C->alloc[sp];
  return a < C->sp[sp].cap ? a : C->sp[sp].cap;
}

__device__ __forceinline__ void lds_add(unsigned long long* a, long long v) {
  atomicAdd(a, (unsigned long long)v);
}
__device__ __forceinline__ void gl_add(int64_t* a, long long v) {
  atomicAdd((unsigned long long*)a, (unsigned long long)v);
}

// LDS counters of a particle workgroup.
enum { kLAbsPow = 0, kLAbsGnd, kLColl, kLIoniz, kLAnom, kLDrop, kLLiveE, kLLiveI, kLN };

// ---------------------------------------------------------------------------
// Step 2: density -> rho -> potential -> field, one workgroup per case.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(1024) k_field(CaseDev* __restrict__ C) {
  extern __shared__ double fsm[];
  const int ng = C->ng;
  double* sRho = fsm;
  double* sPhi = fsm + ng;
  double* sR = fsm + 2 * ng;
  const int64_t s = C->step;
  const int nsub = C->nsub;
  const int64_t k = s / nsub;
  const bool ion_step = (s % nsub) == 0;
  const uint32_t fl = C->flags;
  const int64_t* cntE = C->cnt_e + (s % 3) * ng;
  const int64_t* cntI = C->cnt_i + (k % 3) * ng;
  int64_t* zeroE = C->cnt_e + ((s + 2) % 3) * ng;
  int64_t* zeroI = C->cnt_i + ((k + 2) % 3) * ng;
  const int64_t fold = ((s + 2) % 3) * ng;  // per-step sums of step s-1
  const double scale = C->dens_scale;
  for (int p = threadIdx.x; p < ng; p += blockDim.x) {
    double ne = (double)cntE[p] * scale;
    double ni = (double)cntI[p] * scale;
    if (p == 0 || p == ng - 1) {
      ne *= 2.0;
      ni *= 2.0;
    }
    const double rho = kECharge * (ni - ne);
    sRho[p] = rho;
    sR[p] = C->rden[p];
    sPhi[p] = rho * C->kpois;  // right-hand side d_p (boundary term below)
    if (fl & kDiagDensity) {
      C->sum_ne[p] += ne;
      C->sum_ni[p] += ni;
    }
    zeroE[p] = 0;
    if (ion_step) zeroI[p] = 0;
    if (fl & kDiagCurrent) {
      C->sum_je[p] += (double)C->acc_je[fold + p];
      C->acc_je[fold + p] = 0;
      C->sum_ji[p] += (double)C->acc_ji[fold + p];
      C->acc_ji[fold + p] = 0;
    }
    if (fl & kDiagMeanE) {
      C->sum_w[p] += (double)C->acc_w[fold + p];
      C->sum_e[p] += (double)C->acc_e[fold + p];
      C->acc_w[fold + p] = 0;
      C->acc_e[fold + p] = 0;
    }
  }
  __syncthreads();
  const double V = C->volt[s % kVoltChunk];
  if (threadIdx.x == 0) {
    // Thomas algorithm (constant tridiagonal matrix): forward sweep
    // y_p = (d_p + y_{p-1}) r_p, back substitution phi_p = y_p + r_p phi_{p+1}.
    const int m = ng - 2;
    double prev = 0.0;
    for (int p = 1; p <= m; ++p) {
      double d = sPhi[p];
      if (p == 1) d = d + V;
      prev = (d + prev) * sR[p];
      sPhi[p] = prev;
    }
    for (int p = m - 1; p >= 1; --p) sPhi[p] = sPhi[p] + sR[p] * sPhi[p + 1];
    sPhi[0] = V;
    sPhi[ng - 1] = 0.0;
    // per-step bookkeeping: snapshot the particle slots of this step; after a
    // capacity overflow alloc may have run past the capacity, never process
    // beyond it
    for (int sp = 0; sp < 2; ++sp) {
      int64_t a = C->alloc[sp];
      if (a > C->sp[sp].cap) {
        a = C->sp[sp].cap;
        C->alloc[sp] = a;
      }
      C->n[sp] = a;
    }
    C->ctr[kPstepE] += C->ctr[kLiveE];
    if (ion_step) C->ctr[kPstepI] += C->ctr[kLiveI];
    C->diag_steps += 1;
    if (ion_step) C->diag_ion_steps += 1;
    C->step = s + 1;  // particle kernels of this step read step-1
  }
  __syncthreads();
  const double dx = C->dx;
  for (int p = threadIdx.x; p < ng; p += blockDim.x) {
    double e;
    if (p == 0)
      e = (sPhi[0] - sPhi[1]) / dx - sRho[0] * dx / (2.0 * kEps0);
    else if (p == ng - 1)
      e = (sPhi[ng - 2] - sPhi[ng - 1]) / dx + sRho[ng - 1] * dx / (2.0 * kEps0);
    else
      e = (sPhi[p - 1] - sPhi[p + 1]) / (2.0 * dx);
    C->efield[p] = e;
    C->phi[p] = sPhi[p];
    C->rho[p] = sRho[p];
  }
}

// ---------------------------------------------------------------------------
// Steps 3-6 for one species, fused, plus the deposit for step s+1.
// Dynamic LDS: E[ng] double, H[ng] deposit; with particle diagnostics also
// J[ng], W[ng], En[ng] (int64) and EEPF[n_eepf] (uint32).
// ---------------------------------------------------------------------------
template <int SP>
__global__ void __launch_bounds__(256) k_particles(CaseDev* __restrict__ C) {
  extern __shared__ double psm[];
  __shared__ unsigned long long sCtr[kLN];
  const int ng = C->ng;
  const int64_t s = C->step - 1;  // k_field of this step already advanced it
  const int nsub = C->nsub;
  const int64_t kion = s / nsub;
  const uint32_t fl = C->flags;
  const bool pdiag = (fl & kDiagParticle) != 0;
  double* sE = psm;
  unsigned long long* sH = (unsigned long long*)(psm + ng);
  unsigned long long* sJ = sH + ng;
  unsigned long long* sW = sJ + ng;
  unsigned long long* sEn = sW + ng;
  unsigned int* sF = (unsigned int*)(sEn + ng);
  const int n_eepf = C->n_eepf;
  for (int p = threadIdx.x; p < ng; p += blockDim.x) {
    sE[p] = C->efield[p];
    sH[p] = 0;
    if (pdiag) {
      sJ[p] = 0;
      sW[p] = 0;
      sEn[p] = 0;
    }
  }
  if (SP == 0 && (fl & kDiagEepf))
    for (int b = threadIdx.x; b < n_eepf; b += blockDim.x) sF[b] = 0;
  if (threadIdx.x < kLN) sCtr[threadIdx.x] = 0;
  __syncthreads();

  const int cur = C->cur[SP];
  double* __restrict__ X = C->sp[SP].x[cur];
  double* __restrict__ VX = C->sp[SP].vx[cur];
  double* __restrict__ VY = C->sp[SP].vy[cur];
  double* __restrict__ VZ = C->sp[SP].vz[cur];
  const uint64_t* __restrict__ UID = C->sp[SP].uid[cur];
  const int64_t n = C->n[SP];
  const double inv_dx = C->inv_dx, L = C->L;
  const double dt = SP == 0 ? C->dt_e : C->dt_i;
  const double factor = SP == 0 ? C->factor_e : C->factor_i;
  const double* __restrict__ nsig = SP == 0 ? C->nsig_e : C->nsig_i;
  const double de_cs = C->de_cs;
  const int nbins = C->nbins;
  const uint64_t seed = C->seed;
  const uint32_t st = (uint32_t)s;
  const double x_lo = C->x_lo, x_hi = C->x_hi;

  unsigned long long my_abs_pow = 0, my_abs_gnd = 0, my_coll = 0;
  const int64_t G = gridDim.x;
  const int64_t per = (n + G - 1) / G;
  const int64_t lo = (int64_t)blockIdx.x * per;
  const int64_t hi = lo + per < n ? lo + per : n;
  for (int64_t i = lo + threadIdx.x; i < hi; i += blockDim.x) {
    const double x = X[i];
    if (!(x == x)) continue;  // absorbed earlier: tombstone
    const double vx = VX[i];
    double vy = VY[i], vz = VZ[i];
    const uint64_t uid = UID[i];
    // Steps 3-4: field at the particle and leapfrog.
    const double c0 = x * inv_dx;
    int p = (int)c0;
    p = p > ng - 2 ? ng - 2 : (p < 0 ? 0 : p);
    const double c1 = (double)(p + 1) - c0;
    const double c2 = c0 - (double)p;
    const double ex = c1 * sE[p] + c2 * sE[p + 1];
    double vxn;
    if (SP == 0)
      vxn = vx - ex * factor;
    else
      vxn = vx + ex * factor;
    const double xn = x + vxn * dt;
    if (pdiag) {
      // measurement at integer time: old position, mean of the half-step velocities
      const double vbar = 0.5 * (vx + vxn);
      if (fl & kDiagCurrent) {
        lds_add(&sJ[p], (long long)(c1 * vbar * kDiagJS));
        lds_add(&sJ[p + 1], (long long)(c2 * vbar * kDiagJS));
      }
      if (SP == 0 && (fl & (kDiagMeanE | kDiagEepf))) {
        const double en = 0.5 * kEMass * (vbar * vbar + vy * vy + vz * vz) / kEvToJ;
        if (fl & kDiagMeanE) {
          lds_add(&sW[p], (long long)(c1 * kDiagWS));
          lds_add(&sW[p + 1], (long long)(c2 * kDiagWS));
          lds_add(&sEn[p], (long long)(c1 * en * kDiagES));
          lds_add(&sEn[p + 1], (long long)(c2 * en * kDiagES));
        }
        if ((fl & kDiagEepf) && x >= x_lo && x <= x_hi) {
          const double t = en / C->de_eepf;
          if (t < (double)n_eepf) atomicAdd(&sF[(int)t], 1u);
        }
      }
    }
    // Step 5: absorbing electrodes.
    if (xn < 0.0 || xn > L) {
      if (xn < 0.0)
        ++my_abs_pow;
      else
        ++my_abs_gnd;
      X[i] = __longlong_as_double(0x7FF8000000000000LL);
      continue;
    }
    // Step 6: collision test and event.
    if (SP == 0) {
      const double v2 = vxn * vxn + vy * vy + vz * vz;
      const double v = sqrt(v2);
      const double energy = 0.5 * kEMass * v2 / kEvToJ;
      const int idx = energy_bin(energy, de_cs, nbins);
      const double nu = nsig[idx] * v;
      const double p_coll = 1.0 - exp(-nu * dt);
      double r_coll, r_proc;
      uniform2(seed, uid, st, tag(0, 0, 0), r_coll, r_proc);
      if (r_coll < p_coll) {
        double r_chi, r_eta, r_share, r_unused;
        uniform2(seed, uid, st, tag(0, 0, 1), r_chi, r_eta);
        uniform2(seed, uid, st, tag(0, 0, 2), r_share, r_unused);
        const double f1 = kEMass / (kEMass + kArMass);
        const double f2 = kArMass / (kEMass + kArMass);
        const double wx = f1 * vxn, wy = f1 * vy, wz = f1 * vz;
        const double s_el = C->sig_el[idx], s_exc = C->sig_exc[idx], s_ion = C->sig_ion[idx];
        const double s_tot = s_el + s_exc + s_ion;
        int proc;
        if (!(s_tot > 0.0) || r_proc < s_el / s_tot)
          proc = 0;
        else if (r_proc < (s_el + s_exc) / s_tot)
          proc = 1;
        else
          proc = 2;
        const double eta = kTwoPi * r_eta;
        double ox, oy, oz;
        if (proc < 2) {
          double gnew = v;
          if (proc == 1) {
            double ec = 0.5 * kMuEAr * v2 - C->thr_exc * kEvToJ;
            if (ec < 0.0) {
              ec = 0.0;
              atomicAdd(&sCtr[kLAnom], 1ull);
            }
            gnew = sqrt(2.0 * ec / kMuEAr);
          }
          const double cos_chi = 1.0 - 2.0 * r_chi;
          const double sin_chi = sqrt(1.0 - cos_chi * cos_chi);
          scatter(vxn, vy, vz, v, gnew, f2, cos_chi, sin_chi, eta, wx, wy, wz, ox, oy, oz);
        } else {
          double e_ev = 0.5 * kMuEAr * v2 / kEvToJ - C->thr_ion;
          if (e_ev < 0.0) {
            e_ev = 0.0;
            atomicAdd(&sCtr[kLAnom], 1ull);
          }
          const double w_ion = C->w_ion;
          const double e_ej = w_ion * tan(r_share * atan(e_ev / (2.0 * w_ion)));
          const double e_sc = e_ev - e_ej;
          const double g_sc = sqrt(2.0 * e_sc * kEvToJ / kMuEAr);
          const double g_ej = sqrt(2.0 * e_ej * kEvToJ / kMuEAr);
          double cs_sc, sn_sc, cs_ej, sn_ej;
          if (fl & kIonizLiteral) {
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
          scatter(vxn, vy, vz, v, g_sc, f2, cs_sc, sn_sc, eta, wx, wy, wz, ox, oy, oz);
          double ex_, ey_, ez_;
          scatter(vxn, vy, vz, v, g_ej, f2, cs_ej, sn_ej, eta + kPi, wx, wy, wz, ex_, ey_, ez_);
          // births: the ejected electron and the new ion at the parent's position
          atomicAdd(&sCtr[kLIoniz], 1ull);
          const uint64_t ue = child_uid(uid, s, 1), ui = child_uid(uid, s, 2);
          const unsigned long long se = atomicAdd((unsigned long long*)&C->alloc[0], 1ull);
          if ((int64_t)se < C->sp[0].cap) {
            X[se] = xn;
            VX[se] = ex_;
            VY[se] = ey_;
            VZ[se] = ez_;
            C->sp[0].uid[cur][se] = ue;
            long long r;
            const int q = deposit_split(xn, inv_dx, ng, r);
            lds_add(&sH[q], 4294967296LL - r);
            lds_add(&sH[q + 1], r);
            atomicAdd(&sCtr[kLLiveE], 1ull);
          } else {
            atomicAdd(&sCtr[kLDrop], 1ull);
          }
          const int ci = C->cur[1];
          const unsigned long long si = atomicAdd((unsigned long long*)&C->alloc[1], 1ull);
          if ((int64_t)si < C->sp[1].cap) {
            double z0, z1, z2;
            normals3(seed, ui, st, 1u, 2u, 1u, z0, z1, z2);
            const double sa = C->sigma_a;
            C->sp[1].x[ci][si] = xn;
            C->sp[1].vx[ci][si] = sa * z0;
            C->sp[1].vy[ci][si] = sa * z1;
            C->sp[1].vz[ci][si] = sa * z2;
            C->sp[1].uid[ci][si] = ui;
            long long r;
            const int q = deposit_split(xn, inv_dx, ng, r);
            int64_t* ci_next = C->cnt_i + ((kion + 1) % 3) * ng;
            gl_add(&ci_next[q], 4294967296LL - r);
            gl_add(&ci_next[q + 1], r);
            atomicAdd(&sCtr[kLLiveI], 1ull);
          } else {
            atomicAdd(&sCtr[kLDrop], 1ull);
          }
        }
        VY[i] = oy;
        VZ[i] = oz;
        vxn = ox;
        ++my_coll;
      }
    } else {
      double z0, z1, z2;
      normals3(seed, uid, st, 1u, 0u, 0u, z0, z1, z2);
      const double sa = C->sigma_a;
      const double vax = sa * z0, vay = sa * z1, vaz = sa * z2;
      const double gx = vxn - vax, gy = vy - vay, gz = vz - vaz;
      const double g2 = gx * gx + gy * gy + gz * gz;
      const double g = sqrt(g2);
      const double energy = 0.5 * kMuArAr * g2 / kEvToJ;
      const int idx = energy_bin(energy, de_cs, nbins);
      const double nu = nsig[idx] * g;
      const double p_coll = 1.0 - exp(-nu * dt);
      double r_coll, r_proc;
      uniform2(seed, uid, st, tag(1, 0, 2), r_coll, r_proc);
      if (r_coll < p_coll) {
        double r_chi, r_eta;
        uniform2(seed, uid, st, tag(1, 0, 3), r_chi, r_eta);
        const double wx = 0.5 * (vxn + vax), wy = 0.5 * (vy + vay), wz = 0.5 * (vz + vaz);
        const double s_iso = C->sig_iso[idx], s_back = C->sig_back[idx];
        double cos_chi, sin_chi;
        if (!(s_iso + s_back > 0.0) || r_proc < s_iso / (s_iso + s_back)) {
          cos_chi = 1.0 - 2.0 * r_chi;
          sin_chi = sqrt(1.0 - cos_chi * cos_chi);
        } else {
          cos_chi = -1.0;
          sin_chi = 0.0;
        }
        double ox, oy, oz;
        scatter(gx, gy, gz, g, g, 0.5, cos_chi, sin_chi, kTwoPi * r_eta, wx, wy, wz, ox, oy, oz);
        VY[i] = oy;
        VZ[i] = oz;
        vxn = ox;
        ++my_coll;
      }
    }
    X[i] = xn;
    VX[i] = vxn;
    long long r;
    const int q = deposit_split(xn, inv_dx, ng, r);
    lds_add(&sH[q], 4294967296LL - r);
    lds_add(&sH[q + 1], r);
  }
  if (my_abs_pow) atomicAdd(&sCtr[kLAbsPow], my_abs_pow);
  if (my_abs_gnd) atomicAdd(&sCtr[kLAbsGnd], my_abs_gnd);
  if (my_coll) atomicAdd(&sCtr[kLColl], my_coll);
  __syncthreads();
  // flush: deposit for step s+1, diagnostics of step s, counters
  int64_t* dst = SP == 0 ? C->cnt_e + ((s + 1) % 3) * ng : C->cnt_i + ((kion + 1) % 3) * ng;
  for (int q = threadIdx.x; q < ng; q += blockDim.x) {
    const unsigned long long h = sH[q];
    if (h) gl_add(&dst[q], (long long)h);
    if (pdiag) {
      const int64_t off = (s % 3) * ng + q;
      if (sJ[q]) gl_add(&(SP == 0 ? C->acc_je : C->acc_ji)[off], (long long)sJ[q]);
      if (SP == 0 && sW[q]) gl_add(&C->acc_w[off], (long long)sW[q]);
      if (SP == 0 && sEn[q]) gl_add(&C->acc_e[off], (long long)sEn[q]);
    }
  }
  if (SP == 0 && (fl & kDiagEepf))
    for (int b = threadIdx.x; b < n_eepf; b += blockDim.x)
      if (sF[b]) gl_add(&C->eepf[b], (long long)sF[b]);
  if (threadIdx.x == 0) {
    const unsigned long long a_pow = sCtr[kLAbsPow], a_gnd = sCtr[kLAbsGnd];
    if (a_pow) gl_add(&C->ctr[SP == 0 ? kAbsEPow : kAbsIPow], (long long)a_pow);
    if (a_gnd) gl_add(&C->ctr[SP == 0 ? kAbsEGnd : kAbsIGnd], (long long)a_gnd);
    if (sCtr[kLColl]) gl_add(&C->ctr[SP == 0 ? kCollE : kCollI], (long long)sCtr[kLColl]);
    if (sCtr[kLIoniz]) gl_add(&C->ctr[kIoniz], (long long)sCtr[kLIoniz]);
    if (sCtr[kLAnom]) gl_add(&C->ctr[kAnomaly], (long long)sCtr[kLAnom]);
    if (sCtr[kLDrop]) {
      gl_add(&C->ctr[kDropped], (long long)sCtr[kLDrop]);
      atomicExch(&C->error, 1);
    }
    const long long dl = -(long long)(a_pow + a_gnd);
    if (SP == 0) {
      const long long de = dl + (long long)sCtr[kLLiveE];
      if (de) gl_add(&C->ctr[kLiveE], de);
      if (sCtr[kLLiveI]) gl_add(&C->ctr[kLiveI], (long long)sCtr[kLLiveI]);
    } else if (dl) {
      gl_add(&C->ctr[kLiveI], dl);
    }
  }
}

// ---------------------------------------------------------------------------
// Seeding (Algorithm 1, init) and redeposit.
// ---------------------------------------------------------------------------
__global__ void k_seed(CaseDev* __restrict__ C, int sp, int64_t n, double sigma) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int cur = C->cur[sp];
  double u0, u1, z0, z1, z2;
  uniform2(C->seed, (uint64_t)i, 0u, tag((uint32_t)sp, 1u, 0u), u0, u1);
  normals3(C->seed, (uint64_t)i, 0u, (uint32_t)sp, 1u, 1u, z0, z1, z2);
  C->sp[sp].x[cur][i] = C->L * u0;
  C->sp[sp].vx[cur][i] = sigma * z0;
  C->sp[sp].vy[cur][i] = sigma * z1;
  C->sp[sp].vz[cur][i] = sigma * z2;
  C->sp[sp].uid[cur][i] = (uint64_t)i;
}

// Deposit the live particles [0, alloc) of a species into one or two buffers.
__global__ void __launch_bounds__(256) k_deposit(CaseDev* __restrict__ C, int sp, int64_t* dst1,
                                                 int64_t* dst2) {
  extern __shared__ double dsm[];
  unsigned long long* sH = (unsigned long long*)dsm;
  const int ng = C->ng;
  for (int p = threadIdx.x; p < ng; p += blockDim.x) sH[p] = 0;
  __syncthreads();
  const int cur = C->cur[sp];
  const double* __restrict__ X = C->sp[sp].x[cur];
  const int64_t n = slots(C, sp);
  const double inv_dx = C->inv_dx;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const double x = X[i];
    if (!(x == x)) continue;
    long long r;
    const int q = deposit_split(x, inv_dx, ng, r);
    lds_add(&sH[q], 4294967296LL - r);
    lds_add(&sH[q + 1], r);
  }
  __syncthreads();
  for (int q = threadIdx.x; q < ng; q += blockDim.x) {
    const unsigned long long h = sH[q];
    if (!h) continue;
    gl_add(&dst1[q], (long long)h);
    if (dst2) gl_add(&dst2[q], (long long)h);
  }
}

// ---------------------------------------------------------------------------
// Compaction + counting sort by cell: drops tombstones, merges births and
// restores spatial locality (contiguous particle ranges then touch few nodes,
// so the per-workgroup deposit flush stays small).  Order within a cell is
// arbitrary; results do not depend on it.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int cell_of(double x, double inv_dx, int ng) {
  int p = (int)(x * inv_dx);
  return p > ng - 2 ? ng - 2 : (p < 0 ? 0 : p);
}



__global__ void __launch_bounds__(256) k_sort_hist(CaseDev* __restrict__ C, int sp) {
  extern __shared__ double hsm[];
  unsigned int* sC = (unsigned int*)hsm;
  const int ng = C->ng;
  for (int p = threadIdx.x; p < ng; p += blockDim.x) sC[p] = 0;
  __syncthreads();
  const int cur = C->cur[sp];
  const double* __restrict__ X = C->sp[sp].x[cur];
  const int64_t n = slots(C, sp);
  const int64_t G = gridDim.x, per = (n + G - 1) / G;
  const int64_t lo = (int64_t)blockIdx.x * per, hi = lo + per < n ? lo + per : n;
  for (int64_t i = lo + threadIdx.x; i < hi; i += blockDim.x) {
    const double x = X[i];
    if (x == x) atomicAdd(&sC[cell_of(x, C->inv_dx, ng)], 1u);
  }
  __syncthreads();
  for (int p = threadIdx.x; p < ng - 1; p += blockDim.x)
    if (sC[p]) gl_add(&C->sort_cnt[p], (long long)sC[p]);
}

// Exclusive scan of the ng-1 cell counts (one workgroup); total -> sort_cnt[ng].
__global__ void __launch_bounds__(1024) k_sort_scan(CaseDev* __restrict__ C) {
  __shared__ int64_t sPart[1024];
  const int m = C->ng - 1;
  const int t = threadIdx.x, T = blockDim.x;
  const int per = (m + T - 1) / T;
  const int lo = t * per, hi = lo + per < m ? lo + per : m;
  int64_t acc = 0;
  for (int p = lo; p < hi; ++p) acc += C->sort_cnt[p];
  sPart[t] = acc;
  __syncthreads();
  if (t == 0) {
    int64_t run = 0;
    for (int j = 0; j < T; ++j) {
      const int64_t v = sPart[j];
      sPart[j] = run;
      run += v;
    }
    C->sort_cnt[C->ng] = run;
  }
  __syncthreads();
  int64_t run = sPart[t];
  for (int p = lo; p < hi; ++p) {
    const int64_t v = C->sort_cnt[p];
    C->sort_cnt[p] = run;
    run += v;
  }
}

__global__ void __launch_bounds__(256) k_sort_scatter(CaseDev* __restrict__ C, int sp) {
  extern __shared__ double ssm[];
  unsigned int* sC = (unsigned int*)ssm;
  unsigned long long* sB = (unsigned long long*)(ssm + (C->ng + 1) / 2);
  const int ng = C->ng;
  for (int p = threadIdx.x; p < ng; p += blockDim.x) sC[p] = 0;
  __syncthreads();
  const int cur = C->cur[sp], nxt = cur ^ 1;
  const SpeciesDev& S = C->sp[sp];
  const double* __restrict__ X = S.x[cur];
  const int64_t n = slots(C, sp);
  const int64_t G = gridDim.x, per = (n + G - 1) / G;
  const int64_t lo = (int64_t)blockIdx.x * per, hi = lo + per < n ? lo + per : n;
  const double inv_dx = C->inv_dx;
  for (int64_t i = lo + threadIdx.x; i < hi; i += blockDim.x) {
    const double x = X[i];
    if (x == x) atomicAdd(&sC[cell_of(x, inv_dx, ng)], 1u);
  }
  __syncthreads();
  for (int p = threadIdx.x; p < ng - 1; p += blockDim.x) {
    const unsigned int c = sC[p];
    sB[p] = c ? atomicAdd((unsigned long long*)&C->sort_cnt[p], (unsigned long long)c) : 0ull;
    sC[p] = 0;
  }
  __syncthreads();
  for (int64_t i = lo + threadIdx.x; i < hi; i += blockDim.x) {
    const double x = X[i];
    if (!(x == x)) continue;
    const int c = cell_of(x, inv_dx, ng);
    const int64_t d = (int64_t)sB[c] + atomicAdd(&sC[c], 1u);
    S.x[nxt][d] = x;
    S.vx[nxt][d] = S.vx[cur][i];
    S.vy[nxt][d] = S.vy[cur][i];
    S.vz[nxt][d] = S.vz[cur][i];
    S.uid[nxt][d] = S.uid[cur][i];
  }
}

__global__ void k_sort_finish(CaseDev* __restrict__ C, int sp) {
  const int ng = C->ng;
  if (threadIdx.x == 0) {
    C->alloc[sp] = C->sort_cnt[ng];
    C->cur[sp] ^= 1;
  }
  __syncthreads();
  for (int p = threadIdx.x; p <= ng; p += blockDim.x) C->sort_cnt[p] = 0;
}

// Fold the pending per-step diagnostic sums of the last completed step.
__global__ void k_fold_diag(CaseDev* __restrict__ C) {
  const int ng = C->ng;
  const int64_t s = C->step;  // next step to run; the pending sums are those of s-1
  const int64_t off = ((s + 2) % 3) * ng;
  const uint32_t fl = C->flags;
  for (int p = threadIdx.x; p < ng; p += blockDim.x) {
    if (fl & kDiagCurrent) {
      C->sum_je[p] += (double)C->acc_je[off + p];
      C->acc_je[off + p] = 0;
      C->sum_ji[p] += (double)C->acc_ji[off + p];
      C->acc_ji[off + p] = 0;
    }
    if (fl & kDiagMeanE) {
      C->sum_w[p] += (double)C->acc_w[off + p];
      C->sum_e[p] += (double)C->acc_e[off + p];
      C->acc_w[off + p] = 0;
      C->acc_e[off + p] = 0;
    }
  }
}

__global__ void k_zero(int64_t* __restrict__ p, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0;
}

// ---------------------------------------------------------------------------
// Host-side launchers (same translation unit as the kernels).
// ---------------------------------------------------------------------------
size_t particle_lds_bytes(int ng, uint32_t flags, int n_eepf, int sp) {
  size_t b = (size_t)ng * 16;
  if (flags & kDiagParticle) b += (size_t)ng * 24 + (sp == 0 ? (size_t)n_eepf * 4 : 0);
  return b;
}

hipError_t launch_field(CaseDev* d, int ng, hipStream_t st) {
  hipLaunchKernelGGL(k_field, dim3(1), dim3(1024), (size_t)ng * 24, st, d);
  return hipGetLastError();
}

hipError_t launch_particles(CaseDev* d, int sp, int blocks, int ng, uint32_t flags, int n_eepf,
                            hipStream_t st) {
  const size_t lds = particle_lds_bytes(ng, flags, n_eepf, sp);
  if (sp == 0)
    hipLaunchKernelGGL(k_particles<0>, dim3(blocks), dim3(256), lds, st, d);
  else
    hipLaunchKernelGGL(k_particles<1>, dim3(blocks), dim3(256), lds, st, d);
  return hipGetLastError();
}

hipError_t launch_zero(void* p, int64_t bytes, hipStream_t st) {
  const int64_t n = bytes / 8;
  if (n <= 0) return hipSuccess;
  int64_t blocks = (n + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(k_zero, dim3((unsigned)blocks), dim3(256), 0, st, (int64_t*)p, n);
  return hipGetLastError();
}

hipError_t launch_seed(CaseDev* d, int sp, int64_t n, double sigma, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  const int64_t blocks = (n + 255) / 256;
  hipLaunchKernelGGL(k_seed, dim3((unsigned)blocks), dim3(256), 0, st, d, sp, n, sigma);
  return hipGetLastError();
}

hipError_t launch_deposit(CaseDev* d, int sp, int64_t* dst1, int64_t* dst2, int ng, int blocks,
                          hipStream_t st) {
  hipLaunchKernelGGL(k_deposit, dim3(blocks), dim3(256), (size_t)ng * 8, st, d, sp, dst1, dst2);
  return hipGetLastError();
}

hipError_t launch_sort(CaseDev* d, int sp, int ng, int blocks, hipStream_t st) {
  hipLaunchKernelGGL(k_sort_hist, dim3(blocks), dim3(256), (size_t)ng * 4, st, d, sp);
  hipLaunchKernelGGL(k_sort_scan, dim3(1), dim3(1024), 0, st, d);
  const size_t lds = (size_t)((ng + 1) / 2) * 8 + (size_t)ng * 8;
  hipLaunchKernelGGL(k_sort_scatter, dim3(blocks), dim3(256), lds, st, d, sp);
  hipLaunchKernelGGL(k_sort_finish, dim3(1), dim3(1024), 0, st, d, sp);
  return hipGetLastError();
}

hipError_t launch_fold(CaseDev* d, hipStream_t st) {
  hipLaunchKernelGGL(k_fold_diag, dim3(1), dim3(1024), 0, st, d);
  return hipGetLastError();
}

}  // namespace edp
