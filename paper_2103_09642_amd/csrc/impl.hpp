// Internal layout shared by the HIP kernels and the host runtime of the
// library.  One CaseDev block per discharge case lives in the case's device
// arena; kernels reach it through their workgroup's role and read every
// constant, array pointer and dynamic counter from there.  A launch's only
// other argument is the offset of its step in the window, so a window of
// steps can be captured into a hipGraph once and replayed.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace edp {

// Physical constants: CODATA 2018 (the paper does not list its values).
constexpr double kECharge = 1.602176634e-19;  // C
constexpr double kEMass = 9.1093837015e-31;   // kg
constexpr double kBoltzmann = 1.380649e-23;   // J/K
constexpr double kEps0 = 8.8541878128e-12;    // F/m
constexpr double kAmu = 1.66053906660e-27;    // kg
constexpr double kArMass = 39.948 * kAmu;
constexpr double kMuArAr = kArMass / 2.0;                          // Ar+ + Ar
constexpr double kMuEAr = kEMass * kArMass / (kEMass + kArMass);   // e + Ar
constexpr double kEvToJ = kECharge;
constexpr double kPi = 3.14159265358979323846;
constexpr double kTwoPi = 6.28318530717958647692;
constexpr double kTwo32 = 4294967296.0;

// The float nearest above a non-negative double: an upper bound that costs
// half the bytes (+inf past the float range).
__host__ __device__ inline float float_above(double d) {
  const float f = (float)d;
  // next float up when rounding went down (f is then finite and >= 0)
  return (double)f < d ? __builtin_bit_cast(float, __builtin_bit_cast(uint32_t, f) + 1u) : f;
}

// Fixed-point scales of the per-step diagnostic sums.
constexpr double kDiagJS = 1024.0;     // c * vbar_x [m/s]
constexpr double kDiagWS = 1048576.0;  // c
constexpr double kDiagES = 1048576.0;  // c * energy [eV]
constexpr double kDiagIZS = 4294967296.0;  // c * nu_ion dt_e

// Workgroup size of most kernels, and of the small-case kernel's chunks.
constexpr int kBlock = 256;
constexpr int kChunk = kBlock;  // slots per chunk of the host's size estimates and the sort
// Workgroup size of the lockstep particle kernels; a chunk of their
// streaming loop is one slot per thread.  Candidate lists are sized for the
// largest chunk.
#ifndef EDP_PART_BLOCK
#define EDP_PART_BLOCK 256
#endif
constexpr int kPartBlock = EDP_PART_BLOCK;
constexpr int kMaxChunk = 1024;
static_assert(kPartBlock % 256 == 0 && kPartBlock <= kMaxChunk, "particle workgroup size");
constexpr int kMaxApply = 1024;   // collision workgroups per case and application
constexpr int kMaxPartWG = 8192;  // particle workgroups per case and species
constexpr int kMaxNodes = 2048;                      // largest n_grid accepted
constexpr int kMaxPb = 256;  // blocks of the collision pre-test's bound table
constexpr int kVoltChunk = 1 << 16;  // steps of V(t) resident on the device

// Flags (same values as EDP_* in edupic.h).
constexpr uint32_t kDiagDensity = 1u, kDiagEepf = 2u, kDiagCurrent = 4u, kDiagMeanE = 8u,
                   kIonizLiteral = 16u, kNullCollision = 64u, kDiagXT = 128u, kDiagIfed = 256u;
constexpr uint32_t kDiagParticle = kDiagEepf | kDiagCurrent | kDiagMeanE | kDiagXT | kDiagIfed;

// Sums of the xt arrays, each [n_xt][ng] (time bin major).  kXtFlux holds
// sum F_q for q < ng-1 and sum V in slot ng-1, from which the potential is
// rebuilt as phi_p = V - sum_{q<p} F_q.
enum XtSum {
  kXtFlux = 0, kXtEf, kXtNe, kXtNi, kXtJe, kXtJi, kXtPe, kXtPi, kXtWe, kXtEe, kXtWi, kXtEi, kXtIz,
  kNumXt
};

// Dynamic counters (int64 slots of CaseDev::ctr).
enum Ctr {
  kAbsEPow = 0, kAbsEGnd, kAbsIPow, kAbsIGnd, kCollE, kCollI, kIoniz, kAnomaly, kDropped,
  kLiveE, kLiveI, kPstepE, kPstepI, kSeePow, kSeeGnd, kRefl, kNumCtr
};

struct SpeciesDev {
  double *x[2], *vx[2], *vy[2], *vz[2];  // two buffer sets: current and sort target
  uint64_t *uid[2];
  // electrons: an upper bound of vy*vy + vz*vz of the same slot as a float
  // (the double value rounded up), kept with vy and vz by every writer, so
  // that the streaming pass reads 4 bytes instead of 16 to rule out the
  // electrons too fast for its collision pre-test (ions: null)
  float* vp2[2];
  int64_t cap;
};

struct CaseDev {
  // ---- constants -------------------------------------------------------
  int32_t ng, nbins, nsub, n_eepf;
  uint32_t flags;
  int32_t nt;         // steps per RF period
  int32_t n_xt_bin;   // steps per xt time bin
  int32_t n_xt;       // xt time bins (nt / n_xt_bin)
  int32_t n_ifed;     // IFEDF bins per electrode (plus one beyond the range)
  int32_t pad0;
  double de_ifed;
  double L, dx, inv_dx, dt_e, dt_i, factor_w, factor_e, factor_i;
  double sigma_a, de_cs, thr_exc, thr_ion, w_ion, de_eepf, x_lo, x_hi;
  double dens_scale;  // factor_w / 2^32
  double n_gas;                     // gas density p / (k_B T_g)
  double nu_star_e, nu_star_i;      // null-collision maximum frequencies
  double p_null_e, p_null_i;        // 1 - exp(-nu* dt) per species
  // collision candidates of the direct test: R below p_bound (P* with a
  // relative margin), or electrons with v^2 > v2_lim_e, ions with
  // 2 (v^2 + a2_i) > g2_lim_i (a2_i bounds the squared thermal target speed
  // the generator can give), i.e. beyond the energy range P* covers
  double p_bound_e, p_bound_i, v2_lim_e, g2_lim_i, a2_i;
  // the same bound by energy: pbound[sp][b] bounds P over every table row
  // up to the last of block b (rows r with r >> pb_shift <= b), a prefix
  // maximum, so that the block of any upper bound of a particle's energy
  // gives a bound of its P
  const double* pbound[2];
  int32_t pb_shift, pb_n;
  double kpois;       // dx*dx/eps0
  // surface processes, [0] powered electrode (x = 0), [1] grounded (x = L)
  double gamma_see[2];  // ion-induced secondary electron yield
  double eta_refl[2];   // elastic electron reflection probability
  double see_sigma;     // sqrt(k T_see / m_e) of the emitted electrons
  int32_t see_on, refl_on;
  uint64_t seed;
  SpeciesDev sp[2];
  const double *nsig_e, *nsig_i, *sig_el, *sig_exc, *sig_ion, *sig_iso, *sig_back;
  const double *rden;   // Thomas reciprocals r_p, p = 0..ng-1 (r_0 unused)
  const double *volt;   // V(t_s) at volt[s % kVoltChunk]
  int64_t *cnt_e;       // [3][ng] electron deposit, ring by step % 3
  int64_t *cnt_i;       // [3][ng] ion deposit, ring by (step / nsub) % 3
  double *rho, *phi, *efield;
  double* flux;         // F_q = phi_q - phi_{q+1}, q < ng-1; flux[ng-1] = V of the step
  double *sum_ne, *sum_ni, *sum_je, *sum_ji, *sum_w, *sum_e;  // [ng] time sums
  int64_t *acc_je, *acc_ji, *acc_w, *acc_e;                   // [3][ng] per step
  int64_t *acc_wi, *acc_ei, *acc_iz;  // [3][ng] per step: ion weight, ion energy, c nu_ion dt
  double* xt;                         // [kNumXt][n_xt][ng] sums
  int64_t* xt_cnt;                    // [2][n_xt]: steps and ion steps per bin
  int64_t* ifed;                      // [2][n_ifed + 1] impacts per energy bin
  int64_t *eepf;                                              // [n_eepf]
  int64_t *sort_cnt;                                          // [ng + 1] scratch
  // Step totals of the lockstep particle workgroups, [2][kShards][kRec]:
  // workgroup j of a species adds its totals to shard j % kShards (few
  // workgroups share an address); the window-end kernel folds the shards
  // into the counters and clears them.
  int64_t* shard;
  // Collision candidates a particle workgroup's streaming loop could not
  // keep in LDS, per species [cap]: workgroup j writes their slots into its
  // own chunk range and tests them after the loop.
  int64_t* clist[2];
  // ---- dynamic (device-mutated) -----------------------------------------
  int64_t step;       // next step to run (advanced at the end of a window)
  int64_t n[2];       // slots in use (live + tombstones) at `step`, between windows
  int64_t alloc[2];   // the same (kept for the host's asynchronous size estimate)
  int32_t cur[2];     // current buffer set per species
  // Slot counts inside a window: the slots at the start of step s are
  // min(nbase[sp][(s+2)%3] + born[sp][(s+2)%3], cap) -- the slots at the start
  // of step s-1 and the births that step placed.  Newborns of step s take
  // slots nbase + born[sp][s%3]++ (so a step's loops never see its own
  // newborns); step s stores its own count in nbase[sp][s%3] and clears
  // born[sp][(s+1)%3] for the next step.
  int64_t nbase[2][3];
  int64_t born[2][3];
  int64_t diag_steps, diag_ion_steps;
  int64_t ctr[kNumCtr];
  int32_t error;      // 1: capacity overflow
  int32_t phi_valid;  // 1: phi[] holds the potential of the last step, 0: use flux[]
};

// Fields of a particle workgroup's step totals (one shard record).
enum Rec { kRecColl = 0, kRecIoniz, kRecAbsPow, kRecAbsGnd, kRecLive, kRecBornE, kRecBornI, kRecDropped, kRec };
constexpr int kShards = 64;

// A batch of cases stepped together: every launch advances each case by one
// step.  Each workgroup of a batched launch reads its role from a table the
// host builds with the batch -- its case, the case's deposit rings and V(t)
// ring, the case's step at the start of the window (refreshed on the device
// by the window's first kernel), its index among that case's workgroups of
// the same kind and their number, and the case's node count and ion
// subcycle, and for a particle workgroup its share of the case's chunks --
// in one scalar load, so that its first loads of the deposit need not wait
// for the case block.  A launch of a window gets its step offset as an
// argument: step = step0 + dstep.
constexpr int kMaxBatch = 256;
struct BlockRole {
  CaseDev* c;
  const int64_t* cnt_e;  // [3][ng] electron deposit rings
  const int64_t* cnt_i;  // [3][ng] ion deposit rings
  const double* volt;    // V(t_s) ring
  int64_t step0;
  int32_t j, n;
  int32_t ng, nsub;
  // particle workgroups: chunks [nch*f_lo, nch*f_hi) / 2^31 of the case's nch
  // chunks of a step (consecutive workgroups share their bounds, the first
  // starts at 0 and the last ends at 2^31)
  uint32_t f_lo, f_hi;
};

}  // namespace edp
