// HIP kernels of the PIC/MCC time step for gfx950.
//
// One step s of a case (section 2.1; Algorithms 2-6) is one launch per
// species (ions only on steps with s % N_SUB == 0: ion subcycling).  Every
// workgroup of k_particles first solves the field of step s from the
// fixed-point densities into its own LDS (steps 1-2: rho, the discrete
// Poisson equation, E on the nodes) and then streams its share of the
// particles: gather E, leapfrog push, wall absorption, the collision test,
// the colliders' scattering and the ionization births, and the deposit of
// the new position for step s+1 -- fused, so each particle's state is
// streamed from HBM once per step and no launch sits between two steps'
// particle passes.
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
#include <hip/hip_ext.h>

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
    // one 32x32->64 multiply each (v_mad_u64_u32) gives both halves
    const uint64_t p0 = (uint64_t)0xD2511F53u * c.x;
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * c.z;
    c = make_uint4((uint32_t)(p1 >> 32) ^ c.y ^ k0, (uint32_t)p1, (uint32_t)(p0 >> 32) ^ c.w ^ k1,
                   (uint32_t)p0);
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
  // sincos: one argument reduction for both (the same values as separate
  // sin and cos calls)
  double sn, cs;
  sincos(kTwoPi * u1, &sn, &cs);
  z0 = r * cs;
  z1 = r * sn;
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

// Cross-section table row of a kinetic energy: the nearest of the tabulated
// energies i * de (section 3.2), every energy past the end in the last row.
__device__ __forceinline__ int energy_bin(double e_ev, double de, int nbins) {
  const double rows = e_ev / de + 0.5;
  return rows >= (double)(nbins - 1) ? nbins - 1 : (int)rows;
}

// Post-collision velocity w + f2 g' R(theta,phi)(cos chi, sin chi cos eta,
// sin chi sin eta) with the Euler angles of g from its components (phi = 0
// when g is along x); the components follow the final velocity equation of
// section 2.1.6 term by term.
struct Frame {
  double cos_theta, sin_theta, cos_phi, sin_phi;
};
__device__ __forceinline__ Frame frame_of(double gx, double gy, double gz, double gmag) {
  Frame F;
  if (gmag > 0.0) {
    const double gyz = sqrt(gy * gy + gz * gz);
    F.cos_theta = gx / gmag;
    F.sin_theta = gyz / gmag;
    if (gyz > 0.0) {
      F.cos_phi = gy / gyz;
      F.sin_phi = gz / gyz;
    } else {
      F.cos_phi = 1.0;
      F.sin_phi = 0.0;
    }
  } else {
    F.cos_theta = 1.0;
    F.sin_theta = 0.0;
    F.cos_phi = 1.0;
    F.sin_phi = 0.0;
  }
  return F;
}
__device__ __forceinline__ void rotate(const Frame& F, double gnew, double f2, double cos_chi, double sin_chi,
                                       double cos_eta, double sin_eta, double wx, double wy, double wz, double& ox,
                                       double& oy, double& oz) {
  const double a = f2 * gnew;
  ox = wx + a * (F.cos_theta * cos_chi - F.sin_theta * sin_chi * cos_eta);
  oy = wy + a * (F.sin_theta * F.cos_phi * cos_chi + F.cos_theta * F.cos_phi * sin_chi * cos_eta -
                 F.sin_phi * sin_chi * sin_eta);
  oz = wz + a * (F.sin_theta * F.sin_phi * cos_chi + F.cos_theta * F.sin_phi * sin_chi * cos_eta +
                 F.cos_phi * sin_chi * sin_eta);
}
__device__ __forceinline__ void scatter(double gx, double gy, double gz, double gmag, double gnew,
                                        double f2, double cos_chi, double sin_chi, double eta,
                                        double wx, double wy, double wz, double& ox, double& oy,
                                        double& oz) {
  const Frame F = frame_of(gx, gy, gz, gmag);
  double cos_eta, sin_eta;
  sincos(eta, &sin_eta, &cos_eta);
  rotate(F, gnew, f2, cos_chi, sin_chi, cos_eta, sin_eta, wx, wy, wz, ox, oy, oz);
}

// Fixed-point split of one particle between nodes p and p+1 (charge
// assignment equations): in cell units xi = x/dx, p = int(xi) clamped to
// N_g-2, the share of node p+1 (xi - p) 2^32 truncated, capped at 2^32.
__device__ __forceinline__ int deposit_split(double x, double inv_dx, int ng, long long& r) {
  const double xi = x * inv_dx;
  int p = (int)xi;
  p = p > ng - 2 ? ng - 2 : (p < 0 ? 0 : p);
  const double f = xi - (double)p;
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

// Arrays reached through the CaseDev block are global memory, but the
// compiler cannot prove it for pointers loaded from memory and would emit
// FLAT instructions, which count against the LDS wait counter too: every LDS
// access would then wait for the in-flight HBM traffic.  G() states the
// address space so loads, stores and atomics are global_* instructions.
#define EDP_GLOBAL __attribute__((address_space(1)))
template <class T>
__device__ __forceinline__ EDP_GLOBAL T* G(T* p) {
  return (EDP_GLOBAL T*)p;
}
// A case's constants (and the counters no thread of the running kernel
// writes) are read through the constant address space: uniform reads then
// become scalar loads and stay in scalar registers.  Every write goes
// through the ordinary pointer.
#define EDP_CONST __attribute__((address_space(4)))
template <class T>
__device__ __forceinline__ const EDP_CONST T* KC(const T* p) {
  return (const EDP_CONST T*)p;
}
__device__ __forceinline__ void gl_add(int64_t* a, long long v) {
  __hip_atomic_fetch_add(G((unsigned long long*)a), (unsigned long long)v, __ATOMIC_RELAXED,
                         __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ unsigned long long gl_fetch_add(int64_t* a, unsigned long long v) {
  return __hip_atomic_fetch_add(G((unsigned long long*)a), v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}


// Exclusive scan of one integer per thread across the workgroup; *total
// gets the sum.  scratch: 64 int64 of LDS.
template <class T>
__device__ __forceinline__ T block_exclusive_scan_t(T x, int64_t* scratch, T* total) {
  T* sW = (T*)scratch;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
  T inc = x;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const T y = __shfl_up(inc, off, 64);
    if (lane >= off) inc += y;
  }
  if (lane == 63) sW[wv] = inc;
  __syncthreads();
  T before = 0, tot = 0;
  for (int w = 0; w < nw; ++w) {
    const T v = sW[w];
    if (w < wv) before += v;
    tot += v;
  }
  *total = tot;
  __syncthreads();
  return before + inc - x;
}

// ---------------------------------------------------------------------------
// Steps 1-2: density -> rho -> potential -> field.  MODE 0 (default)
// solves the discrete Poisson equation through the fluxes between nodes, in
// parallel (two workgroup scans instead of 2 N_g dependent steps); it agrees
// with an 80-bit solution to ~1e-15 of the field scale, closer than the
// sequential sweep.  MODE 1 runs the Thomas algorithm itself in one thread,
// operation for operation as the sequential definition (bit-reproducible,
// slow).
// ---------------------------------------------------------------------------
constexpr int kWave = 64;

// Fold the per-step particle sums of one node (ring slot `fold`, the step
// before the one about to run) into the time sums and, with the xt arrays,
// into time-bin row `row_prev`; the power density j E takes the field that
// step used, still in efield[] (the caller overwrites it after a barrier).
__device__ __forceinline__ void fold_particle_sums(const EDP_CONST CaseDev* __restrict__ C, int p,
                                                   int64_t fold, size_t row_prev, size_t plane) {
  const uint32_t fl = C->flags;
  EDP_GLOBAL int64_t* aJe = G(C->acc_je) + fold + p;
  EDP_GLOBAL int64_t* aJi = G(C->acc_ji) + fold + p;
  EDP_GLOBAL int64_t* aW = G(C->acc_w) + fold + p;
  EDP_GLOBAL int64_t* aE = G(C->acc_e) + fold + p;
  const int64_t je = *aJe, ji = *aJi, w = *aW, e = *aE;
  if (fl & kDiagCurrent) {
    G(C->sum_je)[p] += (double)je;
    G(C->sum_ji)[p] += (double)ji;
  }
  if (fl & kDiagMeanE) {
    G(C->sum_w)[p] += (double)w;
    G(C->sum_e)[p] += (double)e;
  }
  *aJe = 0;
  *aJi = 0;
  *aW = 0;
  *aE = 0;
  if (fl & kDiagXT) {
    EDP_GLOBAL int64_t* aWi = G(C->acc_wi) + fold + p;
    EDP_GLOBAL int64_t* aEi = G(C->acc_ei) + fold + p;
    EDP_GLOBAL int64_t* aIz = G(C->acc_iz) + fold + p;
    const int64_t wi = *aWi, ei = *aEi, iz = *aIz;
    const double eo = G(C->efield)[p];
    EDP_GLOBAL double* __restrict__ X = G(C->xt) + row_prev + p;
    X[kXtJe * plane] += (double)je;
    X[kXtPe * plane] += (double)je * eo;
    X[kXtJi * plane] += (double)ji;
    X[kXtPi * plane] += (double)ji * eo;
    X[kXtWe * plane] += (double)w;
    X[kXtEe * plane] += (double)e;
    X[kXtWi * plane] += (double)wi;
    X[kXtEi * plane] += (double)ei;
    X[kXtIz * plane] += (double)iz;
    *aWi = 0;
    *aEi = 0;
    *aIz = 0;
  }
}

// Per-node duties of a step's writer: rho for reads, the time sums of the
// densities, the deposit rings the next steps refill cleared, the particle
// sums of step s-1 folded with the field that step used (still in efield[];
// it is overwritten after the workgroup's next barrier), the xt rows of the
// densities.
struct FieldWriter {
  const EDP_CONST CaseDev* C;
  int64_t s, k;
  int ng;
  bool ion_step, xt;
  size_t plane, row, row_prev;
  __device__ __forceinline__ void node(int p, double ne, double ni, double rho) const {
    const uint32_t fl = C->flags;
    G(C->rho)[p] = rho;
    if (fl & kDiagDensity) {
      G(C->sum_ne)[p] += ne;
      G(C->sum_ni)[p] += ni;
    }
    G(C->cnt_e)[((s + 2) % 3) * ng + p] = 0;
    if (ion_step) G(C->cnt_i)[((k + 2) % 3) * ng + p] = 0;
    if (fl & (kDiagCurrent | kDiagMeanE | kDiagXT)) fold_particle_sums(C, p, ((s + 2) % 3) * ng, row_prev, plane);
    if (xt) {
      EDP_GLOBAL double* __restrict__ X = G(C->xt);
      X[kXtNe * plane + row + p] += ne;
      X[kXtNi * plane + row + p] += ni;
    }
  }
  // the node's field E and flux f (phi for the Thomas solve: MODE 1)
  template <int MODE>
  __device__ __forceinline__ void out(int p, double e, double f, double phi) const {
    G(C->efield)[p] = e;
    if (MODE == 1)
      G(C->phi)[p] = phi;
    else
      G(C->flux)[p] = f;
    if (xt) {
      EDP_GLOBAL double* __restrict__ X = G(C->xt);
      X[kXtEf * plane + row + p] += e;
      X[kXtFlux * plane + row + p] += f;
    }
  }
};

// Steps 1-2 of step s, computed by every workgroup that needs E (each
// particle workgroup of a lockstep launch, the small-case workgroup): the
// densities of the deposit rings read at step s, rho, the potential and E on
// the nodes into sE (LDS).  sF: ng doubles of LDS scratch (the Thomas
// solve).  The ring and V(t) pointers come with the workgroup's role.  The
// results depend only on the deposit, so every workgroup gets the same bits.
// The writer (one workgroup per case and step) also stores rho, E and the
// fluxes (or phi) for reads, clears the deposit rings the next steps refill,
// adds the measurement sums and counts the step.
template <int MODE, int NB>
__device__ __forceinline__ void solve_field(CaseDev* __restrict__ Cw, const int64_t* __restrict__ cnt_e,
                                            const int64_t* __restrict__ cnt_i, const double* __restrict__ volt,
                                            const int ng, const int nsub, const int64_t s, double* sE, double* sF,
                                            const bool writer) {
  // rows of the flux scan and nodes per thread at the largest grid
  constexpr int kRows = (kMaxNodes - 2 + NB - 1) / NB;
  constexpr int kNodes = (kMaxNodes + NB - 1) / NB;
  __shared__ double sWave[2][NB / kWave];
  const EDP_CONST CaseDev* __restrict__ C = KC(Cw);
  const int64_t k = s / nsub;
  const bool ion_step = (s % nsub) == 0;
  const EDP_GLOBAL int64_t* cntE = G(cnt_e) + (s % 3) * ng;
  const EDP_GLOBAL int64_t* cntI = G(cnt_i) + (k % 3) * ng;
  const int t = (int)threadIdx.x;
  const int lane = t % kWave, wv = t / kWave;
  const double V = G(volt)[s % kVoltChunk];
  const double scale = C->dens_scale;
  const double kp = C->kpois;
  const double dx = C->dx;
  FieldWriter W;
  W.C = C;
  W.s = s;
  W.k = k;
  W.ng = ng;
  W.ion_step = ion_step;
  W.xt = writer && (C->flags & kDiagXT) != 0;
  const int64_t nt = C->nt, nxb = C->n_xt_bin;
  W.plane = (size_t)C->n_xt * (size_t)ng;
  W.row = W.xt ? (size_t)((s % nt) / nxb) * (size_t)ng : 0;
  W.row_prev = W.xt ? (size_t)(((s + nt - 1) % nt) / nxb) * (size_t)ng : 0;
  // densities (the electrodes' half cells count twice) and rho of node p
  auto dens = [&](int p, int64_t ce, int64_t ci, double& ne, double& ni) {
    ne = (double)ce * scale;
    ni = (double)ci * scale;
    if (p == 0 || p == ng - 1) {
      ne *= 2.0;
      ni *= 2.0;
    }
    return kECharge * (ni - ne);
  };
  if (MODE == 1) {
    // node p = t + q NB: rho and the right-hand side d_p = rho_p dx^2/eps0
    int64_t ce[kNodes], ci[kNodes];
#pragma unroll
    for (int q = 0; q < kNodes; ++q) {
      const int p = t + q * NB;
      ce[q] = p < ng ? cntE[p] : 0;
      ci[q] = p < ng ? cntI[p] : 0;
    }
#pragma unroll
    for (int q = 0; q < kNodes; ++q) {
      const int p = t + q * NB;
      if (p >= ng) break;
      double ne, ni;
      const double rho = dens(p, ce[q], ci[q], ne, ni);
      sE[p] = rho;
      sF[p] = rho * kp;
      if (writer) W.node(p, ne, ni, rho);
    }
    __syncthreads();
    const double rho0 = sE[0], rhoN = sE[ng - 1];
    if (t == 0) {
      // Thomas algorithm: forward sweep y_p = (d_p + y_{p-1}) r_p, back
      // substitution phi_p = y_p + r_p phi_{p+1}, with the reciprocals r_p
      // precomputed on the host
      const EDP_GLOBAL double* __restrict__ rd = G(C->rden);
      const int m = ng - 2;
      double prev = 0.0;
      for (int p = 1; p <= m; ++p) {
        double d = sF[p];
        if (p == 1) d = d + V;
        prev = (d + prev) * rd[p];
        sF[p] = prev;
      }
      for (int p = m - 1; p >= 1; --p) sF[p] = sF[p] + rd[p] * sF[p + 1];
      sF[0] = V;
      sF[ng - 1] = 0.0;
    }
    __syncthreads();
    for (int p = t; p < ng; p += NB) {
      double e;
      if (p == 0)
        e = (sF[0] - sF[1]) / dx - rho0 * dx / (2.0 * kEps0);
      else if (p == ng - 1)
        e = (sF[ng - 2] - sF[ng - 1]) / dx + rhoN * dx / (2.0 * kEps0);
      else
        e = (sF[p - 1] - sF[p + 1]) / (2.0 * dx);
      sE[p] = e;
      if (writer) W.out<1>(p, e, p < ng - 1 ? sF[p] - sF[p + 1] : V, sF[p]);
    }
  } else {
    // The flux form of the same tridiagonal system: with F_q = phi_q -
    // phi_{q+1}, row p of the Poisson equation says F_p - F_{p-1} = d_p, so
    // F_p = F_0 + S_p with S the prefix sum of d over the interior nodes; the
    // fluxes add up to phi_0 - phi_{N-1} = V, which fixes
    // F_0 = (V - sum_q S_q)/(N_g - 1), and sum_q S_q = sum_r (m - r) d_r over
    // the m = N_g - 2 interior rows.  Thread t owns the contiguous rows
    // q0 <= q < q0 + nq (row q is node q + 1): it loads their densities,
    // forms its prefix and its share of the weighted sum, and one workgroup
    // pass (wave scans, one exchange of the wave totals) gives every thread
    // the rows before its own and the weighted total.  E of its nodes then
    // follows in registers: E_p = (F_{p-1} + F_p)/(2 dx) inside, the boundary
    // forms (Gauss's law over the half cell) at the electrodes.
    const int m = ng - 2;
    const int R = (m + NB - 1) / NB;  // <= kRows
    const int q0 = t * R < m ? t * R : m;
    const int nq = (q0 + R < m ? q0 + R : m) - q0;
    int64_t ce[kRows], ci[kRows];
#pragma unroll
    for (int r = 0; r < kRows; ++r) {
      ce[r] = r < nq ? cntE[q0 + 1 + r] : 0;
      ci[r] = r < nq ? cntI[q0 + 1 + r] : 0;
    }
    const int64_t ce0 = cntE[0], ci0 = cntI[0], ceN = cntE[ng - 1], ciN = cntI[ng - 1];
    double v[kRows];
    double acc = 0.0, wsum = 0.0;
#pragma unroll
    for (int r = 0; r < kRows; ++r) {
      if (r < nq) {
        const int p = q0 + 1 + r;
        double ne, ni;
        const double rho = dens(p, ce[r], ci[r], ne, ni);
        if (writer) W.node(p, ne, ni, rho);
        const double d = rho * kp;
        acc += d;
        wsum += d * (double)(m - (q0 + r));
      }
      v[r] = acc;  // prefix within the thread
    }
    double ne0, ni0, neN, niN;
    const double rho0 = dens(0, ce0, ci0, ne0, ni0);
    const double rhoN = dens(ng - 1, ceN, ciN, neN, niN);
    if (writer && t == 0) {
      W.node(0, ne0, ni0, rho0);
      W.node(ng - 1, neN, niN, rhoN);
    }
    // the workgroup pass: inclusive scan of acc and sum of wsum per wave
    double inc = acc;
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1) {
      const double y = __shfl_up(inc, off, kWave);
      if (lane >= off) inc += y;
    }
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) wsum += __shfl_xor(wsum, off, kWave);
    if (lane == kWave - 1) {
      sWave[0][wv] = inc;
      sWave[1][wv] = wsum;
    }
    __syncthreads();
    double before = inc - acc, sum_s = 0.0;
#pragma unroll
    for (int u = 0; u < NB / kWave; ++u) {
      if (u < wv) before += sWave[0][u];
      sum_s += sWave[1][u];
    }
    const double F0 = (V - sum_s) / (double)(ng - 1);
    double f_prev = F0 + before;  // F_{q0}: F0 plus the rows before this thread's
#pragma unroll
    for (int r = 0; r < kRows; ++r) {
      if (r < nq) {
        const int p = q0 + 1 + r;
        const double f = F0 + (before + v[r]);  // F_{q+1} = F_p
        const double e = (f_prev + f) / (2.0 * dx);
        sE[p] = e;
        if (writer) W.out<0>(p, e, f, 0.0);
        f_prev = f;
      }
    }
    // the electrodes: node 0 by thread 0, node N_g-1 by the owner of the
    // last row (thread 0 when there are no interior rows)
    if (t == 0) {
      const double e = F0 / dx - rho0 * dx / (2.0 * kEps0);
      sE[0] = e;
      if (writer) W.out<0>(0, e, F0, 0.0);
    }
    if (nq > 0 ? q0 + nq == m : t == 0) {
      const double e = f_prev / dx + rhoN * dx / (2.0 * kEps0);
      sE[ng - 1] = e;
      if (writer) W.out<0>(ng - 1, e, V, 0.0);  // the last flux slot keeps V for phi on demand
    }
  }
  if (writer && t == 0) {
    if (W.xt) {
      G(C->xt_cnt)[W.row / ng] += 1;
      if (ion_step) G(C->xt_cnt)[C->n_xt + W.row / ng] += 1;
    }
    Cw->phi_valid = MODE == 1;
    Cw->diag_steps += 1;
    if (ion_step) Cw->diag_ion_steps += 1;
  }
  __syncthreads();  // sE complete; sF free again
}

// ---------------------------------------------------------------------------
// Collisions (step 6): the particle kernels test every particle, pick the
// process of those that collide (partition of [0,1) into sigma_k/sigma_tot),
// and apply it at once -- COM kinematics, scattering angles, Euler rotation,
// the ionization energy split and the newborns -- in dense passes over the
// colliders (see species_pass).
// ---------------------------------------------------------------------------

// Arrays the scattering code touches, loaded once per workgroup.
struct ScatterPtrs {
  EDP_GLOBAL double *ex, *evx, *evy, *evz, *ix, *ivx, *ivy, *ivz;
  EDP_GLOBAL float* evp2;
  EDP_GLOBAL uint64_t *euid, *iuid;
  int64_t* anomaly;
};

// The arrays of buffer sets ce (electrons) and ci (ions).
__device__ __forceinline__ ScatterPtrs scatter_ptrs_at(CaseDev* __restrict__ Cw, int ce, int ci) {
  const EDP_CONST CaseDev* __restrict__ C = KC(Cw);
  ScatterPtrs P;
  P.anomaly = &Cw->ctr[kAnomaly];
  P.ex = G(C->sp[0].x[ce]);
  P.evx = G(C->sp[0].vx[ce]);
  P.evy = G(C->sp[0].vy[ce]);
  P.evz = G(C->sp[0].vz[ce]);
  P.evp2 = G(C->sp[0].vp2[ce]);
  P.euid = G(C->sp[0].uid[ce]);
  P.ix = G(C->sp[1].x[ci]);
  P.ivx = G(C->sp[1].vx[ci]);
  P.ivy = G(C->sp[1].vy[ci]);
  P.ivz = G(C->sp[1].vz[ci]);
  P.iuid = G(C->sp[1].uid[ci]);
  return P;
}

// Electron-Ar collisions, from the colliding electron's state after the push
// (velocity, identity; position for an ionization).  The post-collision
// velocity is w + f2 g' R(theta,phi)(cos chi, sin chi cos eta, sin chi sin
// eta) about the centre-of-mass velocity w, with the frame of g from its
// components and the azimuth eta = 2 pi R_eta; an ionization shares the
// energy above its threshold between the scattered and the ejected
// electron, which leaves at the azimuth eta + pi, and creates an ion with a
// thermal gas velocity.  The three parts are separate functions that
// recompute what they share from the same inputs (same operations, same
// bits), so that the scattering code after a particle loop keeps few values
// alive at once.

// The energy share of an ionization: the COM energy above the threshold
// [eV] (clamped at 0, counted as an anomaly) and the ejected electron's part
// e_ej = w tan(R atan(E/(2w))).
__device__ __forceinline__ void ionization_share(const EDP_CONST CaseDev* __restrict__ C, const ScatterPtrs& P,
                                                 double v2, uint64_t uid, uint32_t st, double& e_ev, double& e_ej) {
  double r_share, r_unused;
  uniform2(C->seed, uid, st, tag(0, 0, 2), r_share, r_unused);
  e_ev = 0.5 * kMuEAr * v2 / kEvToJ - C->thr_ion;
  if (e_ev < 0.0) e_ev = 0.0;
  const double w_ion = C->w_ion;
  e_ej = w_ion * tan(r_share * atan(e_ev / (2.0 * w_ion)));
}

// Scattering angle of one of the two electrons of an ionization from its
// energy e and the shared energy e_ev: cos chi = sqrt(e / e_ev) (or, with the
// literal reading, chi itself).
__device__ __forceinline__ void ionization_angle(const EDP_CONST CaseDev* __restrict__ C, double e, double e_ev,
                                                 double& cs, double& sn) {
  if (C->flags & kIonizLiteral) {
    const double chi = e_ev > 0.0 ? sqrt(e / e_ev) : 0.0;
    sincos(chi, &sn, &cs);
  } else {
    cs = e_ev > 0.0 ? sqrt(e / e_ev) : 1.0;
    sn = sqrt(1.0 - cs * cs);
  }
}

// An outgoing electron of a collision: the colliding electron itself
// (process proc: 0 elastic, 1 excitation, 2 ionization) or, with `eject`,
// the electron its ionization ejects (proc 2), from the parent's pushed
// velocity and identity.  Both take the frame of g and the draws of the
// parent's counter; the ejected one leaves with the other share of the
// energy at the azimuth eta + pi.  Returns the new velocity.
__device__ __forceinline__ void electron_outgoing(const EDP_CONST CaseDev* __restrict__ C, const ScatterPtrs& P,
                                                  bool eject, int proc, int64_t s, double vxn, double vy,
                                                  double vz, uint64_t uid, double& ox, double& oy, double& oz) {
  const uint32_t st = (uint32_t)s;
  // squared speed, the squares summed from x to z as the collision test does
  const double v2 = vxn * vxn + vy * vy + vz * vz;
  const double v = sqrt(v2);
  double r_chi, r_eta;
  uniform2(C->seed, uid, st, tag(0, 0, 1), r_chi, r_eta);
  double gnew = v, cos_chi, sin_chi;
  if (proc < 2) {
    if (proc == 1) {
      double ec = 0.5 * kMuEAr * v2 - C->thr_exc * kEvToJ;
      if (ec < 0.0) {
        ec = 0.0;
        gl_add(P.anomaly, 1);
      }
      gnew = sqrt(2.0 * ec / kMuEAr);
    }
    cos_chi = 1.0 - 2.0 * r_chi;
    sin_chi = sqrt(1.0 - cos_chi * cos_chi);
  } else {
    double e_ev, e_ej;
    ionization_share(C, P, v2, uid, st, e_ev, e_ej);
    if (!eject && 0.5 * kMuEAr * v2 / kEvToJ - C->thr_ion < 0.0) gl_add(P.anomaly, 1);
    const double e_out = eject ? e_ej : e_ev - e_ej;
    gnew = sqrt(2.0 * e_out * kEvToJ / kMuEAr);
    ionization_angle(C, e_out, e_ev, cos_chi, sin_chi);
  }
  const double f1 = kEMass / (kEMass + kArMass);
  const double f2 = kArMass / (kEMass + kArMass);
  const Frame F = frame_of(vxn, vy, vz, v);
  double cos_eta, sin_eta;
  const double eta = kTwoPi * r_eta;
  sincos(eject ? eta + kPi : eta, &sin_eta, &cos_eta);
  rotate(F, gnew, f2, cos_chi, sin_chi, cos_eta, sin_eta, f1 * vxn, f1 * vy, f1 * vz, ox, oy, oz);
}

// Stores of an electron's velocity (and the float bound of vy^2 + vz^2).
__device__ __forceinline__ void store_electron_v(const ScatterPtrs& P, int64_t i, double ox, double oy, double oz) {
  P.evx[i] = ox;
  P.evy[i] = oy;
  P.evz[i] = oz;
  P.evp2[i] = float_above(oy * oy + oz * oz);
}

// The ion an ionization creates, at slot bi at the parent's position: a
// thermal gas velocity from the newborn's own counter.
__device__ __forceinline__ void ion_birth_at(const EDP_CONST CaseDev* __restrict__ C, const ScatterPtrs& P,
                                             int64_t bi, int64_t s, uint64_t uid, double x) {
  const uint64_t cu = child_uid(uid, s, 2);
  double z0, z1, z2;
  normals3(C->seed, cu, (uint32_t)s, 1u, 2u, 1u, z0, z1, z2);
  const double sa = C->sigma_a;
  P.ix[bi] = x;
  P.ivx[bi] = sa * z0;
  P.ivy[bi] = sa * z1;
  P.ivz[bi] = sa * z2;
  P.iuid[bi] = cu;
}

// Ar+ + Ar scattering of colliding ion i (proc 0 isotropic, 1 backward) with the
// thermal target of its test (redrawn from the same counter: the same atom).
__device__ __forceinline__ void ion_scatter_at(const EDP_CONST CaseDev* __restrict__ C, const ScatterPtrs& P, int64_t i,
                                               int proc, int64_t s, double vxn, double vy, double vz, uint64_t uid) {
  const uint64_t seed = C->seed;
  const uint32_t st = (uint32_t)s;
  double z0, z1, z2;
  normals3(seed, uid, st, 1u, 0u, 0u, z0, z1, z2);
  const double sa = C->sigma_a;
  const double vax = sa * z0, vay = sa * z1, vaz = sa * z2;
  const double gx = vxn - vax, gy = vy - vay, gz = vz - vaz;
  const double g = sqrt(gx * gx + gy * gy + gz * gz);
  double r_chi, r_eta;
  uniform2(seed, uid, st, tag(1, 0, 3), r_chi, r_eta);
  const double wx = 0.5 * (vxn + vax), wy = 0.5 * (vy + vay), wz = 0.5 * (vz + vaz);
  double cos_chi, sin_chi;
  if (proc == 0) {
    cos_chi = 1.0 - 2.0 * r_chi;
    sin_chi = sqrt(1.0 - cos_chi * cos_chi);
  } else {
    cos_chi = -1.0;
    sin_chi = 0.0;
  }
  double ox, oy, oz;
  scatter(gx, gy, gz, g, g, 0.5, cos_chi, sin_chi, kTwoPi * r_eta, wx, wy, wz, ox, oy, oz);
  P.ivx[i] = ox;
  P.ivy[i] = oy;
  P.ivz[i] = oz;
}
// Secondary electron of ion i, absorbed at electrode `side` (0 at
// x = 0, 1 at x = L): it starts on the surface with the velocity of a thermal
// flux at T_see -- a Rayleigh normal component into the gap and two normal
// tangential ones (Box-Muller) -- from purpose 3 of the ion's counter; its
// identity is the ion's child of kind 3.  be < 0: dropped at capacity.
__device__ __forceinline__ void see_emit_at(const EDP_CONST CaseDev* __restrict__ C, const ScatterPtrs& P,
                                            uint64_t uid, int side, int64_t be, int64_t s) {
  if (be < 0) return;
  const uint32_t st = (uint32_t)s;
  double a0, a1, b0, b1;
  uniform2(C->seed, uid, st, tag(1, 3, 1), a0, a1);
  uniform2(C->seed, uid, st, tag(1, 3, 2), b0, b1);
  const double sig = C->see_sigma;
  const double vn = sig * sqrt(-2.0 * log(1.0 - a0));
  const double vt = sig * sqrt(-2.0 * log(1.0 - a1));
  P.ex[be] = side == 0 ? 0.0 : C->L;
  P.evx[be] = side == 0 ? vn : -vn;
  double sn, cs;
  sincos(kTwoPi * b0, &sn, &cs);
  const double vy = vt * cs, vz = vt * sn;
  P.evy[be] = vy;
  P.evz[be] = vz;
  P.evp2[be] = float_above(vy * vy + vz * vz);
  P.euid[be] = child_uid(uid, s, 3);
}
// ---------------------------------------------------------------------------
// Steps 3-6 for one species plus the deposit for step s+1.
//
// A case's particle slots are cut into chunks of NB slots (the workgroup
// size).  In the lockstep kernels a case gets a fixed number of workgroups
// (its share, by expected particle count, of the resident slots the batch
// uses); each takes a contiguous range of the step's chunks by the share
// its role gives it (the later a workgroup is dispatched, the smaller its
// share, when the host weights them so), so the launch shape never depends
// on the count.  The small-case kernel runs every chunk of its case
// in one workgroup.  Inside a workgroup the range is worked in slices of 64
// slots, one per lane: wave w takes slices w, w + W, w + 2W, ... of its
// workgroup's W waves.
//
// Every particle: gather E from LDS, leapfrog, wall test, deposit the new x
// into the workgroup's LDS histogram, store x and v_x, and one Philox call
// for its collision uniform R.  Only R below a bound of the collision
// probability over the tables (the null-collision P*, with a relative
// margin for the direct test), or a speed beyond the range that bound
// covers, can give a collision; such candidates (a few percent) go to the
// wave's LDS segment and everyone else is done.  The candidates get the
// exact test -- energy bin, table lookups, exp, for ions the thermal target
// first -- and the colliders their scattering, in dense passes after the
// loop: each wave its own segment, then the workgroup's overflow list (the
// segments that filled during the loop), 64 entries per pass from an LDS
// counter.  So the table work and the transcendentals run on full waves
// instead of on every wave with one candidate lane.  An ionization takes
// slots for its newborns from the step's birth counters, writes them, and
// adds their charge (the electron a second share at the parent's x, the ion
// to the next ion step's density).
//
// Dynamic LDS: E[ng] double, then the region of H[ng] deposit (also the field
// solve's scratch); with particle diagnostics also J[ng], W[ng], En[ng]
// (int64) and EEPF[n_eepf] (uint32).  Static: the candidate segments (ions
// 4 KiB of slots; electrons 10 KiB of slots, v^2 and uids) and a few
// counters.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int lane_rank(uint64_t mask) {
  // set bits of mask below this lane
  return (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

// Candidate segment entries per wave: ions keep the slot only (their exact
// test reloads the state); electrons keep the slot, the pushed v_x and the
// uid, so that their exact test reads only v_y and v_z back.
constexpr int kSegI = 256;
constexpr int kSegE = 128;
template <int SP>
constexpr int seg_len() { return SP == 0 ? kSegE : kSegI; }

// Birth slots of one step: a species' newborns take consecutive slots after
// its slot count at the step's start, from a counter of the step's births
// (LDS in the small-case kernel, born[sp][s % 3] in global memory in the
// lockstep kernels); a slot at or beyond the capacity drops the birth.
template <bool SMALL>
struct Births {
  int64_t base[2], cap[2];
  int* lds;           // SMALL: this step's counters per species
  int64_t* glob[2];   // lockstep: this step's counters per species
  // Slot of this lane's newborn of species sp (mine), -1 if none or dropped;
  // every lane of the wave calls it.  placed / dropped count the wave's.
  __device__ __forceinline__ int64_t take(int sp, bool mine, int lane, int& placed, int& dropped) const {
    const uint64_t m = __ballot(mine);
    if (m == 0) return -1;
    long long b = 0;
    if (lane == 0) {
      const int c = (int)__popcll(m);
      if (SMALL)
        b = atomicAdd(&lds[sp], c);
      else
        b = (long long)gl_fetch_add(glob[sp], (unsigned long long)c);
    }
    b = __shfl(b, 0);
    const int64_t slot = base[sp] + (int64_t)b + lane_rank(m);
    const bool ok = slot < cap[sp];
    placed += (int)__popcll(__ballot(mine && ok));
    dropped += (int)__popcll(__ballot(mine && !ok));
    return mine && ok ? slot : -1;
  }
  // Slots of the newborn pairs (an electron and an ion) of the wave's `cnt`
  // ionizations: issue() takes them from both counters (lane 0; the
  // atomics go out together and their values are needed only by
  // first_slots()), newborn r of the wave then has slot first + r.
  __device__ __forceinline__ void issue_pair(int cnt, int lane, long long& a_e, long long& a_i) const {
    a_e = a_i = 0;
    if (lane == 0) {
      if (SMALL) {
        a_e = atomicAdd(&lds[0], cnt);
        a_i = atomicAdd(&lds[1], cnt);
      } else {
        a_e = (long long)gl_fetch_add(glob[0], (unsigned long long)cnt);
        a_i = (long long)gl_fetch_add(glob[1], (unsigned long long)cnt);
      }
    }
  }
  __device__ __forceinline__ void first_slots(long long a_e, long long a_i, int64_t& f_e, int64_t& f_i) const {
    f_e = base[0] + (int64_t)__shfl(a_e, 0);
    f_i = base[1] + (int64_t)__shfl(a_i, 0);
  }
};

// Totals of one species' step in one workgroup (kRec fields, summed over the
// waves).
struct SpTot {
  int v[kRec];
};

// Steps 3-6 of species SP at step s over chunks [c_lo, c_hi) of slots [0, n)
// of buffer set `cur` (the other species' current set `cur_o`), E in sE,
// `reg` the LDS region for the deposit histogram (and the particle
// diagnostics), B the step's birth counters.
template <int SP, bool SMALL, int NB>
__device__ __forceinline__ SpTot species_pass(CaseDev* __restrict__ Cw, const double* sE, double* reg,
                                              const int64_t s, const int64_t n, const int64_t c_lo,
                                              const int64_t c_hi, const int cur, const int cur_o,
                                              const Births<SMALL>& B, const int pretest) {
  const EDP_CONST CaseDev* __restrict__ C = KC(Cw);
  constexpr int kSeg = seg_len<SP>();
  constexpr int kPay = SP == 0 ? NB / kWave : 1;
  __shared__ int32_t sSeg[NB / kWave][kSeg];
  __shared__ double sVx[kPay][SP == 0 ? kSeg : 1];
  __shared__ uint64_t sUid[kPay][SP == 0 ? kSeg : 1];
  __shared__ int sTot[NB / kWave][kRec];
  // entries of the overflow list, next pass over it
  __shared__ int sOvf, sFin;
  // the pre-test's bound of P by energy block (direct collision test)
  __shared__ double sPB[kMaxPb];
  // lanes of a pass's ionizing colliders by rank (electrons)
  __shared__ int sIon[SP == 0 ? NB / kWave : 1][SP == 0 ? kWave : 1];
  const int ng = C->ng;
  const int nsub = C->nsub;
  const int64_t kion = s / nsub;
  const uint32_t fl = C->flags;
  const bool pdiag = (fl & kDiagParticle) != 0;
  const bool xt = (fl & kDiagXT) != 0;
  const int n_eepf = C->n_eepf;
  const int n_ifed = C->n_ifed;
  // histogram: the EEPF for electrons, the IFEDF of both electrodes for ions
  const int n_hist = SP == 0 ? ((fl & kDiagEepf) ? n_eepf : 0) : ((fl & kDiagIfed) ? 2 * (n_ifed + 1) : 0);
  unsigned long long* sH = (unsigned long long*)reg;
  unsigned long long* sJ = sH + ng;
  unsigned long long* sW = sJ + ng;
  unsigned long long* sEn = sW + ng;
  unsigned long long* sIz = sEn + ng;  // electrons with the xt arrays only
  unsigned int* sF = (unsigned int*)(sIz + (SP == 0 && xt ? ng : 0));
  for (int p = threadIdx.x; p < ng; p += blockDim.x) {
    sH[p] = 0;
    if (pdiag) {
      sJ[p] = 0;
      sW[p] = 0;
      sEn[p] = 0;
      if (SP == 0 && xt) sIz[p] = 0;
    }
  }
  for (int b = threadIdx.x; b < n_hist; b += blockDim.x) sF[b] = 0;
  constexpr int kWaves = NB / kWave;
  // candidate pre-test: R below a bound of P, or a speed beyond the bound's
  // range.  The direct test's bound is P* (with its margin), or, when a
  // wave's slots would give enough candidates by it, the
  // bound by energy: the block of the table row of an upper bound of the
  // particle's (relative) energy -- from g2u, a bound of its squared speed,
  // times (1 + 1e-12) against the rounding of the exact test's own v^2 and
  // energy -- in sPB.  The lookup costs every particle a few instructions
  // and an LDS load, so it is taken when P* would give a wave more than a
  // quarter round of candidates (measured: 2% slower on the large case with
  // 8 per wave, 4-12% faster on the batched sets with 20-400).
  const bool null_coll = (fl & kNullCollision) != 0;
  const double p_null = SP == 0 ? C->p_null_e : C->p_null_i;
  const double p_cand = null_coll ? p_null : (SP == 0 ? C->p_bound_e : C->p_bound_i);
  const bool by_energy =
      !null_coll && (pretest == 2 || (pretest == 0 && (double)(c_hi - c_lo) * kWave * p_cand > (double)(kWave / 4)));
  if (by_energy) {
    const int pb_n = C->pb_n;
    const EDP_GLOBAL double* __restrict__ pbg = G(C->pbound[SP]);
    for (int b = threadIdx.x; b < pb_n; b += blockDim.x) sPB[b] = pbg[b];
  }
  if (threadIdx.x == 0) {
    sOvf = 0;
    sFin = 0;
  }
  __syncthreads();
  EDP_GLOBAL double* __restrict__ X = G(C->sp[SP].x[cur]);
  // this workgroup's overflow list of candidates: its chunk range of the
  // species' list (as many entries as the range has slots)
  EDP_GLOBAL int64_t* __restrict__ CL = G(C->clist[SP]) + c_lo * NB;
  EDP_GLOBAL double* __restrict__ VX = G(C->sp[SP].vx[cur]);
  const EDP_GLOBAL double* __restrict__ VY = G(C->sp[SP].vy[cur]);
  const EDP_GLOBAL double* __restrict__ VZ = G(C->sp[SP].vz[cur]);
  const EDP_GLOBAL uint64_t* __restrict__ UID = G(C->sp[SP].uid[cur]);
  // electrons: a float bound of vy*vy + vz*vz per slot, read in place of vy
  // and vz for the pre-test (those only by the candidates' exact test and the
  // measurement sums)
  const EDP_GLOBAL float* __restrict__ VP2 = G(C->sp[SP].vp2[cur]);
  const ScatterPtrs P = SP == 0 ? scatter_ptrs_at(Cw, cur, cur_o) : scatter_ptrs_at(Cw, cur_o, cur);
  const double inv_dx = C->inv_dx, L_gap = C->L;
  const double dt = SP == 0 ? C->dt_e : C->dt_i;
  const double kick = SP == 0 ? C->factor_e : C->factor_i;
  const EDP_GLOBAL double* __restrict__ nsig = G(SP == 0 ? C->nsig_e : C->nsig_i);
  const EDP_GLOBAL double* __restrict__ sig0 = G(SP == 0 ? C->sig_el : C->sig_iso);
  const EDP_GLOBAL double* __restrict__ sig1 = G(SP == 0 ? C->sig_exc : C->sig_back);
  const EDP_GLOBAL double* __restrict__ sig2 = G(C->sig_ion);
  int64_t* const cnt_i_next = C->cnt_i + ((kion + 1) % 3) * ng;
  // this species' deposit for step s+1 (next ion step for ions)
  int64_t* const dst = SP == 0 ? C->cnt_e + ((s + 1) % 3) * ng : C->cnt_i + ((kion + 1) % 3) * ng;
  int64_t* const cnt_e_next = C->cnt_e + ((s + 1) % 3) * ng;
  const double de_cs = C->de_cs;
  const int nbins = C->nbins;
  const uint64_t seed = C->seed;
  const uint32_t st = (uint32_t)s;
  const double x_lo = C->x_lo, x_hi = C->x_hi, de_eepf = C->de_eepf, de_ifed = C->de_ifed;
  const double sa = C->sigma_a;
  // surface processes of this species' electrode hits
  const bool surf_on = SP == 0 ? C->refl_on != 0 : C->see_on != 0;
  const double p_surf0 = SP == 0 ? C->eta_refl[0] : C->gamma_see[0];
  const double p_surf1 = SP == 0 ? C->eta_refl[1] : C->gamma_see[1];
  const double n_gas = C->n_gas;
  const double nu_star = SP == 0 ? C->nu_star_e : C->nu_star_i;
  const double v2_cand = null_coll ? __builtin_huge_val() : (SP == 0 ? C->v2_lim_e : C->g2_lim_i);
  const double rows_per_g2 = 0.5 * (SP == 0 ? kEMass : kMuArAr) / kEvToJ / C->de_cs * (1.0 + 1e-12);
  const int pb_shift = C->pb_shift;
  const double a2_i = C->a2_i;
  const uint32_t r_tag = SP == 0 ? tag(0, 0, 0) : tag(1, 0, 2);
  const int w = (int)threadIdx.x / kWave, lane = (int)threadIdx.x % kWave;
  // this wave's totals (uniform over the wave)
  int t_coll = 0, t_ioniz = 0, t_pow = 0, t_gnd = 0, t_live = 0, t_be = 0, t_bi = 0, t_drop = 0;
  int ncw = 0;  // entries in this wave's candidate segment

  // Step 6 for candidates.  exact_test: the exact test of one candidate
  // (direct: P = 1 - exp(-n sigma_tot g dt), collide iff R < P, process by
  // sigma_k / sigma_tot; null collision: process by R nu* against the
  // cumulative nu_k, the rest null) from its pushed v_x, v_y, v_z and uid;
  // returns the process or -1.
  auto exact_test = [&](const double vxn, const double vy, const double vz, const uint64_t uid) -> int {
    int proc = -1;
    double r_coll, r_proc;
    uniform2(seed, uid, st, r_tag, r_coll, r_proc);
    if (null_coll) {
      double g, c1, c2, c3;
      int idx;
      if (SP == 0) {
        const double v2 = vxn * vxn + vy * vy + vz * vz;
        g = sqrt(v2);
        const double energy = 0.5 * kEMass * v2 / kEvToJ;
        idx = energy_bin(energy, de_cs, nbins);
        c1 = (n_gas * sig0[idx]) * g;
        c2 = c1 + (n_gas * sig1[idx]) * g;
        c3 = c2 + (n_gas * sig2[idx]) * g;
      } else {
        double z0, z1, z2;
        normals3(seed, uid, st, 1u, 0u, 0u, z0, z1, z2);
        const double gx = vxn - sa * z0, gy = vy - sa * z1, gz = vz - sa * z2;
        const double g2 = gx * gx + gy * gy + gz * gz;
        g = sqrt(g2);
        const double energy = 0.5 * kMuArAr * g2 / kEvToJ;
        idx = energy_bin(energy, de_cs, nbins);
        c1 = (n_gas * sig0[idx]) * g;
        c2 = c1 + (n_gas * sig1[idx]) * g;
        c3 = c2;
      }
      if (c3 > nu_star) gl_add(&Cw->ctr[kAnomaly], 1);
      const double t = r_proc * nu_star;
      proc = t < c1 ? 0 : (t < c2 ? 1 : (SP == 0 && t < c3 ? 2 : -1));
    } else {
      double p_coll, s_a, s_b, s_c = 0.0;
      int idx;
      if (SP == 0) {
        // squared speed summed from x to z (Algorithm 6)
        const double v2 = vxn * vxn + vy * vy + vz * vz;
        const double v = sqrt(v2);
        const double energy = 0.5 * kEMass * v2 / kEvToJ;
        idx = energy_bin(energy, de_cs, nbins);
        // the process tables with the total (one round trip; idx is a
        // valid bin whatever the outcome)
        s_a = sig0[idx];
        s_b = sig1[idx];
        s_c = sig2[idx];
        const double nu = nsig[idx] * v;
        p_coll = 1.0 - exp(-nu * dt);
      } else {
        double z0, z1, z2;
        normals3(seed, uid, st, 1u, 0u, 0u, z0, z1, z2);
        const double gx = vxn - sa * z0, gy = vy - sa * z1, gz = vz - sa * z2;
        const double g2 = gx * gx + gy * gy + gz * gz;
        const double g = sqrt(g2);
        const double energy = 0.5 * kMuArAr * g2 / kEvToJ;
        idx = energy_bin(energy, de_cs, nbins);
        s_a = sig0[idx];
        s_b = sig1[idx];
        const double nu = nsig[idx] * g;
        p_coll = 1.0 - exp(-nu * dt);
      }
      if (r_coll < p_coll) {
        if (SP == 0) {
          const double s_tot = s_a + s_b + s_c;
          if (!(s_tot > 0.0) || r_proc < s_a / s_tot)
            proc = 0;
          else if (r_proc < (s_a + s_b) / s_tot)
            proc = 1;
          else
            proc = 2;
        } else {
          proc = (!(s_a + s_b > 0.0) || r_proc < s_a / (s_a + s_b)) ? 0 : 1;
        }
      }
    }
    return proc;
  };

  // A wave's full segment inside the streaming loop goes to the
  // workgroup's overflow list (entries taken from an LDS counter; the
  // workgroup's candidates are at most its slots) and is tested after the
  // loop: the loop holds no table or transcendental code, so it keeps few
  // registers.
  auto spill_segment = [&](const int count) {
    int off = 0;
    if (lane == 0) off = atomicAdd(&sOvf, count);
    off = __builtin_amdgcn_readfirstlane(__shfl(off, 0));
    for (int k = lane; k < count; k += kWave) CL[off + k] = sSeg[w][k];
  };

  // After the loop and the histogram's flush, in rounds of 64 entries: each
  // wave what is left in its segment, then rounds of the workgroup's
  // overflow list (state reloaded) from an LDS counter, until none is left.
  // Each round runs the exact test, moves the round's
  // colliders with their state to the low lanes (one push permutation), and
  // gives each its scattering; an ionization also gets its newborns (slots
  // from the step's counters, charge at the parent's new position: the
  // electron a second share of this step's deposit, the ion the next ion
  // step's density).  No workgroup barrier: waves finish at their own pace.
  auto finish = [&]() {
    const int npool = sOvf;  // written before the barrier after the loop
    const int own = (ncw + kWave - 1) / kWave;
    for (int round = 0;; ++round) {
      bool pool = false;
      int b0, count;
      if (round < own) {
        b0 = round * kWave;
        count = ncw;
      } else {
        int g = 0;
        if (lane == 0) g = atomicAdd(&sFin, 1);
        b0 = __builtin_amdgcn_readfirstlane(__shfl(g, 0)) * kWave;
        if (b0 >= npool) break;
        pool = true;
        count = npool;
      }
      const int k = b0 + lane;
      int64_t i = 0;
      double vxn = 0.0, vy = 0.0, vz = 0.0;
      uint64_t uid = 0;
      int proc = -1;
      if (k < count) {
        if (pool) {
          i = CL[k];
          vxn = VX[i];
          uid = UID[i];
        } else {
          i = sSeg[w][k];
          if (SP == 0) {
            // the pushed v_x and the uid from the segment
            vxn = sVx[SP == 0 ? w : 0][SP == 0 ? k : 0];
            uid = sUid[SP == 0 ? w : 0][SP == 0 ? k : 0];
          } else {
            vxn = VX[i];
            uid = UID[i];
          }
        }
        // v_y and v_z are not changed by the push
        vy = VY[i];
        vz = VZ[i];
        proc = exact_test(vxn, vy, vz, uid);
      }
      const bool hit = proc >= 0;
      const uint64_t mc = __ballot(hit);
      const int ncol = (int)__popcll(mc);
      t_coll += ncol;
      if (ncol == 0) continue;
      // colliders to lanes [0, ncol), the others after them
      const int to = 4 * (hit ? lane_rank(mc) : ncol + lane_rank(~mc));
      auto push32 = [&](int v) { return __builtin_amdgcn_ds_permute(to, v); };
      auto push64 = [&](uint64_t v) {
        return (uint64_t)(uint32_t)push32((int)(uint32_t)v) | ((uint64_t)(uint32_t)push32((int)(v >> 32)) << 32);
      };
      i = (int64_t)push64((uint64_t)i);
      proc = push32(proc);
      vxn = __longlong_as_double((long long)push64((uint64_t)__double_as_longlong(vxn)));
      vy = __longlong_as_double((long long)push64((uint64_t)__double_as_longlong(vy)));
      vz = __longlong_as_double((long long)push64((uint64_t)__double_as_longlong(vz)));
      uid = push64(uid);
      const bool coll = lane < ncol;
      if (SP == 0) {
        const bool ioniz = coll && proc == 2;
        const uint64_t mi = __ballot(ioniz);
        if (mi == 0) {
          if (coll) {
            double ox, oy, oz;
            electron_outgoing(C, P, false, proc, s, vxn, vy, vz, uid, ox, oy, oz);
            store_electron_v(P, i, ox, oy, oz);
          }
        } else {
          // Ionizations.  The parent's new position and the newborns' slots
          // are loaded and taken first and used only at the stores; the
          // ejected electrons are worked on the lanes the colliders leave
          // free, beside the colliders, in rank order (more passes if they
          // do not fit); the new ions on their parents' lanes after that.
          const int ni = (int)__popcll(mi);
          t_ioniz += ni;
          const int ri = lane_rank(mi);
          const double xb = ioniz ? X[i] : 0.0;
          long long a_e, a_i;
          B.issue_pair(ni, lane, a_e, a_i);
          if (ioniz) sIon[SP == 0 ? w : 0][SP == 0 ? ri : 0] = lane;
          int64_t f_e = 0, f_i = 0;
          bool have_slots = false;
          for (int e0 = 0, pass = 0; pass == 0 || e0 < ni; ++pass) {
            const int lane0 = pass == 0 ? ncol : 0;
            const int e = e0 + lane - lane0;  // the ejected electron of this lane, by rank
            const bool ej = lane >= lane0 && e < ni;
            const bool par = pass == 0 && coll;
            const int src = ej ? sIon[SP == 0 ? w : 0][SP == 0 ? e : 0] : lane;
            const double tvx = __shfl(vxn, src), tvy = __shfl(vy, src), tvz = __shfl(vz, src);
            const uint64_t tuid = (uint64_t)__shfl((long long)uid, src);
            double ox = 0.0, oy = 0.0, oz = 0.0;
            if (par || ej) electron_outgoing(C, P, ej, ej ? 2 : proc, s, tvx, tvy, tvz, tuid, ox, oy, oz);
            if (!have_slots) {
              B.first_slots(a_e, a_i, f_e, f_i);
              have_slots = true;
            }
            const double tx = __shfl(xb, src);
            if (par) store_electron_v(P, i, ox, oy, oz);
            const int64_t be = f_e + e;
            if (ej && be < B.cap[0]) {
              P.ex[be] = tx;
              store_electron_v(P, be, ox, oy, oz);
              P.euid[be] = child_uid(tuid, s, 1);
            }
            e0 += kWave - lane0;
          }
          const bool ok_e = f_e + ri < B.cap[0], ok_i = f_i + ri < B.cap[1];
          t_be += (int)__popcll(__ballot(ioniz && ok_e));
          t_bi += (int)__popcll(__ballot(ioniz && ok_i));
          t_drop += (int)__popcll(__ballot(ioniz && !ok_e)) + (int)__popcll(__ballot(ioniz && !ok_i));
          if (ioniz) {
            long long r;
            const int q = deposit_split(xb, inv_dx, ng, r);
            gl_add(&dst[q], 4294967296LL - r);
            gl_add(&dst[q + 1], r);
            gl_add(&cnt_i_next[q], 4294967296LL - r);
            gl_add(&cnt_i_next[q + 1], r);
            if (ok_i) ion_birth_at(C, P, f_i + ri, s, uid, xb);
          }
        }
      } else if (coll) {
        ion_scatter_at(C, P, i, proc, s, vxn, vy, vz, uid);
      }
    }
  };

  // The state of a wave's next slice is loaded before its current one is
  // worked on, so each wave keeps two slices' loads in flight (the loop is
  // bound by memory latency, not by its arithmetic).
  const int64_t q_lo = c_lo * kWaves;
  const int64_t q_end = (n + kWave - 1) / kWave;
  const int64_t q_hi = c_hi * kWaves < q_end ? c_hi * kWaves : q_end;
  double nx = 0.0, nvx = 0.0, nvy = 0.0, nvz = 0.0;
  float nvp2 = 0.0f;
  uint64_t nuid = 0;
  auto fetch = [&](const int64_t q) {
    const int64_t i = q * kWave + lane;
    nx = __longlong_as_double(0x7FF8000000000000LL);
    nvx = nvy = nvz = 0.0;
    nvp2 = 0.0f;
    nuid = 0;
    if (i < n) {
      nx = X[i];
      nvx = VX[i];
      if (SP == 1 || pdiag) {
        nvy = VY[i];
        nvz = VZ[i];
      }
      if (SP == 0) nvp2 = VP2[i];
      nuid = UID[i];
    }
  };
  int64_t q = q_lo + w;
  if (q < q_hi) fetch(q);
  while (q < q_hi) {
    const int64_t i = q * kWave + lane;
    const double x = nx, vx = nvx, vy = nvy, vz = nvz, vp2 = (double)nvp2;
    const uint64_t uid = nuid;
    const int64_t qn = q + kWaves;
    if (qn < q_hi) fetch(qn);
    bool live = x == x;  // past the end, or absorbed earlier (tombstone)
    t_live += (int)__popcll(__ballot(live));
    bool abs_pow = false, abs_gnd = false, surf = false, cand = false;
    double xn = 0.0, vxn = 0.0, v2 = 0.0;
    if (live) {
      // Steps 3-4: linear interpolation of the nodal field (section 2.1.3)
      // from cell coordinate xi = x/dx, then the leapfrog equations of
      // section 2.1.4, the kick being e dt/m per unit field (subtracted for
      // the electron's negative charge).
      const double xi = x * inv_dx;
      int cell = (int)xi;
      cell = cell > ng - 2 ? ng - 2 : (cell < 0 ? 0 : cell);
      const double w_lo = (double)(cell + 1) - xi;  // weight of node `cell`
      const double w_hi = xi - (double)cell;        // weight of node `cell + 1`
      const double e_here = sE[cell] * w_lo + sE[cell + 1] * w_hi;
      vxn = SP == 0 ? vx - e_here * kick : vx + e_here * kick;
      xn = x + vxn * dt;
      // the pre-test's bound of P for this particle by energy, looked up now
      // so that the LDS load is in flight during the wall test, the deposit
      // and the Philox call (a reflection below keeps |v|)
      double pc = p_cand, g2u = 0.0;
      if (by_energy) {
        v2 = SP == 0 ? vxn * vxn + vp2 : vxn * vxn + vy * vy + vz * vz;
        g2u = SP == 0 ? v2 : 2.0 * (v2 + a2_i);
        double rows = g2u * rows_per_g2 + 0.5;
        rows = rows < (double)(nbins - 1) ? rows : (double)(nbins - 1);
        pc = sPB[(int)rows >> pb_shift];
      }
      if (pdiag) {
        // measurement at integer time: old position, mean of the half-step
        // velocities; the ionization rate as the expected n sigma_ion |v|
        const double vbar = 0.5 * (vx + vxn);
        if (fl & (kDiagCurrent | kDiagXT)) {
          lds_add(&sJ[cell], (long long)(w_lo * vbar * kDiagJS));
          lds_add(&sJ[cell + 1], (long long)(w_hi * vbar * kDiagJS));
        }
        if (SP == 1) {
          if (xt) {
            const double en = 0.5 * kArMass * (vbar * vbar + vy * vy + vz * vz) / kEvToJ;
            lds_add(&sW[cell], (long long)(w_lo * kDiagWS));
            lds_add(&sW[cell + 1], (long long)(w_hi * kDiagWS));
            lds_add(&sEn[cell], (long long)(w_lo * en * kDiagES));
            lds_add(&sEn[cell + 1], (long long)(w_hi * en * kDiagES));
          }
        } else if (fl & (kDiagMeanE | kDiagEepf | kDiagXT)) {
          const double en = 0.5 * kEMass * (vbar * vbar + vy * vy + vz * vz) / kEvToJ;
          if (xt) {
            const double vmag = sqrt(vbar * vbar + vy * vy + vz * vz);
            const double pdt = (n_gas * sig2[energy_bin(en, de_cs, nbins)]) * vmag * dt;
            lds_add(&sIz[cell], (long long)(w_lo * pdt * kDiagIZS));
            lds_add(&sIz[cell + 1], (long long)(w_hi * pdt * kDiagIZS));
          }
          if (fl & (kDiagMeanE | kDiagXT)) {
            lds_add(&sW[cell], (long long)(w_lo * kDiagWS));
            lds_add(&sW[cell + 1], (long long)(w_hi * kDiagWS));
            lds_add(&sEn[cell], (long long)(w_lo * en * kDiagES));
            lds_add(&sEn[cell + 1], (long long)(w_hi * en * kDiagES));
          }
          if ((fl & kDiagEepf) && x >= x_lo && x <= x_hi) {
            const double t = en / de_eepf;
            if (t < (double)n_eepf) atomicAdd(&sF[(int)t], 1u);
          }
        }
      }
      // Step 5: absorbing electrodes; an absorbed ion adds its impact energy
      // to its electrode's IFEDF (bin n_ifed: beyond the range).  Surface
      // processes (purpose 3 of the particle's counter): an electron is
      // reflected specularly with the electrode's probability eta (unless
      // its mirror image lies outside the gap); an absorbed ion emits an
      // electron with probability gamma, whose charge goes on the electrode
      // node of the next step's deposit now and which takes its slot from
      // the step's electron births below.
      abs_pow = xn < 0.0;
      abs_gnd = xn > L_gap;
      if (surf_on && (abs_pow || abs_gnd)) {
        double r_surf, r_unused;
        uniform2(seed, uid, st, tag(SP, 3, 0), r_surf, r_unused);
        if (r_surf < (abs_pow ? p_surf0 : p_surf1)) {
          if (SP == 0) {
            const double xm = abs_pow ? -xn : 2.0 * L_gap - xn;
            if (xm >= 0.0 && xm <= L_gap) {
              xn = xm;
              vxn = -vxn;
              abs_pow = abs_gnd = false;
              surf = true;
            }
          } else {
            surf = true;
            long long r;
            const int q = deposit_split(abs_pow ? 0.0 : L_gap, inv_dx, ng, r);
            gl_add(&cnt_e_next[q], 4294967296LL - r);
            if (r) gl_add(&cnt_e_next[q + 1], r);
          }
        }
      }
      if (abs_pow || abs_gnd) {
        live = false;
        if (SP == 1 && (fl & kDiagIfed)) {
          const double en = 0.5 * kArMass * (vxn * vxn + vy * vy + vz * vz) / kEvToJ;
          const double t = en / de_ifed;
          const int b = t < (double)n_ifed ? (int)t : n_ifed;
          atomicAdd(&sF[(abs_gnd ? n_ifed + 1 : 0) + b], 1u);
        }
      } else {
        // Step 7 for step s+1: deposit the new position.  Step 6 pre-test:
        // a particle can collide only if its R is below the bound of
        // 1 - exp(-nu dt) over the tables (exactly P* for null collisions),
        // or if it is faster than the range that bound covers; the others
        // are settled here with no table work, the candidates go to the
        // wave's segment for the exact test.
        long long r;
        const int q = deposit_split(xn, inv_dx, ng, r);
        lds_add(&sH[q], 4294967296LL - r);
        lds_add(&sH[q + 1], r);
        double r_coll, r_proc;
        uniform2(seed, uid, st, r_tag, r_coll, r_proc);
        if (!by_energy) {
          v2 = SP == 0 ? vxn * vxn + vp2 : vxn * vxn + vy * vy + vz * vz;
          g2u = SP == 0 ? v2 : 2.0 * (v2 + a2_i);
        }
        cand = r_coll < pc || g2u > v2_cand;
      }
    }
    if (i < n && x == x) {
      X[i] = live ? xn : __longlong_as_double(0x7FF8000000000000LL);
      VX[i] = vxn;
    }
    if (surf_on) {
      // reflections (electrons) or emissions per electrode (ions); an ion's
      // secondary electron takes its slot after this step's births so far
      const uint64_t m_s0 = __ballot(surf && (SP == 0 || abs_pow));
      const uint64_t m_s1 = SP == 1 ? __ballot(surf && abs_gnd) : 0ull;
      if (lane == 0 && m_s0) gl_add(&Cw->ctr[SP == 0 ? kRefl : kSeePow], (long long)__popcll(m_s0));
      if (lane == 0 && m_s1) gl_add(&Cw->ctr[kSeeGnd], (long long)__popcll(m_s1));
      if (SP == 1 && (m_s0 | m_s1)) {
        const int64_t be = B.take(0, surf, lane, t_be, t_drop);
        if (surf) see_emit_at(C, P, uid, abs_pow ? 0 : 1, be, s);
      }
    }
    const uint64_t m_c = __ballot(cand);
    if (m_c) {
      if (cand) {
        const int at = ncw + lane_rank(m_c);
        sSeg[w][at] = (int32_t)i;
        if (SP == 0) {
          sVx[SP == 0 ? w : 0][SP == 0 ? at : 0] = vxn;
          sUid[SP == 0 ? w : 0][SP == 0 ? at : 0] = uid;
        }
      }
      ncw += (int)__popcll(m_c);
      if (ncw > kSeg - kWave) {
        spill_segment(ncw);
        ncw = 0;
      }
    }
    t_pow += (int)__popcll(__ballot(abs_pow));
    t_gnd += (int)__popcll(__ballot(abs_gnd));
    q = qn;
  }
  __syncthreads();
  // flush first (deposit for step s+1 and diagnostics of step s): the
  // last candidate pass below adds its newborns' charge to global memory
  // directly, so the flush's atomics are in flight during its table loads
  for (int q = threadIdx.x; q < ng; q += blockDim.x) {
    const unsigned long long h = sH[q];
    if (h) gl_add(&dst[q], (long long)h);
    if (pdiag) {
      const int64_t off3 = (s % 3) * ng + q;
      if (sJ[q]) gl_add(&(SP == 0 ? C->acc_je : C->acc_ji)[off3], (long long)sJ[q]);
      if (sW[q]) gl_add(&(SP == 0 ? C->acc_w : C->acc_wi)[off3], (long long)sW[q]);
      if (sEn[q]) gl_add(&(SP == 0 ? C->acc_e : C->acc_ei)[off3], (long long)sEn[q]);
      if (SP == 0 && xt && sIz[q]) gl_add(&C->acc_iz[off3], (long long)sIz[q]);
    }
  }
  int64_t* hist = SP == 0 ? C->eepf : C->ifed;
  for (int b = threadIdx.x; b < n_hist; b += blockDim.x)
    if (sF[b]) gl_add(&hist[b], (long long)sF[b]);
  // this wave's segment, then the workgroup's overflow list
  finish();
  if (lane == 0) {
    sTot[w][kRecColl] = t_coll;
    sTot[w][kRecIoniz] = t_ioniz;
    sTot[w][kRecAbsPow] = t_pow;
    sTot[w][kRecAbsGnd] = t_gnd;
    sTot[w][kRecLive] = t_live;
    sTot[w][kRecBornE] = t_be;
    sTot[w][kRecBornI] = t_bi;
    sTot[w][kRecDropped] = t_drop;
  }
  __syncthreads();
  SpTot T;
#pragma unroll
  for (int f = 0; f < kRec; ++f) T.v[f] = 0;
#pragma unroll 1
  for (int u = 0; u < NB / kWave; ++u)
#pragma unroll
    for (int f = 0; f < kRec; ++f) T.v[f] += sTot[u][f];
  __syncthreads();  // sTot, the segments and the histograms are free again
  return T;
}

// Slot count of species sp at the start of step s inside a window.
__device__ __forceinline__ int64_t step_slots(const EDP_CONST CaseDev* __restrict__ C, int sp, int64_t s) {
  const int r = (int)((s + 2) % 3);
  const int64_t a = C->nbase[sp][r] + C->born[sp][r];
  return a < C->sp[sp].cap ? a : C->sp[sp].cap;
}

// Steps 1-7 of one species for every case of a lockstep group, at step
// step0 + dstep of each case.  At most 128 VGPRs (four workgroups per CU):
// the streaming loop needs about 100; the scattering code after the loop
// would take twice that if left alone, and spills there instead (colliders
// are a few percent of the particles).  Every workgroup solves its case's field into
// LDS, then takes its chunk range.  The electron launch's workgroup 0 of
// each case is the writer of the step (field outputs, ring clearing,
// measurement sums) and publishes the step's slot counts.  Each workgroup
// adds its totals to its shard of the case's counters.
template <int SP, int MODE>
__global__ void __launch_bounds__(kPartBlock) __attribute__((amdgpu_waves_per_eu(4)))
k_particles(const BlockRole* __restrict__ R, int dstep, int pretest) {
  extern __shared__ double psm[];
  const EDP_CONST BlockRole* r = KC(R) + blockIdx.x;
  CaseDev* Cw = r->c;
  const int ng = r->ng, nsub = r->nsub, j = r->j;
  const int64_t s = r->step0 + dstep;
  if (SP == 1 && (s % nsub) != 0) return;  // ions move on ion steps only
  double* sE = psm;
  double* reg = psm + ng;
  const bool writer = SP == 0 && j == 0;
  const EDP_CONST CaseDev* __restrict__ C = KC(Cw);
  const int64_t n_e = step_slots(C, 0, s), n_i = step_slots(C, 1, s);
  const int64_t n = SP == 0 ? n_e : n_i;
  const uint64_t nch = (uint64_t)((n + kPartBlock - 1) / kPartBlock);
  const int64_t c_lo = (int64_t)((nch * r->f_lo) >> 31);
  const int64_t c_hi = (int64_t)((nch * r->f_hi) >> 31);
  const int cur = C->cur[SP];
  solve_field<MODE, kPartBlock>(Cw, r->cnt_e, r->cnt_i, r->volt, ng, nsub, s, sE, reg, writer);
  if (writer && threadIdx.x == 0) {
    for (int sp = 0; sp < 2; ++sp) {
      Cw->nbase[sp][s % 3] = sp == 0 ? n_e : n_i;
      Cw->born[sp][(s + 1) % 3] = 0;
    }
  }
  if (c_lo >= c_hi) return;  // whole workgroup: nothing to do this step
  Births<false> B;
  B.base[0] = n_e;
  B.base[1] = n_i;
  B.cap[0] = C->sp[0].cap;
  B.cap[1] = C->sp[1].cap;
  B.lds = nullptr;
  B.glob[0] = &Cw->born[0][s % 3];
  B.glob[1] = &Cw->born[1][s % 3];
  const SpTot T = species_pass<SP, false, kPartBlock>(Cw, sE, reg, s, n, c_lo, c_hi, cur, C->cur[1 - SP], B, pretest);
  if (threadIdx.x == 0) {
    int64_t* sh = C->shard + ((int64_t)SP * kShards + j % kShards) * kRec;
#pragma unroll
    for (int f = 0; f < kRec; ++f)
      if (T.v[f]) gl_add(&sh[f], T.v[f]);
    if (T.v[kRecDropped]) Cw->error = 1;
  }
}

// First kernel of a lockstep window: every role's step0 from its case, and
// each case's slot-count rings from its slot counts (so that any host-side
// change of a case between windows is picked up).  Workgroups [0, ncase)
// take the cases of `cases`, the others the roles.
__global__ void __launch_bounds__(kBlock) k_window_begin(BlockRole* __restrict__ roles, int nroles,
                                                         const BlockRole* __restrict__ cases, int ncase) {
  const int b = (int)blockIdx.x;
  if (b < ncase) {
    if (threadIdx.x == 0) {
      CaseDev* C = cases[b].c;
      const int64_t s = C->step;
      for (int sp = 0; sp < 2; ++sp) {
        C->nbase[sp][(s + 2) % 3] = C->n[sp];
        C->born[sp][(s + 2) % 3] = 0;
        C->born[sp][s % 3] = 0;
      }
    }
    return;
  }
  const int i = (b - ncase) * kBlock + (int)threadIdx.x;
  if (i < nroles) roles[i].step0 = roles[i].c->step;
}

// Last kernel of a lockstep window of `steps` steps, one workgroup per case:
// the case's step, its slot counts, and the workgroups' shards folded into
// the counters (then cleared).
__global__ void __launch_bounds__(kBlock) k_window_end(const BlockRole* __restrict__ cases, int steps) {
  __shared__ int64_t sSum[kBlock / kWave][2 * kRec];
  CaseDev* Cw = (KC(cases) + blockIdx.x)->c;
  const EDP_CONST CaseDev* __restrict__ C = KC(Cw);
  // thread t sums field t % (2 kRec) of every shard of both species
  constexpr int kF = 2 * kRec;
  const int t = (int)threadIdx.x;
  static_assert(kBlock == 4 * kWave && kWave == 4 * kF, "shard fold layout");
  int64_t acc = 0;
  EDP_GLOBAL int64_t* sh = G(C->shard);
  {
    const int f = t % kF, sp = f / kRec, fld = f % kRec;
    for (int k = t / kF; k < kShards; k += kBlock / kF) {
      EDP_GLOBAL int64_t* a = sh + ((int64_t)sp * kShards + k) * kRec + fld;
      acc += *a;
      *a = 0;
    }
  }
  const int lane = t % kWave, wv = t / kWave;
  // lanes l and l + 16, l + 32, l + 48 hold the same field (64 = 4 * kF)
  acc += __shfl_xor(acc, 16, kWave);
  acc += __shfl_xor(acc, 32, kWave);
  if (lane < kF) sSum[wv][lane] = acc;
  __syncthreads();
  if (t == 0) {
    int64_t v[kF];
    for (int f = 0; f < kF; ++f) v[f] = sSum[0][f] + sSum[1][f] + sSum[2][f] + sSum[3][f];
    const int64_t* e = v;
    const int64_t* ii = v + kRec;
    int64_t* ctr = Cw->ctr;
    ctr[kCollE] += e[kRecColl];
    ctr[kIoniz] += e[kRecIoniz];
    ctr[kAbsEPow] += e[kRecAbsPow];
    ctr[kAbsEGnd] += e[kRecAbsGnd];
    ctr[kPstepE] += e[kRecLive];
    ctr[kCollI] += ii[kRecColl];
    ctr[kAbsIPow] += ii[kRecAbsPow];
    ctr[kAbsIGnd] += ii[kRecAbsGnd];
    ctr[kPstepI] += ii[kRecLive];
    ctr[kLiveE] += e[kRecBornE] + ii[kRecBornE] - e[kRecAbsPow] - e[kRecAbsGnd];
    ctr[kLiveI] += e[kRecBornI] + ii[kRecBornI] - ii[kRecAbsPow] - ii[kRecAbsGnd];
    ctr[kDropped] += e[kRecDropped] + ii[kRecDropped];
    const int64_t s = Cw->step + steps;
    Cw->step = s;
    for (int sp = 0; sp < 2; ++sp) {
      const int r = (int)((s + 2) % 3);
      const int64_t a = Cw->nbase[sp][r] + Cw->born[sp][r];
      const int64_t cap = C->sp[sp].cap;
      Cw->n[sp] = Cw->alloc[sp] = a < cap ? a : cap;
    }
  }
}

// Cell of a position (the deposit's node p, clamped to N_g - 2).
__device__ __forceinline__ int cell_of(double x, double inv_dx, int ng) {
  int p = (int)(x * inv_dx);
  return p > ng - 2 ? ng - 2 : (p < 0 ? 0 : p);
}

// ---------------------------------------------------------------------------
// Persistent small cases: one workgroup advances one case through a whole
// window of steps inside one launch, and every case of the launch runs at its
// own pace -- no lockstep with the other cases, no launch between two steps,
// no wait between workgroups.  Each step is the same method as the lockstep
// path's and gives the same results bit for bit: the field solve into LDS
// (steps 1-2), then per species the push, walls, collision test, the
// colliders' scattering and the newborns (steps 3-6) and the deposit for the
// next step, then the step's bookkeeping; compaction and cell sort every
// `sort_every` steps as in the lockstep path.  Meant for cases of a few
// thousand particles, whose steps are latency-bound: one workgroup per case
// keeps the chip's other CUs for the other cases.
//
// The workgroup owns the case for the launch: the step, the slot counts and
// the buffer sets live in LDS and are written back at the end.
// ---------------------------------------------------------------------------

// Compaction + counting sort by cell of species sp in one workgroup: the
// live slots of [0, n) of set `cur` go to the other set, cell by cell (order
// within a cell arbitrary); returns the live count.  sC: LDS for ng counters.
__device__ __forceinline__ int64_t small_sort(CaseDev* __restrict__ Cw, int sp, int cur, int64_t n, unsigned int* sC) {
  __shared__ int64_t sRed[64];
  const EDP_CONST CaseDev* __restrict__ C = KC(Cw);
  const int ng = C->ng;
  const double inv_dx = C->inv_dx;
  const EDP_CONST SpeciesDev& S = C->sp[sp];
  const EDP_GLOBAL double* __restrict__ X = G(S.x[cur]);
  for (int p = threadIdx.x; p < ng; p += blockDim.x) sC[p] = 0;
  __syncthreads();
  for (int64_t i = threadIdx.x; i < n; i += kBlock) {
    const double x = X[i];
    if (x == x) atomicAdd(&sC[cell_of(x, inv_dx, ng)], 1u);
  }
  __syncthreads();
  // exclusive scan of the ng - 1 cell counts, a contiguous range per thread
  const int m = ng - 1;
  const int per = (m + kBlock - 1) / kBlock;
  const int lo = (int)threadIdx.x * per < m ? (int)threadIdx.x * per : m;
  const int hi = lo + per < m ? lo + per : m;
  int64_t acc = 0;
  for (int p = lo; p < hi; ++p) acc += sC[p];
  int64_t total;
  int64_t run = block_exclusive_scan_t<int64_t>(acc, sRed, &total);
  for (int p = lo; p < hi; ++p) {
    const unsigned int v = sC[p];
    sC[p] = (unsigned int)run;
    run += v;
  }
  __syncthreads();
  const int nxt = cur ^ 1;
  const EDP_GLOBAL double* __restrict__ VX = G(S.vx[cur]);
  const EDP_GLOBAL double* __restrict__ VY = G(S.vy[cur]);
  const EDP_GLOBAL double* __restrict__ VZ = G(S.vz[cur]);
  const EDP_GLOBAL uint64_t* __restrict__ UID = G(S.uid[cur]);
  EDP_GLOBAL double* __restrict__ X2 = G(S.x[nxt]);
  EDP_GLOBAL double* __restrict__ VX2 = G(S.vx[nxt]);
  EDP_GLOBAL double* __restrict__ VY2 = G(S.vy[nxt]);
  EDP_GLOBAL double* __restrict__ VZ2 = G(S.vz[nxt]);
  EDP_GLOBAL uint64_t* __restrict__ UID2 = G(S.uid[nxt]);
  EDP_GLOBAL float* __restrict__ VP22 = sp == 0 ? G(S.vp2[nxt]) : nullptr;
  for (int64_t i = threadIdx.x; i < n; i += kBlock) {
    const double x = X[i];
    if (!(x == x)) continue;
    const double vx = VX[i], vy = VY[i], vz = VZ[i];
    const uint64_t uid = UID[i];
    const int64_t d = atomicAdd(&sC[cell_of(x, inv_dx, ng)], 1u);
    X2[d] = x;
    VX2[d] = vx;
    VY2[d] = vy;
    VZ2[d] = vz;
    UID2[d] = uid;
    if (sp == 0) VP22[d] = float_above(vy * vy + vz * vz);
  }
  __syncthreads();
  return total;
}

// Window of steps of the small cases: workgroup b advances the case of role
// b by role.j steps.  Dynamic LDS: E, then the largest of the particle
// phase's histograms (also the field solve's scratch) and the sort's
// counters.
template <int MODE>
__global__ void __launch_bounds__(kBlock) k_small(const BlockRole* __restrict__ R, int sort_every, int pretest) {
  extern __shared__ double ssm2[];
  __shared__ int64_t sState[5];  // step, n_e, n_i, cur_e, cur_i
  __shared__ int sBirth[2];
  const EDP_CONST BlockRole* r = KC(R) + blockIdx.x;
  CaseDev* Cw = r->c;
  const int steps = r->j;
  const EDP_CONST CaseDev* __restrict__ C = KC(Cw);
  const int ng = C->ng;
  const int nsub = C->nsub;
  double* sE = ssm2;
  double* reg = ssm2 + ng;
  if (threadIdx.x == 0) {
    sState[0] = Cw->step;
    sState[1] = Cw->n[0];
    sState[2] = Cw->n[1];
    sState[3] = Cw->cur[0];
    sState[4] = Cw->cur[1];
  }
  __syncthreads();
  for (int t = 0; t < steps; ++t) {
    const int64_t s = sState[0];
    int64_t n_e = sState[1], n_i = sState[2];
    int cur_e = (int)sState[3], cur_i = (int)sState[4];
    const bool ion_step = (s % nsub) == 0;
    // compaction + cell sort on the lockstep path's schedule
    if (s % sort_every == 0) {
      n_e = small_sort(Cw, 0, cur_e, n_e, (unsigned int*)ssm2);
      cur_e ^= 1;
    }
    if (s % ((int64_t)sort_every * nsub) == 0) {
      n_i = small_sort(Cw, 1, cur_i, n_i, (unsigned int*)ssm2);
      cur_i ^= 1;
    }
    if (threadIdx.x < 2) sBirth[threadIdx.x] = 0;
    // steps 1-2
    solve_field<MODE, kBlock>(Cw, C->cnt_e, C->cnt_i, C->volt, ng, nsub, s, sE, reg, true);
    Births<true> B;
    B.base[0] = n_e;
    B.base[1] = n_i;
    B.cap[0] = C->sp[0].cap;
    B.cap[1] = C->sp[1].cap;
    B.lds = sBirth;
    B.glob[0] = B.glob[1] = nullptr;
    const int64_t nch_e = (n_e + kChunk - 1) / kChunk, nch_i = (n_i + kChunk - 1) / kChunk;
    const SpTot te = species_pass<0, true, kBlock>(Cw, sE, reg, s, n_e, 0, nch_e, cur_e, cur_i, B, pretest);
    SpTot ti{};
    if (ion_step) ti = species_pass<1, true, kBlock>(Cw, sE, reg, s, n_i, 0, nch_i, cur_i, cur_e, B, pretest);
    if (threadIdx.x == 0) {
      int64_t* ctr = Cw->ctr;
      ctr[kCollE] += te.v[kRecColl];
      ctr[kIoniz] += te.v[kRecIoniz];
      ctr[kAbsEPow] += te.v[kRecAbsPow];
      ctr[kAbsEGnd] += te.v[kRecAbsGnd];
      ctr[kPstepE] += te.v[kRecLive];
      ctr[kCollI] += ti.v[kRecColl];
      ctr[kAbsIPow] += ti.v[kRecAbsPow];
      ctr[kAbsIGnd] += ti.v[kRecAbsGnd];
      ctr[kPstepI] += ti.v[kRecLive];
      const int64_t ge = te.v[kRecBornE] + ti.v[kRecBornE], gi = te.v[kRecBornI] + ti.v[kRecBornI];
      ctr[kLiveE] += ge - te.v[kRecAbsPow] - te.v[kRecAbsGnd];
      ctr[kLiveI] += gi - ti.v[kRecAbsPow] - ti.v[kRecAbsGnd];
      const int64_t dropped = te.v[kRecDropped] + ti.v[kRecDropped];
      if (dropped) {
        ctr[kDropped] += dropped;
        Cw->error = 1;
      }
      sState[0] = s + 1;
      sState[1] = n_e + ge;
      sState[2] = n_i + gi;
      sState[3] = cur_e;
      sState[4] = cur_i;
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    Cw->step = sState[0];
    Cw->n[0] = Cw->alloc[0] = sState[1];
    Cw->n[1] = Cw->alloc[1] = sState[2];
    Cw->cur[0] = (int32_t)sState[3];
    Cw->cur[1] = (int32_t)sState[4];
  }
}

__global__ void k_seed(CaseDev* __restrict__ C, int sp, int64_t n, double sigma) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int cur = C->cur[sp];
  double u0, u1, z0, z1, z2;
  uniform2(C->seed, (uint64_t)i, 0u, tag((uint32_t)sp, 1u, 0u), u0, u1);
  normals3(C->seed, (uint64_t)i, 0u, (uint32_t)sp, 1u, 1u, z0, z1, z2);
  G(C->sp[sp].x[cur])[i] = C->L * u0;
  const double vy = sigma * z1, vz = sigma * z2;
  G(C->sp[sp].vx[cur])[i] = sigma * z0;
  G(C->sp[sp].vy[cur])[i] = vy;
  G(C->sp[sp].vz[cur])[i] = vz;
  if (sp == 0) G(C->sp[0].vp2[cur])[i] = float_above(vy * vy + vz * vz);
  G(C->sp[sp].uid[cur])[i] = (uint64_t)i;
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
  const EDP_GLOBAL double* __restrict__ X = G(C->sp[sp].x[cur]);
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



// The sort kernels serve a batch: one role per workgroup (a case's sort
// workgroups, or one per case for the scan and the finish).  A case sorts its
// electrons at steps that are multiples of `every` and its ions at multiples
// of every * N_SUB; the workgroups of a case that is not due return at once,
// so the host launches the four kernels only at steps where some case is due.
constexpr int kSortUnroll = 4;

// Step of a sort launch of a window for role r, and whether species sp of
// its case is due at that step.
__device__ __forceinline__ bool sort_due(const EDP_CONST BlockRole* r, int sp, int every, int dstep, int64_t& s) {
  s = r->step0 + dstep;
  const int64_t per = sp == 0 ? (int64_t)every : (int64_t)every * r->nsub;
  return s % per == 0;
}

__global__ void __launch_bounds__(256) k_sort_hist(const BlockRole* __restrict__ R, int sp, int every, int dstep) {
  extern __shared__ double hsm[];
  const EDP_CONST BlockRole* r = KC(R) + blockIdx.x;
  CaseDev* C = r->c;
  int64_t s;
  if (!sort_due(r, sp, every, dstep, s)) return;
  unsigned int* sC = (unsigned int*)hsm;
  const int ng = C->ng;
  for (int p = threadIdx.x; p < ng; p += blockDim.x) sC[p] = 0;
  __syncthreads();
  const int cur = C->cur[sp];
  const EDP_GLOBAL double* __restrict__ X = G(C->sp[sp].x[cur]);
  const int64_t n = step_slots(KC(C), sp, s);
  const int64_t nb = r->n, per = (n + nb - 1) / nb;
  const int64_t lo = (int64_t)r->j * per, hi = lo + per < n ? lo + per : n;
  const double inv_dx = C->inv_dx;
  // kSortUnroll particles per thread and round: their loads are in flight
  // together
  for (int64_t i0 = lo + threadIdx.x; i0 < hi; i0 += kSortUnroll * kBlock) {
    double x[kSortUnroll];
#pragma unroll
    for (int u = 0; u < kSortUnroll; ++u) {
      const int64_t i = i0 + u * kBlock;
      x[u] = i < hi ? X[i] : __longlong_as_double(0x7FF8000000000000LL);
    }
#pragma unroll
    for (int u = 0; u < kSortUnroll; ++u)
      if (x[u] == x[u]) atomicAdd(&sC[cell_of(x[u], inv_dx, ng)], 1u);
  }
  __syncthreads();
  for (int p = threadIdx.x; p < ng - 1; p += blockDim.x)
    if (sC[p]) gl_add(&C->sort_cnt[p], (long long)sC[p]);
}

// Exclusive scan of the ng-1 cell counts (one workgroup); total -> sort_cnt[ng].
__global__ void __launch_bounds__(1024) k_sort_scan(const BlockRole* __restrict__ R, int sp, int every, int dstep) {
  __shared__ int64_t sRed[64];
  const EDP_CONST BlockRole* r = KC(R) + blockIdx.x;
  CaseDev* C = r->c;
  int64_t s;
  if (!sort_due(r, sp, every, dstep, s)) return;
  const int m = C->ng - 1;
  const int t = threadIdx.x, T = blockDim.x;
  const int per = (m + T - 1) / T;
  const int lo = t * per < m ? t * per : m, hi = lo + per < m ? lo + per : m;
  int64_t acc = 0;
  for (int p = lo; p < hi; ++p) acc += C->sort_cnt[p];
  int64_t total;
  int64_t run = block_exclusive_scan_t<int64_t>(acc, sRed, &total);
  if (t == 0) C->sort_cnt[C->ng] = total;
  for (int p = lo; p < hi; ++p) {
    const int64_t v = C->sort_cnt[p];
    C->sort_cnt[p] = run;
    run += v;
  }
}

__global__ void __launch_bounds__(256) k_sort_scatter(const BlockRole* __restrict__ R, int sp, int every,
                                                      int dstep) {
  extern __shared__ double ssm[];
  const EDP_CONST BlockRole* r = KC(R) + blockIdx.x;
  CaseDev* C = r->c;
  int64_t s;
  if (!sort_due(r, sp, every, dstep, s)) return;
  unsigned int* sC = (unsigned int*)ssm;
  unsigned long long* sB = (unsigned long long*)(ssm + (C->ng + 1) / 2);
  const int ng = C->ng;
  for (int p = threadIdx.x; p < ng; p += blockDim.x) sC[p] = 0;
  __syncthreads();
  const int cur = C->cur[sp], nxt = cur ^ 1;
  const SpeciesDev& S = C->sp[sp];
  const EDP_GLOBAL double* __restrict__ X = G(S.x[cur]);
  const int64_t n = step_slots(KC(C), sp, s);
  const int64_t nb = r->n, per = (n + nb - 1) / nb;
  const int64_t lo = (int64_t)r->j * per, hi = lo + per < n ? lo + per : n;
  const double inv_dx = C->inv_dx;
  for (int64_t i0 = lo + threadIdx.x; i0 < hi; i0 += kSortUnroll * kBlock) {
    double x[kSortUnroll];
#pragma unroll
    for (int u = 0; u < kSortUnroll; ++u) {
      const int64_t i = i0 + u * kBlock;
      x[u] = i < hi ? X[i] : __longlong_as_double(0x7FF8000000000000LL);
    }
#pragma unroll
    for (int u = 0; u < kSortUnroll; ++u)
      if (x[u] == x[u]) atomicAdd(&sC[cell_of(x[u], inv_dx, ng)], 1u);
  }
  __syncthreads();
  for (int p = threadIdx.x; p < ng - 1; p += blockDim.x) {
    const unsigned int c = sC[p];
    sB[p] = c ? gl_fetch_add(&C->sort_cnt[p], (unsigned long long)c) : 0ull;
    sC[p] = 0;
  }
  __syncthreads();
  const EDP_GLOBAL double* __restrict__ VX = G(S.vx[cur]);
  const EDP_GLOBAL double* __restrict__ VY = G(S.vy[cur]);
  const EDP_GLOBAL double* __restrict__ VZ = G(S.vz[cur]);
  const EDP_GLOBAL uint64_t* __restrict__ UID = G(S.uid[cur]);
  EDP_GLOBAL double* __restrict__ X2 = G(S.x[nxt]);
  EDP_GLOBAL double* __restrict__ VX2 = G(S.vx[nxt]);
  EDP_GLOBAL double* __restrict__ VY2 = G(S.vy[nxt]);
  EDP_GLOBAL double* __restrict__ VZ2 = G(S.vz[nxt]);
  EDP_GLOBAL uint64_t* __restrict__ UID2 = G(S.uid[nxt]);
  // electrons also carry vy*vy + vz*vz: formed again from the moved vy and
  // vz, as every writer forms it, rather than read
  const bool p2 = sp == 0;
  EDP_GLOBAL float* __restrict__ VP22 = G(S.vp2[nxt]);
  for (int64_t i0 = lo + threadIdx.x; i0 < hi; i0 += kSortUnroll * kBlock) {
    double x[kSortUnroll], vx[kSortUnroll], vy[kSortUnroll], vz[kSortUnroll];
    uint64_t uid[kSortUnroll];
#pragma unroll
    for (int u = 0; u < kSortUnroll; ++u) {
      const int64_t i = i0 + u * kBlock;
      x[u] = __longlong_as_double(0x7FF8000000000000LL);
      if (i < hi) {
        x[u] = X[i];
        vx[u] = VX[i];
        vy[u] = VY[i];
        vz[u] = VZ[i];
        uid[u] = UID[i];
      }
    }
#pragma unroll
    for (int u = 0; u < kSortUnroll; ++u) {
      if (!(x[u] == x[u])) continue;
      const int c = cell_of(x[u], inv_dx, ng);
      const int64_t d = (int64_t)sB[c] + atomicAdd(&sC[c], 1u);
      X2[d] = x[u];
      VX2[d] = vx[u];
      VY2[d] = vy[u];
      VZ2[d] = vz[u];
      UID2[d] = uid[u];
      if (p2) VP22[d] = float_above(vy[u] * vy[u] + vz[u] * vz[u]);
    }
  }
}

__global__ void k_sort_finish(const BlockRole* __restrict__ R, int sp, int every, int dstep) {
  const EDP_CONST BlockRole* r = KC(R) + blockIdx.x;
  CaseDev* C = r->c;
  int64_t s;
  if (!sort_due(r, sp, every, dstep, s)) return;
  const int ng = C->ng;
  if (threadIdx.x == 0) {
    // the step's slot count: the live particles, now in the other set
    C->nbase[sp][(s + 2) % 3] = C->sort_cnt[ng];
    C->born[sp][(s + 2) % 3] = 0;
    C->cur[sp] ^= 1;
  }
  __syncthreads();
  for (int p = threadIdx.x; p <= ng; p += blockDim.x) C->sort_cnt[p] = 0;
}

// Fold the pending per-step diagnostic sums of the last completed step.
__global__ void k_fold_diag(CaseDev* __restrict__ Cw) {
  const EDP_CONST CaseDev* __restrict__ C = KC(Cw);
  const int ng = C->ng;
  const int64_t s = Cw->step;  // next step to run; the pending sums are those of s-1
  const int64_t off = ((s + 2) % 3) * ng;
  if (!(C->flags & (kDiagCurrent | kDiagMeanE | kDiagXT))) return;
  const int64_t nt = C->nt, nxb = C->n_xt_bin;
  const size_t plane = (size_t)C->n_xt * (size_t)ng;
  const size_t row_prev = (C->flags & kDiagXT) ? (size_t)(((s + nt - 1) % nt) / nxb) * (size_t)ng : 0;
  for (int p = threadIdx.x; p < ng; p += blockDim.x) fold_particle_sums(C, p, off, row_prev, plane);
}

__global__ void k_zero(int64_t* __restrict__ p, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0;
}

// ---------------------------------------------------------------------------
// Host-side launchers (same translation unit as the kernels).
// ---------------------------------------------------------------------------
// Static LDS of a species' particle kernel: the candidate segments with
// their payload, plus a bound on the counters, the totals, a round's
// colliders and the field scan's scratch.
size_t particle_static_lds(int sp) {
  const size_t waves = kPartBlock / kWave;
  return (sp == 0 ? waves * kSegE * (4 + 8 + 8) : waves * kSegI * 4) + kMaxPb * 8 + 2048;
}

size_t particle_lds_bytes(int ng, uint32_t flags, int n_eepf, int n_ifed, int sp) {
  size_t doubles = (size_t)2 * ng;
  if (flags & kDiagParticle) {
    doubles += (size_t)3 * ng + (sp == 0 && (flags & kDiagXT) ? (size_t)ng : 0);
    const size_t hist = sp == 0 ? ((flags & kDiagEepf) ? (size_t)n_eepf : 0)
                                : ((flags & kDiagIfed) ? 2 * (size_t)(n_ifed + 1) : 0);
    doubles += (hist + 1) / 2;
  }
  return doubles * 8;
}

// One species of a window step of a batch: `blocks` workgroups with their
// roles; `lds` = the largest per-case need; mode 1: the Thomas solve.  With
// ev0/ev1 the launch records its own start and end (the dispatch's
// timestamps, not those of separate event packets around it).
template <int SP, int MODE>
void launch_particles_t(const BlockRole* roles, int blocks, size_t lds, int dstep, int pretest, hipStream_t st, hipEvent_t ev0,
                        hipEvent_t ev1) {
  if (ev0)
    hipExtLaunchKernelGGL((k_particles<SP, MODE>), dim3(blocks), dim3(kPartBlock), lds, st, ev0, ev1, 0, roles, dstep,
                          pretest);
  else
    hipLaunchKernelGGL((k_particles<SP, MODE>), dim3(blocks), dim3(kPartBlock), lds, st, roles, dstep, pretest);
}

hipError_t launch_particles(const BlockRole* roles, int sp, int blocks, size_t lds, int mode, int dstep, int pretest,
                            hipStream_t st, hipEvent_t ev0, hipEvent_t ev1) {
  switch (sp * 2 + (mode == 1)) {
    case 0: launch_particles_t<0, 0>(roles, blocks, lds, dstep, pretest, st, ev0, ev1); break;
    case 1: launch_particles_t<0, 1>(roles, blocks, lds, dstep, pretest, st, ev0, ev1); break;
    case 2: launch_particles_t<1, 0>(roles, blocks, lds, dstep, pretest, st, ev0, ev1); break;
    default: launch_particles_t<1, 1>(roles, blocks, lds, dstep, pretest, st, ev0, ev1); break;
  }
  return hipGetLastError();
}

// The first and last kernels of a lockstep window (see k_window_begin and
// k_window_end): `roles` the group's nroles roles, `cases` its ncase case
// roles.
hipError_t launch_window_begin(BlockRole* roles, int nroles, const BlockRole* cases, int ncase, hipStream_t st) {
  const int blocks = ncase + (nroles + kBlock - 1) / kBlock;
  hipLaunchKernelGGL(k_window_begin, dim3(blocks), dim3(kBlock), 0, st, roles, nroles, cases, ncase);
  return hipGetLastError();
}

hipError_t launch_window_end(const BlockRole* cases, int ncase, int steps, hipStream_t st) {
  hipLaunchKernelGGL(k_window_end, dim3(ncase), dim3(kBlock), 0, st, cases, steps);
  return hipGetLastError();
}

// Resident workgroups per CU of a species' particle kernel with `lds` bytes
// of dynamic LDS.
int particle_occupancy(int sp, size_t lds) {
  int nb = 0;
  const hipError_t e = sp == 0 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_particles<0, 0>, kPartBlock, lds)
                               : hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_particles<1, 0>, kPartBlock, lds);
  return e == hipSuccess && nb > 0 ? nb : 1;
}

// Dynamic LDS of the small-case kernel for a case: E, then the largest of
// either species' particle region (which also holds the field solve's
// scratch and the sort's counters).
size_t small_lds_bytes(int ng, uint32_t flags, int n_eepf, int n_ifed) {
  size_t region = (size_t)ng;
  for (int sp = 0; sp < 2; ++sp) {
    const size_t r = particle_lds_bytes(ng, flags, n_eepf, n_ifed, sp) / 8 - (size_t)ng;
    region = region > r ? region : r;
  }
  return ((size_t)ng + region) * 8;
}

size_t small_static_lds() {
  const size_t waves = kBlock / kWave;
  return waves * kSegE * (4 + 8 + 8) + waves * kSegI * 4 + 2 * kMaxPb * 8 + 6144;
}

// One window of the small cases: workgroup b runs the case of roles[b] for
// roles[b].j steps.
hipError_t launch_small(const BlockRole* roles, int ncase, size_t lds, int mode, int sort_every, int pretest,
                        hipStream_t st) {
  if (mode == 1)
    hipLaunchKernelGGL(k_small<1>, dim3(ncase), dim3(kBlock), lds, st, roles, sort_every, pretest);
  else
    hipLaunchKernelGGL(k_small<0>, dim3(ncase), dim3(kBlock), lds, st, roles, sort_every, pretest);
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

// Compaction + cell sort of species sp for every case of a batch that is due
// (see sort_due): `blocks` workgroups with roles `roles` for the histogram
// and the scatter, one per case (`case_roles`, ncase of them) for the scan
// and the finish; `max_ng` sizes the LDS.
hipError_t launch_sort(const BlockRole* roles, const BlockRole* case_roles, int sp, int blocks, int ncase, int max_ng,
                       int every, int dstep, hipStream_t st) {
  hipLaunchKernelGGL(k_sort_hist, dim3(blocks), dim3(256), (size_t)max_ng * 4, st, roles, sp, every, dstep);
  hipLaunchKernelGGL(k_sort_scan, dim3(ncase), dim3(1024), 0, st, case_roles, sp, every, dstep);
  const size_t lds = (size_t)((max_ng + 1) / 2) * 8 + (size_t)max_ng * 8;
  hipLaunchKernelGGL(k_sort_scatter, dim3(blocks), dim3(256), lds, st, roles, sp, every, dstep);
  hipLaunchKernelGGL(k_sort_finish, dim3(ncase), dim3(1024), 0, st, case_roles, sp, every, dstep);
  return hipGetLastError();
}

hipError_t launch_fold(CaseDev* d, hipStream_t st) {
  hipLaunchKernelGGL(k_fold_diag, dim3(1), dim3(1024), 0, st, d);
  return hipGetLastError();
}

}  // namespace edp
