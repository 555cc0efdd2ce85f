// HIP kernels of the PIC/MCC time step for gfx950.
//
// One step s of a case (section 2.1; Algorithms 2-6):
//   k_head       workgroup 0: fixed-point densities -> rho -> the discrete
//                Poisson equation -> grid field E; the other workgroups
//                finish the collisions of step s-1 (new velocities).
//   k_particles  every particle of a species: gather E, leapfrog push, wall
//                absorption, the collision test and process selection with
//                ionization births, and the deposit of the new position for
//                step s+1 -- fused, so each particle's state is streamed
//                from HBM once per step.
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
// Step 2: density -> rho -> potential -> field, one workgroup per case.
// MODE 0 (default) solves the discrete Poisson equation through the fluxes
// F_q = phi_q - phi_{q+1}: each row of the equation says F_p - F_{p-1} = d_p
// with d_p = rho_p dx^2/eps0, so F_p = F_0 + S_p with S_p the prefix sum of
// d, and the fluxes add up to phi_0 - phi_{N-1} = V, which fixes
// F_0 = (V - sum_p S_p)/(N_g - 1).  The field follows from the fluxes
// without forming phi: E_p = (F_{p-1} + F_p)/(2 dx) inside, and the boundary
// forms use F_0 and F_{N_g-2}.  This is the same linear system as the Thomas
// algorithm solves, in parallel (two wave scans instead of 2 N_g dependent
// steps); it agrees with an 80-bit solution to ~1e-15 of the field scale,
// closer than the sequential sweep.
// MODE 1 runs the Thomas algorithm itself in one thread, operation for
// operation as the sequential definition (bit-reproducible, slow).
// ---------------------------------------------------------------------------
constexpr int kWave = 64;

// Fold the per-step particle sums of one node (ring slot `fold`, the step
// before the one about to run) into the time sums and, with the xt arrays,
// into time-bin row `row_prev`; the power density j E takes the field that
// step used, still in efield[] (it is overwritten later in the same thread).
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

// Interior rows per lane of the flux scan at the largest grid.
constexpr int kScanRows = (kMaxNodes - 2 + kWave - 1) / kWave;

template <int MODE>
__device__ __forceinline__ void field_solve(CaseDev* __restrict__ Cw, double* fsm) {
  const EDP_CONST CaseDev* __restrict__ C = KC(Cw);
  const int ng = C->ng;
  // LDS rows padded by one slot per 16 nodes (node p at lp(p)): the flux
  // scan's lanes own 16-node blocks, which would otherwise fall on the same
  // banks
  const int np = ng + (ng >> 4) + 1;
  auto lp = [](int p) { return p + (p >> 4); };
  double* sRho = fsm;
  double* sPhi = fsm + np;    // MODE 1: d then phi; MODE 0: S_p then fluxes F_q
  double* sR = fsm + 2 * np;  // MODE 1: Thomas reciprocals
  const int64_t s = C->step;
  const int nsub = C->nsub;
  const int64_t k = s / nsub;
  const bool ion_step = (s % nsub) == 0;
  const uint32_t fl = C->flags;
  const EDP_GLOBAL int64_t* cntE = G(C->cnt_e + (s % 3) * ng);
  const EDP_GLOBAL int64_t* cntI = G(C->cnt_i + (k % 3) * ng);
  EDP_GLOBAL int64_t* zeroE = G(C->cnt_e + ((s + 2) % 3) * ng);
  EDP_GLOBAL int64_t* zeroI = G(C->cnt_i + ((k + 2) % 3) * ng);
  const int64_t fold = ((s + 2) % 3) * ng;  // per-step sums of step s-1
  const double scale = C->dens_scale;
  const double V = G(C->volt)[s % kVoltChunk];
  // xt rows: this step's grid values go to its time bin, the particle sums
  // of step s-1 to the bin of s-1
  const bool xt = (fl & kDiagXT) != 0;
  const int64_t nt = C->nt, nxb = C->n_xt_bin;
  const size_t plane = (size_t)C->n_xt * (size_t)ng;
  const size_t row = xt ? (size_t)((s % nt) / nxb) * (size_t)ng : 0;
  const size_t row_prev = xt ? (size_t)(((s + nt - 1) % nt) / nxb) * (size_t)ng : 0;
  EDP_GLOBAL double* __restrict__ X = G(C->xt);
  // every load of the thread's nodes before any store (one memory round trip)
  int64_t ce[kGridPerThread], ci[kGridPerThread];
#pragma unroll
  for (int j = 0; j < kGridPerThread; ++j) {
    const int p = threadIdx.x + j * kBlock;
    ce[j] = p < ng ? cntE[p] : 0;
    ci[j] = p < ng ? cntI[p] : 0;
  }
#pragma unroll
  for (int j = 0; j < kGridPerThread; ++j) {
    const int p = threadIdx.x + j * kBlock;
    if (p >= ng) break;
    double ne = (double)ce[j] * scale;
    double ni = (double)ci[j] * scale;
    if (p == 0 || p == ng - 1) {
      ne *= 2.0;
      ni *= 2.0;
    }
    const double rho = kECharge * (ni - ne);
    sRho[lp(p)] = rho;
    if (MODE == 1) {
      sR[lp(p)] = G(C->rden)[p];
      sPhi[lp(p)] = rho * C->kpois;  // right-hand side d_p (boundary term below)
    }
    if (fl & kDiagDensity) {
      G(C->sum_ne)[p] += ne;
      G(C->sum_ni)[p] += ni;
    }
    zeroE[p] = 0;
    if (ion_step) zeroI[p] = 0;
    if (fl & (kDiagCurrent | kDiagMeanE | kDiagXT)) fold_particle_sums(C, p, fold, row_prev, plane);
    if (xt) {
      X[kXtNe * plane + row + p] += ne;
      X[kXtNi * plane + row + p] += ni;
    }
  }
  __syncthreads();
  const double dx = C->dx;
  if (MODE == 1) {
    if (threadIdx.x == 0) {
      // Thomas algorithm: forward sweep y_p = (d_p + y_{p-1}) r_p, back
      // substitution phi_p = y_p + r_p phi_{p+1}.
      const int m = ng - 2;
      double prev = 0.0;
      for (int p = 1; p <= m; ++p) {
        double d = sPhi[lp(p)];
        if (p == 1) d = d + V;
        prev = (d + prev) * sR[lp(p)];
        sPhi[lp(p)] = prev;
      }
      for (int p = m - 1; p >= 1; --p) sPhi[lp(p)] = sPhi[lp(p)] + sR[lp(p)] * sPhi[lp(p + 1)];
      sPhi[lp(0)] = V;
      sPhi[lp(ng - 1)] = 0.0;
    }
    __syncthreads();
    for (int p = threadIdx.x; p < ng; p += blockDim.x) {
      double e;
      if (p == 0)
        e = (sPhi[lp(0)] - sPhi[lp(1)]) / dx - sRho[lp(0)] * dx / (2.0 * kEps0);
      else if (p == ng - 1)
        e = (sPhi[lp(ng - 2)] - sPhi[lp(ng - 1)]) / dx + sRho[lp(ng - 1)] * dx / (2.0 * kEps0);
      else
        e = (sPhi[lp(p - 1)] - sPhi[lp(p + 1)]) / (2.0 * dx);
      G(C->efield)[p] = e;
      G(C->phi)[p] = sPhi[lp(p)];
      G(C->rho)[p] = sRho[lp(p)];
      if (xt) {
        X[kXtEf * plane + row + p] += e;
        X[kXtFlux * plane + row + p] += p < ng - 1 ? sPhi[lp(p)] - sPhi[lp(p + 1)] : V;
      }
    }
  } else {
    // One wave does the two scans (no workgroup barriers in between): lane l
    // owns the contiguous rows q0 <= q < q1 of the m = N_g - 2 interior rows
    // (row q is node q+1), and node q+1's slot becomes F_{q+1}.  A lane's
    // rows stay in registers between one batch of LDS loads and one of
    // stores.
    if (threadIdx.x < kWave) {
      const int lane = (int)threadIdx.x;
      const int m = ng - 2;
      const double kp = C->kpois;
      const int R = (m + kWave - 1) / kWave;  // <= kScanRows
      const int q0 = lane * R < m ? lane * R : m;
      const int nq = (q0 + R < m ? q0 + R : m) - q0;
      double v[kScanRows];
#pragma unroll
      for (int t = 0; t < kScanRows; ++t) v[t] = t < nq ? sRho[lp(q0 + t + 1)] : 0.0;
      double acc = 0.0;
#pragma unroll
      for (int t = 0; t < kScanRows; ++t) {
        if (t < nq) acc += v[t] * kp;
        v[t] = acc;  // prefix within the lane
      }
      double inc = acc;
#pragma unroll
      for (int off = 1; off < kWave; off <<= 1) {
        const double y = __shfl_up(inc, off, kWave);
        if (lane >= off) inc += y;
      }
      const double before = inc - acc;
      double mine = 0.0;
#pragma unroll
      for (int t = 0; t < kScanRows; ++t) {
        v[t] = before + v[t];  // S_q
        if (t < nq) mine += v[t];
      }
      for (int off = kWave / 2; off > 0; off >>= 1) mine += __shfl_xor(mine, off, kWave);
      const double F0 = (V - mine) / (double)(ng - 1);
#pragma unroll
      for (int t = 0; t < kScanRows; ++t)
        if (t < nq) sPhi[lp(q0 + t + 1)] = F0 + v[t];
      if (lane == 0) sPhi[lp(0)] = F0;
    }
    __syncthreads();
    for (int p = threadIdx.x; p < ng; p += blockDim.x) {
      double e;
      if (p == 0)
        e = sPhi[lp(0)] / dx - sRho[lp(0)] * dx / (2.0 * kEps0);
      else if (p == ng - 1)
        e = sPhi[lp(ng - 2)] / dx + sRho[lp(ng - 1)] * dx / (2.0 * kEps0);
      else
        e = (sPhi[lp(p - 1)] + sPhi[lp(p)]) / (2.0 * dx);
      G(C->efield)[p] = e;
      const double f = p < ng - 1 ? sPhi[lp(p)] : V;  // last slot keeps V for phi on demand
      G(C->flux)[p] = f;
      G(C->rho)[p] = sRho[lp(p)];
      if (xt) {
        X[kXtEf * plane + row + p] += e;
        X[kXtFlux * plane + row + p] += f;
      }
    }
  }
  if (threadIdx.x == 0) {
    if (xt) {
      G(C->xt_cnt)[row / ng] += 1;
      if (ion_step) G(C->xt_cnt)[C->n_xt + row / ng] += 1;
    }
    Cw->phi_valid = MODE == 1;
    Cw->pstep = s;  // the particle kernels of this step read it
  }
}

// The same solve for a workgroup that keeps E of step s in its own LDS (sE)
// instead of handing it to other launches, with the step given: the
// persistent small-case kernel below, where the step changes inside the
// launch.  fsm: two padded rows of scratch.  The writer also stores rho, E
// and the fluxes (or phi) for reads, clears the deposit rings the next steps
// refill, folds the per-step diagnostics and counts the step.
template <int MODE>
__device__ __forceinline__ void field_to_lds(CaseDev* __restrict__ Cw, double* sE, double* fsm, const bool writer,
                                             const int64_t s) {
  const EDP_CONST CaseDev* __restrict__ C = KC(Cw);
  const int ng = C->ng;
  // LDS rows padded by one slot per 16 nodes (node p at lp(p)): the flux
  // scan's lanes own 16-node blocks, which would otherwise fall on the same
  // banks
  const int np = ng + (ng >> 4) + 1;
  auto lp = [](int p) { return p + (p >> 4); };
  double* sRho = fsm;
  double* sPhi = fsm + np;  // MODE 1: d then phi; MODE 0: S_p then fluxes F_q
  const int nsub = C->nsub;
  const int64_t k = s / nsub;
  const bool ion_step = (s % nsub) == 0;
  const uint32_t fl = C->flags;
  const EDP_GLOBAL int64_t* cntE = G(C->cnt_e + (s % 3) * ng);
  const EDP_GLOBAL int64_t* cntI = G(C->cnt_i + (k % 3) * ng);
  EDP_GLOBAL int64_t* zeroE = G(C->cnt_e + ((s + 2) % 3) * ng);
  EDP_GLOBAL int64_t* zeroI = G(C->cnt_i + ((k + 2) % 3) * ng);
  const int64_t fold = ((s + 2) % 3) * ng;  // per-step sums of step s-1
  const double scale = C->dens_scale;
  const double V = G(C->volt)[s % kVoltChunk];
  // xt rows: this step's grid values go to its time bin, the particle sums
  // of step s-1 to the bin of s-1
  const bool xt = writer && (fl & kDiagXT) != 0;
  const int64_t nt = C->nt, nxb = C->n_xt_bin;
  const size_t plane = (size_t)C->n_xt * (size_t)ng;
  const size_t row = xt ? (size_t)((s % nt) / nxb) * (size_t)ng : 0;
  const size_t row_prev = xt ? (size_t)(((s + nt - 1) % nt) / nxb) * (size_t)ng : 0;
  EDP_GLOBAL double* __restrict__ X = G(C->xt);
  // every load of the thread's nodes before any store (one memory round trip)
  int64_t ce[kGridPerThread], ci[kGridPerThread];
#pragma unroll
  for (int j = 0; j < kGridPerThread; ++j) {
    const int p = threadIdx.x + j * kBlock;
    ce[j] = p < ng ? cntE[p] : 0;
    ci[j] = p < ng ? cntI[p] : 0;
  }
#pragma unroll
  for (int j = 0; j < kGridPerThread; ++j) {
    const int p = threadIdx.x + j * kBlock;
    if (p >= ng) break;
    double ne = (double)ce[j] * scale;
    double ni = (double)ci[j] * scale;
    if (p == 0 || p == ng - 1) {
      ne *= 2.0;
      ni *= 2.0;
    }
    const double rho = kECharge * (ni - ne);
    sRho[lp(p)] = rho;
    if (MODE == 1) sPhi[lp(p)] = rho * C->kpois;  // right-hand side d_p (boundary term below)
    if (writer) {
      if (fl & kDiagDensity) {
        G(C->sum_ne)[p] += ne;
        G(C->sum_ni)[p] += ni;
      }
      zeroE[p] = 0;
      if (ion_step) zeroI[p] = 0;
      if (fl & (kDiagCurrent | kDiagMeanE | kDiagXT)) fold_particle_sums(C, p, fold, row_prev, plane);
      if (xt) {
        X[kXtNe * plane + row + p] += ne;
        X[kXtNi * plane + row + p] += ni;
      }
    }
  }
  __syncthreads();
  const double dx = C->dx;
  if (MODE == 1) {
    if (threadIdx.x == 0) {
      // Thomas algorithm: forward sweep y_p = (d_p + y_{p-1}) r_p, back
      // substitution phi_p = y_p + r_p phi_{p+1}, with the reciprocals r_p
      // precomputed on the host
      const EDP_GLOBAL double* __restrict__ rd = G(C->rden);
      const int m = ng - 2;
      double prev = 0.0;
      for (int p = 1; p <= m; ++p) {
        double d = sPhi[lp(p)];
        if (p == 1) d = d + V;
        prev = (d + prev) * rd[p];
        sPhi[lp(p)] = prev;
      }
      for (int p = m - 1; p >= 1; --p) sPhi[lp(p)] = sPhi[lp(p)] + rd[p] * sPhi[lp(p + 1)];
      sPhi[lp(0)] = V;
      sPhi[lp(ng - 1)] = 0.0;
    }
    __syncthreads();
    for (int p = threadIdx.x; p < ng; p += blockDim.x) {
      double e;
      if (p == 0)
        e = (sPhi[lp(0)] - sPhi[lp(1)]) / dx - sRho[lp(0)] * dx / (2.0 * kEps0);
      else if (p == ng - 1)
        e = (sPhi[lp(ng - 2)] - sPhi[lp(ng - 1)]) / dx + sRho[lp(ng - 1)] * dx / (2.0 * kEps0);
      else
        e = (sPhi[lp(p - 1)] - sPhi[lp(p + 1)]) / (2.0 * dx);
      sE[p] = e;
      if (writer) {
        G(C->efield)[p] = e;
        G(C->phi)[p] = sPhi[lp(p)];
        G(C->rho)[p] = sRho[lp(p)];
        if (xt) {
          X[kXtEf * plane + row + p] += e;
          X[kXtFlux * plane + row + p] += p < ng - 1 ? sPhi[lp(p)] - sPhi[lp(p + 1)] : V;
        }
      }
    }
  } else {
    // One wave does the two scans (no workgroup barriers in between): lane l
    // owns the contiguous rows q0 <= q < q1 of the m = N_g - 2 interior rows
    // (row q is node q+1), and node q+1's slot becomes F_{q+1}.  A lane's
    // rows stay in registers between one batch of LDS loads and one of
    // stores.
    if (threadIdx.x < kWave) {
      const int lane = (int)threadIdx.x;
      const int m = ng - 2;
      const double kp = C->kpois;
      const int R = (m + kWave - 1) / kWave;  // <= kScanRows
      const int q0 = lane * R < m ? lane * R : m;
      const int nq = (q0 + R < m ? q0 + R : m) - q0;
      double v[kScanRows];
#pragma unroll
      for (int t = 0; t < kScanRows; ++t) v[t] = t < nq ? sRho[lp(q0 + t + 1)] : 0.0;
      double acc = 0.0;
#pragma unroll
      for (int t = 0; t < kScanRows; ++t) {
        if (t < nq) acc += v[t] * kp;
        v[t] = acc;  // prefix within the lane
      }
      double inc = acc;
#pragma unroll
      for (int off = 1; off < kWave; off <<= 1) {
        const double y = __shfl_up(inc, off, kWave);
        if (lane >= off) inc += y;
      }
      const double before = inc - acc;
      double mine = 0.0;
#pragma unroll
      for (int t = 0; t < kScanRows; ++t) {
        v[t] = before + v[t];  // S_q
        if (t < nq) mine += v[t];
      }
      for (int off = kWave / 2; off > 0; off >>= 1) mine += __shfl_xor(mine, off, kWave);
      const double F0 = (V - mine) / (double)(ng - 1);
#pragma unroll
      for (int t = 0; t < kScanRows; ++t)
        if (t < nq) sPhi[lp(q0 + t + 1)] = F0 + v[t];
      if (lane == 0) sPhi[lp(0)] = F0;
    }
    __syncthreads();
    for (int p = threadIdx.x; p < ng; p += blockDim.x) {
      double e;
      if (p == 0)
        e = sPhi[lp(0)] / dx - sRho[lp(0)] * dx / (2.0 * kEps0);
      else if (p == ng - 1)
        e = sPhi[lp(ng - 2)] / dx + sRho[lp(ng - 1)] * dx / (2.0 * kEps0);
      else
        e = (sPhi[lp(p - 1)] + sPhi[lp(p)]) / (2.0 * dx);
      sE[p] = e;
      if (writer) {
        G(C->efield)[p] = e;
        const double f = p < ng - 1 ? sPhi[lp(p)] : V;  // last slot keeps V for phi on demand
        G(C->flux)[p] = f;
        G(C->rho)[p] = sRho[lp(p)];
        if (xt) {
          X[kXtEf * plane + row + p] += e;
          X[kXtFlux * plane + row + p] += f;
        }
      }
    }
  }
  if (writer && threadIdx.x == 0) {
    if (xt) {
      G(C->xt_cnt)[row / ng] += 1;
      if (ion_step) G(C->xt_cnt)[C->n_xt + row / ng] += 1;
    }
    Cw->phi_valid = MODE == 1;
    Cw->diag_steps += 1;
    if (ion_step) Cw->diag_ion_steps += 1;
  }
  __syncthreads();  // sE complete; fsm free again
}

// ---------------------------------------------------------------------------
// Collisions (step 6).  The particle kernel tests every particle, picks the
// process of those that collide (partition of [0,1) into sigma_k/sigma_tot),
// deposits the charge of the particles an ionization creates, and queues the
// event in its chunk's part of the queue.  The new velocities -- COM
// kinematics, scattering angles, Euler rotation, the ionization energy
// split -- and the newborns' slots are computed from the queue by extra
// workgroups of the next step's field launch (they do not depend on each
// other), so this long transcendental code runs off the streaming path and
// overlaps the field solve.
// ---------------------------------------------------------------------------

// Arrays the collision workgroups touch, loaded once per workgroup.
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
__device__ __forceinline__ ScatterPtrs scatter_ptrs(CaseDev* __restrict__ Cw) {
  const EDP_CONST CaseDev* __restrict__ C = KC(Cw);
  return scatter_ptrs_at(Cw, C->cur[0], C->cur[1]);
}

// Electron-Ar scattering of queued particle i (state after the push) by
// process proc (0 elastic, 1 excitation, 2 ionization).  An ionization also
// writes its newborns: the ejected electron at slot be and the ion at slot
// bi (-1: dropped at capacity), both at the parent's position.
// electron_scatter_at takes the particle's state (velocity after the push,
// identity, position) from the caller; electron_scatter loads it.
__device__ __forceinline__ void electron_scatter_at(const EDP_CONST CaseDev* __restrict__ C, const ScatterPtrs& P,
                                                    int64_t i, int proc, int64_t be, int64_t bi, int64_t s,
                                                    double vxn, double vy, double vz, uint64_t uid, double x) {
  const uint64_t seed = C->seed;
  const uint32_t st = (uint32_t)s;
  // squared speed, the squares summed from x to z as the collision test does
  const double v2 = vxn * vxn + vy * vy + vz * vz;
  const double v = sqrt(v2);
  double r_chi, r_eta;
  uniform2(seed, uid, st, tag(0, 0, 1), r_chi, r_eta);
  const double f1 = kEMass / (kEMass + kArMass);
  const double f2 = kArMass / (kEMass + kArMass);
  const double wx = f1 * vxn, wy = f1 * vy, wz = f1 * vz;
  const double eta = kTwoPi * r_eta;
  // the frame of g and the azimuth are the same for every process: computed
  // once, outside the branch, so that a wave holding both an ionization and
  // other events runs them once (the results are those of the same
  // operations taken per process)
  const Frame F = frame_of(vxn, vy, vz, v);
  double cos_eta, sin_eta;
  sincos(eta, &sin_eta, &cos_eta);
  double gnew, cos_chi, sin_chi;
  if (proc < 2) {
    gnew = v;
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
    // Every draw of the ionization -- the energy share and the new ion's
    // thermal velocity -- is taken before the dependent chains, and only the
    // stores are conditional, so that the independent chains overlap (an
    // ionization is the longest event of the queue).
    double r_share, r_unused;
    uniform2(seed, uid, st, tag(0, 0, 2), r_share, r_unused);
    const uint64_t cu = child_uid(uid, s, 2);
    double z0, z1, z2;
    normals3(seed, cu, st, 1u, 2u, 1u, z0, z1, z2);
    double cos_eta2, sin_eta2;
    sincos(eta + kPi, &sin_eta2, &cos_eta2);
    double e_ev = 0.5 * kMuEAr * v2 / kEvToJ - C->thr_ion;
    if (e_ev < 0.0) {
      e_ev = 0.0;
      gl_add(P.anomaly, 1);
    }
    const double w_ion = C->w_ion;
    const double e_ej = w_ion * tan(r_share * atan(e_ev / (2.0 * w_ion)));
    const double e_sc = e_ev - e_ej;
    const double g_sc = sqrt(2.0 * e_sc * kEvToJ / kMuEAr);
    const double g_ej = sqrt(2.0 * e_ej * kEvToJ / kMuEAr);
    double cs_sc, sn_sc, cs_ej, sn_ej;
    if (C->flags & kIonizLiteral) {
      const double chi_sc = e_ev > 0.0 ? sqrt(e_sc / e_ev) : 0.0;
      const double chi_ej = e_ev > 0.0 ? sqrt(e_ej / e_ev) : 0.0;
      sincos(chi_sc, &sn_sc, &cs_sc);
      sincos(chi_ej, &sn_ej, &cs_ej);
    } else {
      cs_sc = e_ev > 0.0 ? sqrt(e_sc / e_ev) : 1.0;
      cs_ej = e_ev > 0.0 ? sqrt(e_ej / e_ev) : 1.0;
      sn_sc = sqrt(1.0 - cs_sc * cs_sc);
      sn_ej = sqrt(1.0 - cs_ej * cs_ej);
    }
    // the scattered electron is rotated below with the other processes; the
    // ejected one, scattered about the same w, here
    gnew = g_sc;
    cos_chi = cs_sc;
    sin_chi = sn_sc;
    double ex_, ey_, ez_;
    rotate(F, g_ej, f2, cs_ej, sn_ej, cos_eta2, sin_eta2, wx, wy, wz, ex_, ey_, ez_);
    if (be >= 0) {
      P.ex[be] = x;
      P.evx[be] = ex_;
      P.evy[be] = ey_;
      P.evz[be] = ez_;
      P.evp2[be] = float_above(ey_ * ey_ + ez_ * ez_);
      P.euid[be] = child_uid(uid, s, 1);
    }
    if (bi >= 0) {  // the new ion: a thermal gas velocity
      const double sa = C->sigma_a;
      P.ix[bi] = x;
      P.ivx[bi] = sa * z0;
      P.ivy[bi] = sa * z1;
      P.ivz[bi] = sa * z2;
      P.iuid[bi] = cu;
    }
  }
  double ox, oy, oz;
  rotate(F, gnew, f2, cos_chi, sin_chi, cos_eta, sin_eta, wx, wy, wz, ox, oy, oz);
  P.evx[i] = ox;
  P.evy[i] = oy;
  P.evz[i] = oz;
  P.evp2[i] = float_above(oy * oy + oz * oz);
}
__device__ __forceinline__ void electron_scatter(const EDP_CONST CaseDev* __restrict__ C, const ScatterPtrs& P, int64_t i,
                                                 int proc, int64_t be, int64_t bi, int64_t s) {
  electron_scatter_at(C, P, i, proc, be, bi, s, P.evx[i], P.evy[i], P.evz[i], P.euid[i], proc == 2 ? P.ex[i] : 0.0);
}

// Ar+ + Ar scattering of queued ion i (proc 0 isotropic, 1 backward) with the
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
__device__ __forceinline__ void ion_scatter(const EDP_CONST CaseDev* __restrict__ C, const ScatterPtrs& P, int64_t i, int proc,
                                            int64_t s) {
  ion_scatter_at(C, P, i, proc, s, P.ivx[i], P.ivy[i], P.ivz[i], P.iuid[i]);
}

// Secondary electron of queued ion i, absorbed at electrode `side` (0 at
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
__device__ __forceinline__ void see_emit(const EDP_CONST CaseDev* __restrict__ C, const ScatterPtrs& P, int64_t i,
                                         int side, int64_t be, int64_t s) {
  if (be < 0) return;
  see_emit_at(C, P, P.iuid[i], side, be, s);
}

typedef int rec4 __attribute__((ext_vector_type(4)));  // per-workgroup queue record

// Apply the pending collision queue.  Every particle workgroup of the last
// step left one event list (in its chunk range of the queue) and a record
// {events, births, absorbed at x=0, absorbed at x=L}; an event is
// slot | process << 32 | birth rank in the list << 34.  Workgroup blk of
// nblk takes a contiguous range of those lists, a group of LANES lanes one
// list (events carry their birth ranks, so any lane can take any event: more
// lanes per list shorten long lists, fewer serve more lists per workgroup).
// Newborns of list j go to q_base + (births of the lists before j) + rank;
// secondary electrons of ion impacts (ion events of process 2, 3) follow
// every electron birth of the step.  No atomics: every slot follows from the
// records alone.
template <int LANES>
__device__ __forceinline__ void apply_queue(CaseDev* __restrict__ Cw, int blk, int nblk) {
  static_assert(LANES >= 1 && LANES <= kWave && kBlock % LANES == 0, "collision workgroup shape");
  constexpr int kApplyLanes = LANES;
  constexpr int kApplyGroups = kBlock / LANES;  // lists per round of a workgroup
  __shared__ int64_t sRed[64];
  const EDP_CONST CaseDev* __restrict__ C = KC(Cw);
  const int64_t s = C->q_step;
  const ScatterPtrs P = scatter_ptrs(Cw);
  const int grp = (int)threadIdx.x / kApplyLanes, l = (int)threadIdx.x % kApplyLanes;
  const int64_t base_e = C->q_base[0], base_i = C->q_base[1];
  const int64_t cap_e = C->sp[0].cap, cap_i = C->sp[1].cap;
  const bool see_on = C->see_on != 0;
  // no pending queue: no lists (a value, not an early exit, so that every
  // field of the case is loaded in one round trip)
  const bool valid = C->q_valid != 0;
  for (int sp = 0; sp < 2; ++sp) {
    const int64_t per = valid ? C->q_per[sp] : 0;
    const int64_t nwg = per > 0 ? (C->q_nblk[sp] + per - 1) / per : 0;
    const int64_t j0 = nwg * blk / nblk, j1 = nwg * (blk + 1) / nblk;
    if (j0 >= j1) continue;  // uniform
    const EDP_GLOBAL rec4* __restrict__ wg = (const EDP_GLOBAL rec4*)G(C->q_wg[sp]);
    const EDP_GLOBAL int64_t* __restrict__ ent = G(C->cq_ent[sp]);
    const bool births = sp == 0 || see_on;
    int64_t zrun = 0;  // births before the current round
    for (int64_t jb = j0; jb < j1; jb += kApplyGroups) {
      const bool first = jb == j0;
      const int64_t jj = jb + grp;
      const bool valid = jj < j1;
      rec4 r = {0, 0, 0, 0};
      int64_t code0 = 0;
      const EDP_GLOBAL int64_t* __restrict__ e = ent + jj * per * kChunk;
      if (valid) {
        // the first event of this lane is loaded with the record, not after
        // it (a list region holds at least kChunk entries; unused ones are
        // ignored below)
        r = wg[jj];
        code0 = e[l];
      }
      int64_t zbase = 0;
      if (births) {
        // first round: the births of the lists before this range (for ions,
        // after every electron birth), loads all in flight together and
        // summed in the same scan as the round's births (low and high word;
        // both totals stay below 2^31)
        int64_t zp = 0;
        if (first) {
#pragma unroll 8
          for (int64_t k = threadIdx.x; k < j0; k += kBlock) zp += wg[k].y;
          if (sp == 1) {
            const int64_t pe = C->q_per[0];
            const int64_t nwe = pe > 0 ? (C->q_nblk[0] + pe - 1) / pe : 0;
            const EDP_GLOBAL rec4* __restrict__ wge = (const EDP_GLOBAL rec4*)G(C->q_wg[0]);
#pragma unroll 8
            for (int64_t k = threadIdx.x; k < nwe; k += kBlock) zp += wge[k].y;
          }
        }
        int64_t tot;
        const int64_t exc = block_exclusive_scan_t<int64_t>(((int64_t)(l == 0 ? r.y : 0) << 32) | zp, sRed, &tot);
        if (first) zrun = tot & 0xFFFFFFFFLL;
        zbase = zrun + (__shfl(exc, 0, kApplyLanes) >> 32);  // births of the lower groups of this round
        zrun += tot >> 32;
      }
      for (int k = l; k < r.x; k += kApplyLanes) {
        const int64_t code = k == l ? code0 : e[k];
        const int64_t i = code & 0xFFFFFFFFLL;
        const int proc = (int)((code >> 32) & 3);
        const int64_t kk = zbase + (code >> 34);
        if (sp == 0) {
          int64_t be = -1, bi = -1;
          if (proc == 2) {
            if (base_e + kk < cap_e) be = base_e + kk;
            if (base_i + kk < cap_i) bi = base_i + kk;
          }
          electron_scatter(C, P, i, proc, be, bi, s);
        } else if (proc < 2) {
          ion_scatter(C, P, i, proc, s);
        } else {  // 2, 3: absorbed at x = 0 / x = L with an emitted electron
          see_emit(C, P, i, proc - 2, base_e + kk < cap_e ? base_e + kk : -1, s);
        }
      }
    }
  }
}

// Add the totals of the last particle step to the counters and place its
// newborns (one workgroup): the particle workgroups' records give collisions,
// births and absorptions; the newborns occupy q_base + [0, births) up to the
// capacity, births being ionizations plus, for electrons, the secondaries of
// ion impacts (ion records count those as events and births).
__device__ __forceinline__ void fold_queue(CaseDev* __restrict__ Cw) {
  __shared__ int64_t sRed[64];
  const EDP_CONST CaseDev* __restrict__ C = KC(Cw);
  int64_t v[2][4] = {{0, 0, 0, 0}, {0, 0, 0, 0}};
  for (int sp = 0; sp < 2; ++sp) {
    const int64_t per = C->q_per[sp];
    const int64_t nwg = per > 0 ? (C->q_nblk[sp] + per - 1) / per : 0;
    const EDP_GLOBAL rec4* wg = (const EDP_GLOBAL rec4*)G(C->q_wg[sp]);
#pragma unroll 4
    for (int64_t k = threadIdx.x; k < nwg; k += blockDim.x) {
      const rec4 t = wg[k];
      v[sp][0] += t.x;
      v[sp][1] += t.y;
      v[sp][2] += t.z;
      v[sp][3] += t.w;
    }
  }
  // two sums per scan word (each total is at most the slot count, < 2^31)
  int64_t t[4];
  (void)block_exclusive_scan_t<int64_t>((v[0][0] << 32) | v[0][1], sRed, &t[0]);
  (void)block_exclusive_scan_t<int64_t>((v[0][2] << 32) | v[0][3], sRed, &t[1]);
  (void)block_exclusive_scan_t<int64_t>((v[1][0] << 32) | v[1][2], sRed, &t[2]);
  (void)block_exclusive_scan_t<int64_t>((v[1][1] << 32) | v[1][3], sRed, &t[3]);
  if (threadIdx.x == 0) {
    const int64_t coll_e = t[0] >> 32, z = t[0] & 0xFFFFFFFFLL;
    const int64_t ap_e = t[1] >> 32, ag_e = t[1] & 0xFFFFFFFFLL;
    const int64_t see = t[3] >> 32, ag_i = t[3] & 0xFFFFFFFFLL;
    const int64_t coll_i = (t[2] >> 32) - see, ap_i = t[2] & 0xFFFFFFFFLL;
    const int64_t base_e = C->q_base[0], base_i = C->q_base[1];
    const int64_t room_e = C->sp[0].cap - base_e, room_i = C->sp[1].cap - base_i;
    const int64_t ze = z + see;
    const int64_t ok_e = ze < room_e ? ze : (room_e > 0 ? room_e : 0);
    const int64_t ok_i = z < room_i ? z : (room_i > 0 ? room_i : 0);
    Cw->alloc[0] = Cw->n[0] = base_e + ok_e;
    Cw->alloc[1] = Cw->n[1] = base_i + ok_i;
    Cw->ctr[kCollE] += coll_e;
    Cw->ctr[kCollI] += coll_i;
    Cw->ctr[kIoniz] += z;
    Cw->ctr[kAbsEPow] += ap_e;
    Cw->ctr[kAbsEGnd] += ag_e;
    Cw->ctr[kAbsIPow] += ap_i;
    Cw->ctr[kAbsIGnd] += ag_i;
    Cw->ctr[kLiveE] += ok_e - ap_e - ag_e;
    Cw->ctr[kLiveI] += ok_i - ap_i - ag_i;
    if (ok_e < ze || ok_i < z) {
      Cw->ctr[kDropped] += (ze - ok_e) + (z - ok_i);
      Cw->error = 1;
    }
  }
}

// Head of step s for every case of the batch.  Workgroups [0, nc) solve the
// fields, the next na apply the queues of step s-1 (a range per case), the
// last nc fold each queue's totals into the counters and do the step's
// bookkeeping.  R: one role per workgroup.
template <int MODE, int LANES>
__global__ void __launch_bounds__(kBlock) k_head(const BlockRole* __restrict__ R, int nc, int na) {
  extern __shared__ double hsm[];
  const int bid = (int)blockIdx.x;
  const EDP_CONST BlockRole* r = KC(R) + bid;
  CaseDev* C = r->c;
  if (bid < nc) {
    field_solve<MODE>(C, hsm);
    return;
  }
  if (bid < nc + na) {
    apply_queue<LANES>(C, r->j, r->n);
    return;
  }
  if (C->q_valid) fold_queue(C);
  if (threadIdx.x == 0) {
    const int64_t s = C->step;
    const bool ion_step = (s % C->nsub) == 0;
    C->ctr[kPstepE] += C->ctr[kLiveE];
    if (ion_step) C->ctr[kPstepI] += C->ctr[kLiveI];
    C->diag_steps += 1;
    if (ion_step) C->diag_ion_steps += 1;
  }
}

// Apply the pending queue before the host looks at the state (the last
// workgroup folds the totals).
__global__ void __launch_bounds__(kBlock) k_drain(CaseDev* __restrict__ C) {
  apply_queue<kWave>(C, (int)blockIdx.x, (int)gridDim.x);
}
__global__ void __launch_bounds__(kBlock) k_drain_done(CaseDev* __restrict__ C) {
  if (C->q_valid) fold_queue(C);
  __syncthreads();
  if (threadIdx.x == 0) C->q_valid = 0;
}

// ---------------------------------------------------------------------------
// Steps 3-6 for one species plus the deposit for step s+1.
//
// A case's particle slots are cut into chunks of kChunk = 256 slots; wave w
// of a workgroup owns slots [c*256 + 64w, c*256 + 64w + 64) of chunk c, one
// per lane.  The case gets a fixed number of workgroups (its share, by
// expected particle count, of the resident slots the batch uses); workgroup
// j takes the contiguous chunk range [j*per, (j+1)*per) with per computed
// from the live slot count at run time, so the launch shape never depends
// on the count,
// every workgroup does the same amount of work, and E is loaded and the
// deposit flushed once per workgroup.
//
// Every particle: gather E from LDS, leapfrog, wall test, deposit the new x
// into the workgroup's LDS histogram, store x and v_x, and one Philox call
// for its collision uniform R.  Only R below a bound of the collision
// probability over the tables (the null-collision P*, with a relative
// margin for the direct test), or a speed beyond the range that bound
// covers, can give a collision; such candidates (a few percent) go to the
// wave's LDS segment and everyone else is done.  The candidates get the
// exact test -- energy bin, table lookups, exp, for ions the thermal target
// first -- in dense passes: all of the workgroup's at the end as one list,
// or a wave's own when its segment fills.  So the table work and the
// transcendentals run on full waves instead of on every wave with one
// candidate lane.  An ionization adds its newborns' charge (the electron a
// second share at the parent's x, the ion to the next ion step's density).
// Colliders are appended to the workgroup's event list (one LDS atomic per
// wave) and the workgroup writes one record {events, births, absorbed at
// x=0, absorbed at x=L}.  There are no global returning atomics and no
// counter shared between workgroups.
//
// Dynamic LDS: E[ng] double, H[ng] deposit; with particle diagnostics also
// J[ng], W[ng], En[ng] (int64) and EEPF[n_eepf] (uint32).  Static: the
// candidate segments (ions 4 KiB of slots; electrons 10 KiB of slots, v^2
// and uids) and a few counters.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int lane_rank(uint64_t mask) {
  // set bits of mask below this lane
  return (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

// Candidate segment entries per wave of a particle workgroup.
// Candidate segment per wave: ions keep the slot only (their exact test
// reloads the state); electrons keep the slot, v^2 and uid, which is all
// their exact test needs, so it reads nothing back from HBM.
constexpr int kSegI = 256;
constexpr int kSegE = 128;
template <int SP>
constexpr int seg_len() { return SP == 0 ? kSegE : kSegI; }

// Event of a particle step: slot | process << 32 | birth rank << 34.
__device__ __forceinline__ int64_t event_code(int64_t i, int proc, int64_t brank) {
  return i | ((int64_t)proc << 32) | (brank << 34);
}

// Append one wave's events (lanes with ev) to its workgroup's list; list
// positions and birth ranks come from the workgroup's LDS counters, one
// atomic per wave.  Called by every lane of the wave.
__device__ __forceinline__ void push_events(bool ev, bool birth, int64_t i, int proc, int* sCnt,
                                            EDP_GLOBAL int64_t* ent, int lane) {
  const uint64_t me = __ballot(ev);
  if (me == 0) return;
  const uint64_t mb = __ballot(birth);
  int e0 = 0, b0 = 0;
  if (lane == 0) {
    e0 = atomicAdd(&sCnt[0], (int)__popcll(me));
    if (mb) b0 = atomicAdd(&sCnt[1], (int)__popcll(mb));
  }
  e0 = __shfl(e0, 0);
  b0 = __shfl(b0, 0);
  if (ev) ent[e0 + lane_rank(me)] = event_code(i, proc, birth ? b0 + lane_rank(mb) : 0);
}

template <int SP>
__device__ __forceinline__ void particles_block(CaseDev* __restrict__ Cw, const double* __restrict__ efield,
                                                const int ng, const int j, const int nwg) {
  const EDP_CONST CaseDev* __restrict__ C = KC(Cw);
  extern __shared__ double psm[];
  // candidate segments (one per wave; electrons with v^2 and uid), their
  // fill, the workgroup's event and birth counters, the per-wave absorption
  // totals
  constexpr int kSeg = seg_len<SP>();
  constexpr int kPay = SP == 0 ? kBlock / kWave : 1;
  __shared__ int32_t sSeg[kBlock / kWave][kSeg];
  __shared__ double sVx[kPay][SP == 0 ? kSeg : 1];
  __shared__ uint64_t sUid[kPay][SP == 0 ? kSeg : 1];
  __shared__ int sNc[kBlock / kWave];
  __shared__ int sCnt[2];
  __shared__ int sAbs[kBlock / kWave][2];
  // E into LDS first: its address and size come with the workgroup's role,
  // so these loads go out with those of the case block (a workgroup with no
  // work this step returns below, after the barrier)
  double* sE = psm;
  {
    double ev[kGridPerThread];
#pragma unroll
    for (int q = 0; q < kGridPerThread; ++q) {
      const int p = threadIdx.x + q * kBlock;
      ev[q] = p < ng ? G(efield)[p] : 0.0;
    }
#pragma unroll
    for (int q = 0; q < kGridPerThread; ++q) {
      const int p = threadIdx.x + q * kBlock;
      if (p < ng) sE[p] = ev[q];
    }
  }
  const int64_t s = C->pstep;
  const int64_t n = C->n[SP];
  if (SP == 1 && (s % C->nsub) != 0) return;  // ions move on ion steps only
  const int64_t nch = (n + kChunk - 1) / kChunk;
  if (j == 0 && threadIdx.x == 0) {
    // this step's queue: read by the next head (or a drain)
    Cw->q_step = s;
    Cw->q_base[SP] = n;
    Cw->q_nblk[SP] = (int32_t)nch;
    if (SP == 0) {
      Cw->q_base[1] = C->n[1];
      Cw->q_nblk[1] = 0;  // set by the ion kernel on ion steps
      Cw->q_valid = 1;
      Cw->step = s + 1;
    }
  }
  const int64_t per = (nch + nwg - 1) / nwg;
  if (j == 0 && threadIdx.x == 0) Cw->q_per[SP] = per;
  const int64_t c_lo = (int64_t)j * per;
  const int64_t c_hi = c_lo + per < nch ? c_lo + per : nch;
  if (c_lo >= c_hi) return;  // whole workgroup: nothing to do this step
  const int nsub = C->nsub;
  const int64_t kion = s / nsub;
  const uint32_t fl = C->flags;
  const bool pdiag = (fl & kDiagParticle) != 0;
  const bool xt = (fl & kDiagXT) != 0;
  const int n_eepf = C->n_eepf;
  const int n_ifed = C->n_ifed;
  // histogram: the EEPF for electrons, the IFEDF of both electrodes for ions
  const int n_hist = SP == 0 ? ((fl & kDiagEepf) ? n_eepf : 0) : ((fl & kDiagIfed) ? 2 * (n_ifed + 1) : 0);
  unsigned long long* sH = (unsigned long long*)(psm + ng);
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
  if (threadIdx.x < 2) sCnt[threadIdx.x] = 0;
  __syncthreads();

  const int cur = C->cur[SP];
  EDP_GLOBAL double* __restrict__ X = G(C->sp[SP].x[cur]);
  EDP_GLOBAL double* __restrict__ VX = G(C->sp[SP].vx[cur]);
  const EDP_GLOBAL double* __restrict__ VY = G(C->sp[SP].vy[cur]);
  const EDP_GLOBAL double* __restrict__ VZ = G(C->sp[SP].vz[cur]);
  const EDP_GLOBAL uint64_t* __restrict__ UID = G(C->sp[SP].uid[cur]);
  // electrons: a float bound of vy*vy + vz*vz per slot, read in place of vy
  // and vz for the pre-test (those only by the candidates' exact test and the
  // measurement sums)
  const EDP_GLOBAL float* __restrict__ VP2 = G(C->sp[SP].vp2[cur]);
  // this workgroup's event list: its chunk range of the queue
  EDP_GLOBAL int64_t* __restrict__ ENT = G(C->cq_ent[SP]) + c_lo * kChunk;
  const int64_t base_slot = c_lo * kChunk;
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
  const double de_cs = C->de_cs;
  const int nbins = C->nbins;
  const uint64_t seed = C->seed;
  const uint32_t st = (uint32_t)s;
  const double x_lo = C->x_lo, x_hi = C->x_hi, de_eepf = C->de_eepf, de_ifed = C->de_ifed;
  const double sa = C->sigma_a;
  const bool null_coll = (fl & kNullCollision) != 0;
  // surface processes of this species' electrode hits
  const bool surf_on = SP == 0 ? C->refl_on != 0 : C->see_on != 0;
  const double p_surf0 = SP == 0 ? C->eta_refl[0] : C->gamma_see[0];
  const double p_surf1 = SP == 0 ? C->eta_refl[1] : C->gamma_see[1];
  int64_t* const cnt_e_next = C->cnt_e + ((s + 1) % 3) * ng;
  const double n_gas = C->n_gas;
  const double nu_star = SP == 0 ? C->nu_star_e : C->nu_star_i;
  const double p_null = SP == 0 ? C->p_null_e : C->p_null_i;
  // candidate pre-test: R below this bound, or a speed beyond the bound's range
  const double p_cand = null_coll ? p_null : (SP == 0 ? C->p_bound_e : C->p_bound_i);
  const double v2_cand = null_coll ? __builtin_huge_val() : (SP == 0 ? C->v2_lim_e : C->g2_lim_i);
  const double a2_i = C->a2_i;
  const uint32_t r_tag = SP == 0 ? tag(0, 0, 0) : tag(1, 0, 2);
  const int w = (int)threadIdx.x / kWave, lane = (int)threadIdx.x % kWave;
  int tap = 0, tag_ = 0;  // this wave's absorptions over the workgroup's chunks
  int ncw = 0;             // entries in this wave's candidate segment

  // Step 6 for candidates, in dense passes: entry k of `count` (k = first,
  // first + stride, ...; the loop bound is uniform over the participating
  // waves) is the particle at slot base_slot + list(k).  The exact test
  // (direct: P = 1 - exp(-n sigma_tot g dt), collide iff R < P, process by
  // sigma_k / sigma_tot; null collision: process by R nu* against the
  // cumulative nu_k, the rest null), then an ionization's newborn charge and
  // the events of the colliders.
  auto process = [&](const bool wg_list, const int count, const int first, const int stride) {
    for (int b0 = 0; b0 < count; b0 += stride) {
      const int k = b0 + first;
      const bool act = k < count;
      int64_t i = 0;
      double vxn = 0.0, vy = 0.0, vz = 0.0;
      uint64_t uid = 0;
      if (act) {
        int sg = w, kk = k;
        if (wg_list) {  // the workgroup's segments, one after another
          sg = 0;
          while (kk >= sNc[sg]) kk -= sNc[sg++];
        }
        i = base_slot + sSeg[sg][kk];
        if (SP == 0) {
          // the pushed v_x and the uid from the segment, v_y and v_z (not
          // changed by the push) from memory
          vxn = sVx[SP == 0 ? sg : 0][SP == 0 ? kk : 0];
          uid = sUid[SP == 0 ? sg : 0][SP == 0 ? kk : 0];
        } else {
          vxn = VX[i];
          uid = UID[i];
        }
        vy = VY[i];
        vz = VZ[i];
      }
      int proc = -1;
      if (act) {
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
              const double s_el = s_a, s_exc = s_b, s_ion = s_c;
              const double s_tot = s_el + s_exc + s_ion;
              if (!(s_tot > 0.0) || r_proc < s_el / s_tot)
                proc = 0;
              else if (r_proc < (s_el + s_exc) / s_tot)
                proc = 1;
              else
                proc = 2;
            } else {
              const double s_iso = s_a, s_back = s_b;
              proc = (!(s_iso + s_back > 0.0) || r_proc < s_iso / (s_iso + s_back)) ? 0 : 1;
            }
          }
        }
      }
      const bool coll = proc >= 0;
      const bool ioniz = SP == 0 && proc == 2;
      if (ioniz) {
        // the newborns sit at the parent's position: the electron adds a
        // second share to this step's deposit, the ion goes to the next ion
        // step's density
        // (the parent's new x: stored by this workgroup before the fence or
        // barrier that precedes every dense pass; the last pass runs after
        // the histogram's flush and adds the electron's share to global
        // memory)
        long long r;
        const int q = deposit_split(X[i], inv_dx, ng, r);
        if (wg_list) {
          gl_add(&dst[q], 4294967296LL - r);
          gl_add(&dst[q + 1], r);
        } else {
          lds_add(&sH[q], 4294967296LL - r);
          lds_add(&sH[q + 1], r);
        }
        gl_add(&cnt_i_next[q], 4294967296LL - r);
        gl_add(&cnt_i_next[q + 1], r);
      }
      push_events(coll, ioniz, i, proc, sCnt, ENT, lane);
    }
  };

  // The state of chunk c + 1 is loaded before chunk c is worked on, so each
  // wave keeps two chunks' loads in flight (the loop is bound by memory
  // latency, not by its arithmetic).
  const int slot = w * kWave + lane;  // slot in the chunk
  double nx, nvx, nvy, nvz;
  float nvp2;
  uint64_t nuid;
  auto fetch = [&](const int64_t c) {
    const int64_t i = c * kChunk + slot;
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
  fetch(c_lo);
  for (int64_t c = c_lo; c < c_hi; ++c) {
    const int64_t i = c * kChunk + slot;
    const double x = nx, vx = nvx, vy = nvy, vz = nvz, vp2 = (double)nvp2;
    const uint64_t uid = nuid;
    if (c + 1 < c_hi) fetch(c + 1);
    bool live = x == x;  // past the end, or absorbed earlier (tombstone)
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
      // node of the next step's deposit now and whose slot and velocity the
      // next head's queue pass writes.
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
        v2 = SP == 0 ? vxn * vxn + vp2 : vxn * vxn + vy * vy + vz * vz;
        cand = r_coll < p_cand || (SP == 0 ? v2 : 2.0 * (v2 + a2_i)) > v2_cand;
      }
    }
    if (i < n && x == x) {
      X[i] = live ? xn : __longlong_as_double(0x7FF8000000000000LL);
      VX[i] = vxn;
    }
    if (surf_on) {
      // reflections (electrons) or emissions per electrode (ions); an ion's
      // secondary emission is an event of process 2 (x = 0) or 3 (x = L)
      // with one electron birth
      const uint64_t m_s0 = __ballot(surf && (SP == 0 || abs_pow));
      const uint64_t m_s1 = SP == 1 ? __ballot(surf && abs_gnd) : 0ull;
      if (lane == 0 && m_s0) gl_add(&Cw->ctr[SP == 0 ? kRefl : kSeePow], (long long)__popcll(m_s0));
      if (lane == 0 && m_s1) gl_add(&Cw->ctr[kSeeGnd], (long long)__popcll(m_s1));
      if (SP == 1) push_events(surf, surf, i, abs_pow ? 2 : 3, sCnt, ENT, lane);
    }
    const uint64_t m_c = __ballot(cand);
    if (m_c) {
      if (cand) {
        const int at = ncw + lane_rank(m_c);
        sSeg[w][at] = (int32_t)(i - base_slot);
        if (SP == 0) {
          sVx[SP == 0 ? w : 0][SP == 0 ? at : 0] = vxn;
          sUid[SP == 0 ? w : 0][SP == 0 ? at : 0] = uid;
        }
      }
      ncw += __popcll(m_c);
      if (ncw > kSeg - kWave) {
        // a full segment: the wave finishes its own candidates now (the
        // fence makes the other lanes' stores of x and v_x visible)
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "workgroup");
        process(false, ncw, lane, kWave);
        ncw = 0;
      }
    }
    tap += __popcll(__ballot(abs_pow));
    tag_ += __popcll(__ballot(abs_gnd));
  }
  if (lane == 0) {
    sNc[w] = ncw;
    sAbs[w][0] = tap;
    sAbs[w][1] = tag_;
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
  // the remaining candidates of all waves, as one list over the workgroup
  process(true, sNc[0] + sNc[1] + sNc[2] + sNc[3], (int)threadIdx.x, kBlock);
  __syncthreads();
  if (threadIdx.x == 0)
    ((EDP_GLOBAL rec4*)G(Cw->q_wg[SP]))[j] =
        rec4{sCnt[0], sCnt[1], sAbs[0][0] + sAbs[1][0] + sAbs[2][0] + sAbs[3][0],
             sAbs[0][1] + sAbs[1][1] + sAbs[2][1] + sAbs[3][1]};
}

// One launch per species covers the chunks of every case of the batch.
template <int SP>
__global__ void __launch_bounds__(kBlock) k_particles(const BlockRole* __restrict__ R) {
  const EDP_CONST BlockRole* r = KC(R) + blockIdx.x;
  particles_block<SP>(r->c, r->efield, r->ng, r->j, r->n);
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
// the buffer sets live in LDS and are written back at the end (with a
// pending collision queue of the lockstep path applied first).
// ---------------------------------------------------------------------------

// Slots for the newborns of a wave from an LDS counter: lanes with `mine`
// take consecutive slots after base0 (the slot count at the step's start)
// and the step's births so far; -1 past the capacity.
__device__ __forceinline__ int64_t take_slot_lds(bool mine, int* births, int64_t base0, int64_t cap, int lane) {
  const uint64_t m = __ballot(mine);
  if (m == 0) return -1;
  int b = 0;
  if (lane == 0) b = atomicAdd(births, (int)__popcll(m));
  b = __shfl(b, 0);
  const int64_t slot = base0 + (int64_t)b + lane_rank(m);
  return mine && slot < cap ? slot : -1;
}

// Totals of one species' step in a small case (summed over the waves).
struct SmallTot {
  int coll, ioniz, pow, gnd, live;
};

// Steps 3-6 of species SP for the case of this workgroup at step s: slots
// [0, n) of buffer set `cur` (the other species' current set `cur_o`), E in
// sE, `reg` the LDS region for the deposit histogram (and the particle
// diagnostics), sBirth the step's birth counters (electron slots, ion slots)
// after the slot counts n_e0, n_i0 at the step's start.
template <int SP>
__device__ __forceinline__ SmallTot small_species(CaseDev* __restrict__ Cw, const double* sE, double* reg, int64_t s,
                                                  int64_t n, int cur, int cur_o, int64_t n_e0, int64_t n_i0,
                                                  int* sBirth) {
  const EDP_CONST CaseDev* __restrict__ C = KC(Cw);
  constexpr int kSeg = seg_len<SP>();
  constexpr int kPay = SP == 0 ? kBlock / kWave : 1;
  __shared__ int32_t sSeg[kBlock / kWave][kSeg];
  __shared__ double sVx[kPay][SP == 0 ? kSeg : 1];
  __shared__ uint64_t sUid[kPay][SP == 0 ? kSeg : 1];
  __shared__ int sNc[kBlock / kWave];
  __shared__ int sTot[kBlock / kWave][5];
  const int ng = C->ng;
  const int64_t cap_e = C->sp[0].cap, cap_i = C->sp[1].cap;
  const int64_t nch = (n + kChunk - 1) / kChunk;
  const int nsub = C->nsub;
  const int64_t kion = s / nsub;
  const uint32_t fl = C->flags;
  const bool pdiag = (fl & kDiagParticle) != 0;
  const bool xt = (fl & kDiagXT) != 0;
  const int n_eepf = C->n_eepf;
  const int n_ifed = C->n_ifed;
  const int n_hist = SP == 0 ? ((fl & kDiagEepf) ? n_eepf : 0) : ((fl & kDiagIfed) ? 2 * (n_ifed + 1) : 0);
  unsigned long long* sH = (unsigned long long*)reg;
  unsigned long long* sJ = sH + ng;
  unsigned long long* sW = sJ + ng;
  unsigned long long* sEn = sW + ng;
  unsigned long long* sIz = sEn + ng;
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
  __syncthreads();
  EDP_GLOBAL double* __restrict__ X = G(C->sp[SP].x[cur]);
  EDP_GLOBAL double* __restrict__ VX = G(C->sp[SP].vx[cur]);
  const EDP_GLOBAL double* __restrict__ VY = G(C->sp[SP].vy[cur]);
  const EDP_GLOBAL double* __restrict__ VZ = G(C->sp[SP].vz[cur]);
  const EDP_GLOBAL uint64_t* __restrict__ UID = G(C->sp[SP].uid[cur]);
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
  int64_t* const dst = SP == 0 ? C->cnt_e + ((s + 1) % 3) * ng : C->cnt_i + ((kion + 1) % 3) * ng;
  int64_t* const cnt_e_next = C->cnt_e + ((s + 1) % 3) * ng;
  const double de_cs = C->de_cs;
  const int nbins = C->nbins;
  const uint64_t seed = C->seed;
  const uint32_t st = (uint32_t)s;
  const double x_lo = C->x_lo, x_hi = C->x_hi, de_eepf = C->de_eepf, de_ifed = C->de_ifed;
  const double sa = C->sigma_a;
  const bool null_coll = (fl & kNullCollision) != 0;
  const bool surf_on = SP == 0 ? C->refl_on != 0 : C->see_on != 0;
  const double p_surf0 = SP == 0 ? C->eta_refl[0] : C->gamma_see[0];
  const double p_surf1 = SP == 0 ? C->eta_refl[1] : C->gamma_see[1];
  const double n_gas = C->n_gas;
  const double nu_star = SP == 0 ? C->nu_star_e : C->nu_star_i;
  const double p_null = SP == 0 ? C->p_null_e : C->p_null_i;
  const double p_cand = null_coll ? p_null : (SP == 0 ? C->p_bound_e : C->p_bound_i);
  const double v2_cand = null_coll ? __builtin_huge_val() : (SP == 0 ? C->v2_lim_e : C->g2_lim_i);
  const double a2_i = C->a2_i;
  const uint32_t r_tag = SP == 0 ? tag(0, 0, 0) : tag(1, 0, 2);
  const int w = (int)threadIdx.x / kWave, lane = (int)threadIdx.x % kWave;
  int t_coll = 0, t_ioniz = 0, t_pow = 0, t_gnd = 0, t_live = 0;
  int ncw = 0;

  // The exact test of the candidates (as in the lockstep path), then at once
  // the colliders' scattering and an ionization's newborns and their charge.
  auto process = [&](const bool wg_list, const int count, const int first, const int stride) {
    for (int b0 = 0; b0 < count; b0 += stride) {
      const int k = b0 + first;
      const bool act = k < count;
      int64_t i = 0;
      double vxn = 0.0, vy = 0.0, vz = 0.0;
      uint64_t uid = 0;
      if (act) {
        int sg = w, kk = k;
        if (wg_list) {
          sg = 0;
          while (kk >= sNc[sg]) kk -= sNc[sg++];
        }
        i = sSeg[sg][kk];
        if (SP == 0) {
          vxn = sVx[SP == 0 ? sg : 0][SP == 0 ? kk : 0];
          uid = sUid[SP == 0 ? sg : 0][SP == 0 ? kk : 0];
        } else {
          vxn = VX[i];
          uid = UID[i];
        }
        vy = VY[i];
        vz = VZ[i];
      }
      int proc = -1;
      if (act) {
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
            const double v2 = vxn * vxn + vy * vy + vz * vz;
            const double v = sqrt(v2);
            const double energy = 0.5 * kEMass * v2 / kEvToJ;
            idx = energy_bin(energy, de_cs, nbins);
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
      }
      const bool coll = proc >= 0;
      t_coll += __popcll(__ballot(coll));
      if (SP == 0) {
        const bool ioniz = proc == 2;
        double xb = 0.0;
        int64_t be = -1, bi = -1;
        const uint64_t mi = __ballot(ioniz);
        if (mi) {
          t_ioniz += __popcll(mi);
          be = take_slot_lds(ioniz, &sBirth[0], n_e0, cap_e, lane);
          bi = take_slot_lds(ioniz, &sBirth[1], n_i0, cap_i, lane);
          if (ioniz) {
            xb = X[i];
            long long r;
            const int q = deposit_split(xb, inv_dx, ng, r);
            if (wg_list) {
              gl_add(&dst[q], 4294967296LL - r);
              gl_add(&dst[q + 1], r);
            } else {
              lds_add(&sH[q], 4294967296LL - r);
              lds_add(&sH[q + 1], r);
            }
            gl_add(&cnt_i_next[q], 4294967296LL - r);
            gl_add(&cnt_i_next[q + 1], r);
          }
        }
        if (coll) electron_scatter_at(C, P, i, proc, be, bi, s, vxn, vy, vz, uid, xb);
      } else if (coll) {
        ion_scatter_at(C, P, i, proc, s, vxn, vy, vz, uid);
      }
    }
  };

  for (int64_t c = 0; c < nch; ++c) {
    const int slot = w * kWave + lane;
    const int64_t i = c * kChunk + slot;
    double x = __longlong_as_double(0x7FF8000000000000LL), vx = 0.0, vy = 0.0, vz = 0.0, vp2 = 0.0;
    uint64_t uid = 0;
    if (i < n) {
      x = X[i];
      vx = VX[i];
      if (SP == 1 || pdiag) {
        vy = VY[i];
        vz = VZ[i];
      }
      if (SP == 0) vp2 = (double)VP2[i];
      uid = UID[i];
    }
    bool live = x == x;
    t_live += __popcll(__ballot(live));
    bool abs_pow = false, abs_gnd = false, surf = false, cand = false;
    double xn = 0.0, vxn = 0.0, v2 = 0.0;
    if (live) {
      // steps 3-4: field at the particle (section 2.1.3) and leapfrog
      // (section 2.1.4), as in the lockstep kernel
      const double xi = x * inv_dx;
      int cell = (int)xi;
      cell = cell > ng - 2 ? ng - 2 : (cell < 0 ? 0 : cell);
      const double w_lo = (double)(cell + 1) - xi;
      const double w_hi = xi - (double)cell;
      const double e_here = sE[cell] * w_lo + sE[cell + 1] * w_hi;
      vxn = SP == 0 ? vx - e_here * kick : vx + e_here * kick;
      xn = x + vxn * dt;
      if (pdiag) {
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
      // step 5: walls and surface processes, as in the lockstep kernel
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
        long long r;
        const int q = deposit_split(xn, inv_dx, ng, r);
        lds_add(&sH[q], 4294967296LL - r);
        lds_add(&sH[q + 1], r);
        double r_coll, r_proc;
        uniform2(seed, uid, st, r_tag, r_coll, r_proc);
        v2 = SP == 0 ? vxn * vxn + vp2 : vxn * vxn + vy * vy + vz * vz;
        cand = r_coll < p_cand || (SP == 0 ? v2 : 2.0 * (v2 + a2_i)) > v2_cand;
      }
    }
    if (i < n && x == x) {
      X[i] = live ? xn : __longlong_as_double(0x7FF8000000000000LL);
      VX[i] = vxn;
    }
    if (surf_on) {
      const uint64_t m_s0 = __ballot(surf && (SP == 0 || abs_pow));
      const uint64_t m_s1 = SP == 1 ? __ballot(surf && abs_gnd) : 0ull;
      if (lane == 0 && m_s0) gl_add(&Cw->ctr[SP == 0 ? kRefl : kSeePow], (long long)__popcll(m_s0));
      if (lane == 0 && m_s1) gl_add(&Cw->ctr[kSeeGnd], (long long)__popcll(m_s1));
      if (SP == 1 && (m_s0 | m_s1)) {
        // a secondary electron takes its slot after this step's births so far
        const int64_t be = take_slot_lds(surf, &sBirth[0], n_e0, cap_e, lane);
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
      ncw += __popcll(m_c);
      if (ncw > kSeg - kWave) {
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "workgroup");
        process(false, ncw, lane, kWave);
        ncw = 0;
      }
    }
    t_pow += __popcll(__ballot(abs_pow));
    t_gnd += __popcll(__ballot(abs_gnd));
  }
  if (lane == 0) sNc[w] = ncw;
  __syncthreads();
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
  process(true, sNc[0] + sNc[1] + sNc[2] + sNc[3], (int)threadIdx.x, kBlock);
  if (lane == 0) {
    sTot[w][0] = t_coll;
    sTot[w][1] = t_ioniz;
    sTot[w][2] = t_pow;
    sTot[w][3] = t_gnd;
    sTot[w][4] = t_live;
  }
  __syncthreads();
  SmallTot T{0, 0, 0, 0, 0};
  for (int v = 0; v < kBlock / kWave; ++v) {
    T.coll += sTot[v][0];
    T.ioniz += sTot[v][1];
    T.pow += sTot[v][2];
    T.gnd += sTot[v][3];
    T.live += sTot[v][4];
  }
  __syncthreads();  // sTot and the segments are free for the next call
  return T;
}

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
// b by role.j steps.  Dynamic LDS: E, then the largest of the field solve's
// two padded rows, the particle phase's histograms and the sort's counters.
template <int MODE>
__global__ void __launch_bounds__(kBlock) k_small(const BlockRole* __restrict__ R, int sort_every) {
  extern __shared__ double ssm2[];
  __shared__ int64_t sState[6];  // step, n_e, n_i, cur_e, cur_i, spare
  __shared__ int sBirth[2];
  const EDP_CONST BlockRole* r = KC(R) + blockIdx.x;
  CaseDev* Cw = r->c;
  const int steps = r->j;
  const EDP_CONST CaseDev* __restrict__ C = KC(Cw);
  const int ng = C->ng;
  const int nsub = C->nsub;
  double* sE = ssm2;
  double* reg = ssm2 + ng;
  // a collision queue the lockstep path left pending is applied first
  if (Cw->q_valid) {
    apply_queue<kWave>(Cw, 0, 1);
    __syncthreads();
    fold_queue(Cw);
    __syncthreads();
    if (threadIdx.x == 0) Cw->q_valid = 0;
  }
  if (threadIdx.x == 0) {
    // vector loads (the scalar cache does not see this launch's stores)
    auto ld = [](const int64_t* a) { return __hip_atomic_load(a, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP); };
    auto ld32 = [](const int32_t* a) { return __hip_atomic_load(a, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP); };
    sState[0] = ld(&Cw->step);
    sState[1] = ld(&Cw->n[0]);
    sState[2] = ld(&Cw->n[1]);
    sState[3] = ld32(&Cw->cur[0]);
    sState[4] = ld32(&Cw->cur[1]);
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
    field_to_lds<MODE>(Cw, sE, reg, true, s);
    const SmallTot te = small_species<0>(Cw, sE, reg, s, n_e, cur_e, cur_i, n_e, n_i, sBirth);
    SmallTot ti{0, 0, 0, 0, 0};
    if (ion_step) ti = small_species<1>(Cw, sE, reg, s, n_i, cur_i, cur_e, n_e, n_i, sBirth);
    if (threadIdx.x == 0) {
      int64_t* ctr = Cw->ctr;
      ctr[kCollE] += te.coll;
      ctr[kIoniz] += te.ioniz;
      ctr[kAbsEPow] += te.pow;
      ctr[kAbsEGnd] += te.gnd;
      ctr[kPstepE] += te.live;
      ctr[kCollI] += ti.coll;
      ctr[kAbsIPow] += ti.pow;
      ctr[kAbsIGnd] += ti.gnd;
      ctr[kPstepI] += ti.live;
      const int64_t be = sBirth[0], bi = sBirth[1];
      const int64_t room_e = C->sp[0].cap - n_e, room_i = C->sp[1].cap - n_i;
      const int64_t ge = be < room_e ? be : (room_e > 0 ? room_e : 0);
      const int64_t gi = bi < room_i ? bi : (room_i > 0 ? room_i : 0);
      ctr[kLiveE] += ge - te.pow - te.gnd;
      ctr[kLiveI] += gi - ti.pow - ti.gnd;
      if (ge < be || gi < bi) {
        ctr[kDropped] += (be - ge) + (bi - gi);
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

__device__ __forceinline__ bool sort_due(const CaseDev* C, int sp, int every) {
  const EDP_CONST CaseDev* K = KC(C);
  const int64_t per = sp == 0 ? (int64_t)every : (int64_t)every * K->nsub;
  return K->step % per == 0;
}

__global__ void __launch_bounds__(256) k_sort_hist(const BlockRole* __restrict__ R, int sp, int every) {
  extern __shared__ double hsm[];
  const EDP_CONST BlockRole* r = KC(R) + blockIdx.x;
  CaseDev* C = r->c;
  if (!sort_due(C, sp, every)) return;
  unsigned int* sC = (unsigned int*)hsm;
  const int ng = C->ng;
  for (int p = threadIdx.x; p < ng; p += blockDim.x) sC[p] = 0;
  __syncthreads();
  const int cur = C->cur[sp];
  const EDP_GLOBAL double* __restrict__ X = G(C->sp[sp].x[cur]);
  const int64_t n = slots(C, sp);
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
__global__ void __launch_bounds__(1024) k_sort_scan(const BlockRole* __restrict__ R, int sp, int every) {
  __shared__ int64_t sRed[64];
  CaseDev* C = (KC(R) + blockIdx.x)->c;
  if (!sort_due(C, sp, every)) return;
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

__global__ void __launch_bounds__(256) k_sort_scatter(const BlockRole* __restrict__ R, int sp, int every) {
  extern __shared__ double ssm[];
  const EDP_CONST BlockRole* r = KC(R) + blockIdx.x;
  CaseDev* C = r->c;
  if (!sort_due(C, sp, every)) return;
  unsigned int* sC = (unsigned int*)ssm;
  unsigned long long* sB = (unsigned long long*)(ssm + (C->ng + 1) / 2);
  const int ng = C->ng;
  for (int p = threadIdx.x; p < ng; p += blockDim.x) sC[p] = 0;
  __syncthreads();
  const int cur = C->cur[sp], nxt = cur ^ 1;
  const SpeciesDev& S = C->sp[sp];
  const EDP_GLOBAL double* __restrict__ X = G(S.x[cur]);
  const int64_t n = slots(C, sp);
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

__global__ void k_sort_finish(const BlockRole* __restrict__ R, int sp, int every) {
  CaseDev* C = (KC(R) + blockIdx.x)->c;
  if (!sort_due(C, sp, every)) return;
  const int ng = C->ng;
  if (threadIdx.x == 0) {
    C->alloc[sp] = C->sort_cnt[ng];
    C->n[sp] = C->sort_cnt[ng];  // the step's snapshot, taken before the sort
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
// their payload, plus a bound on the small per-wave counters.
size_t particle_static_lds(int sp) {
  const size_t waves = kBlock / kWave;
  return sp == 0 ? waves * kSegE * (4 + 8 + 8) + 256 : waves * kSegI * 4 + 256;
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

// Head of a batch step: ncase field workgroups, `apply_blocks` collision
// workgroups in total and ncase totals workgroups, with their roles in this
// order.  `max_ng` sizes the field workgroups' LDS; `lanes` (16, 32, 64) per
// event list in the collision workgroups.
hipError_t launch_head(const BlockRole* roles, int ncase, int apply_blocks, int max_ng, int mode, int lanes,
                       hipStream_t st) {
  const size_t lds = (size_t)(max_ng + (max_ng >> 4) + 1) * 24;  // three padded rows
  const dim3 grid(2 * ncase + apply_blocks);
#define EDP_HEAD(M, LN) hipLaunchKernelGGL((k_head<M, LN>), grid, dim3(kBlock), lds, st, roles, ncase, apply_blocks)
  switch (lanes * 2 + (mode == 1)) {
    case 32: EDP_HEAD(0, 16); break;
    case 33: EDP_HEAD(1, 16); break;
    case 64: EDP_HEAD(0, 32); break;
    case 65: EDP_HEAD(1, 32); break;
    case 128: EDP_HEAD(0, 64); break;
    case 129: EDP_HEAD(1, 64); break;
    default: return hipErrorInvalidValue;
  }
#undef EDP_HEAD
  return hipGetLastError();
}

hipError_t launch_drain(CaseDev* d, int blocks, hipStream_t st) {
  hipLaunchKernelGGL(k_drain, dim3(blocks), dim3(kBlock), 0, st, d);
  hipLaunchKernelGGL(k_drain_done, dim3(1), dim3(kBlock), 0, st, d);
  return hipGetLastError();
}

// One species of a batch: `blocks` workgroups with their roles; `lds` = the
// largest per-case need.  With ev0/ev1 the launch records its own
// start and end (the dispatch's timestamps, not those of separate event
// packets around it).
hipError_t launch_particles(const BlockRole* roles, int sp, int blocks, size_t lds, hipStream_t st, hipEvent_t ev0,
                            hipEvent_t ev1) {
  if (ev0) {
    if (sp == 0)
      hipExtLaunchKernelGGL(k_particles<0>, dim3(blocks), dim3(kBlock), lds, st, ev0, ev1, 0, roles);
    else
      hipExtLaunchKernelGGL(k_particles<1>, dim3(blocks), dim3(kBlock), lds, st, ev0, ev1, 0, roles);
  } else if (sp == 0) {
    hipLaunchKernelGGL(k_particles<0>, dim3(blocks), dim3(kBlock), lds, st, roles);
  } else {
    hipLaunchKernelGGL(k_particles<1>, dim3(blocks), dim3(kBlock), lds, st, roles);
  }
  return hipGetLastError();
}

// Resident workgroups per CU of the head for grids of up to max_ng nodes.
int head_occupancy(int max_ng) {
  const size_t lds = (size_t)(max_ng + (max_ng >> 4) + 1) * 24;
  int nb = 0;
  const hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_head<0, 16>, kBlock, lds);
  return e == hipSuccess && nb > 0 ? nb : 1;
}

// Resident workgroups per CU of a species' particle kernel with `lds` bytes
// of dynamic LDS.
int particle_occupancy(int sp, size_t lds) {
  int nb = 0;
  const hipError_t e = sp == 0 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_particles<0>, kBlock, lds)
                               : hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_particles<1>, kBlock, lds);
  return e == hipSuccess && nb > 0 ? nb : 1;
}

// Dynamic LDS of the small-case kernel for a case: E, then the largest of
// the field solve's rows and either species' particle region.
size_t small_lds_bytes(int ng, uint32_t flags, int n_eepf, int n_ifed) {
  size_t region = 2 * (size_t)(ng + (ng >> 4) + 1);
  for (int sp = 0; sp < 2; ++sp) {
    const size_t r = particle_lds_bytes(ng, flags, n_eepf, n_ifed, sp) / 8 - (size_t)ng;
    region = region > r ? region : r;
  }
  return ((size_t)ng + region) * 8;
}

size_t small_static_lds() { return particle_static_lds(0) + particle_static_lds(1) + 2048; }

// One window of the small cases: workgroup b runs the case of roles[b] for
// roles[b].j steps.
hipError_t launch_small(const BlockRole* roles, int ncase, size_t lds, int mode, int sort_every, hipStream_t st) {
  if (mode == 1)
    hipLaunchKernelGGL(k_small<1>, dim3(ncase), dim3(kBlock), lds, st, roles, sort_every);
  else
    hipLaunchKernelGGL(k_small<0>, dim3(ncase), dim3(kBlock), lds, st, roles, sort_every);
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
                       int every, hipStream_t st) {
  hipLaunchKernelGGL(k_sort_hist, dim3(blocks), dim3(256), (size_t)max_ng * 4, st, roles, sp, every);
  hipLaunchKernelGGL(k_sort_scan, dim3(ncase), dim3(1024), 0, st, case_roles, sp, every);
  const size_t lds = (size_t)((max_ng + 1) / 2) * 8 + (size_t)max_ng * 8;
  hipLaunchKernelGGL(k_sort_scatter, dim3(blocks), dim3(256), lds, st, roles, sp, every);
  hipLaunchKernelGGL(k_sort_finish, dim3(ncase), dim3(1024), 0, st, case_roles, sp, every);
  return hipGetLastError();
}

hipError_t launch_fold(CaseDev* d, hipStream_t st) {
  hipLaunchKernelGGL(k_fold_diag, dim3(1), dim3(1024), 0, st, d);
  return hipGetLastError();
}

}  // namespace edp
