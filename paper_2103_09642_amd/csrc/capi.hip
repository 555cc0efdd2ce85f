// Host runtime and C ABI of the PIC/MCC library (see include/edupic.h).
//
// A case lives entirely in a caller-owned device arena: the CaseDev control
// block, two buffer sets of FP64 structure-of-arrays particles per species,
// the per-case n*sigma tables, Thomas reciprocals, a ring of V(t_s) values and
// the grid and diagnostic arrays.  The runtime only computes constants and
// host-side inputs (V(t), Thomas reciprocals, n*sigma_tot), uploads them and
// enqueues kernels; every step of the method runs on the GPU.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstddef>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <numeric>
#include <string>
#include <vector>

#include "edupic.h"
#include "impl.hpp"

namespace edp {
hipError_t launch_particles(const BlockRole* roles, int sp, int blocks, size_t lds, int mode, int dstep, int pretest,
                            hipStream_t st, hipEvent_t ev0, hipEvent_t ev1);
hipError_t launch_window_begin(BlockRole* roles, int nroles, const BlockRole* cases, int ncase, hipStream_t st);
hipError_t launch_window_end(const BlockRole* cases, int ncase, int steps, hipStream_t st);
size_t particle_lds_bytes(int ng, uint32_t flags, int n_eepf, int n_ifed, int sp);
size_t particle_static_lds(int sp);
int particle_occupancy(int sp, size_t lds);
hipError_t launch_seed(CaseDev* d, int sp, int64_t n, double sigma, hipStream_t st);
hipError_t launch_deposit(CaseDev* d, int sp, int64_t* dst1, int64_t* dst2, int ng, int blocks,
                          hipStream_t st);
hipError_t launch_sort(const BlockRole* roles, const BlockRole* case_roles, int sp, int blocks, int ncase, int max_ng,
                       int every, int dstep, hipStream_t st);
hipError_t launch_fold(CaseDev* d, hipStream_t st);
size_t small_lds_bytes(int ng, uint32_t flags, int n_eepf, int n_ifed);
size_t small_static_lds();
hipError_t launch_small(const BlockRole* roles, int ncase, size_t lds, int mode, int sort_every, int pretest,
                        hipStream_t st);
hipError_t launch_zero(void* p, int64_t bytes, hipStream_t st);
}  // namespace edp

using namespace edp;

namespace {

thread_local std::string g_err;

int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

#define HIPCHK(expr)                                                                 \
  do {                                                                               \
    hipError_t e_ = (expr);                                                          \
    if (e_ != hipSuccess) return fail(EDP_EHIP, "%s: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

constexpr size_t kAlign = 256;
inline size_t align_up(size_t v) { return (v + kAlign - 1) & ~(kAlign - 1); }

struct Case {
  edp_case id = 0;
  edp_case_desc desc{};
  CaseDev h{};  // host copy of constants and pointers
  CaseDev* d = nullptr;
  char* arena = nullptr;
  int64_t arena_bytes = 0;
  int64_t step = 0;        // next step to run (host view)
  int64_t est[2] = {0, 0}; // estimate of the slots in use, for launch sizing
  int64_t* est_pinned = nullptr;  // async read-back of alloc[] .. ctr[] (kEstSpan bytes)
  // collisions per particle step of each species over the last read-backs
  // far enough apart (kRateSteps particle steps), and that read-back's counters
  double coll_rate[2] = {0.0, 0.0};
  int64_t rate_coll[2] = {0, 0}, rate_pst[2] = {0, 0};
  hipEvent_t est_ev = nullptr;
  bool est_pending = false;
  double* vstage = nullptr;  // pinned staging of V(t_s)
  hipEvent_t vev = nullptr;
  bool vev_pending = false;
  bool failed = false;
};

// Workgroups per case of each batched launch: prefix offsets, one range per
// case in case order.
struct BatchTable {
  int32_t ncase;
  int32_t part_off[2][kMaxBatch + 1];  // particle workgroups per species
  int32_t sort_off[2][kMaxBatch + 1];  // sort workgroups per species
};

// The cases of one lockstep run and everything derived from them: the
// workgroup tables, grid sizes, and the captured graph.
struct Batch {
  std::vector<Case*> cases;
  BatchTable h{};
  int parts[2] = {0, 0};  // particle workgroups per species
  int sorts[2] = {0, 0};  // sort workgroups per species
  // roles of the electron and ion launches' workgroups, one per case (the
  // window kernels, the sort scan and finish), and of the electron-sort and
  // ion-sort launches' workgroups, in the context's device table
  size_t role_off[5] = {0, 0, 0, 0, 0};
  size_t nroles = 0;
  int max_ng = 2;
  size_t lds[2] = {0, 0};
  // graph of one window of g_steps steps, valid for these cases at these
  // step phases and sort grids
  hipGraphExec_t gexec = nullptr;
  int g_steps = 0;
  std::vector<int64_t> g_phase;
};

// One lockstep group of cases: its batch tables, its device role table, and
// the stream its launches go to.  A multi-case advance runs as one group on
// the caller's stream, or as up to kMaxGroups groups whose launches go to
// streams of their own, so that one group's launch tail overlaps another's
// streaming (the groups share nothing; each keeps its own order).
constexpr int kMaxGroups = 4;
constexpr int kAutoSkew = -1;  // EDP_OPT_PART_SKEW default
struct Group {
  Batch batch;
  BlockRole* roles_d = nullptr;
  size_t roles_cap = 0;
  std::vector<BlockRole> roles_h;  // host copy of the last upload
  bool valid = false;  // the tables match batch.cases
  hipStream_t stream = nullptr;  // where this advance enqueues the group's work
  // groups 1.. : the library's own stream (default priority) and the event
  // the caller's stream waits on at the end of an advance
  hipStream_t own = nullptr;
  hipEvent_t join = nullptr;
  // the allocation-free advance's group: its role table is the device's
  // file-scope array (roles_d, roles_cap fixed), it launches plainly (no
  // graph, no timing events) on the context's stream and never allocates
  bool fixed = false;
};

// Workgroup roles the allocation-free advance can hold: its role table is a
// file-scope device array of this many entries (1 MiB) per GPU.
constexpr int kScratchRoles = 16384;

}  // namespace

// The allocation-free advance's role table.  On the host this name is a
// stand-in, not a device address: host code uses it only to ask
// hipGetSymbolAddress, with a device current, for that device's copy, and
// then only that address (kept per device by scratch_roles()).
static_assert(sizeof(BlockRole) == 64, "role size named in the ABI header (16384 roles: 1 MiB)");
__device__ __align__(256) BlockRole scratch[kScratchRoles];


struct edp_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  int num_cu = 256;
  // cross sections
  bool has_xs = false;
  int nbins = 0;
  double de = 0, thr_exc = 0, thr_ion = 0, w_ion = 0;
  std::vector<double> el, exc, ion, iso, back;
  std::map<edp_case, Case*> cases;
  edp_case next_id = 1;
  // options
  int mode = 0, sort_every = 100, profile = 0, graph_steps = 0, poisson = 0;
  int part_wg_per_cu = 0;  // 0: every resident slot
  int pretest = 0;  // EDP_OPT_PRETEST
  int part_skew = kAutoSkew;  // per mille: the last layer's weight below the first's; -1 automatic
  int groups = 2;  // lockstep groups of a multi-case advance (1..kMaxGroups)
  // cases of at most this many slots per species (estimate) run in the
  // persistent one-workgroup-per-case kernel (0: none)
  int64_t small_max = 0;
  // the persistent small cases' stream (default priority) and role table
  hipStream_t small_stream = nullptr;
  hipEvent_t small_join = nullptr;
  BlockRole* small_roles = nullptr;
  size_t small_cap = 0;
  std::vector<BlockRole> small_h;
  // the groups' tables and run state; group 0 runs on `stream`, the others
  // on streams of their own, forked from and joined back into `stream` by an
  // advance
  Group grp[kMaxGroups];
  hipEvent_t fork_ev = nullptr;
  // the allocation-free advance (edp_advance_steps_noalloc): one group on
  // `stream` whose role table is the device's scratch array
  Group na;
  // profiling
  std::vector<std::pair<hipEvent_t, hipEvent_t>> ev_pairs;  // recorded, not yet read
  std::vector<std::pair<hipEvent_t, hipEvent_t>> ev_free;   // created, ready for reuse
  double prof_ms = 0.0;
  int64_t prof_launches = 0;
};

namespace {

struct Layout {
  size_t off_case, off_part[2][2][5], off_vp2[2], off_cl[2], off_tab[7], off_pb[2], off_rden, off_volt, off_cnt_e, off_cnt_i,
      off_shard, off_rho, off_phi, off_ef, off_flux, off_sum[6], off_acc[7], off_eepf, off_xt, off_xtcnt, off_ifed,
      off_sort, total;
  int64_t cap[2];
};

constexpr int64_t kMaxCap = (int64_t(1) << 31) - 1024;  // slots are int32 in the candidate lists

int validate(const edp_case_desc* c) {
  if (!c) return fail(EDP_EINVAL, "null descriptor");
  if (c->n_grid < 2 || c->n_grid > kMaxNodes) return fail(EDP_EINVAL, "n_grid must be 2..%d", kMaxNodes);
  if (c->ion_subcycle < 1) return fail(EDP_EINVAL, "ion_subcycle must be >= 1");
  if (c->steps_per_cycle < 1) return fail(EDP_EINVAL, "steps_per_cycle must be >= 1");
  if (!(c->dt_e > 0.0) || !(c->gap_m > 0.0) || !(c->area_m2 > 0.0))
    return fail(EDP_EINVAL, "dt_e, gap and area must be > 0");
  if (!(c->gas_temp_k > 0.0) || !(c->pressure_pa >= 0.0) || !(c->weight >= 0.0))
    return fail(EDP_EINVAL, "bad gas temperature, pressure or weight");
  if (c->n_harm < 0 || c->n_harm > 4) return fail(EDP_EINVAL, "n_harm must be 0..4");
  if (c->n_init_e < 0 || c->n_init_i < 0 || c->cap_e < 0 || c->cap_i < 0)
    return fail(EDP_EINVAL, "negative particle count");
  if (c->cap_e > kMaxCap || c->cap_i > kMaxCap || 2 * c->n_init_e > kMaxCap || 2 * c->n_init_i > kMaxCap)
    return fail(EDP_EINVAL, "capacity above 2^31 slots");
  if ((c->flags & EDP_DIAG_EEPF) && (c->n_eepf < 1 || c->n_eepf > 4096 || !(c->de_eepf_ev > 0.0)))
    return fail(EDP_EINVAL, "bad EEPF binning (1..4096 bins)");
  if ((c->flags & EDP_DIAG_XT) &&
      (c->n_xt_bin < 1 || c->steps_per_cycle % c->n_xt_bin != 0 || c->steps_per_cycle / c->n_xt_bin > 100000))
    return fail(EDP_EINVAL, "n_xt_bin must divide steps_per_cycle (at most 100000 time bins)");
  if ((c->flags & EDP_DIAG_IFED) && (c->n_ifed < 1 || c->n_ifed > 4096 || !(c->de_ifed_ev > 0.0)))
    return fail(EDP_EINVAL, "bad IFEDF binning (1..4096 bins)");
  for (int k = 0; k < 2; ++k)
    if (!(c->gamma_see[k] >= 0.0 && c->gamma_see[k] <= 1.0) || !(c->eta_refl[k] >= 0.0 && c->eta_refl[k] <= 1.0))
      return fail(EDP_EINVAL, "surface probabilities must be in [0, 1]");
  if ((c->gamma_see[0] > 0.0 || c->gamma_see[1] > 0.0) && !(c->see_te_ev > 0.0))
    return fail(EDP_EINVAL, "see_te_ev must be > 0 with secondary emission");
  // particle-kernel LDS: E + deposit (16 B/node), with measurements 24-32 B/node
  // more and the EEPF / IFEDF histograms
  const uint32_t meas = EDP_DIAG_EEPF | EDP_DIAG_CURRENT | EDP_DIAG_MEANE | EDP_DIAG_XT | EDP_DIAG_IFED;
  if ((c->flags & meas) && c->n_grid > 1024) return fail(EDP_EINVAL, "measurements support n_grid <= 1024");
  for (int sp = 0; sp < 2; ++sp)
    if (particle_lds_bytes(c->n_grid, c->flags, c->n_eepf, c->n_ifed, sp) + particle_static_lds(sp) > 65536)
      return fail(EDP_EINVAL, "measurement histograms and grid exceed the workgroup's LDS");
  return EDP_OK;
}

int64_t auto_cap(int64_t n_init, int64_t cap) {
  int64_t c = cap > 0 ? cap : std::max<int64_t>(2 * n_init, int64_t(1) << 18);
  return (c + 255) / 256 * 256;
}

Layout layout(const edp_case_desc* c, int nbins) {
  Layout L{};
  size_t o = 0;
  auto take = [&](size_t bytes) {
    size_t r = o;
    o = align_up(o + bytes);
    return r;
  };
  L.off_case = take(sizeof(CaseDev));
  L.cap[0] = auto_cap(c->n_init_e, c->cap_e);
  L.cap[1] = auto_cap(c->n_init_i, c->cap_i);
  for (int sp = 0; sp < 2; ++sp)
    for (int set = 0; set < 2; ++set)
      for (int a = 0; a < 5; ++a) L.off_part[sp][set][a] = take((size_t)L.cap[sp] * 8);
  for (int set = 0; set < 2; ++set) L.off_vp2[set] = take((size_t)L.cap[0] * 4);  // electrons only (float)
  for (int sp = 0; sp < 2; ++sp) {
    const size_t chunks = (size_t)((L.cap[sp] + kMaxChunk - 1) / kMaxChunk);
    L.off_cl[sp] = take(chunks * kMaxChunk * 8);  // candidates (per-workgroup lists over its chunk range)
  }
  for (int t = 0; t < 7; ++t) L.off_tab[t] = take((size_t)nbins * 8);
  for (int sp = 0; sp < 2; ++sp) L.off_pb[sp] = take((size_t)kMaxPb * 8);
  const size_t ng = (size_t)c->n_grid;
  L.off_rden = take(ng * 8);
  L.off_volt = take((size_t)kVoltChunk * 8);
  L.off_cnt_e = take(3 * ng * 8);
  L.off_cnt_i = take(3 * ng * 8);
  L.off_shard = take((size_t)2 * kShards * kRec * 8);
  L.off_rho = take(ng * 8);
  L.off_phi = take(ng * 8);
  L.off_ef = take(ng * 8);
  L.off_flux = take(ng * 8);
  for (int k = 0; k < 6; ++k) L.off_sum[k] = take(ng * 8);
  for (int k = 0; k < 7; ++k) L.off_acc[k] = take(3 * ng * 8);
  L.off_eepf = take((size_t)std::max(1, c->n_eepf) * 8);
  const size_t n_xt = (c->flags & EDP_DIAG_XT) ? (size_t)(c->steps_per_cycle / c->n_xt_bin) : 0;
  L.off_xt = take(std::max<size_t>(1, (size_t)kNumXt * n_xt * ng) * 8);
  L.off_xtcnt = take(std::max<size_t>(1, 2 * n_xt) * 8);
  L.off_ifed = take(2 * (size_t)((c->flags & EDP_DIAG_IFED) ? c->n_ifed + 1 : 1) * 8);
  L.off_sort = take((ng + 1) * 8);
  L.total = o;
  return L;
}

// The array pointers of a case's control block for an arena laid out as L
// (the capacities too).
void set_pointers(CaseDev& h, char* arena, const Layout& L) {
  for (int sp = 0; sp < 2; ++sp) {
    h.sp[sp].cap = L.cap[sp];
    for (int set = 0; set < 2; ++set) {
      h.sp[sp].x[set] = (double*)(arena + L.off_part[sp][set][0]);
      h.sp[sp].vx[set] = (double*)(arena + L.off_part[sp][set][1]);
      h.sp[sp].vy[set] = (double*)(arena + L.off_part[sp][set][2]);
      h.sp[sp].vz[set] = (double*)(arena + L.off_part[sp][set][3]);
      h.sp[sp].uid[set] = (uint64_t*)(arena + L.off_part[sp][set][4]);
      h.sp[sp].vp2[set] = sp == 0 ? (float*)(arena + L.off_vp2[set]) : nullptr;
    }
  }
  for (int sp = 0; sp < 2; ++sp) h.clist[sp] = (int64_t*)(arena + L.off_cl[sp]);
  double* tabs[7];
  for (int t = 0; t < 7; ++t) tabs[t] = (double*)(arena + L.off_tab[t]);
  h.nsig_e = tabs[0];
  h.nsig_i = tabs[1];
  h.sig_el = tabs[2];
  h.sig_exc = tabs[3];
  h.sig_ion = tabs[4];
  h.sig_iso = tabs[5];
  h.sig_back = tabs[6];
  for (int sp = 0; sp < 2; ++sp) h.pbound[sp] = (const double*)(arena + L.off_pb[sp]);
  h.rden = (double*)(arena + L.off_rden);
  h.volt = (double*)(arena + L.off_volt);
  h.cnt_e = (int64_t*)(arena + L.off_cnt_e);
  h.cnt_i = (int64_t*)(arena + L.off_cnt_i);
  h.shard = (int64_t*)(arena + L.off_shard);
  h.rho = (double*)(arena + L.off_rho);
  h.phi = (double*)(arena + L.off_phi);
  h.efield = (double*)(arena + L.off_ef);
  h.flux = (double*)(arena + L.off_flux);
  double** sums[6] = {&h.sum_ne, &h.sum_ni, &h.sum_je, &h.sum_ji, &h.sum_w, &h.sum_e};
  for (int k = 0; k < 6; ++k) *sums[k] = (double*)(arena + L.off_sum[k]);
  int64_t** accs[7] = {&h.acc_je, &h.acc_ji, &h.acc_w, &h.acc_e, &h.acc_wi, &h.acc_ei, &h.acc_iz};
  for (int k = 0; k < 7; ++k) *accs[k] = (int64_t*)(arena + L.off_acc[k]);
  h.eepf = (int64_t*)(arena + L.off_eepf);
  h.xt = (double*)(arena + L.off_xt);
  h.xt_cnt = (int64_t*)(arena + L.off_xtcnt);
  h.ifed = (int64_t*)(arena + L.off_ifed);
  h.sort_cnt = (int64_t*)(arena + L.off_sort);
}

// Driving voltage V(t_s) = sum_k V_k sin(2 pi f_k t_s + phi_k) + V_dc, t_s = s dt_e.
double voltage(const edp_case_desc& c, int64_t s) {
  const double t = (double)s * c.dt_e;
  double v = 0.0;
  for (int k = 0; k < c.n_harm; ++k)
    v += c.v_amp[k] * std::sin(kTwoPi * c.freq_hz[k] * t + c.phase_rad[k]);
  return v + c.v_dc;
}

// Null-collision maximum frequency of a table of n sigma_tot: the largest
// n sigma_tot(E) g(E) with g at the upper end of each bin's energy range
// (energies round to the nearest bin) and, for the last bin, which also holds
// every higher energy, at four times the table's range.
// Collision-frequency bound of table row i: n sigma_tot at the row's upper
// energy (energies round to the nearest row), the last row (which also
// holds every higher energy) taken at four times the table range.
double row_nu(const std::vector<double>& nsig, int i, double de_ev, double mass) {
  const int nb = (int)nsig.size();
  const double e_hi = i == nb - 1 ? 4.0 * (double)nb * de_ev : ((double)i + 0.5) * de_ev;
  return nsig[i] * std::sqrt(2.0 * e_hi * kEvToJ / mass);
}

// Rows per block of the pre-test's bound table: a power of two giving at
// most kMaxPb blocks.
int pb_shift(int nbins) {
  int s = 0;
  while (((nbins - 1) >> s) >= kMaxPb) ++s;
  return s;
}

// The pre-test's bound by energy (CaseDev::pbound): for block b the prefix
// maximum of P = 1 - exp(-nu dt) over rows 0 .. the block's last, with the
// relative margin of p_bound.
std::vector<double> pbound_table(const std::vector<double>& nsig, double de_ev, double mass, double dt) {
  const int nb = (int)nsig.size();
  const int sh = pb_shift(nb);
  std::vector<double> t((size_t)kMaxPb, 1.0);
  double m = 0.0;
  for (int i = 0; i < nb; ++i) {
    m = std::max(m, row_nu(nsig, i, de_ev, mass));
    if (i == nb - 1 || ((i + 1) >> sh) != (i >> sh))
      t[(size_t)(i >> sh)] = std::min(1.0, (1.0 - std::exp(-m * dt)) * (1.0 + 1e-9));
  }
  return t;
}

double nu_star(const std::vector<double>& nsig, double de_ev, double mass) {
  double m = 0.0;
  for (int i = 0; i < (int)nsig.size(); ++i) m = std::max(m, row_nu(nsig, i, de_ev, mass));
  return m;
}

Case* find(edp_ctx* ctx, edp_case id) {
  auto it = ctx->cases.find(id);
  return it == ctx->cases.end() ? nullptr : it->second;
}

// The dynamic tail of CaseDev (from `step` on) is read and written whole.
constexpr size_t kDynOff = offsetof(CaseDev, step);
constexpr size_t kDynBytes = sizeof(CaseDev) - kDynOff;

int read_dyn(edp_ctx* ctx, Case* c, CaseDev& t) {
  HIPCHK(hipStreamSynchronize(ctx->stream));
  HIPCHK(hipMemcpy((char*)&t + kDynOff, (char*)c->d + kDynOff, kDynBytes, hipMemcpyDeviceToHost));
  return EDP_OK;
}

int write_dyn(edp_ctx* ctx, Case* c, const CaseDev& t) {
  HIPCHK(hipStreamSynchronize(ctx->stream));
  HIPCHK(hipMemcpy((char*)c->d + kDynOff, (const char*)&t + kDynOff, kDynBytes, hipMemcpyHostToDevice));
  return EDP_OK;
}

// Grid of the deposit/sort kernels for about n particles.
int blocks_for(const edp_ctx* ctx, int64_t n) {
  const int64_t per_block = 256 * 4;
  int64_t b = (n + per_block - 1) / per_block;
  b = std::max<int64_t>(1, std::min<int64_t>(b, (int64_t)ctx->num_cu * 8));
  return (int)b;
}

// Expected chunks of a species of a case (10% headroom over the estimate).
int64_t est_chunks(const Case* c, int sp) { return (c->est[sp] + c->est[sp] / 10 + kChunk) / kChunk; }

// Expected work of a case's electron share of a particle launch: its chunks
// weighted by the collision work per particle step.  Timestamps of every
// workgroup of batched launches (the 32 dual-frequency and the 64
// heterogeneous cases) put a workgroup's time at about 10.5 ns per electron
// of its range plus about 200 ns per collider (exact test and scattering):
// a collider weighs as much as 20 electrons.  Ions are weighted by their
// chunks alone (not measured).
constexpr double kCollWeight[2] = {20.0, 0.0};
double est_cost(const Case* c, int sp) {
  return (double)est_chunks(c, sp) * (1.0 + kCollWeight[sp] * c->coll_rate[sp]);
}
// Bytes read back by request_estimate: CaseDev from alloc[] to the end of ctr[].
constexpr size_t kEstSpan = offsetof(CaseDev, ctr) + sizeof(int64_t) * kNumCtr - offsetof(CaseDev, alloc);
constexpr int64_t kRateSteps = 1 << 20;

// Upload V(t_s) for steps [s0, s1) (s1 - s0 <= kVoltChunk) into the ring.
int upload_volt(Case* c, int64_t s0, int64_t s1, hipStream_t st) {
  if (c->vev_pending) {
    HIPCHK(hipEventSynchronize(c->vev));
    c->vev_pending = false;
  }
  const int64_t n = s1 - s0;
  for (int64_t k = 0; k < n; ++k) c->vstage[k] = voltage(c->desc, s0 + k);
  double* ring = const_cast<double*>(c->h.volt);
  const int64_t a = s0 % kVoltChunk;
  const int64_t first = std::min<int64_t>(n, kVoltChunk - a);
  HIPCHK(hipMemcpyAsync(ring + a, c->vstage, first * 8, hipMemcpyHostToDevice, st));
  if (first < n) HIPCHK(hipMemcpyAsync(ring, c->vstage + first, (n - first) * 8, hipMemcpyHostToDevice, st));
  HIPCHK(hipEventRecord(c->vev, st));
  c->vev_pending = true;
  return EDP_OK;
}

void poll_estimate(Case* c) {
  if (c->est_pending && hipEventQuery(c->est_ev) == hipSuccess) {
    const char* b = (const char*)c->est_pinned;
    auto at = [&](size_t off) {
      int64_t v;
      std::memcpy(&v, b + off - offsetof(CaseDev, alloc), sizeof v);
      return v;
    };
    c->est[0] = at(offsetof(CaseDev, alloc));
    c->est[1] = at(offsetof(CaseDev, alloc) + 8);
    const size_t ctr = offsetof(CaseDev, ctr);
    const int64_t coll[2] = {at(ctr + 8 * kCollE), at(ctr + 8 * kCollI)};
    const int64_t pst[2] = {at(ctr + 8 * kPstepE), at(ctr + 8 * kPstepI)};
    for (int sp = 0; sp < 2; ++sp) {
      const int64_t dp = pst[sp] - c->rate_pst[sp], dc = coll[sp] - c->rate_coll[sp];
      if (dp < 0 || dc < 0) {  // counters restarted: a new baseline
        c->rate_pst[sp] = pst[sp];
        c->rate_coll[sp] = coll[sp];
      } else if (dp >= kRateSteps) {
        c->coll_rate[sp] = (double)dc / (double)dp;
        c->rate_pst[sp] = pst[sp];
        c->rate_coll[sp] = coll[sp];
      }
    }
    c->est_pending = false;
  }
}

int request_estimate(Case* c, hipStream_t st) {
  if (c->est_pending) return EDP_OK;
  HIPCHK(hipMemcpyAsync(c->est_pinned, (char*)c->d + offsetof(CaseDev, alloc), kEstSpan, hipMemcpyDeviceToHost, st));
  HIPCHK(hipEventRecord(c->est_ev, st));
  c->est_pending = true;
  return EDP_OK;
}

int drain_profile(edp_ctx* ctx) {
  for (auto& pr : ctx->ev_pairs) {
    float ms = 0.f;
    HIPCHK(hipEventSynchronize(pr.second));
    HIPCHK(hipEventElapsedTime(&ms, pr.first, pr.second));
    ctx->prof_ms += ms;
    ctx->prof_launches += 1;
    ctx->ev_free.push_back(pr);
  }
  ctx->ev_pairs.clear();
  return EDP_OK;
}

// A new timing event pair.  Timing only: no system-scope fence (nothing on
// the host reads the memory these events order).
int create_event_pair(hipEvent_t& e0, hipEvent_t& e1) {
  HIPCHK(hipEventCreateWithFlags(&e0, hipEventDisableSystemFence));
  const hipError_t e = hipEventCreateWithFlags(&e1, hipEventDisableSystemFence);
  if (e != hipSuccess) {
    (void)hipEventDestroy(e0);
    return fail(EDP_EHIP, "hipEventCreateWithFlags: %s", hipGetErrorString(e));
  }
  return EDP_OK;
}

// A timing event pair for one electron launch: from the pool, else new.
int take_event_pair(edp_ctx* ctx, hipEvent_t& e0, hipEvent_t& e1) {
  if (ctx->ev_free.empty()) return create_event_pair(e0, e1);
  e0 = ctx->ev_free.back().first;
  e1 = ctx->ev_free.back().second;
  ctx->ev_free.pop_back();
  return EDP_OK;
}

void drop_graph(Group& G) {
  if (G.batch.gexec) {
    (void)hipGraphExecDestroy(G.batch.gexec);
    G.batch.gexec = nullptr;
  }
  G.batch.g_steps = 0;
}

void destroy_group_streams(edp_ctx* ctx) {
  if (ctx->fork_ev) (void)hipEventDestroy(ctx->fork_ev);
  ctx->fork_ev = nullptr;
  if (ctx->small_stream) (void)hipStreamDestroy(ctx->small_stream);
  if (ctx->small_join) (void)hipEventDestroy(ctx->small_join);
  ctx->small_stream = nullptr;
  ctx->small_join = nullptr;
  for (Group& G : ctx->grp) {
    if (G.own) (void)hipStreamDestroy(G.own);
    if (G.join) (void)hipEventDestroy(G.join);
    G.own = nullptr;
    G.join = nullptr;
  }
}

// Drain every group's stream and forget their graphs and tables.
int reset_groups(edp_ctx* ctx) {
  HIPCHK(hipStreamSynchronize(ctx->stream));
  if (ctx->small_stream) HIPCHK(hipStreamSynchronize(ctx->small_stream));
  for (Group& G : ctx->grp)
    if (G.own) HIPCHK(hipStreamSynchronize(G.own));
  for (Group& G : ctx->grp) {
    drop_graph(G);
    G.valid = false;
  }
  return EDP_OK;
}

// Workgroup j of n of case c in a batched launch (an equal share of the
// case's chunks).
BlockRole role(const Case* c, int j, int n) {
  const uint64_t one = 1ull << 31;
  return BlockRole{c->d, c->h.cnt_e, c->h.cnt_i, c->h.volt, c->step, j, n, (int32_t)c->desc.n_grid,
                   (int32_t)c->desc.ion_subcycle, (uint32_t)(one * (uint64_t)j / (uint64_t)n),
                   (uint32_t)(one * (uint64_t)(j + 1) / (uint64_t)n)};
}

// Particle roles of one launch: case k's want[k] workgroups, spread over
// the launch (workgroup j of n at position (j + 1/2)/n of it, cases in order
// on ties) so that each case has workgroups in every dispatch layer, with
// their chunk shares.  A launch's workgroups are dispatched one per CU in
// turn, so block b is in layer b / num_cu; the CUs' wave arbitration favours
// the older waves, and a later layer streams its chunks more slowly.  With
// skew a (per mille) layer l of L gets the weight 1 - a l / (L - 1), and
// each case's chunks are split by the weights of its workgroups.  The
// automatic skew (a < 0) is 200 (L - 1), at most 900, for a launch of one
// case: on the large case (2e6 particles per species, four layers) 600-750
// measured best, 4% above none; a launch of several cases runs without
// (measured neutral with two lockstep groups, 3% slower with one: cases
// differ in their cost per chunk more than layers do).
void particle_roles(std::vector<BlockRole>& roles, const std::vector<Case*>& cs, const std::vector<int>& want,
                    int num_cu, int skew) {
  struct Pos {
    double key;
    int k, j;
  };
  std::vector<Pos> order;
  for (size_t k = 0; k < cs.size(); ++k)
    for (int j = 0; j < want[k]; ++j) order.push_back({(j + 0.5) / want[k], (int)k, j});
  std::stable_sort(order.begin(), order.end(), [](const Pos& a, const Pos& b) { return a.key < b.key; });
  const size_t off = roles.size();
  const int nblocks = (int)order.size();
  std::vector<std::vector<int>> at(cs.size());
  for (int b = 0; b < nblocks; ++b) {
    const Pos& p = order[b];
    roles.push_back(role(cs[p.k], p.j, want[p.k]));
    at[p.k].push_back(b);  // j increasing with b within a case
  }
  const int layers = (nblocks + num_cu - 1) / std::max(1, num_cu);
  if (skew < 0) skew = cs.size() == 1 ? std::min(900, 200 * (layers - 1)) : 0;
  auto weight = [&](int b) {
    if (layers < 2 || skew <= 0) return 1.0;
    return 1.0 - 1e-3 * skew * (double)(b / num_cu) / (double)(layers - 1);
  };
  const double one = (double)(1ull << 31);
  for (size_t k = 0; k < cs.size(); ++k) {
    double total = 0.0;
    for (int b : at[k]) total += weight(b);
    double acc = 0.0;
    uint32_t lo = 0;
    for (size_t j = 0; j < at[k].size(); ++j) {
      BlockRole& r = roles[off + at[k][j]];
      acc += weight(at[k][j]);
      r.f_lo = lo;
      r.f_hi = j + 1 == at[k].size() ? (uint32_t)(1ull << 31) : (uint32_t)std::min(one, std::floor(acc / total * one));
      lo = r.f_hi;
    }
  }
}

// Workgroups of a case's sort histogram and scatter.
int sort_blocks(const edp_ctx* ctx, const Case* c, int sp) { return std::max(1, blocks_for(ctx, c->est[sp]) / 4); }

// Build the batch table for `cs` (in this order) and upload it.  Particle
// workgroups: the chip's resident workgroups (at most part_wg_per_cu per CU
// when that option is set) shared out in proportion to each case's expected
// work (est_cost), so every workgroup has about the same amount of it (any
// count is still covered: the kernels split the live chunks over whatever
// workgroups a case has).  The table is read by
// kernels still in flight, so the stream is drained before it changes;
// grids are rebuilt only when a case's share has moved by a quarter or the
// shares by a sixteenth of the workgroups in all.
int set_batch(edp_ctx* ctx, Group& G, const std::vector<Case*>& cs) {
  Batch& B = G.batch;
  const size_t nc = cs.size();
  size_t lds[2] = {0, 0};
  int max_ng = 2;
  for (const Case* c : cs) {
    for (int sp = 0; sp < 2; ++sp)
      lds[sp] = std::max(lds[sp], particle_lds_bytes(c->desc.n_grid, c->desc.flags, c->desc.n_eepf, c->desc.n_ifed, sp));
    max_ng = std::max(max_ng, (int)c->desc.n_grid);
  }
  std::vector<int> want[2];
  for (int sp = 0; sp < 2; ++sp) {
    const int occ = particle_occupancy(sp, lds[sp]);
    const int per_cu = ctx->part_wg_per_cu > 0 ? std::min(ctx->part_wg_per_cu, occ) : occ;
    const int64_t slots = (int64_t)ctx->num_cu * per_cu;
    double total = 0.0;
    for (const Case* c : cs) total += est_cost(c, sp);
    // every case at least one workgroup, the slots in proportion to the
    // chunks (largest remainders first), never more workgroups than chunks
    // and never more than the slots in all (unless the cases outnumber
    // them): a workgroup beyond the resident slots would wait for a whole
    // workgroup to finish and run after it
    want[sp].assign(nc, 1);
    std::vector<double> frac(nc, 0.0);
    int64_t used = 0;
    for (size_t k = 0; k < nc; ++k) {
      const int64_t ch = est_chunks(cs[k], sp);
      const double ideal = est_cost(cs[k], sp) * (double)slots / std::max(1e-9, total);
      const int64_t w = std::max<int64_t>(1, std::min<int64_t>({(int64_t)ideal, ch, (int64_t)kMaxPartWG}));
      want[sp][k] = (int)w;
      frac[k] = ideal - (double)w;
      used += w;
    }
    std::vector<size_t> order(nc);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](size_t a, size_t b) { return frac[a] > frac[b]; });
    for (size_t k : order) {
      if (used >= slots) break;
      if (frac[k] <= 0.0 || want[sp][k] >= std::min<int64_t>(kMaxPartWG, est_chunks(cs[k], sp))) continue;
      ++want[sp][k];
      ++used;
    }
  }
  std::vector<int> want_sort[2];
  for (int sp = 0; sp < 2; ++sp)
    for (size_t k = 0; k < nc; ++k) want_sort[sp].push_back(sort_blocks(ctx, cs[k], sp));
  // rebuilt when a case's share has moved by a quarter, or the shares by a
  // sixteenth of the workgroups in all
  auto near = [](int a, int a0) { return a <= a0 * 5 / 4 + 1 && a >= a0 * 3 / 4; };
  bool same = G.valid && B.cases == cs;
  int64_t moved[2] = {0, 0};
  for (size_t k = 0; k < nc && same; ++k) {
    for (int sp = 0; sp < 2 && same; ++sp) {
      const int had = B.h.part_off[sp][k + 1] - B.h.part_off[sp][k];
      same = near(want[sp][k], had);
      moved[sp] += std::abs(want[sp][k] - had);
    }
    for (int sp = 0; sp < 2 && same; ++sp) same = near(want_sort[sp][k], B.h.sort_off[sp][k + 1] - B.h.sort_off[sp][k]);
  }
  for (int sp = 0; sp < 2 && same; ++sp) same = 16 * moved[sp] <= B.parts[sp];
  if (same) return EDP_OK;
  HIPCHK(hipStreamSynchronize(G.stream));
  drop_graph(G);
  G.valid = false;
  B.cases = cs;
  B.h = BatchTable{};
  B.h.ncase = (int32_t)nc;
  B.max_ng = max_ng;
  B.lds[0] = lds[0];
  B.lds[1] = lds[1];
  for (size_t k = 0; k < nc; ++k) {
    for (int sp = 0; sp < 2; ++sp) B.h.part_off[sp][k + 1] = B.h.part_off[sp][k] + want[sp][k];
    for (int sp = 0; sp < 2; ++sp) B.h.sort_off[sp][k + 1] = B.h.sort_off[sp][k] + want_sort[sp][k];
  }
  B.parts[0] = B.h.part_off[0][nc];
  B.parts[1] = B.h.part_off[1][nc];
  B.sorts[0] = B.h.sort_off[0][nc];
  B.sorts[1] = B.h.sort_off[1][nc];
  // roles: electrons, ions, one per case, electron sort, ion sort
  std::vector<BlockRole> roles;
  roles.reserve((size_t)B.parts[0] + B.parts[1] + nc + B.sorts[0] + B.sorts[1]);
  for (int sp = 0; sp < 2; ++sp) {
    B.role_off[sp] = roles.size();
    particle_roles(roles, cs, want[sp], ctx->num_cu, ctx->part_skew);
  }
  B.role_off[2] = roles.size();
  for (size_t k = 0; k < nc; ++k) roles.push_back(role(cs[k], 0, 1));
  for (int sp = 0; sp < 2; ++sp) {
    B.role_off[3 + sp] = roles.size();
    for (size_t k = 0; k < nc; ++k)
      for (int j = 0; j < want_sort[sp][k]; ++j) roles.push_back(role(cs[k], j, want_sort[sp][k]));
  }
  B.nroles = roles.size();
  if (roles.size() > G.roles_cap && G.fixed)
    return fail(EDP_EINVAL, "the batch needs %zu workgroup roles; the allocation-free advance holds at most %d",
                roles.size(), kScratchRoles);
  if (roles.size() > G.roles_cap) {
    // no kernel of this group is in flight (drained above)
    if (G.roles_d) HIPCHK(hipFree(G.roles_d));
    G.roles_d = nullptr;
    G.roles_cap = 0;
    HIPCHK(hipMalloc((void**)&G.roles_d, roles.size() * sizeof(BlockRole)));
    G.roles_cap = roles.size();
  }
  // ordered on the group's own stream (a blocking copy would also wait for
  // the other group's work when the caller's stream is the null stream)
  G.roles_h.swap(roles);
  HIPCHK(hipMemcpyAsync(G.roles_d, G.roles_h.data(), G.roles_h.size() * sizeof(BlockRole), hipMemcpyHostToDevice,
                        G.stream));
  G.valid = true;
  return EDP_OK;
}

// Step j of the current window (case k at step s[k] + j), plain launches:
// the compaction/sort of the cases due for it, then one electron launch and,
// when some case has an ion step, one ion launch.
int enqueue_batch_step(edp_ctx* ctx, Group& G, const std::vector<int64_t>& s, int64_t j, bool capture) {
  Batch& B = G.batch;
  hipStream_t st = G.stream;
  const int nc = (int)B.cases.size();
  bool any_ion = false, sort_e = false, sort_i = false;
  for (int k = 0; k < nc; ++k) {
    const int64_t sk = s[k] + j;
    const int64_t nsub = B.cases[k]->desc.ion_subcycle;
    sort_e = sort_e || sk % ctx->sort_every == 0;
    sort_i = sort_i || sk % ((int64_t)ctx->sort_every * nsub) == 0;
    any_ion = any_ion || sk % nsub == 0;
  }
  // one set of sort launches per species for the whole batch; the cases that
  // are not due skip them on the device
  const BlockRole* case_roles = G.roles_d + B.role_off[2];
  const int dj = (int)j;
  if (sort_e)
    HIPCHK(launch_sort(G.roles_d + B.role_off[3], case_roles, 0, B.sorts[0], nc, B.max_ng, ctx->sort_every, dj, st));
  if (sort_i)
    HIPCHK(launch_sort(G.roles_d + B.role_off[4], case_roles, 1, B.sorts[1], nc, B.max_ng, ctx->sort_every, dj, st));
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (ctx->profile && !capture && !G.fixed) {
    const int r = take_event_pair(ctx, e0, e1);
    if (r) return r;
  }
  HIPCHK(launch_particles(G.roles_d + B.role_off[0], 0, B.parts[0], B.lds[0], ctx->poisson, dj, ctx->pretest, st, e0,
                          e1));
  if (e0) ctx->ev_pairs.emplace_back(e0, e1);
  if (any_ion)
    HIPCHK(launch_particles(G.roles_d + B.role_off[1], 1, B.parts[1], B.lds[1], ctx->poisson, dj, ctx->pretest, st,
                            nullptr, nullptr));
  return EDP_OK;
}

// A window of `steps` steps of the group from the cases' steps s: the
// window's first kernel (roles' steps, slot-count rings), the steps, its
// last kernel (counters, steps, slot counts).
int enqueue_window(edp_ctx* ctx, Group& G, const std::vector<int64_t>& s, int64_t steps, bool capture) {
  Batch& B = G.batch;
  const int nc = (int)B.cases.size();
  const BlockRole* case_roles = G.roles_d + B.role_off[2];
  HIPCHK(launch_window_begin(G.roles_d, (int)B.nroles, case_roles, nc, G.stream));
  for (int64_t j = 0; j < steps; ++j) {
    const int r = enqueue_batch_step(ctx, G, s, j, capture);
    if (r) return r;
  }
  HIPCHK(launch_window_end(case_roles, nc, (int)steps, G.stream));
  return EDP_OK;
}

// Capture one window of `steps` batch steps from the cases' current steps
// into a graph.
int build_graph(edp_ctx* ctx, Group& G, const std::vector<int64_t>& s, int steps) {
  Batch& B = G.batch;
  drop_graph(G);
  const int nc = (int)B.cases.size();
  B.g_phase.resize(nc);
  for (int k = 0; k < nc; ++k) B.g_phase[k] = s[k] % steps;
  hipStream_t st = G.stream;
  hipGraph_t g = nullptr;
  HIPCHK(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
  const int r = enqueue_window(ctx, G, s, steps, true);
  const hipError_t ec = hipStreamEndCapture(st, &g);
  if (r) {
    if (g) (void)hipGraphDestroy(g);
    return r;
  }
  if (ec != hipSuccess) return fail(EDP_EHIP, "hipStreamEndCapture: %s", hipGetErrorString(ec));
  const hipError_t e = hipGraphInstantiate(&B.gexec, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e != hipSuccess) return fail(EDP_EHIP, "hipGraphInstantiate: %s", hipGetErrorString(e));
  B.g_steps = steps;
  return EDP_OK;
}

bool graph_matches(const Group& G, const std::vector<int64_t>& s, int steps) {
  const Batch& B = G.batch;
  if (!B.gexec || B.g_steps != steps) return false;
  for (size_t k = 0; k < B.cases.size(); ++k)
    if (s[k] % steps != B.g_phase[k]) return false;
  return true;
}

// One window (up to 4096 steps) of the cases of group G that still have
// steps to go, all in lockstep: the group's tables, the voltages, then graph
// replays (whole graphs of a multiple of sort_every * N_SUB steps) or plain
// steps on the group's stream.  `done`: no case had steps left.
int group_window(edp_ctx* ctx, Group& G, const std::vector<Case*>& cases, std::vector<int64_t>& left, bool& done) {
  std::vector<Case*> act;
  std::vector<int64_t> s;
  int64_t w = 4096;
  int64_t base = 1;
  for (size_t k = 0; k < cases.size(); ++k) {
    if (left[k] <= 0) continue;
    act.push_back(cases[k]);
    s.push_back(cases[k]->step);
    w = std::min(w, left[k]);
    const int64_t p = (int64_t)ctx->sort_every * cases[k]->desc.ion_subcycle;
    base = std::lcm(base, p);
  }
  done = act.empty();
  if (done) return EDP_OK;
  for (Case* c : act) poll_estimate(c);
  int r = set_batch(ctx, G, act);
  if (r) return r;
  int gsteps = 0;
  if (ctx->mode == 1 && base <= 4096 && !G.fixed) {
    gsteps = ctx->graph_steps > 0 ? ctx->graph_steps : (int)(base * std::max<int64_t>(1, 200 / base));
    if (gsteps % base != 0) gsteps = (int)((gsteps / base + 1) * base);
    if (gsteps <= w) w = (w / gsteps) * gsteps; else gsteps = 0;
  }
  for (Case* c : act) {
    r = upload_volt(c, c->step, c->step + w, G.stream);
    if (r) return r;
  }
  int64_t j = 0;
  while (j < w) {
    if (gsteps > 0) {
      std::vector<int64_t> sj(s);
      for (auto& v : sj) v += j;
      if (!graph_matches(G, sj, gsteps)) {
        r = build_graph(ctx, G, sj, gsteps);
        if (r) return r;
      }
      HIPCHK(hipGraphLaunch(G.batch.gexec, G.stream));
      j += gsteps;
      continue;
    }
    // plain launches: the rest of the window as one window of its own
    std::vector<int64_t> sj(s);
    for (auto& v : sj) v += j;
    r = enqueue_window(ctx, G, sj, w - j, false);
    if (r) return r;
    j = w;
  }
  for (size_t k = 0, a = 0; k < cases.size(); ++k) {
    if (left[k] <= 0) continue;
    cases[k]->step += w;
    left[k] -= w;
    r = request_estimate(act[a++], G.stream);
    if (r) return r;
  }
  if (ctx->ev_pairs.size() > 8192) {
    r = drain_profile(ctx);
    if (r) return r;
  }
  return EDP_OK;
}

// Advance cases[k] by n[k] steps.  With G groups (the option, at most one
// per case) the cases are split into G lockstep groups balanced by expected
// work (particles x steps, largest first onto the least loaded group), each
// keeping the call's order; the streams of groups 1.. wait for everything
// enqueued on the caller's stream before they start, windows of the groups
// are enqueued in turn, and the caller's stream waits for every group at
// the end, so every later call on it is ordered after all of them.
// Whether a case runs in the persistent one-workgroup-per-case kernel: few
// enough slots (estimate) and its LDS within one workgroup's 64 KiB.
bool small_case(const edp_ctx* ctx, const Case* c) {
  if (ctx->small_max <= 0 || std::max(c->est[0], c->est[1]) > ctx->small_max) return false;
  const edp_case_desc& D = c->desc;
  return small_lds_bytes(D.n_grid, D.flags, D.n_eepf, D.n_ifed) + small_static_lds() <= 65536;
}

// The persistent small cases of an advance, on the context's small-case
// stream (forked from and joined back into the caller's stream): windows of
// up to 4096 steps, each one launch in which workgroup k runs case k by its
// own window (the cases do not wait for each other).
int run_small(edp_ctx* ctx, const std::vector<Case*>& cases, std::vector<int64_t> left) {
  hipStream_t st = ctx->small_stream;
  // the previous call's table may still be in flight from host memory
  HIPCHK(hipStreamSynchronize(st));
  HIPCHK(hipEventRecord(ctx->fork_ev, ctx->stream));
  HIPCHK(hipStreamWaitEvent(st, ctx->fork_ev, 0));
  size_t lds = 0;
  for (const Case* c : cases)
    lds = std::max(lds, small_lds_bytes(c->desc.n_grid, c->desc.flags, c->desc.n_eepf, c->desc.n_ifed));
  // every window's roles, built up front and uploaded once: window w holds
  // the cases with steps left, each with min(left, 4096) steps
  constexpr int64_t kWin = 4096;
  std::vector<BlockRole>& roles = ctx->small_h;
  roles.clear();
  std::vector<size_t> win_off{0};
  std::vector<int64_t> rem(left);
  for (;;) {
    for (size_t k = 0; k < cases.size(); ++k)
      if (rem[k] > 0) {
        const int64_t w = std::min(rem[k], kWin);
        roles.push_back(role(cases[k], (int)w, 1));
        rem[k] -= w;
      }
    if (roles.size() == win_off.back()) break;
    win_off.push_back(roles.size());
  }
  int r = EDP_OK;
  if (!roles.empty()) {
    if (roles.size() > ctx->small_cap) {
      if (ctx->small_roles) HIPCHK(hipFree(ctx->small_roles));
      ctx->small_roles = nullptr;
      ctx->small_cap = 0;
      HIPCHK(hipMalloc((void**)&ctx->small_roles, roles.size() * sizeof(BlockRole)));
      ctx->small_cap = roles.size();
    }
    HIPCHK(hipMemcpyAsync(ctx->small_roles, roles.data(), roles.size() * sizeof(BlockRole), hipMemcpyHostToDevice, st));
  }
  for (size_t win = 0; win + 1 < win_off.size() && r == EDP_OK; ++win) {
    const size_t lo = win_off[win], hi = win_off[win + 1];
    for (size_t a = lo; a < hi && r == EDP_OK; ++a) {
      Case* c = nullptr;
      for (Case* q : cases)
        if (q->d == roles[a].c) c = q;
      r = upload_volt(c, c->step, c->step + roles[a].j, st);
    }
    if (r) break;
    HIPCHK(launch_small(ctx->small_roles + lo, (int)(hi - lo), lds, ctx->poisson, ctx->sort_every, ctx->pretest, st));
    for (size_t a = lo; a < hi && r == EDP_OK; ++a)
      for (Case* q : cases)
        if (q->d == roles[a].c) {
          q->step += roles[a].j;
          r = request_estimate(q, st);
        }
  }
  const hipError_t e = hipEventRecord(ctx->small_join, st);
  const hipError_t w = e == hipSuccess ? hipStreamWaitEvent(ctx->stream, ctx->small_join, 0) : e;
  if (w != hipSuccess && r == EDP_OK) r = fail(EDP_EHIP, "joining the small cases: %s", hipGetErrorString(w));
  return r;
}

int run_lockstep(edp_ctx* ctx, const std::vector<Case*>& cases, const std::vector<int64_t>& n);

int run_batch(edp_ctx* ctx, const std::vector<Case*>& all, const std::vector<int64_t>& all_n) {
  std::vector<Case*> small, cases;
  std::vector<int64_t> small_n, n;
  for (Case* c : all) poll_estimate(c);
  for (size_t k = 0; k < all.size(); ++k) {
    if (small_case(ctx, all[k])) {
      small.push_back(all[k]);
      small_n.push_back(all_n[k]);
    } else {
      cases.push_back(all[k]);
      n.push_back(all_n[k]);
    }
  }
  int r = EDP_OK;
  if (!small.empty()) r = run_small(ctx, small, small_n);
  if (r == EDP_OK && !cases.empty()) r = run_lockstep(ctx, cases, n);
  return r;
}

int run_lockstep(edp_ctx* ctx, const std::vector<Case*>& cases, const std::vector<int64_t>& n) {
  const int ng = (int)std::min<size_t>((size_t)ctx->groups, std::max<size_t>(1, cases.size()));
  std::vector<Case*> gc[kMaxGroups];
  std::vector<int64_t> gl[kMaxGroups];
  if (ng == 1) {
    gc[0] = cases;
    gl[0] = n;
  } else {
    std::vector<size_t> order(cases.size());
    for (size_t k = 0; k < order.size(); ++k) order[k] = k;
    auto work = [&](size_t k) { return (double)(cases[k]->est[0] + cases[k]->est[1]) * (double)n[k]; };
    std::stable_sort(order.begin(), order.end(), [&](size_t a, size_t b) { return work(a) > work(b); });
    double load[kMaxGroups] = {};
    int count[kMaxGroups] = {};
    std::vector<int> in(cases.size());
    for (size_t k : order) {
      int g = 0;  // least loaded; on a tie (empty cases) the one with fewest cases
      for (int h = 1; h < ng; ++h)
        if (load[h] < load[g] || (load[h] == load[g] && count[h] < count[g])) g = h;
      in[k] = g;
      load[g] += work(k);
      ++count[g];
    }
    for (size_t k = 0; k < cases.size(); ++k) {
      gc[in[k]].push_back(cases[k]);
      gl[in[k]].push_back(n[k]);
    }
  }
  ctx->grp[0].stream = ctx->stream;
  for (int g = 1; g < kMaxGroups; ++g) ctx->grp[g].stream = ctx->grp[g].own;
  if (ng > 1) {
    HIPCHK(hipEventRecord(ctx->fork_ev, ctx->stream));
    for (int g = 1; g < ng; ++g) HIPCHK(hipStreamWaitEvent(ctx->grp[g].own, ctx->fork_ev, 0));
  }
  int r = EDP_OK;
  bool done[kMaxGroups] = {};
  for (int g = ng; g < kMaxGroups; ++g) done[g] = true;
  auto all_done = [&] { return std::all_of(done, done + kMaxGroups, [](bool d) { return d; }); };
  while (r == EDP_OK && !all_done())
    for (int g = 0; g < ng && r == EDP_OK; ++g)
      if (!done[g]) r = group_window(ctx, ctx->grp[g], gc[g], gl[g], done[g]);
  // the joins also after a failed window: whatever the groups did enqueue
  // stays ordered before later work on the caller's stream
  for (int g = 1; g < ng; ++g) {
    const hipError_t e = hipEventRecord(ctx->grp[g].join, ctx->grp[g].own);
    const hipError_t w = e == hipSuccess ? hipStreamWaitEvent(ctx->stream, ctx->grp[g].join, 0) : e;
    if (w != hipSuccess && r == EDP_OK) r = fail(EDP_EHIP, "joining group %d: %s", g, hipGetErrorString(w));
  }
  return r;
}

int deposit_species(edp_ctx* ctx, Case* c, int sp, int64_t step) {
  const edp_case_desc& D = c->desc;
  const int ng = D.n_grid;
  hipStream_t st = ctx->stream;
  const int blocks = blocks_for(ctx, c->est[sp] + 1);
  if (sp == 0) {
    HIPCHK(launch_zero(c->h.cnt_e, 3 * (int64_t)ng * 8, st));
    HIPCHK(launch_deposit(c->d, 0, c->h.cnt_e + (step % 3) * ng, nullptr, ng, blocks, st));
  } else {
    const int64_t k = step / D.ion_subcycle;
    HIPCHK(launch_zero(c->h.cnt_i, 3 * (int64_t)ng * 8, st));
    int64_t* second = (step % D.ion_subcycle == 0) ? nullptr : c->h.cnt_i + ((k + 1) % 3) * ng;
    HIPCHK(launch_deposit(c->d, 1, c->h.cnt_i + (k % 3) * ng, second, ng, blocks, st));
  }
  return EDP_OK;
}

int zero_diag(edp_ctx* ctx, Case* c) {
  hipStream_t st = ctx->stream;
  const int64_t ng = c->desc.n_grid;
  for (double* p : {c->h.sum_ne, c->h.sum_ni, c->h.sum_je, c->h.sum_ji, c->h.sum_w, c->h.sum_e})
    HIPCHK(launch_zero(p, ng * 8, st));
  for (int64_t* p : {c->h.acc_je, c->h.acc_ji, c->h.acc_w, c->h.acc_e, c->h.acc_wi, c->h.acc_ei, c->h.acc_iz})
    HIPCHK(launch_zero(p, 3 * ng * 8, st));
  HIPCHK(launch_zero(c->h.eepf, (int64_t)std::max(1, c->desc.n_eepf) * 8, st));
  if (c->h.n_xt > 0) {
    HIPCHK(launch_zero(c->h.xt, (int64_t)kNumXt * c->h.n_xt * ng * 8, st));
    HIPCHK(launch_zero(c->h.xt_cnt, (int64_t)2 * c->h.n_xt * 8, st));
  }
  if (c->h.n_ifed > 0) HIPCHK(launch_zero(c->h.ifed, (int64_t)2 * (c->h.n_ifed + 1) * 8, st));
  return EDP_OK;
}

int reset_diag(edp_ctx* ctx, Case* c) {
  int r = zero_diag(ctx, c);
  if (r) return r;
  CaseDev t;
  r = read_dyn(ctx, c, t);
  if (r) return r;
  t.diag_steps = 0;
  t.diag_ion_steps = 0;
  return write_dyn(ctx, c, t);
}

// Stability criteria 2 and 3 of section 2.2 at the seed state.
int stability(const edp_ctx* ctx, const edp_case_desc* D, const std::vector<double>& nsig_e) {
  if (D->flags & EDP_ALLOW_UNSTABLE) return EDP_OK;
  const double n_e = D->weight * (double)D->n_init_e / (D->area_m2 * D->gap_m);
  const double wpe = std::sqrt(n_e * kECharge * kECharge / (kEps0 * kEMass));
  if (wpe * D->dt_e >= 2.0) return fail(EDP_EUNSTABLE, "omega_pe dt = %g >= 2", wpe * D->dt_e);
  double pmax = 0.0;
  for (int k = 0; k < ctx->nbins; ++k) {
    const double e = k * ctx->de;
    const double v = std::sqrt(2.0 * e * kEvToJ / kEMass);
    pmax = std::max(pmax, 1.0 - std::exp(-nsig_e[k] * v * D->dt_e));
  }
  if (pmax >= 0.05) return fail(EDP_EUNSTABLE, "max electron collision probability %g >= 0.05", pmax);
  return EDP_OK;
}

}  // namespace

namespace {

// Device address of `scratch` on each device, taken once per device with the
// device current (every GPU holds its own copy at its own address).
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
BlockRole* g_scratch_ptr[kMaxDevices] = {};

int scratch_roles(int device, BlockRole** out) {
  if (device < 0 || device >= kMaxDevices) return fail(EDP_EINVAL, "device %d beyond %d", device, kMaxDevices);
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) return fail(EDP_EHIP, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
    g_scratch_ptr[device] = (BlockRole*)p;
  }
  *out = g_scratch_ptr[device];
  return EDP_OK;
}

// The cases and step counts of an advance call, validated: distinct known
// cases of the context, counts >= 0; cases marked failed are left out
// (*skipped set).
int collect_cases(edp_ctx* ctx, const edp_case* cases, int32_t n_cases, const int64_t* n_steps,
                  std::vector<Case*>& cs, std::vector<int64_t>& n, bool& skipped) {
  if (!ctx || n_cases < 0 || (n_cases > 0 && (!cases || !n_steps))) return fail(EDP_EINVAL, "null argument");
  for (int32_t k = 0; k < n_cases; ++k) {
    Case* c = find(ctx, cases[k]);
    if (!c) return fail(EDP_EINVAL, "unknown case %lld", (long long)cases[k]);
    if (n_steps[k] < 0) return fail(EDP_EINVAL, "negative step count");
  }
  skipped = false;
  for (int32_t k = 0; k < n_cases; ++k) {
    Case* c = find(ctx, cases[k]);
    if (c->failed) {
      skipped = true;
      continue;
    }
    if (std::find(cs.begin(), cs.end(), c) != cs.end()) return fail(EDP_EINVAL, "case listed twice");
    cs.push_back(c);
    n.push_back(n_steps[k]);
  }
  if ((int)cs.size() > kMaxBatch) return fail(EDP_EINVAL, "more than %d cases in one call", kMaxBatch);
  return EDP_OK;
}

}  // namespace

extern "C" {

const char* edp_last_error(void) { return g_err.c_str(); }

int edp_create(edp_ctx** out, int device, void* hip_stream) {
  if (!out) return fail(EDP_EINVAL, "null out");
  int ndev = 0;
  HIPCHK(hipGetDeviceCount(&ndev));
  if (device < 0 || device >= ndev) return fail(EDP_EINVAL, "device %d of %d", device, ndev);
  HIPCHK(hipSetDevice(device));
  edp_ctx* ctx = new edp_ctx();
  ctx->device = device;
  ctx->stream = (hipStream_t)hip_stream;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) == hipSuccess) ctx->num_cu = prop.multiProcessorCount;
  // the other groups' streams (default priority) and the fork/join events
  bool ok = hipEventCreateWithFlags(&ctx->fork_ev, hipEventDisableTiming) == hipSuccess &&
            hipStreamCreateWithFlags(&ctx->small_stream, hipStreamNonBlocking) == hipSuccess &&
            hipEventCreateWithFlags(&ctx->small_join, hipEventDisableTiming) == hipSuccess;
  for (int g = 1; g < kMaxGroups && ok; ++g)
    ok = hipStreamCreateWithFlags(&ctx->grp[g].own, hipStreamNonBlocking) == hipSuccess &&
         hipEventCreateWithFlags(&ctx->grp[g].join, hipEventDisableTiming) == hipSuccess;
  if (!ok) {
    destroy_group_streams(ctx);
    delete ctx;
    return fail(EDP_EHIP, "creating the groups' streams or events failed");
  }
  // the allocation-free advance's table: this device's scratch array
  BlockRole* sp = nullptr;
  const int rs = scratch_roles(device, &sp);
  if (rs) {
    destroy_group_streams(ctx);
    delete ctx;
    return rs;
  }
  ctx->na.fixed = true;
  ctx->na.roles_d = sp;
  ctx->na.roles_cap = kScratchRoles;
  *out = ctx;
  return EDP_OK;
}

int edp_destroy(edp_ctx* ctx) {
  if (!ctx) return EDP_OK;
  (void)reset_groups(ctx);
  if (ctx->small_stream) (void)hipStreamSynchronize(ctx->small_stream);
  for (Group& G : ctx->grp)
    if (G.roles_d) (void)hipFree(G.roles_d);
  if (ctx->small_roles) (void)hipFree(ctx->small_roles);
  destroy_group_streams(ctx);
  for (auto& kv : ctx->cases) {
    Case* c = kv.second;
    if (c->vstage) (void)hipHostFree(c->vstage);
    if (c->est_pinned) (void)hipHostFree(c->est_pinned);
    if (c->vev) (void)hipEventDestroy(c->vev);
    if (c->est_ev) (void)hipEventDestroy(c->est_ev);
    delete c;
  }
  for (auto* v : {&ctx->ev_pairs, &ctx->ev_free})
    for (auto& pr : *v) {
      (void)hipEventDestroy(pr.first);
      (void)hipEventDestroy(pr.second);
    }
  delete ctx;
  return EDP_OK;
}

int edp_set_xsec(edp_ctx* ctx, const edp_xsec* xs) {
  if (!ctx || !xs) return fail(EDP_EINVAL, "null argument");
  if (xs->n_bins < 1 || !(xs->de_ev > 0.0)) return fail(EDP_EINVAL, "bad table size");
  const double* src[5] = {xs->e_el, xs->e_exc, xs->e_ion, xs->i_iso, xs->i_back};
  std::vector<double>* dst[5] = {&ctx->el, &ctx->exc, &ctx->ion, &ctx->iso, &ctx->back};
  for (int k = 0; k < 5; ++k) {
    if (!src[k]) return fail(EDP_EINVAL, "null table");
    dst[k]->assign(src[k], src[k] + xs->n_bins);
  }
  ctx->nbins = xs->n_bins;
  ctx->de = xs->de_ev;
  ctx->thr_exc = xs->e_exc_thr_ev;
  ctx->thr_ion = xs->e_ion_thr_ev;
  ctx->w_ion = xs->w_ioniz_ev;
  ctx->has_xs = true;
  return EDP_OK;
}

int64_t edp_case_bytes(const edp_ctx* ctx, const edp_case_desc* desc) {
  if (!ctx || !ctx->has_xs) return fail(EDP_EINVAL, "cross sections not set");
  int r = validate(desc);
  if (r) return r;
  return (int64_t)layout(desc, ctx->nbins).total;
}

int edp_case_create(edp_ctx* ctx, const edp_case_desc* desc, void* dev_arena, int64_t arena_bytes,
                    edp_case* out) {
  if (!ctx || !out) return fail(EDP_EINVAL, "null argument");
  if (!ctx->has_xs) return fail(EDP_EINVAL, "cross sections not set");
  int r = validate(desc);
  if (r) return r;
  const Layout L = layout(desc, ctx->nbins);
  if (!dev_arena || arena_bytes < (int64_t)L.total)
    return fail(EDP_EARENA, "arena needs %lld bytes, got %lld", (long long)L.total, (long long)arena_bytes);
  if (((uintptr_t)dev_arena) % kAlign) return fail(EDP_EARENA, "arena must be 256-byte aligned");
  if (desc->n_init_e > L.cap[0] || desc->n_init_i > L.cap[1])
    return fail(EDP_EINVAL, "initial particles exceed capacity");
  HIPCHK(hipSetDevice(ctx->device));
  const edp_case_desc& D = *desc;
  const int ng = D.n_grid, nb = ctx->nbins;
  // constants (Table 1 and section 3.1)
  const double gas_n = D.pressure_pa / (kBoltzmann * D.gas_temp_k);
  std::vector<double> nsig_e(nb), nsig_i(nb);
  for (int k = 0; k < nb; ++k) {
    nsig_e[k] = gas_n * (ctx->el[k] + ctx->exc[k] + ctx->ion[k]);
    nsig_i[k] = gas_n * (ctx->iso[k] + ctx->back[k]);
  }
  r = stability(ctx, desc, nsig_e);
  if (r) return r;
  Case* c = new Case();
  c->desc = D;
  c->arena = (char*)dev_arena;
  c->arena_bytes = arena_bytes;
  c->d = (CaseDev*)(c->arena + L.off_case);
  CaseDev& h = c->h;
  std::memset(&h, 0, sizeof h);
  h.ng = ng;
  h.nbins = nb;
  h.nsub = D.ion_subcycle;
  h.n_eepf = D.n_eepf;
  h.flags = D.flags;
  h.nt = D.steps_per_cycle;
  h.n_xt_bin = (D.flags & EDP_DIAG_XT) ? D.n_xt_bin : 1;
  h.n_xt = (D.flags & EDP_DIAG_XT) ? D.steps_per_cycle / D.n_xt_bin : 0;
  h.n_ifed = (D.flags & EDP_DIAG_IFED) ? D.n_ifed : 0;
  h.de_ifed = (D.flags & EDP_DIAG_IFED) ? D.de_ifed_ev : 1.0;
  h.L = D.gap_m;
  h.dx = h.L / (double)(ng - 1);
  h.inv_dx = 1.0 / h.dx;
  h.dt_e = D.dt_e;
  h.dt_i = (double)D.ion_subcycle * D.dt_e;
  const double dv = D.area_m2 * h.dx;
  h.factor_w = D.weight / dv;
  h.factor_e = h.dt_e / kEMass * kECharge;
  h.factor_i = h.dt_i / kArMass * kECharge;
  h.sigma_a = std::sqrt(kBoltzmann * D.gas_temp_k / kArMass);
  h.n_gas = gas_n;
  h.nu_star_e = nu_star(nsig_e, ctx->de, kEMass);
  h.nu_star_i = nu_star(nsig_i, ctx->de, kMuArAr);
  h.p_null_e = 1.0 - std::exp(-h.nu_star_e * h.dt_e);
  h.p_null_i = 1.0 - std::exp(-h.nu_star_i * h.dt_i);
  {
    // Candidates of the direct collision test.  nu* bounds n sigma_tot g up
    // to the energy e_lim its last bin is taken at, up to rounding of the bin
    // edges; the relative margin covers that and the ulps of exp, so a
    // particle with R >= p_bound and an energy below e_lim has R >= P.  An
    // ion's relative speed is at most |v| + |v_a|: each normal of the
    // generator is r cos or r sin with r <= sqrt(2 * 53 ln 2) < 8.58, so
    // |v_a|^2 <= (r1^2 + r2^2) sigma_a^2 < (12.2 sigma_a)^2, and
    // g^2 <= 2 (v^2 + |v_a|^2).
    const double e_lim = 4.0 * (double)nb * ctx->de;
    h.p_bound_e = std::min(1.0, (1.0 - std::exp(-h.nu_star_e * h.dt_e)) * (1.0 + 1e-9));
    h.p_bound_i = std::min(1.0, (1.0 - std::exp(-h.nu_star_i * h.dt_i)) * (1.0 + 1e-9));
    h.v2_lim_e = 2.0 * e_lim * kEvToJ / kEMass * (1.0 - 1e-12);
    h.g2_lim_i = 2.0 * e_lim * kEvToJ / kMuArAr * (1.0 - 1e-12);
    const double amax = 12.2 * h.sigma_a;
    h.a2_i = amax * amax;
    h.pb_shift = pb_shift(nb);
    h.pb_n = ((nb - 1) >> h.pb_shift) + 1;
  }
  h.de_cs = ctx->de;
  h.thr_exc = ctx->thr_exc;
  h.thr_ion = ctx->thr_ion;
  h.w_ion = ctx->w_ion;
  h.de_eepf = D.de_eepf_ev;
  h.x_lo = 0.45 * h.L;
  h.x_hi = 0.55 * h.L;
  h.dens_scale = h.factor_w / kTwo32;
  h.kpois = h.dx * h.dx / kEps0;
  for (int k = 0; k < 2; ++k) {
    h.gamma_see[k] = D.gamma_see[k];
    h.eta_refl[k] = D.eta_refl[k];
  }
  h.see_on = D.gamma_see[0] > 0.0 || D.gamma_see[1] > 0.0;
  h.refl_on = D.eta_refl[0] > 0.0 || D.eta_refl[1] > 0.0;
  h.see_sigma = h.see_on ? std::sqrt(D.see_te_ev * kEvToJ / kEMass) : 0.0;
  h.seed = D.seed;
  set_pointers(h, c->arena, L);
  double* tabs[7] = {(double*)h.nsig_e, (double*)h.nsig_i, (double*)h.sig_el, (double*)h.sig_exc,
                     (double*)h.sig_ion, (double*)h.sig_iso, (double*)h.sig_back};
  // dynamic part
  h.step = 0;
  h.alloc[0] = D.n_init_e;
  h.alloc[1] = D.n_init_i;
  h.n[0] = D.n_init_e;
  h.n[1] = D.n_init_i;
  h.ctr[kLiveE] = D.n_init_e;
  h.ctr[kLiveI] = D.n_init_i;
  // Thomas reciprocals r_1 = 1/2, r_p = 1/(2 - r_{p-1})
  std::vector<double> rden(ng, 0.0);
  if (ng > 2) {
    rden[1] = 0.5;
    for (int p = 2; p <= ng - 2; ++p) rden[p] = 1.0 / (2.0 - rden[p - 1]);
  }
  hipStream_t st = ctx->stream;
  auto cleanup = [&](int code) {
    delete c;
    return code;
  };
  if (hipHostMalloc((void**)&c->vstage, kVoltChunk * 8, hipHostMallocDefault) != hipSuccess ||
      hipHostMalloc((void**)&c->est_pinned, kEstSpan, hipHostMallocDefault) != hipSuccess ||
      hipEventCreateWithFlags(&c->vev, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&c->est_ev, hipEventDisableTiming) != hipSuccess)
    return cleanup(fail(EDP_EHIP, "host staging allocation failed"));
  // zero the whole grid/diagnostic/scratch region, then upload
  const size_t z0 = L.off_cnt_e, z1 = L.total;
  if (launch_zero(c->arena + z0, (int64_t)(z1 - z0), st) != hipSuccess)
    return cleanup(fail(EDP_EHIP, "zero fill failed"));
  const std::vector<double>* tsrc[7] = {&nsig_e, &nsig_i, &ctx->el, &ctx->exc, &ctx->ion, &ctx->iso, &ctx->back};
  hipError_t e = hipSuccess;
  for (int t = 0; t < 7 && e == hipSuccess; ++t)
    e = hipMemcpyAsync(tabs[t], tsrc[t]->data(), (size_t)nb * 8, hipMemcpyHostToDevice, st);
  const std::vector<double> pb[2] = {pbound_table(nsig_e, ctx->de, kEMass, h.dt_e),
                                     pbound_table(nsig_i, ctx->de, kMuArAr, h.dt_i)};
  for (int sp = 0; sp < 2 && e == hipSuccess; ++sp)
    e = hipMemcpyAsync((void*)h.pbound[sp], pb[sp].data(), (size_t)kMaxPb * 8, hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = hipMemcpyAsync((void*)h.rden, rden.data(), (size_t)ng * 8, hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = hipMemcpyAsync(c->d, &h, sizeof(CaseDev), hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return cleanup(fail(EDP_EHIP, "upload: %s", hipGetErrorString(e)));
  c->est[0] = D.n_init_e;
  c->est[1] = D.n_init_i;
  // seed (Algorithm 1, init) and deposit
  const double sig_e = std::sqrt(D.te_init_ev * kEvToJ / kEMass);
  const double sig_i = std::sqrt(kBoltzmann * D.ti_init_k / kArMass);
  if (launch_seed(c->d, 0, D.n_init_e, sig_e, st) != hipSuccess ||
      launch_seed(c->d, 1, D.n_init_i, sig_i, st) != hipSuccess)
    return cleanup(fail(EDP_EHIP, "seed launch failed"));
  if ((r = deposit_species(ctx, c, 0, 0)) || (r = deposit_species(ctx, c, 1, 0))) return cleanup(r);
  e = hipStreamSynchronize(st);
  if (e != hipSuccess) return cleanup(fail(EDP_EHIP, "seed: %s", hipGetErrorString(e)));
  c->id = ctx->next_id++;
  ctx->cases[c->id] = c;
  *out = c->id;
  return EDP_OK;
}

int edp_case_resize(edp_ctx* ctx, edp_case id, int64_t cap_e, int64_t cap_i, void* dev_arena,
                    int64_t arena_bytes) {
  Case* c = ctx ? find(ctx, id) : nullptr;
  if (!c) return fail(EDP_EINVAL, "unknown case");
  if (cap_e < 0 || cap_i < 0) return fail(EDP_EINVAL, "negative capacity");
  edp_case_desc D2 = c->desc;
  if (cap_e > 0) D2.cap_e = cap_e;
  if (cap_i > 0) D2.cap_i = cap_i;
  int r = validate(&D2);
  if (r) return r;
  const Layout Lo = layout(&c->desc, ctx->nbins), Ln = layout(&D2, ctx->nbins);
  if (!dev_arena || arena_bytes < (int64_t)Ln.total)
    return fail(EDP_EARENA, "arena needs %lld bytes, got %lld", (long long)Ln.total, (long long)arena_bytes);
  if (((uintptr_t)dev_arena) % kAlign) return fail(EDP_EARENA, "arena must be 256-byte aligned");
  HIPCHK(hipSetDevice(ctx->device));
  // the batch tables and graphs hold the old control block's address
  if ((r = reset_groups(ctx))) return r;
  CaseDev t;
  if ((r = read_dyn(ctx, c, t))) return r;
  int64_t live[2];
  for (int sp = 0; sp < 2; ++sp) {
    live[sp] = std::min(t.alloc[sp], c->h.sp[sp].cap);
    if (live[sp] > Ln.cap[sp])
      return fail(EDP_ESTATE, "%lld slots in use exceed the new capacity %lld", (long long)live[sp],
                  (long long)Ln.cap[sp]);
  }
  char* na = (char*)dev_arena;
  hipStream_t st = ctx->stream;
  // the slots in use of the current buffer set go to set 0 of the new arena
  for (int sp = 0; sp < 2; ++sp) {
    const int cur = t.cur[sp];
    const size_t n = (size_t)live[sp];
    if (!n) continue;
    for (int a = 0; a < 5; ++a)
      HIPCHK(hipMemcpyAsync(na + Ln.off_part[sp][0][a], c->arena + Lo.off_part[sp][cur][a], n * 8,
                            hipMemcpyDeviceToDevice, st));
    if (sp == 0)
      HIPCHK(hipMemcpyAsync(na + Ln.off_vp2[0], c->arena + Lo.off_vp2[cur], n * 4, hipMemcpyDeviceToDevice, st));
  }
  // tables, V(t), deposit rings, fields and every diagnostic: the same
  // layout after the particle arrays and candidate lists
  const size_t tail = Lo.total - Lo.off_tab[0];
  if (tail != Ln.total - Ln.off_tab[0]) return fail(EDP_EHIP, "internal: layouts differ beyond the particles");
  HIPCHK(hipMemcpyAsync(na + Ln.off_tab[0], c->arena + Lo.off_tab[0], tail, hipMemcpyDeviceToDevice, st));
  CaseDev h = c->h;
  set_pointers(h, na, Ln);
  std::memcpy((char*)&h + kDynOff, (const char*)&t + kDynOff, kDynBytes);
  h.cur[0] = h.cur[1] = 0;
  CaseDev* nd = (CaseDev*)(na + Ln.off_case);
  HIPCHK(hipMemcpyAsync(nd, &h, sizeof(CaseDev), hipMemcpyHostToDevice, st));
  HIPCHK(hipStreamSynchronize(st));
  c->desc = D2;
  c->h = h;
  c->d = nd;
  c->arena = na;
  c->arena_bytes = arena_bytes;
  return EDP_OK;
}

int edp_case_destroy(edp_ctx* ctx, edp_case id) {
  if (!ctx) return fail(EDP_EINVAL, "null context");
  Case* c = find(ctx, id);
  if (!c) return fail(EDP_EINVAL, "unknown case");
  (void)hipStreamSynchronize(ctx->stream);
  for (Group& G : ctx->grp)
    if (G.own) (void)hipStreamSynchronize(G.own);
  for (Group& G : ctx->grp)
    if (std::find(G.batch.cases.begin(), G.batch.cases.end(), c) != G.batch.cases.end()) {
      drop_graph(G);
      G.batch.cases.clear();
      G.valid = false;
    }
  (void)hipHostFree(c->vstage);
  (void)hipHostFree(c->est_pinned);
  (void)hipEventDestroy(c->vev);
  (void)hipEventDestroy(c->est_ev);
  ctx->cases.erase(id);
  delete c;
  return EDP_OK;
}

int edp_advance_steps(edp_ctx* ctx, const edp_case* cases, int32_t n_cases, const int64_t* n_steps) {
  if (!ctx) return fail(EDP_EINVAL, "null context");
  HIPCHK(hipSetDevice(ctx->device));
  std::vector<Case*> cs;
  std::vector<int64_t> n;
  bool skipped = false;
  int r = collect_cases(ctx, cases, n_cases, n_steps, cs, n, skipped);
  if (r) return r;
  r = run_batch(ctx, cs, n);
  if (r) return r;
  if (skipped) return fail(EDP_ESTATE, "failed cases were not advanced");
  return EDP_OK;
}

int edp_advance_steps_noalloc(edp_ctx* ctx, const edp_case* cases, int32_t n_cases, const int64_t* n_steps) {
  if (!ctx) return fail(EDP_EINVAL, "null context");
  HIPCHK(hipSetDevice(ctx->device));
  std::vector<Case*> cs;
  std::vector<int64_t> n;
  bool skipped = false;
  int r = collect_cases(ctx, cases, n_cases, n_steps, cs, n, skipped);
  if (r) return r;
  // One lockstep group on the context's stream, plain launches, the role
  // table in this device's scratch array.  Any call on the device may have
  // rewritten that array since this context last used it: the table is
  // rebuilt and uploaded (ordered on the stream) before the first window.
  Group& G = ctx->na;
  G.stream = ctx->stream;
  G.valid = false;
  G.batch.cases.clear();
  bool done = false;
  while (r == EDP_OK && !done) r = group_window(ctx, G, cs, n, done);
  if (r) return r;
  if (skipped) return fail(EDP_ESTATE, "failed cases were not advanced");
  return EDP_OK;
}

int edp_advance(edp_ctx* ctx, const edp_case* cases, int32_t n_cases, const int32_t* n_cycles) {
  if (!ctx || (n_cases > 0 && (!cases || !n_cycles))) return fail(EDP_EINVAL, "null argument");
  std::vector<int64_t> steps(n_cases);
  for (int32_t k = 0; k < n_cases; ++k) {
    Case* c = find(ctx, cases[k]);
    if (!c) return fail(EDP_EINVAL, "unknown case %lld", (long long)cases[k]);
    if (n_cycles[k] < 0) return fail(EDP_EINVAL, "negative cycle count");
    steps[k] = (int64_t)n_cycles[k] * c->desc.steps_per_cycle;
  }
  return edp_advance_steps(ctx, cases, n_cases, steps.data());
}

int edp_sync(edp_ctx* ctx) {
  if (!ctx) return fail(EDP_EINVAL, "null context");
  HIPCHK(hipStreamSynchronize(ctx->stream));
  for (Group& G : ctx->grp)
    if (G.own) HIPCHK(hipStreamSynchronize(G.own));
  int status = EDP_OK;
  for (auto& kv : ctx->cases) {
    Case* c = kv.second;
    int32_t err = 0;
    HIPCHK(hipMemcpy(&err, (char*)c->d + offsetof(CaseDev, error), 4, hipMemcpyDeviceToHost));
    if (err) {
      c->failed = true;
      status = fail(EDP_ECAPACITY, "case %lld exceeded its particle capacity", (long long)c->id);
    }
  }
  return status;
}

int edp_read_counts(edp_ctx* ctx, edp_case id, edp_counts* out) {
  if (!ctx || !out) return fail(EDP_EINVAL, "null argument");
  Case* c = find(ctx, id);
  if (!c) return fail(EDP_EINVAL, "unknown case");
  CaseDev t;
  int r = read_dyn(ctx, c, t);
  if (r) return r;
  out->n_e = t.ctr[kLiveE];
  out->n_i = t.ctr[kLiveI];
  out->step = t.step;
  out->abs_e_pow = t.ctr[kAbsEPow];
  out->abs_e_gnd = t.ctr[kAbsEGnd];
  out->abs_i_pow = t.ctr[kAbsIPow];
  out->abs_i_gnd = t.ctr[kAbsIGnd];
  out->coll_e = t.ctr[kCollE];
  out->coll_i = t.ctr[kCollI];
  out->ioniz = t.ctr[kIoniz];
  out->anomalies = t.ctr[kAnomaly];
  out->dropped = t.ctr[kDropped];
  out->psteps_e = t.ctr[kPstepE];
  out->psteps_i = t.ctr[kPstepI];
  out->see_pow = t.ctr[kSeePow];
  out->see_gnd = t.ctr[kSeeGnd];
  out->refl = t.ctr[kRefl];
  if (t.error) {
    c->failed = true;
    return fail(EDP_ECAPACITY, "case %lld exceeded its particle capacity", (long long)c->id);
  }
  return EDP_OK;
}

// EDP_ECAPACITY (and the case marked failed) if the case has overflowed its
// particle capacity, so that results read from it are not mistaken for
// physical ones; EDP_OK otherwise.  Waits for the stream.
static int overflow_status(edp_ctx* ctx, Case* c) {
  int32_t err = 0;
  HIPCHK(hipStreamSynchronize(ctx->stream));
  HIPCHK(hipMemcpy(&err, (char*)c->d + offsetof(CaseDev, error), 4, hipMemcpyDeviceToHost));
  if (!err) return EDP_OK;
  c->failed = true;
  return fail(EDP_ECAPACITY, "case %lld exceeded its particle capacity", (long long)c->id);
}

// The status of a time-averaged read: the overflow status, with the
// diagnostics restarted after the read when asked.
static int after_read(edp_ctx* ctx, Case* c, int32_t reset) {
  const int st = overflow_status(ctx, c);
  const int r = reset ? reset_diag(ctx, c) : EDP_OK;
  return st ? st : r;
}

static int read_grid(edp_ctx* ctx, Case* c, const void* dev, void* host, size_t bytes) {
  HIPCHK(hipStreamSynchronize(ctx->stream));
  HIPCHK(hipMemcpy(host, dev, bytes, hipMemcpyDeviceToHost));
  return EDP_OK;
}

int edp_read_density(edp_ctx* ctx, edp_case id, double* ne, double* ni, int32_t n, int32_t reset) {
  Case* c = ctx ? find(ctx, id) : nullptr;
  if (!c || !ne || !ni) return fail(EDP_EINVAL, "bad argument");
  const int ng = c->desc.n_grid;
  if (n < ng) return fail(EDP_EINVAL, "output shorter than n_grid");
  CaseDev t;
  int r = read_dyn(ctx, c, t);
  if (r) return r;
  std::vector<double> a(ng), b(ng);
  if ((r = read_grid(ctx, c, c->h.sum_ne, a.data(), ng * 8)) || (r = read_grid(ctx, c, c->h.sum_ni, b.data(), ng * 8)))
    return r;
  const double steps = t.diag_steps > 0 ? (double)t.diag_steps : 1.0;
  for (int p = 0; p < ng; ++p) {
    ne[p] = a[p] / steps;
    ni[p] = b[p] / steps;
  }
  return after_read(ctx, c, reset);
}

int edp_read_eepf(edp_ctx* ctx, edp_case id, double* f, int64_t* counts, int32_t n, int32_t reset) {
  Case* c = ctx ? find(ctx, id) : nullptr;
  if (!c) return fail(EDP_EINVAL, "bad argument");
  const int nb = c->desc.n_eepf;
  if (n < nb) return fail(EDP_EINVAL, "output shorter than n_eepf");
  std::vector<int64_t> h(nb);
  int r = read_grid(ctx, c, c->h.eepf, h.data(), (size_t)nb * 8);
  if (r) return r;
  const double de = c->desc.de_eepf_ev;
  double tot = 0.0;
  for (int k = 0; k < nb; ++k) tot += (double)h[k];
  for (int k = 0; k < nb; ++k) {
    if (counts) counts[k] = h[k];
    if (f) f[k] = tot > 0.0 ? (double)h[k] / (tot * de * std::sqrt(((double)k + 0.5) * de)) : 0.0;
  }
  return after_read(ctx, c, reset);
}

int edp_read_currents(edp_ctx* ctx, edp_case id, double* je, double* ji, int32_t n, int32_t reset) {
  Case* c = ctx ? find(ctx, id) : nullptr;
  if (!c || !je || !ji) return fail(EDP_EINVAL, "bad argument");
  const int ng = c->desc.n_grid;
  if (n < ng) return fail(EDP_EINVAL, "output shorter than n_grid");
  HIPCHK(launch_fold(c->d, ctx->stream));
  CaseDev t;
  int r = read_dyn(ctx, c, t);
  if (r) return r;
  std::vector<double> a(ng), b(ng);
  if ((r = read_grid(ctx, c, c->h.sum_je, a.data(), ng * 8)) || (r = read_grid(ctx, c, c->h.sum_ji, b.data(), ng * 8)))
    return r;
  const double ns = t.diag_steps > 0 ? (double)t.diag_steps : 1.0;
  const double ni = t.diag_ion_steps > 0 ? (double)t.diag_ion_steps : 1.0;
  for (int p = 0; p < ng; ++p) {
    const double edge = (p == 0 || p == ng - 1) ? 2.0 : 1.0;
    je[p] = edge * (-kECharge * c->h.factor_w) * (a[p] / kDiagJS) / ns;
    ji[p] = edge * (kECharge * c->h.factor_w) * (b[p] / kDiagJS) / ni;
  }
  return after_read(ctx, c, reset);
}

int edp_read_mean_energy(edp_ctx* ctx, edp_case id, double* mee, int32_t n, int32_t reset) {
  Case* c = ctx ? find(ctx, id) : nullptr;
  if (!c || !mee) return fail(EDP_EINVAL, "bad argument");
  const int ng = c->desc.n_grid;
  if (n < ng) return fail(EDP_EINVAL, "output shorter than n_grid");
  HIPCHK(launch_fold(c->d, ctx->stream));
  std::vector<double> w(ng), e(ng);
  int r;
  if ((r = read_grid(ctx, c, c->h.sum_w, w.data(), ng * 8)) || (r = read_grid(ctx, c, c->h.sum_e, e.data(), ng * 8)))
    return r;
  for (int p = 0; p < ng; ++p) mee[p] = w[p] > 0.0 ? (e[p] / kDiagES) / (w[p] / kDiagWS) : 0.0;
  return after_read(ctx, c, reset);
}

int edp_read_xt_steps(edp_ctx* ctx, edp_case id, int64_t* steps, int64_t* ion_steps, int32_t n) {
  Case* c = ctx ? find(ctx, id) : nullptr;
  if (!c) return fail(EDP_EINVAL, "bad argument");
  if (!(c->desc.flags & EDP_DIAG_XT)) return fail(EDP_EINVAL, "the xt arrays are off for this case");
  const int nx = c->h.n_xt;
  if (n < nx) return fail(EDP_EINVAL, "output shorter than the number of xt bins");
  std::vector<int64_t> cnt(2 * (size_t)nx);
  int r = read_grid(ctx, c, c->h.xt_cnt, cnt.data(), cnt.size() * 8);
  if (r) return r;
  for (int t = 0; t < nx; ++t) {
    if (steps) steps[t] = cnt[t];
    if (ion_steps) ion_steps[t] = cnt[nx + t];
  }
  return EDP_OK;
}

// Cell means of the xt sums, in the units of the time-averaged reads.
int edp_read_xt(edp_ctx* ctx, edp_case id, int32_t q, double* out, int64_t n) {
  Case* c = ctx ? find(ctx, id) : nullptr;
  if (!c || !out || q < 0 || q >= EDP_XT_N) return fail(EDP_EINVAL, "bad argument");
  if (!(c->desc.flags & EDP_DIAG_XT)) return fail(EDP_EINVAL, "the xt arrays are off for this case");
  const int ng = c->desc.n_grid, nx = c->h.n_xt;
  const size_t cells = (size_t)nx * ng;
  if (n < (int64_t)cells) return fail(EDP_EINVAL, "output shorter than n_xt * n_grid");
  HIPCHK(launch_fold(c->d, ctx->stream));
  std::vector<int64_t> cnt(2 * (size_t)nx);
  int r = read_grid(ctx, c, c->h.xt_cnt, cnt.data(), cnt.size() * 8);
  if (r) return r;
  auto plane = [&](int k, std::vector<double>& v) {
    v.resize(cells);
    return read_grid(ctx, c, c->h.xt + (size_t)k * cells, v.data(), cells * 8);
  };
  std::vector<double> a, b;
  const double fw = c->h.factor_w;
  switch (q) {
    case EDP_XT_POT: r = plane(kXtFlux, a); break;
    case EDP_XT_EFIELD: r = plane(kXtEf, a); break;
    case EDP_XT_NE: r = plane(kXtNe, a); break;
    case EDP_XT_NI: r = plane(kXtNi, a); break;
    case EDP_XT_JE: r = plane(kXtJe, a); break;
    case EDP_XT_JI: r = plane(kXtJi, a); break;
    case EDP_XT_POWERE: r = plane(kXtPe, a); break;
    case EDP_XT_POWERI: r = plane(kXtPi, a); break;
    case EDP_XT_MEANEE: r = plane(kXtWe, a) ? 1 : plane(kXtEe, b); break;
    case EDP_XT_MEANEI: r = plane(kXtWi, a) ? 1 : plane(kXtEi, b); break;
    default: r = plane(kXtIz, a); break;
  }
  if (r) return r < 0 ? r : fail(EDP_EHIP, "xt read failed");
  for (int t = 0; t < nx; ++t) {
    const double ns = (double)cnt[t], ni = (double)cnt[nx + t];
    const double* A = a.data() + (size_t)t * ng;
    double* o = out + (size_t)t * ng;
    if (q == EDP_XT_POT) {
      // phi_p = V - sum_{q<p} F_q, summed over the bin's steps
      double phi = A[ng - 1];
      for (int p = 0; p < ng; ++p) {
        o[p] = ns > 0 ? (p == ng - 1 ? 0.0 : phi / ns) : 0.0;
        if (p < ng - 1) phi = phi - A[p];
      }
      continue;
    }
    for (int p = 0; p < ng; ++p) {
      const double edge = (p == 0 || p == ng - 1) ? 2.0 : 1.0;
      double v = 0.0;
      switch (q) {
        case EDP_XT_EFIELD:
        case EDP_XT_NE:
        case EDP_XT_NI: v = ns > 0 ? A[p] / ns : 0.0; break;
        case EDP_XT_JE:
        case EDP_XT_POWERE: v = ns > 0 ? edge * (-kECharge * fw) * (A[p] / kDiagJS) / ns : 0.0; break;
        case EDP_XT_JI:
        case EDP_XT_POWERI: v = ni > 0 ? edge * (kECharge * fw) * (A[p] / kDiagJS) / ni : 0.0; break;
        case EDP_XT_MEANEE:
        case EDP_XT_MEANEI: {
          const double* B = b.data() + (size_t)t * ng;
          v = A[p] > 0 ? (B[p] / kDiagES) / (A[p] / kDiagWS) : 0.0;
          break;
        }
        default: v = ns > 0 ? edge * fw * (A[p] / kDiagIZS) / c->h.dt_e / ns : 0.0; break;
      }
      o[p] = v;
    }
  }
  return EDP_OK;
}

int edp_read_ifed(edp_ctx* ctx, edp_case id, double* f_pow, double* f_gnd, int64_t* counts, int32_t n) {
  Case* c = ctx ? find(ctx, id) : nullptr;
  if (!c) return fail(EDP_EINVAL, "bad argument");
  if (!(c->desc.flags & EDP_DIAG_IFED)) return fail(EDP_EINVAL, "the IFEDF is off for this case");
  const int nb = c->h.n_ifed;
  if (n < nb) return fail(EDP_EINVAL, "output shorter than n_ifed");
  std::vector<int64_t> h(2 * (size_t)(nb + 1));
  int r = read_grid(ctx, c, c->h.ifed, h.data(), h.size() * 8);
  if (r) return r;
  double* f[2] = {f_pow, f_gnd};
  for (int side = 0; side < 2; ++side) {
    const int64_t* H = h.data() + (size_t)side * (nb + 1);
    double tot = 0.0;
    for (int k = 0; k < nb; ++k) tot += (double)H[k];
    if (counts)
      for (int k = 0; k <= nb; ++k) counts[(size_t)side * (nb + 1) + k] = H[k];
    if (f[side])
      for (int k = 0; k < nb; ++k) f[side][k] = tot > 0.0 ? (double)H[k] / (tot * c->h.de_ifed) : 0.0;
  }
  return EDP_OK;
}

int edp_read_info(edp_ctx* ctx, edp_case id, double* out, int32_t n) {
  Case* c = ctx ? find(ctx, id) : nullptr;
  if (!c || !out) return fail(EDP_EINVAL, "bad argument");
  if (n < EDP_INFO_N) return fail(EDP_EINVAL, "output shorter than EDP_INFO_N");
  const int ng = c->desc.n_grid;
  const uint32_t fl = c->desc.flags;
  HIPCHK(launch_fold(c->d, ctx->stream));
  CaseDev t;
  int r = read_dyn(ctx, c, t);
  if (r) return r;
  for (int k = 0; k < EDP_INFO_N; ++k) out[k] = 0.0;
  std::vector<double> ne(ng), w(ng), e(ng);
  if ((r = read_grid(ctx, c, c->h.sum_ne, ne.data(), ng * 8)) || (r = read_grid(ctx, c, c->h.sum_w, w.data(), ng * 8)) ||
      (r = read_grid(ctx, c, c->h.sum_e, e.data(), ng * 8)))
    return r;
  const double nst = t.diag_steps > 0 ? (double)t.diag_steps : 1.0;
  double ne_max = 0.0, sw = 0.0, se = 0.0;
  for (int p = 0; p < ng; ++p) {
    ne_max = std::max(ne_max, ne[p] / nst);
    sw += w[p];
    se += e[p];
  }
  const double mean_e = sw > 0.0 ? (se / kDiagES) / (sw / kDiagWS) : 0.0;
  out[EDP_INFO_MEAN_E] = mean_e;
  out[EDP_INFO_NE_MAX] = ne_max;
  int bad = 0;
  if (ne_max > 0.0 && mean_e > 0.0) {
    // criterion 1 with T_e = 2/3 <eps>, criterion 2 at the peak density
    const double te = 2.0 / 3.0 * mean_e;
    const double lam = std::sqrt(kEps0 * te * kEvToJ / (ne_max * kECharge * kECharge));
    const double wpe = std::sqrt(ne_max * kECharge * kECharge / (kEps0 * kEMass));
    out[EDP_INFO_DEBYE] = lam;
    out[EDP_INFO_DX_DEBYE] = c->h.dx / lam;
    out[EDP_INFO_WPE_DT] = wpe * c->h.dt_e;
    if (!(out[EDP_INFO_DX_DEBYE] < 1.0)) bad |= 1;
    if (!(out[EDP_INFO_WPE_DT] < 2.0)) bad |= 2;
  }
  // criterion 3: the largest collision probabilities over the tables
  out[EDP_INFO_PMAX_E] = c->h.p_null_e;
  out[EDP_INFO_PMAX_I] = c->h.p_null_i;
  if (!(c->h.p_null_e < 0.05) || !(c->h.p_null_i < 0.05)) bad |= 4;
  // criterion 4: the electron energy that crosses one cell per step
  const double vc = c->h.dx / c->h.dt_e;
  out[EDP_INFO_CFL_EV] = 0.5 * kEMass * vc * vc / kEvToJ;
  if (fl & EDP_DIAG_XT) {
    const int nx = c->h.n_xt;
    const size_t cells = (size_t)nx * ng;
    std::vector<int64_t> cnt(2 * (size_t)nx);
    std::vector<double> pe(cells), pi(cells);
    if ((r = read_grid(ctx, c, c->h.xt_cnt, cnt.data(), cnt.size() * 8)) ||
        (r = read_grid(ctx, c, c->h.xt + (size_t)kXtPe * cells, pe.data(), cells * 8)) ||
        (r = read_grid(ctx, c, c->h.xt + (size_t)kXtPi * cells, pi.data(), cells * 8)))
      return r;
    // trapezoid mean over x: the edge weight 1/2 cancels the edge doubling
    double spe = 0.0, spi = 0.0, ns = 0.0, ni = 0.0;
    for (int k = 0; k < nx; ++k) {
      ns += (double)cnt[k];
      ni += (double)cnt[nx + k];
      for (int p = 0; p < ng; ++p) {
        spe += pe[(size_t)k * ng + p];
        spi += pi[(size_t)k * ng + p];
      }
    }
    const double fw = c->h.factor_w;
    if (ns > 0) out[EDP_INFO_POWER_E] = (-kECharge * fw) * (spe / kDiagJS) / ((double)(ng - 1) * ns);
    if (ni > 0) out[EDP_INFO_POWER_I] = (kECharge * fw) * (spi / kDiagJS) / ((double)(ng - 1) * ni);
  }
  if (fl & EDP_DIAG_IFED) {
    const int nb = c->h.n_ifed;
    std::vector<int64_t> h(2 * (size_t)(nb + 1));
    if ((r = read_grid(ctx, c, c->h.ifed, h.data(), h.size() * 8))) return r;
    const double tspan = (double)t.diag_steps * c->h.dt_e;
    for (int side = 0; side < 2; ++side) {
      const int64_t* H = h.data() + (size_t)side * (nb + 1);
      double all = 0.0, in = 0.0, en = 0.0;
      for (int k = 0; k <= nb; ++k) all += (double)H[k];
      for (int k = 0; k < nb; ++k) {
        in += (double)H[k];
        en += (double)H[k] * ((double)k + 0.5) * c->h.de_ifed;
      }
      if (tspan > 0) out[side ? EDP_INFO_FLUX_I_GND : EDP_INFO_FLUX_I_POW] = all * c->desc.weight / (c->desc.area_m2 * tspan);
      if (in > 0) out[side ? EDP_INFO_EI_GND : EDP_INFO_EI_POW] = en / in;
    }
  }
  out[EDP_INFO_FAIL] = (double)bad;
  return EDP_OK;
}

int edp_set_voltage(edp_ctx* ctx, edp_case id, const double* v_amp, int32_t n_harm, double v_dc) {
  Case* c = ctx ? find(ctx, id) : nullptr;
  if (!c || (n_harm > 0 && !v_amp)) return fail(EDP_EINVAL, "bad argument");
  if (n_harm != c->desc.n_harm) return fail(EDP_EINVAL, "n_harm %d differs from the case's %d", n_harm, c->desc.n_harm);
  if (!std::isfinite(v_dc)) return fail(EDP_EINVAL, "v_dc must be finite");
  for (int k = 0; k < n_harm; ++k)
    if (!std::isfinite(v_amp[k])) return fail(EDP_EINVAL, "amplitudes must be finite");
  // the V(t) ring is filled from the descriptor at the start of every advance
  for (int k = 0; k < n_harm; ++k) c->desc.v_amp[k] = v_amp[k];
  c->desc.v_dc = v_dc;
  return EDP_OK;
}

int edp_reset_diag(edp_ctx* ctx, edp_case id) {
  Case* c = ctx ? find(ctx, id) : nullptr;
  if (!c) return fail(EDP_EINVAL, "bad argument");
  return reset_diag(ctx, c);  // also clears the pending per-step sums
}

int edp_read_deposit(edp_ctx* ctx, edp_case id, int64_t* cnt_e, int64_t* cnt_i, int32_t n) {
  Case* c = ctx ? find(ctx, id) : nullptr;
  if (!c || !cnt_e || !cnt_i) return fail(EDP_EINVAL, "bad argument");
  const int ng = c->desc.n_grid;
  if (n < ng) return fail(EDP_EINVAL, "output shorter than n_grid");
  CaseDev t;
  int r = read_dyn(ctx, c, t);
  if (r) return r;
  const int64_t s = t.step, k = s / c->desc.ion_subcycle;
  if ((r = read_grid(ctx, c, c->h.cnt_e + (s % 3) * ng, cnt_e, ng * 8))) return r;
  return read_grid(ctx, c, c->h.cnt_i + (k % 3) * ng, cnt_i, ng * 8);
}

int edp_read_fields(edp_ctx* ctx, edp_case id, double* rho, double* phi, double* ef, int32_t n) {
  Case* c = ctx ? find(ctx, id) : nullptr;
  if (!c) return fail(EDP_EINVAL, "bad argument");
  const int ng = c->desc.n_grid;
  if (n < ng) return fail(EDP_EINVAL, "output shorter than n_grid");
  int r;
  if (rho && (r = read_grid(ctx, c, c->h.rho, rho, ng * 8))) return r;
  if (ef && (r = read_grid(ctx, c, c->h.efield, ef, ng * 8))) return r;
  if (phi) {
    CaseDev t;
    if ((r = read_dyn(ctx, c, t))) return r;
    if (t.phi_valid) return read_grid(ctx, c, c->h.phi, phi, ng * 8);
    // the flux solver keeps F_q = phi_q - phi_{q+1} and V; sum them back up
    std::vector<double> f(ng);
    if ((r = read_grid(ctx, c, c->h.flux, f.data(), ng * 8))) return r;
    phi[0] = f[ng - 1];
    for (int p = 1; p < ng - 1; ++p) phi[p] = phi[p - 1] - f[p - 1];
    phi[ng - 1] = 0.0;
  }
  return EDP_OK;
}

int edp_get_state(edp_ctx* ctx, edp_case id, int32_t species, double* x, double* vx, double* vy,
                  double* vz, uint64_t* uid, int64_t cap, int64_t* n_out) {
  Case* c = ctx ? find(ctx, id) : nullptr;
  if (!c || (species != 0 && species != 1) || cap < 0) return fail(EDP_EINVAL, "bad argument");
  CaseDev t;
  int r = read_dyn(ctx, c, t);
  if (r) return r;
  const int64_t n = t.alloc[species] < c->h.sp[species].cap ? t.alloc[species] : c->h.sp[species].cap;
  const int set = t.cur[species];
  const SpeciesDev& S = c->h.sp[species];
  std::vector<double> hx(n), hvx(n), hvy(n), hvz(n);
  std::vector<uint64_t> hu(n);
  if (n > 0) {
    HIPCHK(hipMemcpy(hx.data(), S.x[set], n * 8, hipMemcpyDeviceToHost));
    HIPCHK(hipMemcpy(hvx.data(), S.vx[set], n * 8, hipMemcpyDeviceToHost));
    HIPCHK(hipMemcpy(hvy.data(), S.vy[set], n * 8, hipMemcpyDeviceToHost));
    HIPCHK(hipMemcpy(hvz.data(), S.vz[set], n * 8, hipMemcpyDeviceToHost));
    HIPCHK(hipMemcpy(hu.data(), S.uid[set], n * 8, hipMemcpyDeviceToHost));
  }
  int64_t m = 0;
  for (int64_t i = 0; i < n; ++i) {
    if (!(hx[i] == hx[i])) continue;
    if (m < cap) {
      if (x) x[m] = hx[i];
      if (vx) vx[m] = hvx[i];
      if (vy) vy[m] = hvy[i];
      if (vz) vz[m] = hvz[i];
      if (uid) uid[m] = hu[i];
    }
    ++m;
  }
  if (n_out) *n_out = m;
  return EDP_OK;
}

int edp_set_state(edp_ctx* ctx, edp_case id, int32_t species, const double* x, const double* vx,
                  const double* vy, const double* vz, const uint64_t* uid, int64_t n, int64_t step) {
  Case* c = ctx ? find(ctx, id) : nullptr;
  if (!c || (species != 0 && species != 1) || n < 0 || step < 0) return fail(EDP_EINVAL, "bad argument");
  if (n > 0 && (!x || !vx || !vy || !vz || !uid)) return fail(EDP_EINVAL, "null array");
  const SpeciesDev& S = c->h.sp[species];
  if (n > S.cap) return fail(EDP_ESTATE, "%lld particles exceed capacity %lld", (long long)n, (long long)S.cap);
  // the kernels rely on every live particle being inside [0, L] with finite
  // velocity components
  for (int64_t i = 0; i < n; ++i) {
    if (!(x[i] >= 0.0 && x[i] <= c->h.L))
      return fail(EDP_EINVAL, "particle %lld at x = %g is outside [0, L]", (long long)i, x[i]);
    if (!std::isfinite(vx[i]) || !std::isfinite(vy[i]) || !std::isfinite(vz[i]))
      return fail(EDP_EINVAL, "particle %lld has a non-finite velocity", (long long)i);
  }
  // the other species keeps its state
  CaseDev t;
  int r = read_dyn(ctx, c, t);
  if (r) return r;
  if (n > 0) {
    HIPCHK(hipMemcpy(S.x[0], x, n * 8, hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(S.vx[0], vx, n * 8, hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(S.vy[0], vy, n * 8, hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(S.vz[0], vz, n * 8, hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(S.uid[0], uid, n * 8, hipMemcpyHostToDevice));
    if (species == 0) {
      // the float bound of vy*vy + vz*vz every kernel writer keeps
      std::vector<float> p2((size_t)n);
      for (int64_t i = 0; i < n; ++i) p2[i] = float_above(vy[i] * vy[i] + vz[i] * vz[i]);
      HIPCHK(hipMemcpy(S.vp2[0], p2.data(), n * 4, hipMemcpyHostToDevice));
    }
  }
  t.step = step;
  t.cur[species] = 0;
  t.alloc[species] = n;
  t.n[species] = n;
  const int64_t live_other = t.ctr[species == 0 ? kLiveI : kLiveE];
  for (int k = 0; k < kNumCtr; ++k) t.ctr[k] = 0;
  t.ctr[species == 0 ? kLiveE : kLiveI] = n;
  t.ctr[species == 0 ? kLiveI : kLiveE] = live_other;
  t.error = 0;
  t.diag_steps = 0;
  t.diag_ion_steps = 0;
  if ((r = write_dyn(ctx, c, t))) return r;
  c->step = step;
  c->est[species] = n;
  c->failed = false;
  if ((r = zero_diag(ctx, c))) return r;
  if ((r = deposit_species(ctx, c, species, step))) return r;
  HIPCHK(hipStreamSynchronize(ctx->stream));
  return EDP_OK;
}

int edp_set_option(edp_ctx* ctx, int32_t key, int64_t value) {
  if (!ctx) return fail(EDP_EINVAL, "null context");
  // every option changes what a captured step sequence contains (and some the
  // tables): drain both groups and rebuild on the next advance
  {
    const int r = reset_groups(ctx);
    if (r) return r;
  }
  switch (key) {
    case EDP_OPT_MODE:
      if (value < 0 || value > 1) return fail(EDP_EINVAL, "mode must be 0 or 1");
      ctx->mode = (int)value;
      break;
    case EDP_OPT_SORT_EVERY:
      if (value < 1) return fail(EDP_EINVAL, "sort interval must be >= 1");
      ctx->sort_every = (int)value;
      break;
    case EDP_OPT_PROFILE:
      ctx->profile = value ? 1 : 0;
      // create the pairs of a whole window up front, so that the host loop
      // that enqueues the timed launches creates none
      for (size_t n = ctx->ev_free.size() + ctx->ev_pairs.size(); ctx->profile && n < 4096; ++n) {
        hipEvent_t e0 = nullptr, e1 = nullptr;
        const int r = create_event_pair(e0, e1);
        if (r) return r;
        ctx->ev_free.emplace_back(e0, e1);
      }
      break;
    case EDP_OPT_GRAPH_STEPS:
      if (value < 0) return fail(EDP_EINVAL, "graph steps must be >= 0");
      ctx->graph_steps = (int)value;
      break;
    case EDP_OPT_POISSON:
      if (value < 0 || value > 1) return fail(EDP_EINVAL, "poisson solver must be 0 or 1");
      ctx->poisson = (int)value;
      break;
    case EDP_OPT_PART_WG_PER_CU:
      if (value < 0 || value > 64) return fail(EDP_EINVAL, "workgroups per CU must be 0..64");
      ctx->part_wg_per_cu = (int)value;
      break;
    case EDP_OPT_PRETEST:
      if (value < 0 || value > 2) return fail(EDP_EINVAL, "pre-test mode must be 0, 1 or 2");
      ctx->pretest = (int)value;
      break;
    case EDP_OPT_PART_SKEW:
      if (value < -1 || value > 900) return fail(EDP_EINVAL, "workgroup share skew must be -1..900 (per mille)");
      ctx->part_skew = (int)value;
      break;
    case EDP_OPT_GROUPS:
      static_assert(kMaxGroups == 4, "the message below names the limit");
      if (value < 1 || value > kMaxGroups) return fail(EDP_EINVAL, "groups must be 1..4");
      ctx->groups = (int)value;
      break;
    case EDP_OPT_SMALL_MAX:
      if (value < 0) return fail(EDP_EINVAL, "small-case limit must be >= 0");
      ctx->small_max = value;
      break;
    default:
      return fail(EDP_EINVAL, "unknown option %d", key);
  }
  return EDP_OK;
}

int edp_read_profile(edp_ctx* ctx, double* ms, int64_t* launches) {
  if (!ctx) return fail(EDP_EINVAL, "null context");
  HIPCHK(hipStreamSynchronize(ctx->stream));
  int r = drain_profile(ctx);
  if (r) return r;
  if (ms) *ms = ctx->prof_ms;
  if (launches) *launches = ctx->prof_launches;
  ctx->prof_ms = 0.0;
  ctx->prof_launches = 0;
  return EDP_OK;
}

}  // extern "C"
