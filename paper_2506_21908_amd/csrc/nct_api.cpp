// Host engine of libnct: the C ABI of include/nct.h.
//
// Owns the device workspace, the FFT tables (twiddles and digit-reversed
// |G|^2 per axis), the projector tables of every atom, and drives the
// kernels of one ETRS step on the caller's stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <complex>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/nct.h"
#include "nct_fft.hpp"
#include "nct_internal.hpp"
#include "nct_tables.hpp"

using namespace nct;
using nct::tables::gl24;

namespace {

constexpr double kPi = 3.14159265358979323846;
constexpr double kMuB = 0.5;  // Bohr magneton, atomic units
constexpr int kObsWidth = 13;

std::string g_create_error;

struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
};

}  // namespace

struct nct_system {
  nct_params prm{};
  int n[3] = {0, 0, 0};
  size_t N = 0;
  int S = 0;
  double dV = 0.0;
  bool fp64 = true;
  size_t cbytes = 16;   // bytes per complex element
  int cache_mode = 0;   // streaming policy of the state-sized passes (see stream_cache_mode)
  hipStream_t st = nullptr;
  hipStream_t st2 = nullptr;       // projector chain, overlapped with the column pass
  hipEvent_t ev_rows = nullptr;    // sphere rows ready (recorded on st)
  hipEvent_t ev_proj = nullptr;    // scatter rows ready (recorded on st2)
  // stream of the early kinetic pass: the next step's first column pass runs there while the
  // density and fields of the new states are formed on st
  hipStream_t stK = nullptr;
  hipEvent_t evK_in = nullptr, evK_out = nullptr;
  // second state group: its Taylor stages run on their own streams, overlapping the first
  // group's (states are contiguous in the state-major layout, so a group is a sub-array)
  int ngroups = 1;
  int S0 = 0;                      // states of group 0 (group 1: S - S0)
  hipStream_t stB = nullptr, stB2 = nullptr;
  hipEvent_t evB_rows = nullptr, evB_proj = nullptr, ev_fork = nullptr, ev_join = nullptr;
  void* CpartB = nullptr;
  void* CB = nullptr;
  void* ECB = nullptr;
  std::string err;
  std::vector<DevBuf> owned;
  // the static scratch array of this system's device (allocation-free entry point), or null
  void* scr = nullptr;
  size_t scr_bytes = 0;
  std::string scr_err;

  // host copies
  std::vector<double> occ_h;
  std::vector<double> positions_h;
  std::vector<nct_channel> channels_h;
  std::vector<nct_pulse> pulses;
  std::vector<nct_laser_pulse> laser;   // uniform electric pulses
  int laser_gauge = NCT_GAUGE_LENGTH;
  double* kv_zero64 = nullptr;          // [S][3] zeros: Bloch vectors for the velocity gauge at Gamma
  float* kv_zero32 = nullptr;
  double B0[3] = {0, 0, 0};
  bool frozen = false;
  bool fields_valid = false;

  // device: FFT tables (double and float)
  void* tw64[3] = {nullptr, nullptr, nullptr};
  void* tw32[3] = {nullptr, nullptr, nullptr};
  double* g2x64 = nullptr;
  double* g2yz64 = nullptr;
  float* g2x32 = nullptr;
  float* g2yz32 = nullptr;
  // signed G per axis (x digit-reversed, y and z per position of the transformed yz plane)
  double *gsx64 = nullptr, *gsy64 = nullptr, *gsz64 = nullptr;
  float *gsx32 = nullptr, *gsy32 = nullptr, *gsz32 = nullptr;
  // Bloch vectors [S][3] of the states (k-point sampling); null: Gamma only
  double* kv64 = nullptr;
  float* kv32 = nullptr;
  bool has_k = false;
  std::vector<int> krun;   // starts of the runs of consecutive states sharing one Bloch vector, + S
  bool krun_split = false; // some Bloch vector occurs in two separate runs

  // device: fields and densities (FP64)
  double* occ = nullptr;
  double* vext = nullptr;
  double* rho = nullptr;
  double* fields = nullptr;    // [4][N] v, b_xc (no B_ext)
  double* fields_scr = nullptr;
  float* fields32 = nullptr;
  void* ncpx = nullptr;        // complex double [N] Poisson work
  double* fpart = nullptr;     // [nblk][kFieldTot]
  double* ftot = nullptr;      // [kFieldTot]
  double* epart = nullptr;     // [2S][ntiles][2]
  double* obs_dev = nullptr;   // [cap][13]
  // per-step watchdog: N_e = sum_i f_i <psi_i|psi_i> after every self-consistent step of a call
  double* ne_hist = nullptr;   // [ne_cap]: slot 0 the initial states, slot k+1 after step k
  int ne_cap = 0;
  double max_ne_drift = 1e-3;  // relative drift of N_e that fails a step (<= 0: finiteness only)
  // ground state: S x S buffers of the orthonormalisation (complex double)
  void* ovl = nullptr;         // [S][S] overlap, then the triangular factor L^-H
  double* dm_atoms = nullptr;  // [natoms][9] atom data of the initial spin-density matrix
  void* ovl_part = nullptr;    // [nchunks][S][S] partial overlaps over chunks of the 2N values
  int ovl_nb = 0;
  std::vector<std::complex<double>> ovl_host;  // host copy of the factor (lives until its upload ends)
  int obs_cap = 0;

  // device: psi-sized work (precision of the system)
  void* psihat = nullptr;
  void* phi = nullptr;
  void* phihat = nullptr;
  void* wbuf = nullptr;
  void* tmp = nullptr;
  void* tmpk_phi = nullptr;   // kinetic column pass of phi (shared by the 2nd and 3rd exponentials)

  // projectors
  ProjTables pt;
  int natoms = 0;
  void* Wpsi = nullptr;
  void* Wphi = nullptr;
  void* Wwork = nullptr;
  void* Y = nullptr;
  void* Yphi = nullptr;       // scatter rows of phi's first stage, shared by the 2nd and 3rd exponentials
  void* Cpart = nullptr;
  void* C = nullptr;
  void* EC = nullptr;
  double* energy_dev = nullptr;

  // adjoint tape: per step 3K state vectors (Taylor iterates of the three exponentials,
  // psi_n, phi, psi~) and the densities / fields of H_n and H~
  struct Tape {
    int cap = 0;
    int valid = 0;
    double t0 = 0.0;
    void* vec = nullptr;      // [cap][3K] states
    double* rho = nullptr;    // [cap][2][4N]  rho(psi_n), rho(psi~)
    double* fld = nullptr;    // [cap][2][4N]  fields of H_n, H~ (without B_ext)
  };
  Tape tape;
  Tape scratch_tape;          // one step, for recompute mode
  void* scratch_out = nullptr;
  double* gA = nullptr;       // [4][N] field gradients
  double* gB = nullptr;
  double* gnm = nullptr;      // [4][N] density gradients
  double* gpart = nullptr;    // [nblk][4]
  double* gtot = nullptr;     // [2][4]: field-adjoint totals of H_n and H~

  // kernel timing (profiling aid)
  struct TimedLaunch {
    int k;
    hipEvent_t a, b;
    double bytes, flops;
  };
  bool timing = false;
  unsigned timing_mask = 0;  // bit k: record class k (1: only the plane pass; all ones: everything)
  int timing_every = 1;      // record one launch in this many of each class
  long long t_seen[NCT_K_COUNT] = {0};
  std::vector<TimedLaunch> pending;
  std::vector<hipEvent_t> free_events;
  double t_ms[NCT_K_COUNT] = {0};
  long long t_count[NCT_K_COUNT] = {0};
  double t_bytes[NCT_K_COUNT] = {0};
  double t_flops[NCT_K_COUNT] = {0};
};

namespace {

nct_status fail(nct_system* s, nct_status code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  if (s) s->err = buf;
  else g_create_error = buf;
  return code;
}

#define HIPCHK(sys, call)                                                                  \
  do {                                                                                     \
    hipError_t e_ = (call);                                                                \
    if (e_ != hipSuccess)                                                                  \
      return fail(sys, NCT_ERR_HIP, "%s failed: %s (%s:%d)", #call, hipGetErrorString(e_), \
                  __FILE__, __LINE__);                                                     \
  } while (0)

nct_status dalloc(nct_system* s, size_t bytes, void** out) {
  void* p = nullptr;
  if (bytes == 0) bytes = 16;
  hipError_t e = hipMalloc(&p, bytes);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return fail(s, NCT_ERR_OOM, "hipMalloc(%zu) failed: %s", bytes, hipGetErrorString(e));
  }
  s->owned.push_back({p, bytes});
  *out = p;
  return NCT_OK;
}

template <typename T>
nct_status upload(nct_system* s, const std::vector<T>& h, T** out) {
  void* p = nullptr;
  nct_status r = dalloc(s, h.size() * sizeof(T), &p);
  if (r != NCT_OK) return r;
  if (!h.empty()) HIPCHK(s, hipMemcpy(p, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice));
  *out = static_cast<T*>(p);
  return NCT_OK;
}

// ---------------------------------------------------------------- kernel timing
hipEvent_t take_event(nct_system* s) {
  if (!s->free_events.empty()) {
    hipEvent_t e = s->free_events.back();
    s->free_events.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

// Runs launch(); when timing is on, brackets it with events and books bytes/flops on class k.
template <typename F>
hipError_t timed_on(nct_system* s, hipStream_t st, int k, double bytes, double flops, F&& launch) {
  if (!s->timing || !((s->timing_mask >> k) & 1u)) return launch();
  if (s->t_seen[k]++ % s->timing_every != 0) return launch();
  hipEvent_t a = take_event(s), b = take_event(s);
  if (!a || !b) return launch();
  (void)st;  // the events ride on the dispatches themselves, on the stream they are launched on
  LaunchEvents& le = launch_events();
  le.start = a;
  le.stop = b;
  le.used = false;
  const hipError_t e = launch();
  const bool used = le.used;
  le = LaunchEvents{};
  if (e != hipSuccess || !used) {
    s->free_events.push_back(a);
    s->free_events.push_back(b);
    return e;
  }
  s->pending.push_back({k, a, b, bytes, flops});
  return hipSuccess;
}
template <typename F>
hipError_t timed(nct_system* s, int k, double bytes, double flops, F&& launch) {
  return timed_on(s, s->st, k, bytes, flops, launch);
}

// Call after the stream has been synchronised.
void harvest_timing(nct_system* s) {
  for (auto& t : s->pending) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, t.a, t.b) == hipSuccess) {
      s->t_ms[t.k] += ms;
      s->t_count[t.k] += 1;
      s->t_bytes[t.k] += t.bytes;
      s->t_flops[t.k] += t.flops;
    }
    s->free_events.push_back(t.a);
    s->free_events.push_back(t.b);
  }
  s->pending.clear();
}

// ---------------------------------------------------------------- FFT tables
// frequency index held at DIF output position pos (mixed radix, digit reversal)
std::vector<int> dif_position_to_freq(int Nl) {
  std::vector<int> rad;
  for (int s = 0; s < 4; ++s) {
    int r = plan_radix(Nl, s);
    if (!r) break;
    rad.push_back(r);
  }
  std::vector<int> m(rad.size());
  int prod = 1;
  for (size_t j = 0; j < rad.size(); ++j) {
    prod *= rad[j];
    m[j] = Nl / prod;
  }
  std::vector<int> k_at(Nl, -1);
  for (int k = 0; k < Nl; ++k) {
    int rem = k, pos = 0;
    for (size_t j = 0; j < rad.size(); ++j) {
      const int pj = rem % rad[j];
      rem /= rad[j];
      pos += pj * m[j];
    }
    k_at[pos] = k;
  }
  return k_at;
}

double gval(int k, int Nl, double Lc) {
  const int ks = (k < (Nl + 1) / 2) ? k : k - Nl;  // fftfreq convention
  return 2.0 * kPi * ks / Lc;
}

// Projector tables: built on the host (nct_tables.hpp), converted to the system's precision and
// uploaded.
template <typename R>
nct_status build_projectors(nct_system* s) {
  const nct_params& p = s->prm;
  s->natoms = (p.nchannels > 0) ? p.natoms : 0;
  if (s->natoms == 0) return NCT_OK;
  int P = 0;
  for (int c = 0; c < p.nchannels; ++c) P += p.channels[c].twoj + 1;
  if (P > 32) return fail(s, NCT_ERR_UNSUPPORTED, "at most 32 projectors per atom (got %d)", P);
  tables::ProjectorTables ht;
  const std::string why = tables::build_projector_tables(s->n, p.cell, s->natoms, p.positions, p.nchannels,
                                                         p.channels, p.r_sphere, ht);
  if (!why.empty()) return fail(s, NCT_ERR_ARG, "projector tables: %s", why.c_str());
  ProjTables& pt = s->pt;
  pt.natoms = s->natoms;
  pt.P = ht.P;
  pt.PP = ht.PP;
  pt.Jtot = ht.Jtot;
  pt.max_kchunks = ht.max_kchunks;
  pt.max_rowtiles = ht.max_rowtiles;
  int *d_row_off, *d_pidx, *d_pr_off, *d_pr_b, *d_pr_e;
  nct_status r;
  if ((r = upload(s, ht.row_off, &d_row_off)) != NCT_OK) return r;
  if ((r = upload(s, ht.pidx, &d_pidx)) != NCT_OK) return r;
  if ((r = upload(s, ht.pr_off, &d_pr_off)) != NCT_OK) return r;
  if ((r = upload(s, ht.pr_begin, &d_pr_b)) != NCT_OK) return r;
  if ((r = upload(s, ht.pr_end, &d_pr_e)) != NCT_OK) return r;
  if ((r = upload(s, ht.energy, &s->energy_dev)) != NCT_OK) return r;
  std::vector<R> braw(ht.beta.size() * 2);
  for (size_t k = 0; k < ht.beta.size(); ++k) {
    braw[2 * k] = R(ht.beta[k].real());
    braw[2 * k + 1] = R(ht.beta[k].imag());
  }
  R* d_beta;
  if ((r = upload(s, braw, &d_beta)) != NCT_OK) return r;
  std::vector<R> disp(ht.disp.begin(), ht.disp.end());
  R* d_disp;
  if ((r = upload(s, disp, &d_disp)) != NCT_OK) return r;
  pt.disp = d_disp;
  pt.row_off = d_row_off;
  pt.pidx = d_pidx;
  pt.pr_off = d_pr_off;
  pt.pr_begin = d_pr_b;
  pt.pr_end = d_pr_e;
  pt.beta = d_beta;
  pt.energy = s->energy_dev;
  const size_t rows = size_t(s->S) * 2 * pt.Jtot * s->cbytes;
  if ((r = dalloc(s, rows, &s->Wpsi)) != NCT_OK) return r;
  if ((r = dalloc(s, rows, &s->Wphi)) != NCT_OK) return r;
  if ((r = dalloc(s, rows, &s->Wwork)) != NCT_OK) return r;
  if ((r = dalloc(s, rows, &s->Y)) != NCT_OK) return r;
  if ((r = dalloc(s, rows, &s->Yphi)) != NCT_OK) return r;
  const size_t cp = size_t(s->natoms) * pt.PP * s->S;
  if ((r = dalloc(s, cp * pt.max_kchunks * 16, &s->Cpart)) != NCT_OK) return r;
  if ((r = dalloc(s, cp * 16, &s->C)) != NCT_OK) return r;
  if ((r = dalloc(s, cp * s->cbytes, &s->EC)) != NCT_OK) return r;
  return NCT_OK;
}

// ---------------------------------------------------------------- B(t)
void bfield_at(const nct_system* s, double t, double B[3]) {
  for (int k = 0; k < 3; ++k) B[k] = s->B0[k];
  for (const nct_pulse& p : s->pulses) {
    const double d = t - p.t0;
    const double g = std::exp(-d * d / (2 * p.tau * p.tau));
    const double ph = p.omega * d + p.phase;
    const double c = std::cos(ph), sn = std::sin(ph);
    for (int k = 0; k < 3; ++k) B[k] += p.A * g * (c * p.e1[k] + sn * p.e2[k]);
  }
}

// Uniform electric field E(t) of the laser pulses (zero without pulses)
void efield_at(const nct_system* s, double t, double E[3]) {
  E[0] = E[1] = E[2] = 0.0;
  for (const nct_laser_pulse& p : s->laser) {
    const double d = t - p.t0;
    const double g = std::exp(-d * d / (2 * p.tau * p.tau));
    const double a = p.A * std::cos(p.omega * t + p.phase) * g;
    for (int k = 0; k < 3; ++k) E[k] += a * p.pol[k];
  }
}

// Velocity-gauge vector potential A(t) = -int_0^t E dt' (composite 24-point Gauss-Legendre on
// panels no wider than a quarter of the shortest pulse width or period).
bool velocity_gauge(const nct_system* s) {
  return s->laser_gauge == NCT_GAUGE_VELOCITY && !s->laser.empty() && !s->frozen;
}
void vector_potential_at(const nct_system* s, double t, double A[3]) {
  A[0] = A[1] = A[2] = 0.0;
  if (s->laser.empty() || t == 0.0) return;
  const std::vector<double>& xs = gl24().x;
  const std::vector<double>& ws = gl24().w;
  double hmax = 1e300;
  for (const nct_laser_pulse& p : s->laser) {
    hmax = std::min(hmax, 0.25 * p.tau);
    if (p.omega != 0.0) hmax = std::min(hmax, 0.25 * 2.0 * kPi / std::fabs(p.omega));
  }
  const int panels = std::max(1, int(std::ceil(std::fabs(t) / hmax)));
  const double h = t / panels;
  for (int q = 0; q < panels; ++q) {
    const double a = q * h;
    for (size_t i = 0; i < xs.size(); ++i) {
      double E[3];
      efield_at(s, a + 0.5 * h * (xs[i] + 1.0), E);
      for (int d = 0; d < 3; ++d) A[d] -= 0.5 * h * ws[i] * E[d];
    }
  }
}

// Length-gauge potential v_E = E.(r - c) at grid point (ix, iy, iz) as lg[0] ix + lg[1] iy +
// lg[2] iz + lg[3]: lg[d] = E_d h_d, lg[3] = -E.c with c the cell centre.
void laser_coeffs(const nct_system* s, double t, double lg[4]) {
  double E[3];
  efield_at(s, t, E);
  lg[3] = 0.0;
  for (int d = 0; d < 3; ++d) {
    lg[d] = E[d] * (s->prm.cell[d] / s->n[d]);
    lg[3] -= E[d] * 0.5 * s->prm.cell[d];
  }
}

// d B / d theta, theta = (A_1..A_k, omega_1..omega_k); out [2k][3]
void bfield_jac(const nct_system* s, double t, std::vector<double>& out) {
  const size_t k = s->pulses.size();
  out.assign(2 * k * 3, 0.0);
  for (size_t i = 0; i < k; ++i) {
    const nct_pulse& p = s->pulses[i];
    const double d = t - p.t0;
    const double g = std::exp(-d * d / (2 * p.tau * p.tau));
    const double ph = p.omega * d + p.phase;
    const double c = std::cos(ph), sn = std::sin(ph);
    for (int q = 0; q < 3; ++q) {
      out[i * 3 + q] = g * (c * p.e1[q] + sn * p.e2[q]);
      out[(k + i) * 3 + q] = p.A * g * d * (-sn * p.e1[q] + c * p.e2[q]);
    }
  }
}

// ---------------------------------------------------------------- S x S host linear algebra
// A (column-major, Hermitian positive definite) = L L^H; on return A holds M = L^(-H) (upper
// triangular), so that Psi M has orthonormal columns when A is their overlap.  False if A is not
// positive definite.
bool cholesky_inverse_h(std::vector<std::complex<double>>& A, int n) {
  using C = std::complex<double>;
  std::vector<C> L(size_t(n) * n, C(0, 0));
  auto a = [&](int i, int j) -> C& { return A[size_t(i) + size_t(j) * n]; };
  auto l = [&](int i, int j) -> C& { return L[size_t(i) + size_t(j) * n]; };
  for (int j = 0; j < n; ++j) {
    double d = a(j, j).real();
    for (int k = 0; k < j; ++k) d -= std::norm(l(j, k));
    // a pivot that rounding alone can produce means linearly dependent columns
    if (!(d > 1e-12 * std::fabs(a(j, j).real())) || !std::isfinite(d)) return false;
    const double ljj = std::sqrt(d);
    l(j, j) = C(ljj, 0);
    for (int i = j + 1; i < n; ++i) {
      C acc = a(i, j);
      for (int k = 0; k < j; ++k) acc -= l(i, k) * std::conj(l(j, k));
      l(i, j) = acc / ljj;
    }
  }
  // M = L^(-H): solve L^H m_j = e_j by back substitution ((L^H)(i, k) = conj(L(k, i)))
  for (int j = 0; j < n; ++j) {
    for (int i = n - 1; i >= 0; --i) {
      C acc = (i == j) ? C(1, 0) : C(0, 0);
      for (int k = i + 1; k < n; ++k) acc -= std::conj(l(k, i)) * a(k, j);
      a(i, j) = acc / std::conj(l(i, i));
    }
  }
  return true;
}

// ---------------------------------------------------------------- engine
template <typename R>
struct Engine {
  nct_system* s;
  const void* twx() const { return sizeof(R) == 8 ? s->tw64[0] : s->tw32[0]; }
  const void* twy() const { return sizeof(R) == 8 ? s->tw64[1] : s->tw32[1]; }
  const void* twz() const { return sizeof(R) == 8 ? s->tw64[2] : s->tw32[2]; }
  const R* g2x() const { return sizeof(R) == 8 ? (const R*)s->g2x64 : (const R*)s->g2x32; }
  const R* g2yz() const { return sizeof(R) == 8 ? (const R*)s->g2yz64 : (const R*)s->g2yz32; }
  const R* kvR() const {
    if (s->has_k) return sizeof(R) == 8 ? (const R*)s->kv64 : (const R*)s->kv32;
    if (velocity_gauge(s)) return sizeof(R) == 8 ? (const R*)s->kv_zero64 : (const R*)s->kv_zero32;
    return nullptr;
  }
  KTables<R> ktab(int state_off = 0) const {
    KTables<R> k;
    k.gx = sizeof(R) == 8 ? (const R*)s->gsx64 : (const R*)s->gsx32;
    k.gy = sizeof(R) == 8 ? (const R*)s->gsy64 : (const R*)s->gsy32;
    k.gz = sizeof(R) == 8 ? (const R*)s->gsz64 : (const R*)s->gsz32;
    k.kv = kvR();
    k.state_off = state_off;
    for (int d = 0; d < 3; ++d) k.ka[d] = R(ka[d]);
    return k;
  }
  const R* fieldsR() const { return sizeof(R) == 8 ? (const R*)s->fields : (const R*)s->fields32; }
  double psiB() const { return 2.0 * s->S * double(s->N) * sizeof(R) * 2; }
  double rowsB() const { return 2.0 * s->S * double(s->pt.Jtot) * sizeof(R) * 2; }

  nct_status check(hipError_t e, const char* what) {
    if (e != hipSuccess) return fail(s, NCT_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
    return NCT_OK;
  }

  // where the next field update also records its electron count (per-step watchdog), or null
  double* ne_slot = nullptr;
  // temporaries of the field update: the system's own buffers unless set (the allocation-free
  // entry point points them into the static scratch array)
  void* w_ncpx = nullptr;     // complex double [N] Poisson work
  double* w_fscr = nullptr;   // [4][N] fields output when they are not kept
  double* w_fpart = nullptr;  // [nblk][kFieldTot] block partial sums
  double* w_ftot = nullptr;   // [kFieldTot] totals
  void* ncpx() const { return w_ncpx ? w_ncpx : s->ncpx; }
  double* fscr() const { return w_fscr ? w_fscr : s->fields_scr; }
  double* fpart() const { return w_fpart ? w_fpart : s->fpart; }
  double* ftot() const { return w_ftot ? w_ftot : s->ftot; }

  // Hartree + exchange fields from the density in s->rho (FP64 throughout)
  nct_status fields_from_rho(bool store) {
    nct_status r;
    void* const pw = ncpx();
    const double* vh = nullptr;
    const double N = double(s->N);
    const int K = NCT_K_FIELDS;
    if (s->prm.hartree) {
      if ((r = check(timed(s, K, 32 * N, 0, [&] {
             return launch_plane_fwd_real(s->n, s->rho, 1, pw, s->tw64[1], s->tw64[2], s->st); }),
                     "poisson fwd")) != NCT_OK) return r;
      if ((r = check(timed(s, K, 32 * N, 0, [&] {
             return launch_xpass<double>(s->n, 1, pw, pw, s->g2x64, s->g2yz64,
                                         4.0 * kPi / double(s->N), 1, s->tw64[0], s->st); }),
                     "poisson x")) != NCT_OK) return r;
      if ((r = check(timed(s, K, 32 * N, 0, [&] {
             return launch_plane_inv<double>(s->n, 1, pw, pw, 1.0, s->tw64[1], s->tw64[2],
                                             s->st); }), "poisson inv")) != NCT_OK) return r;
      vh = reinterpret_cast<const double*>(pw);  // v_H: the real parts
    }
    int nb = 0;
    double* out = store ? s->fields : fscr();
    float* o32 = (store && !s->fp64) ? s->fields32 : nullptr;
    if ((r = check(timed(s, K, (32 + 16 + 32 + (o32 ? 16 : 0)) * N, 0, [&] {
           return launch_fields(s->rho, s->vext, vh, s->prm.xc, s->prm.m_threshold, s->n, s->prm.cell, out, o32,
                                fpart(), &nb, s->st); }), "fields")) != NCT_OK) return r;
    if ((r = check(timed(s, K, 8.0 * kFieldTot * nb, 0, [&] {
           return launch_reduce_rows(fpart(), nb, kFieldTot, ftot(), s->st, ne_slot); }),
                   "reduce")) != NCT_OK) return r;
    if (store) s->fields_valid = true;
    return NCT_OK;
  }

  nct_status density(const void* psi) {
    return check(timed(s, NCT_K_DENSITY, psiB() + 32.0 * s->N, 0, [&] {
                   return launch_density<R>(psi, s->occ, s->S, s->N, s->rho, s->st); }), "density");
  }

  // useful flops of one projector GEMM (contraction or scatter): 8 per complex multiply-add over
  // the P projectors of every atom (not the padded PP columns the MFMA tiles also compute)
  double proj_flops() const { return 8.0 * s->pt.P * 2.0 * s->pt.Jtot * s->S; }
  double beta_bytes() const { return 2.0 * s->pt.Jtot * s->pt.PP * sizeof(R) * 2; }

  nct_status contract(const void* W, hipStream_t st) {
    const double cpB = double(s->natoms) * s->pt.PP * s->S * 16.0;
    return check(timed_on(s, st, NCT_K_PROJ, rowsB() + beta_bytes() + cpB * s->pt.max_kchunks, proj_flops(), [&] {
                   return launch_proj_contract<R>(s->pt, W, s->S, s->dV, s->Cpart, s->C, s->EC, st); }),
                 "proj_contract");
  }

  // NL projections of the sphere rows W -> Y (scatter rows) and C.  Enqueued on the second
  // stream after the rows are ready; join_projections() makes the main stream wait for Y.
  nct_status projections(const void* W) {
    if (s->natoms == 0) return NCT_OK;
    nct_status r;
    HIPCHK(s, hipEventRecord(s->ev_rows, s->st));
    HIPCHK(s, hipStreamWaitEvent(s->st2, s->ev_rows, 0));
    if ((r = contract(W, s->st2)) != NCT_OK) return r;
    const double ecB = double(s->natoms) * s->pt.PP * s->S * sizeof(R) * 2;
    if ((r = check(timed_on(s, s->st2, NCT_K_PROJ, beta_bytes() + ecB + rowsB(), proj_flops(), [&] {
                     return launch_proj_scatter<R>(s->pt, s->EC, s->S, s->Y, s->st2); }), "proj_scatter")) != NCT_OK)
      return r;
    HIPCHK(s, hipEventRecord(s->ev_proj, s->st2));
    return NCT_OK;
  }
  nct_status join_projections() {
    if (s->natoms == 0) return NCT_OK;
    HIPCHK(s, hipStreamWaitEvent(s->st, s->ev_proj, 0));
    return NCT_OK;
  }

  // velocity-gauge vector potential of the H being applied (zero otherwise)
  double ka[3] = {0, 0, 0};
  void at_time(double t) {
    if (velocity_gauge(s)) vector_potential_at(s, t, ka);
    else ka[0] = ka[1] = ka[2] = 0.0;
  }

  // external fields of a plane-pass stage at time t: mu_B B_ext(t) and the laser (length-gauge
  // potential, or the velocity-gauge shift of the Bloch vectors)
  void externals(double t, StageArgs<R>& sa) {
    bext_now(t, sa.bext);
    at_time(t);
    double lg[4] = {0, 0, 0, 0};
    if (!s->frozen && !s->laser.empty() && !velocity_gauge(s)) laser_coeffs(s, t, lg);
    for (int k = 0; k < 4; ++k) sa.lg[k] = R(lg[k]);
    for (int k = 0; k < 3; ++k) sa.ka[k] = R(ka[k]);
  }

  void bext_now(double t, R out[3]) {
    if (s->frozen) {
      out[0] = out[1] = out[2] = R(0);
      return;
    }
    double B[3];
    bfield_at(s, t, B);
    for (int k = 0; k < 3; ++k) out[k] = R(kMuB * B[k]);
  }

  nct_status xpass(const void* src, void* dst) {
    return check(timed(s, NCT_K_XPASS, 2 * psiB(), 0, [&] {
                   return launch_xpass<R>(s->n, 2 * s->S, src, dst, g2x(), g2yz(), R(0.5 / double(s->N)),
                                          0, twx(), s->st, s->cache_mode, ktab()); }), "xpass");
  }

  nct_status plane_stage(const StageArgs<R>& sa) {
    double b = psiB();                                     // tmp_in
    if (sa.w_in) b += psiB();
    if (sa.x_base && sa.x_base != sa.w_in) b += psiB();
    b += 4.0 * s->N * sizeof(R);                           // fields
    if (sa.Y) b += rowsB();
    if (sa.w_out) b += psiB();
    if (sa.tmp_out) b += psiB();
    if (sa.W) b += rowsB();
    if (sa.acc) b += 2 * psiB();
    return check(timed(s, NCT_K_PLANE_STAGE, b, 0, [&] {
                   return launch_plane_stage<R>(s->n, s->S, sa, s->pt, twy(), twz(), s->st); }),
                 "plane_stage");
  }

  // ---- state groups
  struct Group {
    int i0, S;
    hipStream_t st, st2;
    hipEvent_t ev_rows, ev_proj;
    void *Cpart, *C, *EC;
  };
  int groups(Group* g) const {
    g[0] = {0, s->ngroups > 1 ? s->S0 : s->S, s->st, s->st2, s->ev_rows, s->ev_proj, s->Cpart, s->C, s->EC};
    if (s->ngroups == 1) return 1;
    g[1] = {s->S0, s->S - s->S0, s->stB, s->stB2, s->evB_rows, s->evB_proj, s->CpartB, s->CB, s->ECB};
    return 2;
  }
  template <typename P>
  P* offs(P* p, int i0) const {  // states
    return p ? reinterpret_cast<P*>(const_cast<char*>(reinterpret_cast<const char*>(p)) +
                                    size_t(i0) * 2 * s->N * sizeof(R) * 2)
             : nullptr;
  }
  template <typename P>
  P* offr(P* p, int i0) const {  // sphere rows
    return p ? reinterpret_cast<P*>(const_cast<char*>(reinterpret_cast<const char*>(p)) +
                                    size_t(i0) * 2 * s->pt.Jtot * sizeof(R) * 2)
             : nullptr;
  }
  nct_status fork_groups() {
    if (s->ngroups == 1) return NCT_OK;
    HIPCHK(s, hipEventRecord(s->ev_fork, s->st));
    HIPCHK(s, hipStreamWaitEvent(s->stB, s->ev_fork, 0));
    return NCT_OK;
  }
  nct_status join_groups() {
    if (s->ngroups == 1) return NCT_OK;
    HIPCHK(s, hipEventRecord(s->ev_join, s->stB));
    HIPCHK(s, hipStreamWaitEvent(s->st, s->ev_join, 0));
    return NCT_OK;
  }

  // One H application of a state group: projector chain of rows cW (second stream, joined
  // before the plane pass), column pass of chat into tmp, fused plane pass described by sa
  // (full-size pointers; offset here to the group).
  // kin_dst: column-pass output buffer (default s->tmp); chat == nullptr: skip the column pass,
  // sa_full.tmp_in already holds it.
  nct_status stage_group(const Group& g, const void* cW, const void* chat, const StageArgs<R>& sa_full,
                         void* kin_dst = nullptr, void* y_dst = nullptr, const void* y_src = nullptr) {
    nct_status r;
    const double frac = double(g.S) / double(s->S);
    void* ybuf = y_dst ? y_dst : s->Y;
    if (s->natoms && !y_src) {
      HIPCHK(s, hipEventRecord(g.ev_rows, g.st));
      HIPCHK(s, hipStreamWaitEvent(g.st2, g.ev_rows, 0));
      const double cpB = double(s->natoms) * s->pt.PP * g.S * 16.0;
      if ((r = check(timed_on(s, g.st2, NCT_K_PROJ, frac * (rowsB() + beta_bytes()) + cpB * s->pt.max_kchunks,
                              frac * proj_flops(), [&] {
                                return launch_proj_contract<R>(s->pt, offr(cW, g.i0), g.S, s->dV, g.Cpart, g.C,
                                                               g.EC, g.st2); }), "proj_contract")) != NCT_OK)
        return r;
      const double ecB = double(s->natoms) * s->pt.PP * g.S * sizeof(R) * 2;
      if ((r = check(timed_on(s, g.st2, NCT_K_PROJ, beta_bytes() + ecB + frac * rowsB(), frac * proj_flops(), [&] {
                       return launch_proj_scatter<R>(s->pt, g.EC, g.S, offr(ybuf, g.i0), g.st2); }),
                     "proj_scatter")) != NCT_OK)
        return r;
      HIPCHK(s, hipEventRecord(g.ev_proj, g.st2));
    }
    if (chat) {
      void* dst = kin_dst ? kin_dst : s->tmp;
      if ((r = check(timed_on(s, g.st, NCT_K_XPASS, 2 * psiB() * frac, 0, [&] {
             return launch_xpass<R>(s->n, 2 * g.S, offs(chat, g.i0), offs(dst, g.i0), g2x(), g2yz(),
                                    R(0.5 / double(s->N)), 0, twx(), g.st, s->cache_mode, ktab(g.i0)); }), "xpass")) != NCT_OK)
        return r;
    }
    if (s->natoms && !y_src) HIPCHK(s, hipStreamWaitEvent(g.st, g.ev_proj, 0));
    StageArgs<R> sa = sa_full;
    sa.tmp_in = offs(sa.tmp_in, g.i0);
    sa.tmp_out = offs(sa.tmp_out, g.i0);
    sa.w_in = offs(sa.w_in, g.i0);
    sa.x_base = offs(sa.x_base, g.i0);
    sa.w_out = offs(sa.w_out, g.i0);
    sa.acc = offs(sa.acc, g.i0);
    sa.Y = s->natoms ? offr(y_src ? y_src : ybuf, g.i0) : nullptr;
    sa.W = offr(sa.W, g.i0);
    sa.state_off = g.i0;
    double b = psiB();
    if (sa.w_in) b += psiB();
    if (sa.x_base && sa.x_base != sa.w_in) b += psiB();
    if (sa.Y) b += rowsB();
    if (sa.w_out) b += psiB();
    if (sa.tmp_out) b += psiB();
    if (sa.W) b += rowsB();
    if (sa.acc) b += 2 * psiB();
    b = b * frac + 4.0 * s->N * sizeof(R);
    return check(timed_on(s, g.st, NCT_K_PLANE_STAGE, b, 0, [&] {
                   return launch_plane_stage<R>(s->n, g.S, sa, s->pt, twy(), twz(), g.st); }),
                 "plane_stage");
  }

  // imaginary time: when > 0, taylor() forms T_K(-imag_tau H) x (real Horner coefficients)
  double imag_tau = 0.0;

  // Horner coefficient of stage k: -i a/(K-k+1), or -imag_tau/(K-k+1) in imaginary time
  void set_coeff(StageArgs<R>& sa, int k, int K, double a) const {
    if (imag_tau > 0.0) {
      sa.cre = R(-imag_tau / double(K - k + 1));
      sa.cim = R(0);
    } else {
      sa.cre = R(0);
      sa.cim = R(-a / double(K - k + 1));
    }
  }

  // T_K(-i a H) x by Horner stages w_k = x + (-i a/(K-k+1)) H w_{k-1}, w_0 = x.
  // stage_out[k-1] (k = 1..K-1), if given, receives w_k (the adjoint tape); else the work buffer.
  // kin_save: keep the first stage's column pass in this buffer; kin_reuse: take the first
  // stage's column pass from this buffer instead of recomputing it (same x, fields-independent).
  // y_save / y_reuse: the same for the first stage's projector scatter rows (they depend on x
  // and the Bloch phases only).
  nct_status taylor(const void* x, const void* xhat, const void* xW, void* out, void* outhat,
                    void* outW, double t, void* const* stage_out = nullptr, void* kin_save = nullptr,
                    const void* kin_reuse = nullptr, void* y_save = nullptr, const void* y_reuse = nullptr) {
    const int K = s->prm.taylor_order;
    const double a = 0.5 * s->prm.dt;
    const void* cw = x;
    const void* chat = xhat;
    const void* cW = xW;
    StageArgs<R> sa;
    sa.cache_mode = s->cache_mode;
    sa.kv = kvR();
    externals(t, sa);
    sa.fields = fieldsR();
    nct_status r;
    Group G[2];
    const int ng = groups(G);
    if ((r = fork_groups()) != NCT_OK) return r;
    for (int k = 1; k <= K; ++k) {
      const bool last = (k == K);
      const bool first = (k == 1);
      sa.tmp_in = s->tmp;
      if (first && kin_reuse) sa.tmp_in = kin_reuse;
      if (first && kin_save) sa.tmp_in = kin_save;
      sa.w_in = cw;
      sa.x_base = x;
      sa.alpha = R(1);
      set_coeff(sa, k, K, a);
      sa.w_out = last ? out : (stage_out ? stage_out[k - 1] : s->wbuf);
      sa.tmp_out = last ? outhat : s->tmp;
      sa.W = s->natoms ? (last ? outW : s->Wwork) : nullptr;
      sa.acc = nullptr;
      for (int gi = 0; gi < ng; ++gi)
        if ((r = stage_group(G[gi], cW, (first && kin_reuse) ? nullptr : chat, sa, first ? kin_save : nullptr,
                             first ? y_save : nullptr, first ? y_reuse : nullptr)) != NCT_OK)
          return r;
      cw = sa.w_out;
      chat = sa.tmp_out;
      cW = sa.W;
    }
    return join_groups();
  }

  // The next step's first column pass (kinetic part for psi^ at time t) into s->tmp on stK, so
  // that it overlaps the density and field update that follow on st; that step's first Taylor
  // stage takes it as kin_reuse after waiting for evK_out.
  nct_status early_kinetic(double t) {
    at_time(t);
    HIPCHK(s, hipEventRecord(s->evK_in, s->st));
    HIPCHK(s, hipStreamWaitEvent(s->stK, s->evK_in, 0));
    nct_status r = check(timed_on(s, s->stK, NCT_K_XPASS, 2 * psiB(), 0, [&] {
                           return launch_xpass<R>(s->n, 2 * s->S, s->psihat, s->tmp, g2x(), g2yz(),
                                                  R(0.5 / double(s->N)), 0, twx(), s->stK, s->cache_mode,
                                                  ktab()); }), "xpass");
    if (r != NCT_OK) return r;
    HIPCHK(s, hipEventRecord(s->evK_out, s->stK));
    return NCT_OK;
  }

  nct_status prepare(const void* psi, void* hat, void* W) {
    return check(timed(s, NCT_K_PLANE_FWD, 2 * psiB() + (s->natoms ? rowsB() : 0.0), 0, [&] {
                   return launch_plane_fwd<R>(s->n, 2 * s->S, psi, hat, s->natoms ? W : nullptr, &s->pt,
                                              twy(), twz(), s->st, ktab()); }), "plane_fwd");
  }

  nct_status obs_row(double t, double* row) {
    nct_status r;
    int ntiles = 0;
    at_time(t);
    if ((r = check(timed(s, NCT_K_OBS, psiB(), 0, [&] {
           return launch_xpass_energy<R>(s->n, 2 * s->S, s->psihat, g2x(), g2yz(), R(0.5 / double(s->N)),
                                         twx(), s->epart, &ntiles, s->st, ktab()); }), "energy")) != NCT_OK)
      return r;
    if (s->natoms) {
      if ((r = contract(s->Wpsi, s->st)) != NCT_OK) return r;
    }
    ObsInputs in;
    in.field_tot = s->ftot;
    in.epart = s->epart;
    in.ntiles = ntiles;
    in.C = s->natoms ? s->C : nullptr;
    in.energy = s->energy_dev;
    in.occ = s->occ;
    in.S = s->S;
    in.natoms = s->natoms;
    in.PP = s->pt.PP;
    in.precision = s->prm.precision;
    in.dV = s->dV;
    in.invN = 1.0 / double(s->N);
    in.t = t;
    double B[3] = {0, 0, 0}, E[3] = {0, 0, 0};
    if (!s->frozen) {
      bfield_at(s, t, B);
      if (!velocity_gauge(s)) efield_at(s, t, E);
    }
    for (int k = 0; k < 3; ++k) {
      in.muB_B[k] = kMuB * B[k];
      in.efield[k] = E[k];
    }
    return check(timed(s, NCT_K_OBS, 0, 0, [&] { return launch_obs_row(in, row, s->st); }), "obs_row");
  }

  void* tvec(nct_system::Tape& T, int step, int j) const {
    const int K = s->prm.taylor_order;
    const size_t psib = size_t(psiB());
    return static_cast<char*>(T.vec) + (size_t(step) * 3 * K + j) * psib;
  }
  double* trho(nct_system::Tape& T, int step, int which) const {
    return T.rho + (size_t(step) * 2 + which) * 4 * s->N;
  }
  double* tfld(nct_system::Tape& T, int step, int which) const {
    return T.fld + (size_t(step) * 2 + which) * 4 * s->N;
  }
  nct_status save_fields(nct_system::Tape& T, int step, int which) {
    HIPCHK(s, hipMemcpyAsync(trho(T, step, which), s->rho, 4 * s->N * 8, hipMemcpyDeviceToDevice, s->st));
    HIPCHK(s, hipMemcpyAsync(tfld(T, step, which), s->fields, 4 * s->N * 8, hipMemcpyDeviceToDevice, s->st));
    return NCT_OK;
  }

  // nsteps ETRS steps.  With a tape, step k's Taylor iterates are written straight into the tape
  // (slots: exp 1 -> 0..K-1 with slot 0 = psi_n, exp 2 -> K..2K-1 with slot K = phi,
  // exp 3 -> 2K..3K-2, slot 3K-1 = psi~); psi_{n+1} lands in slot 0 of step n+1.
  nct_status step(void* psi, double t0, int nsteps, double* obs_host, nct_system::Tape* T = nullptr) {
    nct_status r;
    const double dt = s->prm.dt;
    const int K = s->prm.taylor_order;
    void* cur = psi;
    if (T) {
      HIPCHK(s, hipMemcpyAsync(tvec(*T, 0, 0), psi, size_t(psiB()), hipMemcpyDeviceToDevice, s->st));
      cur = tvec(*T, 0, 0);
      T->valid = 0;
      T->t0 = t0;
    }
    at_time(t0);
    if ((r = prepare(cur, s->psihat, s->Wpsi)) != NCT_OK) return r;
    if (nsteps > 0 && (r = early_kinetic(t0)) != NCT_OK) return r;
    if (!s->frozen) {
      if ((r = density(cur)) != NCT_OK) return r;
      if ((r = fields_from_rho(true)) != NCT_OK) return r;
    }
    if (obs_host && s->obs_cap < nsteps) {
      void* p;
      if ((r = dalloc(s, size_t(nsteps) * kObsWidth * sizeof(double), &p)) != NCT_OK) return r;
      s->obs_dev = static_cast<double*>(p);
      s->obs_cap = nsteps;
    }
    // per-step watchdog: every self-consistent step already reduces N_e with its fields; that
    // value is kept per step on the device and checked once at the end of the call
    const bool watch = !s->frozen;
    if (watch && s->ne_cap < nsteps + 1) {
      void* p;
      if ((r = dalloc(s, size_t(nsteps + 1) * sizeof(double), &p)) != NCT_OK) return r;
      s->ne_hist = static_cast<double*>(p);
      s->ne_cap = nsteps + 1;
    }
    if (watch) {  // N_e of the initial states (their fields were formed above)
      HIPCHK(s, hipMemcpyAsync(s->ne_hist, s->ftot, sizeof(double), hipMemcpyDeviceToDevice, s->st));
    }
    std::vector<void*> so1(K > 1 ? K - 1 : 1), so2(K > 1 ? K - 1 : 1), so3(K > 1 ? K - 1 : 1);
    for (int k = 0; k < nsteps; ++k) {
      const double t = t0 + k * dt;
      void* phi = s->phi;
      void* ptil = s->wbuf;
      void* next = psi;
      if (T) {
        if ((r = save_fields(*T, k, 0)) != NCT_OK) return r;
        for (int j = 1; j < K; ++j) {
          so1[j - 1] = tvec(*T, k, j);
          so2[j - 1] = tvec(*T, k, K + j);
          so3[j - 1] = tvec(*T, k, 2 * K + j - 1);
        }
        phi = tvec(*T, k, K);
        ptil = tvec(*T, k, 3 * K - 1);
        next = (k + 1 < nsteps) ? tvec(*T, k + 1, 0) : psi;
      }
      // the first column pass ran early on stK (early_kinetic)
      HIPCHK(s, hipStreamWaitEvent(s->st, s->evK_out, 0));
      if ((r = taylor(cur, s->psihat, s->Wpsi, phi, s->phihat, s->Wphi, t, T ? so1.data() : nullptr, nullptr,
                      s->tmp)) != NCT_OK)
        return r;
      // the second and third exponentials share phi's kinetic column pass and first scatter rows
      // unless the kinetic term and the projector phases depend on time (velocity-gauge laser)
      const bool vg = velocity_gauge(s);
      void* yphi = (vg || !s->natoms) ? nullptr : s->Yphi;
      if ((r = taylor(phi, s->phihat, s->Wphi, ptil, nullptr, nullptr, t, T ? so2.data() : nullptr,
                      vg ? nullptr : s->tmpk_phi, nullptr, yphi)) != NCT_OK)
        return r;
      if (!s->frozen) {
        if ((r = density(ptil)) != NCT_OK) return r;
        if ((r = fields_from_rho(true)) != NCT_OK) return r;
      }
      if (T && (r = save_fields(*T, k, 1)) != NCT_OK) return r;
      if (vg && s->natoms) {  // phi's rows were gathered under A(t): carry them to A(t + dt)
        double a0[3], a1[3], dA[3];
        vector_potential_at(s, t, a0);
        vector_potential_at(s, t + dt, a1);
        for (int d = 0; d < 3; ++d) dA[d] = a1[d] - a0[d];
        if ((r = check(launch_rephase_rows<R>(s->pt, s->Wphi, s->S, dA, s->st), "rephase")) != NCT_OK)
          return r;
      }
      if ((r = taylor(phi, s->phihat, s->Wphi, next, s->psihat, s->Wpsi, t + dt, T ? so3.data() : nullptr,
                      nullptr, vg ? nullptr : s->tmpk_phi, nullptr, yphi)) != NCT_OK)
        return r;
      cur = next;
      if (k + 1 < nsteps && (r = early_kinetic(t + dt)) != NCT_OK) return r;
      if (!s->frozen || obs_host) {
        if ((r = density(cur)) != NCT_OK) return r;
        ne_slot = watch ? s->ne_hist + k + 1 : nullptr;
        r = fields_from_rho(!s->frozen);
        ne_slot = nullptr;
        if (r != NCT_OK) return r;
      }
      if (obs_host) {
        if ((r = obs_row(t + dt, s->obs_dev + size_t(k) * kObsWidth)) != NCT_OK) return r;
      }
    }
    if (s->frozen && !obs_host) {  // frozen fields: one density at the end for the finiteness check
      if ((r = density(cur)) != NCT_OK) return r;
      if ((r = fields_from_rho(false)) != NCT_OK) return r;
    }
    double tot[8];
    HIPCHK(s, hipMemcpyAsync(tot, s->ftot, sizeof(tot), hipMemcpyDeviceToHost, s->st));
    if (obs_host)
      HIPCHK(s, hipMemcpyAsync(obs_host, s->obs_dev, size_t(nsteps) * kObsWidth * sizeof(double),
                               hipMemcpyDeviceToHost, s->st));
    std::vector<double> ne(watch ? nsteps + 1 : 0);
    if (watch)
      HIPCHK(s, hipMemcpyAsync(ne.data(), s->ne_hist, ne.size() * sizeof(double), hipMemcpyDeviceToHost, s->st));
    HIPCHK(s, hipStreamSynchronize(s->st));
    harvest_timing(s);
    if (T) T->valid = nsteps;
    for (int k = 1; k <= (watch ? nsteps : 0); ++k) {
      if (!std::isfinite(ne[k]))
        return fail(s, NCT_ERR_NONFINITE, "step %d of the call: non-finite electron count", k - 1);
      const double drift = std::fabs(ne[k] - ne[0]) / std::max(std::fabs(ne[0]), 1e-300);
      if (s->max_ne_drift > 0.0 && drift > s->max_ne_drift)
        return fail(s, NCT_ERR_NONFINITE,
                    "step %d of the call: electron count drifted by %.3e relative (limit %.3e)", k - 1,
                    drift, s->max_ne_drift);
    }
    if (!std::isfinite(tot[0])) return fail(s, NCT_ERR_NONFINITE, "non-finite electron count after step");
    return NCT_OK;
  }

  // ------------------------------------------------------------ adjoint
  nct_status load_fields(const double* f64) {
    HIPCHK(s, hipMemcpyAsync(s->fields, f64, 4 * s->N * 8, hipMemcpyDeviceToDevice, s->st));
    if (!s->fp64) HIPCHK(s, launch_to_float(s->fields, 4 * s->N, s->fields32, s->st));
    return NCT_OK;
  }

  // Adjoint of one Taylor exponential w_K = T(-i a H) x (Horner stages, fields frozen):
  // given mu_K = lam_out, mu_{k-1} = conj(c_k) H mu_k, lam_x = sum_{k=0}^{K} mu_k (into acc,
  // which is set to mu_K first when acc_init, else mu_K is added), and for each stage the pair
  // term of dL/d(v, b) into g.  xs[k] = w_k (k = 0..K-1) from the forward tape.
  nct_status adjoint_taylor(const void* lam_out, void* const* xs, void* acc, bool acc_init, double* g,
                            double t) {
    nct_status r;
    const int K = s->prm.taylor_order;
    const double a = 0.5 * s->prm.dt;
    const size_t cnt = size_t(s->S) * 2 * s->N;
    if (acc_init) {
      HIPCHK(s, hipMemcpyAsync(acc, lam_out, size_t(psiB()), hipMemcpyDeviceToDevice, s->st));
    } else {
      if ((r = check(timed(s, NCT_K_ADJOINT, 3 * psiB(), 0, [&] {
             return launch_axpby<R>(acc, lam_out, cnt, R(1), R(0), R(1), s->st); }), "axpby")) != NCT_OK)
        return r;
    }
    StageArgs<R> sa;
    sa.cache_mode = s->cache_mode;
    sa.kv = kvR();
    externals(t, sa);  // first: the rows gathered below carry the Bloch phases at time t
    sa.fields = fieldsR();
    if ((r = prepare(lam_out, s->tmp, s->Wwork)) != NCT_OK) return r;
    const void* cur = lam_out;
    for (int k = K; k >= 1; --k) {
      const double gamma = a / double(K - k + 1);
      if ((r = check(timed(s, NCT_K_ADJOINT, 2 * psiB() + 64.0 * s->N, 0, [&] {
             return launch_pair<R>(cur, xs[k - 1], s->S, s->N, gamma, g, s->st); }), "pair")) != NCT_OK)
        return r;
      if ((r = projections(s->Wwork)) != NCT_OK) return r;
      if ((r = xpass(s->tmp, s->tmp)) != NCT_OK) return r;
      if ((r = join_projections()) != NCT_OK) return r;
      sa.tmp_in = s->tmp;
      sa.w_in = cur;
      sa.x_base = nullptr;
      sa.alpha = R(0);
      sa.cre = R(0);
      sa.cim = R(gamma);
      sa.Y = s->natoms ? s->Y : nullptr;
      sa.w_out = s->wbuf;
      sa.tmp_out = k > 1 ? s->tmp : nullptr;
      sa.W = (s->natoms && k > 1) ? s->Wwork : nullptr;
      sa.acc = acc;
      if ((r = plane_stage(sa)) != NCT_OK) return r;
      cur = s->wbuf;
    }
    return NCT_OK;
  }

  // (g_v, g_b) at the fields of density rho  ->  (g_n, g_m) into s->gnm; sum_r g_b into
  // s->gtot[4 slot .. 4 slot + 2] (device; read once at the end of the backward step).
  nct_status field_adjoint(const double* rho, const double* g, int slot) {
    nct_status r;
    const double N = double(s->N);
    const double* pgp = nullptr;
    if (s->prm.hartree) {
      if ((r = check(timed(s, NCT_K_ADJOINT, 24 * N, 0, [&] {
             return launch_plane_fwd_real(s->n, g, 2, s->ncpx, s->tw64[1], s->tw64[2], s->st); }),
                     "adj poisson fwd")) != NCT_OK) return r;
      if ((r = check(timed(s, NCT_K_ADJOINT, 32 * N, 0, [&] {
             return launch_xpass<double>(s->n, 1, s->ncpx, s->ncpx, s->g2x64, s->g2yz64,
                                         4.0 * kPi / double(s->N), 1, s->tw64[0], s->st); }),
                     "adj poisson x")) != NCT_OK) return r;
      if ((r = check(timed(s, NCT_K_ADJOINT, 32 * N, 0, [&] {
             return launch_plane_inv<double>(s->n, 1, s->ncpx, s->ncpx, 1.0, s->tw64[1], s->tw64[2],
                                             s->st); }), "adj poisson inv")) != NCT_OK) return r;
      pgp = reinterpret_cast<const double*>(s->ncpx);  // the real parts
    }
    int nb = 0;
    if ((r = check(timed(s, NCT_K_ADJOINT, 96 * N, 0, [&] {
           return launch_field_adjoint(rho, g, pgp, s->prm.xc, s->prm.m_threshold, s->N, s->gnm, s->gpart,
                                       &nb, s->st); }), "field_adjoint")) != NCT_OK) return r;
    return check(launch_reduce_rows(s->gpart, nb, 4, s->gtot + 4 * slot, s->st), "reduce");
  }

  nct_status backprop_density(const void* psi, void* lam, int add) {
    return check(timed(s, NCT_K_ADJOINT, (add ? 3 : 2) * psiB() + 32.0 * s->N, 0, [&] {
                   return launch_density_backprop<R>(psi, s->occ, s->gnm, s->S, s->N, add, lam, s->st); }),
                 "density_backprop");
  }

  // Reverse of one ETRS step (see the forward step for the tape slots).
  nct_status backward(nct_system::Tape& T, int idx, double t_n, const void* lam_np1, void* lam_n,
                      double dLdB[6]) {
    nct_status r;
    const int K = s->prm.taylor_order;
    const double dt = s->prm.dt;
    const size_t gb = 4 * s->N * 8;
    std::vector<void*> xs1(K), xs2(K), xs3(K);
    xs1[0] = tvec(T, idx, 0);
    xs2[0] = tvec(T, idx, K);
    xs3[0] = tvec(T, idx, K);
    for (int j = 1; j < K; ++j) {
      xs1[j] = tvec(T, idx, j);
      xs2[j] = tvec(T, idx, K + j);
      xs3[j] = tvec(T, idx, 2 * K + j - 1);
    }
    void* lamphi = s->phi;
    void* lamtil = s->phihat;
    // third exponential, fields of H~ at t_{n+1}
    if ((r = load_fields(tfld(T, idx, 1))) != NCT_OK) return r;
    HIPCHK(s, hipMemsetAsync(s->gA, 0, gb, s->st));
    if ((r = adjoint_taylor(lam_np1, xs3.data(), lamphi, true, s->gA, t_n + dt)) != NCT_OK) return r;
    if (s->frozen) {
      for (int k = 0; k < 6; ++k) dLdB[k] = 0.0;
    } else {
      if ((r = field_adjoint(trho(T, idx, 1), s->gA, 1)) != NCT_OK) return r;
      // density at psi~ -> lam_psi~, then the second exponential (fields of H_n)
      if ((r = backprop_density(tvec(T, idx, 3 * K - 1), lamtil, 0)) != NCT_OK) return r;
      if ((r = load_fields(tfld(T, idx, 0))) != NCT_OK) return r;
      HIPCHK(s, hipMemsetAsync(s->gB, 0, gb, s->st));
      if ((r = adjoint_taylor(lamtil, xs2.data(), lamphi, false, s->gB, t_n)) != NCT_OK) return r;
    }
    if (s->frozen) {
      HIPCHK(s, hipMemsetAsync(s->gB, 0, gb, s->st));
    } else {
      if ((r = load_fields(tfld(T, idx, 0))) != NCT_OK) return r;
    }
    // first exponential -> lam_n
    if ((r = adjoint_taylor(lamphi, xs1.data(), lam_n, true, s->gB, t_n)) != NCT_OK) return r;
    if (!s->frozen) {
      if ((r = field_adjoint(trho(T, idx, 0), s->gB, 0)) != NCT_OK) return r;
      if ((r = backprop_density(tvec(T, idx, 0), lam_n, 1)) != NCT_OK) return r;
    }
    double tot[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    if (!s->frozen) HIPCHK(s, hipMemcpyAsync(tot, s->gtot, sizeof(tot), hipMemcpyDeviceToHost, s->st));
    HIPCHK(s, hipStreamSynchronize(s->st));
    if (!s->frozen)
      for (int k = 0; k < 3; ++k) {
        dLdB[k] = kMuB * tot[k];
        dLdB[3 + k] = kMuB * tot[4 + k];
      }
    harvest_timing(s);
    return NCT_OK;
  }

  // ------------------------------------------------------------ ground state
  // S x S buffers of the orthonormalisation, allocated on first use
  nct_status ensure_ovl() {
    if (s->ovl_part) return NCT_OK;  // set last: a failed set-up is redone on the next call
    nct_status r;
    const size_t SS = size_t(s->S) * s->S;
    if (!s->ovl && (r = dalloc(s, SS * 16, &s->ovl)) != NCT_OK) return r;
    const int nb = gram_chunks(s->S, 2 * s->N);
    void* p = nullptr;
    if ((r = dalloc(s, size_t(nb) * SS * 16, &p)) != NCT_OK) return r;
    s->ovl_nb = nb;
    s->ovl_part = p;
    return NCT_OK;
  }

  // dst = src L^(-H), L L^H = dV src^H src (states as the columns of a 2N x S matrix)
  // Orthonormalise within each run of states that share one Bloch vector (their periodic
  // parts; states of different k are orthogonal through the Bloch factors).
  nct_status orthonormalize(const void* src, void* dst) {
    nct_status r;
    if ((r = ensure_ovl()) != NCT_OK) return r;
    std::vector<int> runs = s->has_k ? s->krun : std::vector<int>{0, s->S};
    for (size_t b = 0; b + 1 < runs.size(); ++b)
      if ((r = orthonormalize_run(src, dst, runs[b], runs[b + 1] - runs[b])) != NCT_OK) return r;
    return NCT_OK;
  }

  // One run of S states starting at state i0: the overlap dV A^H A on the matrix cores with FP64
  // accumulation (a split-K reduction over the 2N values of each state, summed in a fixed order),
  // its Cholesky factorisation and L^-H on the host, and the triangular change of basis
  // D_j = sum_{i <= j} A_i (L^-H)_ij on the matrix cores.
  nct_status orthonormalize_run(const void* src, void* dst, int i0, int S) {
    const size_t K2 = 2 * s->N;
    const char* A0 = static_cast<const char*>(src) + size_t(i0) * K2 * sizeof(R) * 2;
    char* D0 = static_cast<char*>(dst) + size_t(i0) * K2 * sizeof(R) * 2;
    const int nb = std::min(s->ovl_nb, gram_chunks(S, K2));
    // useful work: the S(S+1)/2 independent entries of the Hermitian overlap, 8 flops per
    // complex multiply-add; algorithmic bytes: the run read once
    const double gram_flops = 8.0 * K2 * double(S) * (S + 1) / 2;
    nct_status r;
    if ((r = check(timed(s, NCT_K_ORTH, double(S) * K2 * sizeof(R) * 2, gram_flops, [&] {
           return launch_gram<R>(A0, S, K2, s->dV, s->ovl_part, nb, s->ovl, s->st); }), "overlap")) != NCT_OK)
      return r;
    const size_t SS = size_t(S) * S;
    std::vector<std::complex<double>> h(SS);
    HIPCHK(s, hipMemcpyAsync(h.data(), s->ovl, SS * 16, hipMemcpyDeviceToHost, s->st));
    HIPCHK(s, hipStreamSynchronize(s->st));
    // column-major copy for the factorisation (row-major [i][j] on the device)
    std::vector<std::complex<double>> A(SS);
    for (int i = 0; i < S; ++i)
      for (int j = 0; j < S; ++j) A[size_t(i) + size_t(j) * S] = h[size_t(i) * S + j];
    if (!cholesky_inverse_h(A, S))
      return fail(s, NCT_ERR_NONFINITE, "overlap of the states is not positive definite");
    s->ovl_host.resize(SS);
    for (int i = 0; i < S; ++i)
      for (int j = 0; j < S; ++j) s->ovl_host[size_t(i) * S + j] = A[size_t(i) + size_t(j) * S];
    HIPCHK(s, hipMemcpyAsync(s->ovl, s->ovl_host.data(), SS * 16, hipMemcpyHostToDevice, s->st));
    const double tflops = 8.0 * K2 * double(S) * (S + 1) / 2;
    if ((r = check(timed(s, NCT_K_ORTH, 2.0 * K2 * S * sizeof(R) * 2 + SS * 16.0, tflops, [&] {
           return launch_basis_transform<R>(A0, s->ovl, S, K2, D0, s->st); }), "basis transform")) != NCT_OK)
      return r;
    HIPCHK(s, hipStreamSynchronize(s->st));  // the factor's host copy is reused by the next run
    return NCT_OK;
  }

  // Self-consistent imaginary-time iterations: psi <- orthonormalise(T_K(-tau H[rho]) psi),
  // rho <- rho(psi); energies[it] = total energy after iteration it.
  nct_status ground_state(void* psi, int niter, double tau, bool keep_fields, double* energies) {
    nct_status r;
    if ((r = orthonormalize(psi, s->phi)) != NCT_OK) return r;
    HIPCHK(s, hipMemcpyAsync(psi, s->phi, psiB(), hipMemcpyDeviceToDevice, s->st));
    if (s->frozen) {
      if (!s->fields_valid) return fail(s, NCT_ERR_STATE, "no fields");
    } else if (!(keep_fields && s->fields_valid)) {
      if ((r = density(psi)) != NCT_OK) return r;
      if ((r = fields_from_rho(true)) != NCT_OK) return r;
    }
    if (s->obs_cap < niter) {
      void* p;
      if ((r = dalloc(s, size_t(niter) * kObsWidth * sizeof(double), &p)) != NCT_OK) return r;
      s->obs_dev = static_cast<double*>(p);
      s->obs_cap = niter;
    }
    imag_tau = tau;
    for (int it = 0; it < niter; ++it) {
      at_time(0.0);
      if ((r = prepare(psi, s->psihat, s->Wpsi)) != NCT_OK) break;
      if ((r = taylor(psi, s->psihat, s->Wpsi, s->phi, nullptr, nullptr, 0.0)) != NCT_OK) break;
      if ((r = orthonormalize(s->phi, psi)) != NCT_OK) break;
      if ((r = density(psi)) != NCT_OK) break;
      if ((r = fields_from_rho(!s->frozen)) != NCT_OK) break;
      if ((r = prepare(psi, s->psihat, s->Wpsi)) != NCT_OK) break;
      if ((r = obs_row(0.0, s->obs_dev + size_t(it) * kObsWidth)) != NCT_OK) break;
    }
    imag_tau = 0.0;
    if (r != NCT_OK) return r;
    std::vector<double> rows(size_t(niter) * kObsWidth);
    if (niter > 0)
      HIPCHK(s, hipMemcpyAsync(rows.data(), s->obs_dev, rows.size() * sizeof(double), hipMemcpyDeviceToHost, s->st));
    HIPCHK(s, hipStreamSynchronize(s->st));
    harvest_timing(s);
    for (int it = 0; it < niter; ++it) {
      const double e = rows[size_t(it) * kObsWidth + 5];
      if (!std::isfinite(e)) return fail(s, NCT_ERR_NONFINITE, "non-finite energy at iteration %d", it);
      if (energies) energies[it] = e;
    }
    return NCT_OK;
  }

  nct_status apply(const void* psi, void* hpsi, double t) {
    nct_status r;
    at_time(t);
    if ((r = prepare(psi, s->tmp, s->Wwork)) != NCT_OK) return r;
    if ((r = projections(s->Wwork)) != NCT_OK) return r;
    if ((r = xpass(s->tmp, s->tmp)) != NCT_OK) return r;
    if ((r = join_projections()) != NCT_OK) return r;
    StageArgs<R> sa;
    sa.cache_mode = s->cache_mode;
    sa.kv = kvR();
    externals(t, sa);
    sa.fields = fieldsR();
    sa.tmp_in = s->tmp;
    sa.w_in = psi;
    sa.x_base = nullptr;
    sa.alpha = R(0);
    sa.cre = R(1);
    sa.cim = R(0);
    sa.Y = s->natoms ? s->Y : nullptr;
    sa.w_out = hpsi;
    return plane_stage(sa);
  }
};

template <typename R>
nct_status build_fft_tables(nct_system* s) {
  nct_status r;
  for (int d = 0; d < 3; ++d) {
    const int Nl = s->n[d];
    std::vector<double> t64(2 * Nl);
    std::vector<float> t32(2 * Nl);
    for (int e = 0; e < Nl; ++e) {
      const double ang = -2.0 * kPi * double(e) / double(Nl);
      t64[2 * e] = std::cos(ang);
      t64[2 * e + 1] = std::sin(ang);
      t32[2 * e] = float(t64[2 * e]);
      t32[2 * e + 1] = float(t64[2 * e + 1]);
    }
    double* p64;
    float* p32;
    if ((r = upload(s, t64, &p64)) != NCT_OK) return r;
    if ((r = upload(s, t32, &p32)) != NCT_OK) return r;
    s->tw64[d] = p64;
    s->tw32[d] = p32;
  }
  std::vector<int> kx = dif_position_to_freq(s->n[0]);
  std::vector<int> ky = dif_position_to_freq(s->n[1]);
  std::vector<int> kz = dif_position_to_freq(s->n[2]);
  std::vector<double> gx(s->n[0]), gyz(size_t(s->n[1]) * s->n[2]);
  for (int i = 0; i < s->n[0]; ++i) {
    const double g = gval(kx[i], s->n[0], s->prm.cell[0]);
    gx[i] = g * g;
  }
  for (int i = 0; i < s->n[1]; ++i)
    for (int j = 0; j < s->n[2]; ++j) {
      const double g1 = gval(ky[i], s->n[1], s->prm.cell[1]);
      const double g2 = gval(kz[j], s->n[2], s->prm.cell[2]);
      gyz[size_t(i) * s->n[2] + j] = g1 * g1 + g2 * g2;
    }
  std::vector<double> sx(s->n[0]), sy(size_t(s->n[1]) * s->n[2]), sz(size_t(s->n[1]) * s->n[2]);
  for (int i = 0; i < s->n[0]; ++i) sx[i] = gval(kx[i], s->n[0], s->prm.cell[0]);
  for (int i = 0; i < s->n[1]; ++i)
    for (int j = 0; j < s->n[2]; ++j) {
      sy[size_t(i) * s->n[2] + j] = gval(ky[i], s->n[1], s->prm.cell[1]);
      sz[size_t(i) * s->n[2] + j] = gval(kz[j], s->n[2], s->prm.cell[2]);
    }
  std::vector<float> sx32(sx.begin(), sx.end()), sy32(sy.begin(), sy.end()), sz32(sz.begin(), sz.end());
  if ((r = upload(s, sx, &s->gsx64)) != NCT_OK) return r;
  if ((r = upload(s, sy, &s->gsy64)) != NCT_OK) return r;
  if ((r = upload(s, sz, &s->gsz64)) != NCT_OK) return r;
  if ((r = upload(s, sx32, &s->gsx32)) != NCT_OK) return r;
  if ((r = upload(s, sy32, &s->gsy32)) != NCT_OK) return r;
  if ((r = upload(s, sz32, &s->gsz32)) != NCT_OK) return r;
  std::vector<float> gx32(gx.begin(), gx.end()), gyz32(gyz.begin(), gyz.end());
  if ((r = upload(s, gx, &s->g2x64)) != NCT_OK) return r;
  if ((r = upload(s, gyz, &s->g2yz64)) != NCT_OK) return r;
  if ((r = upload(s, gx32, &s->g2x32)) != NCT_OK) return r;
  if ((r = upload(s, gyz32, &s->g2yz32)) != NCT_OK) return r;
  return NCT_OK;
}

nct_status alloc_tape(nct_system* s, nct_system::Tape& T, int cap) {
  const size_t psib = size_t(s->S) * 2 * s->N * s->cbytes;
  const int K = s->prm.taylor_order;
  nct_status r;
  void* p;
  if ((r = dalloc(s, size_t(cap) * 3 * K * psib, &T.vec)) != NCT_OK) return r;
  if ((r = dalloc(s, size_t(cap) * 2 * 4 * s->N * 8, &p)) != NCT_OK) return r;
  T.rho = static_cast<double*>(p);
  if ((r = dalloc(s, size_t(cap) * 2 * 4 * s->N * 8, &p)) != NCT_OK) return r;
  T.fld = static_cast<double*>(p);
  T.cap = cap;
  T.valid = 0;
  return NCT_OK;
}

void free_all(nct_system* s) {
  for (hipStream_t q : {s->st2, s->stB, s->stB2})
    if (q) (void)hipStreamSynchronize(q);
  for (auto& b : s->owned) (void)hipFree(b.p);
  s->owned.clear();
  for (hipEvent_t* e : {&s->ev_rows, &s->ev_proj, &s->evB_rows, &s->evB_proj, &s->ev_fork, &s->ev_join,
                        &s->evK_in, &s->evK_out}) {
    if (*e) (void)hipEventDestroy(*e);
    *e = nullptr;
  }
  for (hipStream_t* q : {&s->st2, &s->stB, &s->stB2, &s->stK}) {
    if (*q) {
      (void)hipStreamSynchronize(*q);
      (void)hipStreamDestroy(*q);
    }
    *q = nullptr;
  }
}


// Cache policy of the state-sized passes, from the bytes of one state set |psi|.  Measured on
// MI355X (256 MB Infinity Cache): up to ~64 MiB the buffers stay cache-resident between passes
// and plain accesses are fastest; from there streaming (non-temporal) stores win; from ~192 MiB
// streaming loads win as well.
#ifndef NCT_STREAM_STORE_MIN_BYTES
#define NCT_STREAM_STORE_MIN_BYTES (64ull << 20)
#endif
#ifndef NCT_STREAM_LOAD_MIN_BYTES
#define NCT_STREAM_LOAD_MIN_BYTES (192ull << 20)
#endif
static int stream_cache_mode(size_t psi_bytes) {
  if (psi_bytes >= NCT_STREAM_LOAD_MIN_BYTES) return 2;
  if (psi_bytes >= NCT_STREAM_STORE_MIN_BYTES) return 1;
  return 0;
}

nct_status create_impl(const nct_params* p, nct_system** out) {
  if (!p || !out) return fail(nullptr, NCT_ERR_ARG, "null params or out");
  *out = nullptr;
  for (int d = 0; d < 3; ++d) {
    if (!line_supported(p->n[d]))
      return fail(nullptr, NCT_ERR_UNSUPPORTED, "grid size n[%d] = %d not built", d, p->n[d]);
    if (!(p->cell[d] > 0)) return fail(nullptr, NCT_ERR_ARG, "cell[%d] must be > 0", d);
  }
  if (!plane_pair_supported(p->n[1], p->n[2]))
    return fail(nullptr, NCT_ERR_UNSUPPORTED, "plane (%d, %d) not built", p->n[1], p->n[2]);
  if (p->nstates < 1) return fail(nullptr, NCT_ERR_ARG, "nstates must be >= 1");
  if (p->taylor_order < 1 || p->taylor_order > 16) return fail(nullptr, NCT_ERR_ARG, "taylor_order in 1..16");
  if (p->xc < 0 || p->xc > 2) return fail(nullptr, NCT_ERR_ARG, "xc must be 0, 1 or 2");
  if (p->precision != NCT_FP64 && p->precision != NCT_FP32_MIXED)
    return fail(nullptr, NCT_ERR_ARG, "precision must be NCT_FP64 or NCT_FP32_MIXED");
  if (!(p->dt > 0)) return fail(nullptr, NCT_ERR_ARG, "dt must be > 0");
  if (p->natoms < 0 || (p->natoms > 0 && !p->positions)) return fail(nullptr, NCT_ERR_ARG, "bad atoms");
  if (p->nchannels < 0 || (p->nchannels > 0 && !p->channels)) return fail(nullptr, NCT_ERR_ARG, "bad channels");
  for (int c = 0; c < p->nchannels; ++c) {
    const nct_channel& ch = p->channels[c];
    if (ch.l < 0 || ch.l > 2 || (ch.twoj != 2 * ch.l + 1 && ch.twoj != 2 * ch.l - 1) || !(ch.rc > 0))
      return fail(nullptr, NCT_ERR_ARG, "bad channel %d", c);
  }
  if (p->natoms > 0 && p->nchannels > 0) {
    const double mincell = std::min(p->cell[0], std::min(p->cell[1], p->cell[2]));
    if (!(p->r_sphere > 0) || !(p->r_sphere < 0.5 * mincell))
      return fail(nullptr, NCT_ERR_ARG, "r_sphere must be in (0, cell/2)");
  }
  if (p->tape_steps < 0) return fail(nullptr, NCT_ERR_ARG, "tape_steps must be >= 0");

  nct_system* s = new nct_system();
  s->prm = *p;
  // keep host copies of the caller's arrays; prm points at the copies
  s->prm.occ = nullptr;
  if (p->natoms > 0) s->positions_h.assign(p->positions, p->positions + 3 * size_t(p->natoms));
  if (p->nchannels > 0) s->channels_h.assign(p->channels, p->channels + p->nchannels);
  s->prm.positions = s->positions_h.empty() ? nullptr : s->positions_h.data();
  s->prm.channels = s->channels_h.empty() ? nullptr : s->channels_h.data();
  for (int d = 0; d < 3; ++d) s->n[d] = p->n[d];
  s->N = size_t(p->n[0]) * p->n[1] * p->n[2];
  s->S = p->nstates;
  s->dV = p->cell[0] * p->cell[1] * p->cell[2] / double(s->N);
  s->fp64 = p->precision == NCT_FP64;
  s->cbytes = s->fp64 ? 16 : 8;
  s->cache_mode = stream_cache_mode(size_t(2) * s->S * s->N * s->cbytes);
  s->st = static_cast<hipStream_t>(p->stream);
  s->occ_h.assign(p->nstates, 1.0);
  if (p->occ)
    for (int i = 0; i < p->nstates; ++i) s->occ_h[i] = p->occ[i];

  nct_status r = NCT_OK;
  auto bail = [&](nct_status code) {
    g_create_error = s->err;
    free_all(s);
    delete s;
    return code;
  };
  if ((r = build_fft_tables<double>(s)) != NCT_OK) return bail(r);
  if ((r = upload(s, s->occ_h, &s->occ)) != NCT_OK) return bail(r);
  void* p0;
  const size_t N = s->N;
  if ((r = dalloc(s, N * 8, &p0)) != NCT_OK) return bail(r);
  s->vext = (double*)p0;
  if ((r = dalloc(s, 4 * N * 8, &p0)) != NCT_OK) return bail(r);
  s->rho = (double*)p0;
  if ((r = dalloc(s, 4 * N * 8, &p0)) != NCT_OK) return bail(r);
  s->fields = (double*)p0;
  if ((r = dalloc(s, 4 * N * 8, &p0)) != NCT_OK) return bail(r);
  s->fields_scr = (double*)p0;
  if ((r = dalloc(s, 4 * N * 4, &p0)) != NCT_OK) return bail(r);
  s->fields32 = (float*)p0;
  if ((r = dalloc(s, N * 16, &s->ncpx)) != NCT_OK) return bail(r);
  if ((r = dalloc(s, ((N + 255) / 256) * kFieldTot * 8, &p0)) != NCT_OK) return bail(r);
  s->fpart = (double*)p0;
  if ((r = dalloc(s, kFieldTot * 8, &p0)) != NCT_OK) return bail(r);
  s->ftot = (double*)p0;
  const size_t nyz = size_t(p->n[1]) * p->n[2];
  if ((r = dalloc(s, size_t(2 * s->S) * (nyz / 16) * 2 * 8, &p0)) != NCT_OK) return bail(r);
  s->epart = (double*)p0;
  const size_t psib = size_t(s->S) * 2 * N * s->cbytes;
  if ((r = dalloc(s, psib, &s->psihat)) != NCT_OK) return bail(r);
  if ((r = dalloc(s, psib, &s->phi)) != NCT_OK) return bail(r);
  if ((r = dalloc(s, psib, &s->phihat)) != NCT_OK) return bail(r);
  if ((r = dalloc(s, psib, &s->wbuf)) != NCT_OK) return bail(r);
  if ((r = dalloc(s, psib, &s->tmp)) != NCT_OK) return bail(r);
  if ((r = dalloc(s, psib, &s->tmpk_phi)) != NCT_OK) return bail(r);
  if (s->fp64) r = build_projectors<double>(s);
  else r = build_projectors<float>(s);
  if (r != NCT_OK) return bail(r);
  if ((r = dalloc(s, 4 * N * 8, &p0)) != NCT_OK) return bail(r);
  s->gA = (double*)p0;
  if ((r = dalloc(s, 4 * N * 8, &p0)) != NCT_OK) return bail(r);
  s->gB = (double*)p0;
  if ((r = dalloc(s, 4 * N * 8, &p0)) != NCT_OK) return bail(r);
  s->gnm = (double*)p0;
  if ((r = dalloc(s, ((N + 255) / 256) * 4 * 8, &p0)) != NCT_OK) return bail(r);
  s->gpart = (double*)p0;
  if ((r = dalloc(s, 8 * 8, &p0)) != NCT_OK) return bail(r);
  s->gtot = (double*)p0;
  if (p->tape_steps > 0 && (r = alloc_tape(s, s->tape, p->tape_steps)) != NCT_OK) return bail(r);
  if (hipStreamCreateWithFlags(&s->st2, hipStreamNonBlocking) != hipSuccess ||
      hipStreamCreateWithFlags(&s->stK, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreateWithFlags(&s->ev_rows, hipEventDisableTiming | hipEventDisableSystemFence) != hipSuccess ||
      hipEventCreateWithFlags(&s->ev_proj, hipEventDisableTiming | hipEventDisableSystemFence) != hipSuccess ||
      hipEventCreateWithFlags(&s->evK_in, hipEventDisableTiming | hipEventDisableSystemFence) != hipSuccess ||
      hipEventCreateWithFlags(&s->evK_out, hipEventDisableTiming | hipEventDisableSystemFence) != hipSuccess) {
    fail(s, NCT_ERR_HIP, "stream/event creation failed");
    return bail(NCT_ERR_HIP);
  }
  if (p->overlap && s->S >= 8) {
    s->ngroups = 2;
    s->S0 = (s->S + 1) / 2;
    if (hipStreamCreateWithFlags(&s->stB, hipStreamNonBlocking) != hipSuccess ||
        hipStreamCreateWithFlags(&s->stB2, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&s->evB_rows, hipEventDisableTiming | hipEventDisableSystemFence) != hipSuccess ||
        hipEventCreateWithFlags(&s->evB_proj, hipEventDisableTiming | hipEventDisableSystemFence) != hipSuccess ||
        hipEventCreateWithFlags(&s->ev_fork, hipEventDisableTiming | hipEventDisableSystemFence) != hipSuccess ||
        hipEventCreateWithFlags(&s->ev_join, hipEventDisableTiming | hipEventDisableSystemFence) != hipSuccess) {
      fail(s, NCT_ERR_HIP, "stream/event creation failed");
      return bail(NCT_ERR_HIP);
    }
    if (s->natoms) {
      const size_t cp = size_t(s->natoms) * s->pt.PP * s->S;
      if ((r = dalloc(s, cp * s->pt.max_kchunks * 16, &s->CpartB)) != NCT_OK) return bail(r);
      if ((r = dalloc(s, cp * 16, &s->CB)) != NCT_OK) return bail(r);
      if ((r = dalloc(s, cp * s->cbytes, &s->ECB)) != NCT_OK) return bail(r);
    }
  }
  {  // this device's static scratch (allocation-free entry point): looked up once per device
    void* sp = nullptr;
    size_t sb = 0;
    const hipError_t es = static_scratch(&sp, &sb);
    if (es == hipSuccess) {
      s->scr = sp;
      s->scr_bytes = sb;
    } else {
      (void)hipGetLastError();
      s->scr_err = hipGetErrorString(es);
    }
  }
  hipError_t e = hipMemsetAsync(s->vext, 0, N * 8, s->st);
  if (e == hipSuccess) e = hipMemsetAsync(s->fields, 0, 4 * N * 8, s->st);
  if (e == hipSuccess) e = hipStreamSynchronize(s->st);
  if (e != hipSuccess) {
    fail(s, NCT_ERR_HIP, "init: %s", hipGetErrorString(e));
    return bail(NCT_ERR_HIP);
  }
  *out = s;
  return NCT_OK;
}

}  // namespace

// Same work as nct_density_magnetization; the temporaries of its kernels (Poisson work, the
// fields output when they are not kept, block partial sums and totals) are slices of this
// device's static scratch array, so the call allocates nothing.
template <typename R>
static nct_status density_magnetization_static(nct_system* s, const void* psi, double* rho_v_dev,
                                               double* totals_host, int update_fields) {
  const size_t N = s->N;
  const size_t nblk = (N + 255) / 256;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off = (off + bytes + 255) / 256 * 256;
    return o;
  };
  const size_t o_ncpx = take(N * 16);
  const size_t o_fscr = take(4 * N * 8);
  const size_t o_fpart = take(nblk * kFieldTot * 8);
  const size_t o_ftot = take(kFieldTot * 8);
  if (!s->scr) return fail(s, NCT_ERR_HIP, "static scratch unavailable: %s", s->scr_err.c_str());
  if (off > s->scr_bytes)
    return fail(s, NCT_ERR_UNSUPPORTED, "this grid needs %zu bytes of static scratch; the library holds %zu",
                off, s->scr_bytes);
  char* base = static_cast<char*>(s->scr);
  Engine<R> E{s};
  E.w_ncpx = base + o_ncpx;
  E.w_fscr = reinterpret_cast<double*>(base + o_fscr);
  E.w_fpart = reinterpret_cast<double*>(base + o_fpart);
  E.w_ftot = reinterpret_cast<double*>(base + o_ftot);
  nct_status r = E.density(psi);
  if (r != NCT_OK) return r;
  if (update_fields || totals_host) {
    if ((r = E.fields_from_rho(update_fields != 0)) != NCT_OK) return r;
  }
  if (rho_v_dev) HIPCHK(s, hipMemcpyAsync(rho_v_dev, s->rho, 4 * N * 8, hipMemcpyDeviceToDevice, s->st));
  if (totals_host) {
    double tot[4];
    HIPCHK(s, hipMemcpyAsync(tot, E.w_ftot, sizeof(tot), hipMemcpyDeviceToHost, s->st));
    HIPCHK(s, hipStreamSynchronize(s->st));
    for (int k = 0; k < 4; ++k) totals_host[k] = tot[k] * s->dV;
    if (!std::isfinite(tot[0])) return fail(s, NCT_ERR_NONFINITE, "non-finite density");
  }
  return NCT_OK;
}

// ================================================================ C ABI
extern "C" {

nct_status nct_create_system(const nct_params* params, nct_system** out) {
  try {
    return create_impl(params, out);
  } catch (...) {
    return fail(nullptr, NCT_ERR_OOM, "host allocation failed in nct_create_system");
  }
}

void nct_destroy_system(nct_system* sys) {
  if (!sys) return;
  (void)hipStreamSynchronize(sys->st);
  harvest_timing(sys);
  for (hipEvent_t e : sys->free_events) (void)hipEventDestroy(e);
  sys->free_events.clear();
  free_all(sys);
  delete sys;
}

const char* nct_last_error(const nct_system* sys) {
  return sys ? sys->err.c_str() : g_create_error.c_str();
}

nct_status nct_dm_initialization(nct_system* s, const nct_atom_density* atoms, double* rho_v_dev,
                                 int update_fields) {
  if (!s) return NCT_ERR_ARG;
  const int na = s->prm.natoms;
  if (na <= 0) return fail(s, NCT_ERR_ARG, "the system has no atoms");
  if (!atoms) return fail(s, NCT_ERR_ARG, "atoms is NULL");
  if (update_fields && s->frozen) return fail(s, NCT_ERR_STATE, "fields are frozen");
  std::vector<double> a6(size_t(na) * 6), m3(size_t(na) * 3);
  for (int a = 0; a < na; ++a) {
    const nct_atom_density& q = atoms[a];
    const double mm = std::sqrt(q.moment[0] * q.moment[0] + q.moment[1] * q.moment[1] + q.moment[2] * q.moment[2]);
    if (!(q.Z > 0) || !(q.sigma > 0) || !std::isfinite(q.Z) || !std::isfinite(q.sigma) || !std::isfinite(mm))
      return fail(s, NCT_ERR_ARG, "atom %d: Z and sigma must be positive and finite", a);
    if (mm > q.Z * (1.0 + 1e-12)) return fail(s, NCT_ERR_ARG, "atom %d: |moment| exceeds Z", a);
    for (int k = 0; k < 3; ++k) {
      a6[6 * size_t(a) + k] = s->positions_h[3 * size_t(a) + k];
      m3[3 * size_t(a) + k] = q.moment[k];
    }
    a6[6 * size_t(a) + 3] = q.Z;
    a6[6 * size_t(a) + 4] = q.sigma;
    a6[6 * size_t(a) + 5] = 0.0;
  }
  nct_status r;
  if (!s->dm_atoms) {
    void* p;
    if ((r = dalloc(s, size_t(na) * 9 * sizeof(double), &p)) != NCT_OK) return r;
    s->dm_atoms = static_cast<double*>(p);
  }
  double* d_a = s->dm_atoms;
  double* d_m = s->dm_atoms + size_t(na) * 6;
  HIPCHK(s, hipMemcpyAsync(d_a, a6.data(), a6.size() * sizeof(double), hipMemcpyHostToDevice, s->st));
  HIPCHK(s, hipMemcpyAsync(d_m, m3.data(), m3.size() * sizeof(double), hipMemcpyHostToDevice, s->st));
  HIPCHK(s, launch_dm_init(s->n, s->prm.cell, na, d_a, d_m, s->rho, s->st));
  if (rho_v_dev)
    HIPCHK(s, hipMemcpyAsync(rho_v_dev, s->rho, 4 * s->N * 8, hipMemcpyDeviceToDevice, s->st));
  if (update_fields) {
    if (s->fp64) r = Engine<double>{s}.fields_from_rho(true);
    else r = Engine<float>{s}.fields_from_rho(true);
    if (r != NCT_OK) return r;
  }
  HIPCHK(s, hipStreamSynchronize(s->st));
  return NCT_OK;
}

nct_status nct_ground_state(nct_system* s, void* psi, int niter, double tau, int keep_fields,
                            double* energies_host) {
  if (!s || !psi) return s ? fail(s, NCT_ERR_ARG, "psi is NULL") : NCT_ERR_ARG;
  if (niter < 0) return fail(s, NCT_ERR_ARG, "niter < 0");
  if (!(tau > 0) || !std::isfinite(tau)) return fail(s, NCT_ERR_ARG, "tau must be positive and finite");
  if (s->S > 4096) return fail(s, NCT_ERR_UNSUPPORTED, "at most 4096 states in the ground-state solver");
  if (s->has_k && s->krun_split)
    return fail(s, NCT_ERR_UNSUPPORTED, "the states of each Bloch vector must be consecutive for the ground state");
  if (s->fp64) return Engine<double>{s}.ground_state(psi, niter, tau, keep_fields != 0, energies_host);
  return Engine<float>{s}.ground_state(psi, niter, tau, keep_fields != 0, energies_host);
}

nct_status nct_set_laser_gauge(nct_system* s, int gauge) {
  if (!s) return NCT_ERR_ARG;
  if (gauge != NCT_GAUGE_LENGTH && gauge != NCT_GAUGE_VELOCITY)
    return fail(s, NCT_ERR_ARG, "gauge must be NCT_GAUGE_LENGTH or NCT_GAUGE_VELOCITY");
  if (gauge == NCT_GAUGE_VELOCITY && !s->kv_zero64) {
    const size_t n = size_t(s->S) * 3;
    void* p;
    nct_status r;
    if ((r = dalloc(s, n * sizeof(double), &p)) != NCT_OK) return r;
    s->kv_zero64 = static_cast<double*>(p);
    if ((r = dalloc(s, n * sizeof(float), &p)) != NCT_OK) return r;
    s->kv_zero32 = static_cast<float*>(p);
    HIPCHK(s, hipMemsetAsync(s->kv_zero64, 0, n * sizeof(double), s->st));
    HIPCHK(s, hipMemsetAsync(s->kv_zero32, 0, n * sizeof(float), s->st));
    HIPCHK(s, hipStreamSynchronize(s->st));
  }
  s->laser_gauge = gauge;
  return NCT_OK;
}

nct_status nct_set_kpoints(nct_system* s, const double* kvec) {
  if (!s) return NCT_ERR_ARG;
  if (!kvec) {
    s->has_k = false;
    return NCT_OK;
  }
  const size_t n = size_t(s->S) * 3;
  for (size_t k = 0; k < n; ++k)
    if (!std::isfinite(kvec[k])) return fail(s, NCT_ERR_ARG, "non-finite Bloch vector component %zu", k);
  nct_status r;
  if (!s->kv64) {
    void* p;
    if ((r = dalloc(s, n * sizeof(double), &p)) != NCT_OK) return r;
    s->kv64 = static_cast<double*>(p);
    if ((r = dalloc(s, n * sizeof(float), &p)) != NCT_OK) return r;
    s->kv32 = static_cast<float*>(p);
  }
  s->krun.assign(1, 0);
  for (int i = 1; i < s->S; ++i)
    if (kvec[3 * i] != kvec[3 * i - 3] || kvec[3 * i + 1] != kvec[3 * i - 2] || kvec[3 * i + 2] != kvec[3 * i - 1])
      s->krun.push_back(i);
  s->krun.push_back(s->S);
  s->krun_split = false;
  for (size_t a = 0; a + 1 < s->krun.size(); ++a)
    for (size_t b = a + 1; b + 1 < s->krun.size(); ++b) {
      const double* ka = kvec + 3 * s->krun[a];
      const double* kb = kvec + 3 * s->krun[b];
      if (ka[0] == kb[0] && ka[1] == kb[1] && ka[2] == kb[2]) s->krun_split = true;
    }
  std::vector<float> k32(kvec, kvec + n);
  HIPCHK(s, hipMemcpyAsync(s->kv64, kvec, n * sizeof(double), hipMemcpyHostToDevice, s->st));
  HIPCHK(s, hipMemcpyAsync(s->kv32, k32.data(), n * sizeof(float), hipMemcpyHostToDevice, s->st));
  HIPCHK(s, hipStreamSynchronize(s->st));
  s->has_k = true;
  return NCT_OK;
}

nct_status nct_set_laser(nct_system* s, int npulses, const nct_laser_pulse* pulses) {
  if (!s) return NCT_ERR_ARG;
  if (npulses < 0) return fail(s, NCT_ERR_ARG, "npulses < 0");
  if (npulses > 0 && !pulses) return fail(s, NCT_ERR_ARG, "pulses is NULL");
  for (int k = 0; k < npulses; ++k) {
    const nct_laser_pulse& p = pulses[k];
    const double v[8] = {p.A, p.omega, p.t0, p.tau, p.phase, p.pol[0], p.pol[1], p.pol[2]};
    for (double x : v)
      if (!std::isfinite(x)) return fail(s, NCT_ERR_ARG, "laser pulse %d: non-finite parameter", k);
    if (!(p.tau > 0)) return fail(s, NCT_ERR_ARG, "laser pulse %d: tau must be > 0", k);
  }
  s->laser.assign(pulses, pulses + npulses);
  return NCT_OK;
}

nct_status nct_set_potentials(nct_system* s, const double* v_ext_dev, const nct_bfield* b,
                              const double* fields_dev) {
  if (!s) return NCT_ERR_ARG;
  if (b && b->npulses < 0) return fail(s, NCT_ERR_ARG, "npulses < 0");
  if (b && b->npulses > 0 && !b->pulses) return fail(s, NCT_ERR_ARG, "pulses is NULL");
  if (b) {
    for (int k = 0; k < b->npulses; ++k)
      if (!(b->pulses[k].tau > 0)) return fail(s, NCT_ERR_ARG, "pulse %d: tau must be > 0", k);
  }
  if (v_ext_dev) HIPCHK(s, hipMemcpyAsync(s->vext, v_ext_dev, s->N * 8, hipMemcpyDeviceToDevice, s->st));
  if (b) {
    for (int k = 0; k < 3; ++k) s->B0[k] = b->B0[k];
    s->pulses.assign(b->pulses, b->pulses + b->npulses);
  }
  if (fields_dev) {
    HIPCHK(s, hipMemcpyAsync(s->fields, fields_dev, 4 * s->N * 8, hipMemcpyDeviceToDevice, s->st));
    if (!s->fp64) HIPCHK(s, launch_to_float(s->fields, 4 * s->N, s->fields32, s->st));
    s->frozen = true;
    s->fields_valid = true;
  } else {
    if (s->frozen) s->fields_valid = false;
    s->frozen = false;
    if (v_ext_dev) s->fields_valid = false;
  }
  return NCT_OK;
}

nct_status nct_density_magnetization(nct_system* s, const void* psi, double t, double* rho_v_dev,
                                     double* totals_host, int update_fields) {
  (void)t;
  if (!s || !psi) return s ? fail(s, NCT_ERR_ARG, "psi is NULL") : NCT_ERR_ARG;
  if (update_fields && s->frozen) return fail(s, NCT_ERR_STATE, "fields are frozen");
  nct_status r;
  if (s->fp64) r = Engine<double>{s}.density(psi);
  else r = Engine<float>{s}.density(psi);
  if (r != NCT_OK) return r;
  if (update_fields || totals_host) {
    if (s->fp64) r = Engine<double>{s}.fields_from_rho(update_fields != 0);
    else r = Engine<float>{s}.fields_from_rho(update_fields != 0);
    if (r != NCT_OK) return r;
  }
  if (rho_v_dev)
    HIPCHK(s, hipMemcpyAsync(rho_v_dev, s->rho, 4 * s->N * 8, hipMemcpyDeviceToDevice, s->st));
  if (totals_host) {
    double tot[8];
    HIPCHK(s, hipMemcpyAsync(tot, s->ftot, sizeof(tot), hipMemcpyDeviceToHost, s->st));
    HIPCHK(s, hipStreamSynchronize(s->st));
    for (int k = 0; k < 4; ++k) totals_host[k] = tot[k] * s->dV;
    if (!std::isfinite(tot[0])) return fail(s, NCT_ERR_NONFINITE, "non-finite density");
  }
  return NCT_OK;
}

nct_status nct_density_magnetization_static(nct_system* s, const void* psi, double t, double* rho_v_dev,
                                            double* totals_host, int update_fields) {
  (void)t;
  if (!s || !psi) return s ? fail(s, NCT_ERR_ARG, "psi is NULL") : NCT_ERR_ARG;
  if (update_fields && s->frozen) return fail(s, NCT_ERR_STATE, "fields are frozen");
  if (s->fp64) return density_magnetization_static<double>(s, psi, rho_v_dev, totals_host, update_fields);
  return density_magnetization_static<float>(s, psi, rho_v_dev, totals_host, update_fields);
}

nct_status nct_get_fields(nct_system* s, double t, double* out) {
  if (!s || !out) return s ? fail(s, NCT_ERR_ARG, "out is NULL") : NCT_ERR_ARG;
  if (!s->fields_valid) return fail(s, NCT_ERR_STATE, "fields not computed yet");
  double B[3] = {0, 0, 0}, lg[4] = {0, 0, 0, 0};
  if (!s->frozen) {
    bfield_at(s, t, B);
    for (int k = 0; k < 3; ++k) B[k] *= kMuB;
    if (!s->laser.empty() && !velocity_gauge(s)) laser_coeffs(s, t, lg);
  }
  HIPCHK(s, launch_add_bext(s->fields, s->n, B, lg, out, s->st));
  return NCT_OK;
}

nct_status nct_apply_hamiltonian(nct_system* s, const void* psi, void* hpsi, double t) {
  if (!s || !psi || !hpsi) return s ? fail(s, NCT_ERR_ARG, "null psi/hpsi") : NCT_ERR_ARG;
  if (psi == hpsi) return fail(s, NCT_ERR_ARG, "psi and hpsi must differ");
  if (!s->fields_valid) return fail(s, NCT_ERR_STATE, "fields not computed (call nct_density_magnetization with update_fields)");
  if (s->fp64) return Engine<double>{s}.apply(psi, hpsi, t);
  return Engine<float>{s}.apply(psi, hpsi, t);
}

nct_status nct_step(nct_system* s, void* psi, double t0, int nsteps, double* obs_host, int tape) {
  if (!s || !psi) return s ? fail(s, NCT_ERR_ARG, "psi is NULL") : NCT_ERR_ARG;
  if (nsteps < 0) return fail(s, NCT_ERR_ARG, "nsteps < 0");
  if (tape && nsteps > s->prm.tape_steps) return fail(s, NCT_ERR_ARG, "nsteps exceeds tape_steps");
  if (nsteps == 0) return NCT_OK;
  if (s->frozen && !s->fields_valid) return fail(s, NCT_ERR_STATE, "no fields");
  nct_system::Tape* T = tape ? &s->tape : nullptr;
  if (T) T->valid = 0;
  if (s->fp64) return Engine<double>{s}.step(psi, t0, nsteps, obs_host, T);
  return Engine<float>{s}.step(psi, t0, nsteps, obs_host, T);
}

nct_status nct_magnetization_seed(nct_system* s, const void* psi, const double* w, void* lam) {
  if (!s || !psi || !w || !lam) return s ? fail(s, NCT_ERR_ARG, "null argument") : NCT_ERR_ARG;
  hipError_t e;
  if (s->fp64) e = launch_seed<double>(psi, s->occ, s->S, s->N, w[0], w[1], w[2], 2.0 * s->dV, lam, s->st);
  else e = launch_seed<float>(psi, s->occ, s->S, s->N, w[0], w[1], w[2], 2.0 * s->dV, lam, s->st);
  if (e != hipSuccess) return fail(s, NCT_ERR_HIP, "seed: %s", hipGetErrorString(e));
  return NCT_OK;
}

nct_status nct_backward_step(nct_system* s, int tape_index, const void* psi_n, double t_n,
                             const void* lam_np1, void* lam_n, double* dLdB, double* dLdtheta) {
  if (!s) return NCT_ERR_ARG;
  if (!lam_np1 || !lam_n) return fail(s, NCT_ERR_ARG, "lam_np1 / lam_n is NULL");
  if (s->frozen && !s->fields_valid) return fail(s, NCT_ERR_STATE, "no fields");
  nct_system::Tape* T = nullptr;
  int idx = 0;
  nct_status r;
  if (tape_index >= 0) {
    if (tape_index >= s->tape.valid)
      return fail(s, NCT_ERR_STATE, "tape index %d not recorded (tape holds %d steps)", tape_index,
                  s->tape.valid);
    const double tt = s->tape.t0 + tape_index * s->prm.dt;
    if (std::fabs(tt - t_n) > 1e-9 * std::max(1.0, std::fabs(tt)))
      return fail(s, NCT_ERR_ARG, "t_n = %g does not match the taped time %g", t_n, tt);
    T = &s->tape;
    idx = tape_index;
  } else {
    if (!psi_n) return fail(s, NCT_ERR_ARG, "psi_n is NULL in recompute mode");
    if (s->scratch_tape.cap == 0) {
      if ((r = alloc_tape(s, s->scratch_tape, 1)) != NCT_OK) return r;
      if ((r = dalloc(s, size_t(s->S) * 2 * s->N * s->cbytes, &s->scratch_out)) != NCT_OK) return r;
    }
    HIPCHK(s, hipMemcpyAsync(s->scratch_out, psi_n, size_t(s->S) * 2 * s->N * s->cbytes,
                             hipMemcpyDeviceToDevice, s->st));
    if (s->fp64) r = Engine<double>{s}.step(s->scratch_out, t_n, 1, nullptr, &s->scratch_tape);
    else r = Engine<float>{s}.step(s->scratch_out, t_n, 1, nullptr, &s->scratch_tape);
    if (r != NCT_OK) return r;
    T = &s->scratch_tape;
    idx = 0;
  }
  double dB[6] = {0, 0, 0, 0, 0, 0};
  if (s->fp64) r = Engine<double>{s}.backward(*T, idx, t_n, lam_np1, lam_n, dB);
  else r = Engine<float>{s}.backward(*T, idx, t_n, lam_np1, lam_n, dB);
  if (r != NCT_OK) return r;
  // the system's fields now hold those of H_n; mark them current for later H applications
  s->fields_valid = true;
  if (dLdB)
    for (int k = 0; k < 6; ++k) dLdB[k] = dB[k];
  if (dLdtheta && !s->pulses.empty()) {
    std::vector<double> j0, j1;
    bfield_jac(s, t_n, j0);
    bfield_jac(s, t_n + s->prm.dt, j1);
    const size_t np = 2 * s->pulses.size();
    for (size_t q = 0; q < np; ++q)
      for (int k = 0; k < 3; ++k) dLdtheta[q] += dB[k] * j0[q * 3 + k] + dB[3 + k] * j1[q * 3 + k];
  }
  for (int k = 0; k < 6; ++k)
    if (!std::isfinite(dB[k])) return fail(s, NCT_ERR_NONFINITE, "non-finite field gradient");
  return NCT_OK;
}

nct_status nct_set_watchdog(nct_system* s, double max_rel_drift) {
  if (!s) return NCT_ERR_ARG;
  if (std::isnan(max_rel_drift)) return fail(s, NCT_ERR_ARG, "max_rel_drift is NaN");
  s->max_ne_drift = max_rel_drift;
  return NCT_OK;
}

nct_status nct_set_timing(nct_system* s, int enable) {
  if (!s) return NCT_ERR_ARG;
  HIPCHK(s, hipStreamSynchronize(s->st));
  HIPCHK(s, hipStreamSynchronize(s->st2));
  if (s->stB) HIPCHK(s, hipStreamSynchronize(s->stB));
  if (s->stB2) HIPCHK(s, hipStreamSynchronize(s->stB2));
  harvest_timing(s);
  for (int k = 0; k < NCT_K_COUNT; ++k) {
    s->t_ms[k] = 0;
    s->t_count[k] = 0;
    s->t_bytes[k] = 0;
    s->t_flops[k] = 0;
    s->t_seen[k] = 0;
  }
  s->timing_mask = unsigned(enable);
  s->timing = enable != 0;
  return NCT_OK;
}

nct_status nct_set_timing_sample(nct_system* s, int every) {
  if (!s) return NCT_ERR_ARG;
  if (every < 1) return fail(s, NCT_ERR_ARG, "every must be >= 1");
  s->timing_every = every;
  for (int k = 0; k < NCT_K_COUNT; ++k) s->t_seen[k] = 0;
  return NCT_OK;
}

nct_status nct_get_timing(nct_system* s, int k, double* ms, long long* launches, double* bytes,
                          double* flops) {
  if (!s) return NCT_ERR_ARG;
  if (k < 0 || k >= NCT_K_COUNT) return fail(s, NCT_ERR_ARG, "kernel class out of range");
  HIPCHK(s, hipStreamSynchronize(s->st));
  HIPCHK(s, hipStreamSynchronize(s->st2));
  if (s->stB) HIPCHK(s, hipStreamSynchronize(s->stB));
  if (s->stB2) HIPCHK(s, hipStreamSynchronize(s->stB2));
  harvest_timing(s);
  if (ms) *ms = s->t_ms[k];
  if (launches) *launches = s->t_count[k];
  if (bytes) *bytes = s->t_bytes[k];
  if (flops) *flops = s->t_flops[k];
  return NCT_OK;
}

const char* nct_version(void) {
  return "libnct gfx950; FP64 and FP32-mixed; lines 8,12,16,24,32,48,64,96";
}

}  // extern "C"
