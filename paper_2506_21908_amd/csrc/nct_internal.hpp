// Internal interfaces between the host engine (nct_api.cpp) and the kernel
// launchers (nct_kernels.hip).  Not part of the public ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <cstddef>
#include <cstdint>

namespace nct {

template <typename R>
struct cpx;

// Projector tables on the device.  Sphere rows of all atoms are numbered
// J = 0..Jtot-1; atom a owns rows [row_off[a], row_off[a] + ns[a]), sorted by
// flat grid index, so the rows of one x-plane form a contiguous range.
struct ProjTables {
  int natoms = 0;
  int P = 0;            // projectors per atom
  int PP = 0;           // P padded to a multiple of 16
  int Jtot = 0;         // total sphere rows
  int max_kchunks = 0;  // max over atoms of ceil(2 ns / KC)
  int max_rowtiles = 0; // max over atoms of ceil(2 ns / 16)
  const int* row_off = nullptr;   // [natoms+1]
  const int* pidx = nullptr;      // [Jtot] in-plane index y*NZ + z
  const int* pr_off = nullptr;    // [NX+1] plane -> range list
  const int* pr_begin = nullptr;  // [nranges]
  const int* pr_end = nullptr;    // [nranges]
  const void* beta = nullptr;     // complex R [Jtot][2][PP]
  const void* disp = nullptr;     // R [Jtot][3]: displacement of each sphere row from its atom
  const double* energy = nullptr; // [natoms][PP] (0 beyond P)
};

template <typename R>
struct StageArgs {
  const void* tmp_in = nullptr;   // kinetic-applied mixed representation of w_in
  void* tmp_out = nullptr;        // 2D (y,z) transform of w_out, or null
  const void* w_in = nullptr;     // real-space input of this H application
  const void* x_base = nullptr;   // Taylor base x (null: alpha ignored)
  void* w_out = nullptr;          // alpha x + c H w_in
  const R* fields = nullptr;      // [4][N] {v, b_x, b_y, b_z}
  R bext[3] = {0, 0, 0};          // mu_B B_ext added to b
  R lg[4] = {0, 0, 0, 0};         // laser potential lg[0] ix + lg[1] iy + lg[2] iz + lg[3]
  R cre = 1, cim = 0;             // coefficient c of H w
  R alpha = 0;                    // coefficient of x_base
  const void* Y = nullptr;        // nonlocal scatter rows [S][2][Jtot], or null
  void* W = nullptr;              // output sphere rows [S][2][Jtot] of w_out, or null
  // adjoint extras: acc += w_out (if acc != null)
  void* acc = nullptr;
  // cache policy of the state-sized operands: 0 plain, 1 streaming stores, 2 streaming loads too
  int cache_mode = 0;
  // Bloch vectors [S][3] of the states (null: Gamma only); this launch's state 0 is state_off;
  // ka: velocity-gauge vector potential added to every Bloch vector
  const R* kv = nullptr;
  int state_off = 0;
  R ka[3] = {0, 0, 0};
};

// Kinetic factor with Bloch vectors: |G + k|^2 from signed per-axis G tables (gx in the
// digit-reversed x order of the column transforms, gy / gz per position of the 2D-transformed yz
// plane).  kv null: the |G|^2 tables are used instead (Gamma only).
template <typename R>
struct KTables {
  const R* gx = nullptr;
  const R* gy = nullptr;
  const R* gz = nullptr;
  const R* kv = nullptr;   // [S][3]
  int state_off = 0;       // state of batch entries 0, 1
  R ka[3] = {0, 0, 0};     // velocity-gauge vector potential added to every Bloch vector
};

// Launchers (return hipError_t of the launch).  n = {NX, NY, NZ}.
template <typename R>
hipError_t launch_plane_stage(const int n[3], int S, const StageArgs<R>& a, const ProjTables& pt,
                              const void* twy, const void* twz, hipStream_t st);
// Forward 2D transform of B planes-sets (batch entries, each [NX][NY][NZ]); optionally gathers
// sphere rows of the input into W (batch must then be 2S in state/spinor order).
// With kt.kv (Bloch vectors [S][3], shifted by kt.ka) the gathered rows carry exp(i k.d) (state
// of entry b = b / 2).
// forward (y,z) transform of a real source (B = 1): src 1 = spin density [4][N] (n = rho_uu +
// rho_dd), 2 = real array [N]; out: complex [N]
hipError_t launch_plane_fwd_real(const int n[3], const double* in, int src, void* out, const void* twy,
                                 const void* twz, hipStream_t st);
template <typename R>
hipError_t launch_plane_fwd(const int n[3], int B, const void* in, void* out, void* W,
                            const ProjTables* pt, const void* twy, const void* twz, hipStream_t st,
                            KTables<R> kt = KTables<R>{});
// rows[S][2][Jtot] *= exp(i dA.d_J): sphere rows gathered under one vector potential carried to
// another (dA = A_new - A_old).
template <typename R>
hipError_t launch_rephase_rows(const ProjTables& pt, void* rows, int S, const double dA[3],
                               hipStream_t st);
// Inverse 2D transform; out = scale * result.
template <typename R>
hipError_t launch_plane_inv(const int n[3], int B, const void* in, void* out, R scale,
                            const void* twy, const void* twz, hipStream_t st);
// Column pass along x: dst = IDFT_x( mult * DFT_x(src) ), mult from per-axis |G|^2 tables.
// mode 0: mult = kscale (g2x + g2yz); mode 1: mult = kscale / (g2x + g2yz), 0 at G = 0.
// cache_mode as in StageArgs.
template <typename R>
hipError_t launch_xpass(const int n[3], int B, const void* src, void* dst, const R* g2x,
                        const R* g2yz, R kscale, int mode, const void* twx, hipStream_t st,
                        int cache_mode = 0, KTables<R> kt = KTables<R>{});
// Energy pass: per (batch, tile) partial sums of sum kscale*G^2 |X|^2 and sum |X|^2 of the full
// 3D transform (input in the 2D-transformed form).  part: [B][ntiles][2] doubles.
template <typename R>
hipError_t launch_xpass_energy(const int n[3], int B, const void* src, const R* g2x,
                               const R* g2yz, R kscale, const void* twx, double* part,
                               int* ntiles_out, hipStream_t st, KTables<R> kt = KTables<R>{});

template <typename R>
hipError_t launch_density(const void* psi, const double* occ, int S, size_t N, double* rho,
                          hipStream_t st);

// fields[4][N] = {v_ext + v_H + vbar, b_xc}; fields32 optional float copy;
// part[nblk][kFieldTot] partial sums (slots below)
// Slots of the per-block field partial sums (not scaled by dV).
constexpr int kFieldTot = 12;  // N_e, M_x, M_y, M_z, E_loc, E_H, E_xc, 0, D_x, D_y, D_z, 0
// D = sum (r - c) n, r = (ix hx, iy hy, iz hz), c = cell / 2: the dipole that gives the laser
// energy E.D dV.
// vH: the complex Poisson output (its real parts, stride 2 doubles, are v_H), or null
hipError_t launch_fields(const double* rho, const double* vext, const double* vH, int xc,
                         double thr, const int n[3], const double cell[3], double* fields,
                         float* fields32, double* part, int* nblk_out, hipStream_t st);
// out[w] = sum_r part[r][w] (fixed order); copy0, if non-null, also receives out[0]
hipError_t launch_reduce_rows(const double* part, int nrows, int width, double* out,
                              hipStream_t st, double* copy0 = nullptr);
// out = fields + {v_E, b}: v_E = lg[0] ix + lg[1] iy + lg[2] iz + lg[3] (laser), b added to b_xc
hipError_t launch_add_bext(const double* fields, const int n[3], const double b[3],
                           const double lg[4], double* out, hipStream_t st);
hipError_t launch_to_float(const double* in, size_t n, float* out, hipStream_t st);

// Projectors: C = dV beta^H W (per atom), EC = E * C; Y = beta EC.
template <typename R>
hipError_t launch_proj_contract(const ProjTables& pt, const void* W, int S, double dV,
                                void* Cpart, void* C, void* EC, hipStream_t st);
template <typename R>
hipError_t launch_proj_scatter(const ProjTables& pt, const void* EC, int S, void* Y,
                               hipStream_t st);

// Observables of the current state: assembles one 13-double row.
struct ObsInputs {
  const double* field_tot;  // [8] reduced field partials
  const double* epart;      // [2S][ntiles][2] energy-pass partials
  int ntiles;
  const void* C;            // [natoms][PP][S] complex R (already times dV)
  const double* energy;     // [natoms][PP]
  const double* occ;        // [S]
  int S, natoms, PP, precision;
  double dV, invN, t;
  double muB_B[3];          // mu_B B_ext(t)
  double efield[3];         // laser field E(t) (E_loc gains E.D dV)
};
hipError_t launch_obs_row(const ObsInputs& in, double* row, hipStream_t st);

template <typename R>
hipError_t launch_seed(const void* psi, const double* occ, int S, size_t N, double w0, double w1,
                       double w2, double scale, void* lam, hipStream_t st);
template <typename R>
hipError_t launch_axpby(void* y, const void* x, size_t count, R a_re, R a_im, R b,
                        hipStream_t st);

// Adjoint kernels
template <typename R>
hipError_t launch_pair(const void* mu, const void* w, int S, size_t N, double gamma, double* g,
                       hipStream_t st);
// pg: the complex adjoint Poisson output (its real parts, stride 2 doubles, are used), or null
hipError_t launch_field_adjoint(const double* rho, const double* g, const double* pg, int xc,
                                double thr, size_t N, double* gnm, double* part, int* nblk_out,
                                hipStream_t st);
template <typename R>
hipError_t launch_density_backprop(const void* psi, const double* occ, const double* gnm, int S,
                                   size_t N, int add, void* lam, hipStream_t st);

// HIP events attached to the next kernel dispatches of this host thread (set by the library's
// timing wrapper around one launcher call): 'start' goes with the first dispatch and 'stop' with
// every dispatch, so the pair spans all kernels of the launcher without extra stream packets.
struct LaunchEvents {
  hipEvent_t start = nullptr;
  hipEvent_t stop = nullptr;
  bool used = false;
};
LaunchEvents& launch_events();

// Initial spin-density matrix (initialisation algorithm of Sec. 3.2): every grid point takes its
// nearest atom (minimum image, ties to the lowest index; squared distances formed without fused
// operations), n = Z_a (2 pi s_a^2)^(-3/2) exp(-d^2 / 2 s_a^2), m = M_a / Z_a, and
// rho_v = n {(1 + m_z)/2, (1 - m_z)/2, m_x/2, -m_y/2}.  atoms: device double [natoms][6]
// {X, Y, Z position, charge, sigma, unused} and moments [natoms][3].
hipError_t launch_dm_init(const int n[3], const double cell[3], int natoms, const double* atoms,
                          const double* moments, double* rho, hipStream_t st);

// Orthonormalisation of a run of S states (rows of K = 2N complex values), FP64 arithmetic in
// either precision.  launch_gram: out[S][S] = scale A^H A (Hermitian, both halves written) through
// nchunks partial sums over K in part[nchunks][S][S] (complex double; gram_chunks() chooses
// nchunks).  launch_basis_transform: D_j = sum_{i <= j} Mt[i][j] A_i with Mt [S][S] complex double
// upper triangular (D and A distinct).
int gram_chunks(int S, size_t K);
template <typename R>
hipError_t launch_gram(const void* A, int S, size_t K, double scale, void* part, int nchunks, void* out,
                       hipStream_t st);
template <typename R>
hipError_t launch_basis_transform(const void* A, const void* Mt, int S, size_t K, void* D, hipStream_t st);

// Static device scratch of the allocation-free entry point (nct_density_magnetization_static):
// a file-scope array of NCT_STATIC_SCRATCH_BYTES on every device the library runs on, alive until
// the process ends.  static_scratch() returns its device address on the current device (looked up
// once per device, with that device current) and its size.
#ifndef NCT_STATIC_SCRATCH_BYTES
#define NCT_STATIC_SCRATCH_BYTES (size_t(32) << 20)
#endif
hipError_t static_scratch(void** ptr, size_t* bytes);

bool plane_pair_supported(int ny, int nz);
bool line_supported(int n);

}  // namespace nct
