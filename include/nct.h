/*
 * nct.h -- C ABI of libnct.so: one real-time time step of spin non-collinear
 * TDDFT for a set of two-component spinor Kohn-Sham states on a periodic
 * real-space / plane-wave grid, on one AMD MI355X (gfx950).
 *
 * Physics follows arXiv 2506.21908:
 *   - Hamiltonian: the non-collinear Kohn-Sham Hamiltonian of Eq. (HNC-SDFT),
 *     integrated in time as in Eq. (TDSDFT): kinetic -1/2 nabla^2 (plane-wave
 *     basis), local 2x2 potential [v 1 + b.sigma] with
 *     v = v_ext + v_H + vbar_xc and b = b_xc + mu_B B_ext(t) (mu_B = 1/2),
 *     the Zeeman term of Eq. (zeeman_potential), and Kleinman-Bylander
 *     projectors with j = l +/- 1/2 spinor spherical harmonics, Eqs. (Vps),
 *     (Vps-soc) and the spinor-harmonic formula of the spin-orbit section.
 *   - Spin density matrix stored as rho_v = {rho_uu, rho_dd, Re rho_ud,
 *     Im rho_ud}, Eq. (density4); m_x = 2 Re rho_ud, m_y = -2 Im rho_ud,
 *     m_z = rho_uu - rho_dd, Eqs. (rho1-3).
 *   - Exchange-correlation: adiabatic, locally collinear, Eqs. (LC+ALDA2),
 *     (LC+ALDA); Slater exchange, optionally with the Perdew-Wang 1992 LSDA
 *     correlation (Phys. Rev. B 45, 13244); b_xc = 0 where |m| < m_threshold.
 *   - Hartree: Eq. (KSpot) solved by FFT, G = 0 term dropped.
 *   - Optional uniform electric (laser) pulse E(t) with the temporal profile of
 *     the optical runs of Sec. 4.7, in the length or the velocity gauge (see
 *     nct_set_laser, nct_set_laser_gauge).
 *   - Optional k-point sampling (state index i = (n, k), Eq. KSDFT; see
 *     nct_set_kpoints).
 *   - Initial spin density of the magnetisation-initialisation algorithm
 *     (nct_dm_initialization) and an imaginary-time ground state
 *     (nct_ground_state); the reverse-mode (adjoint) step (nct_backward_step).
 *   - Propagator (the paper names none): enforced time-reversal symmetry with
 *     a truncated Taylor exponential of order taylor_order:
 *        phi = T(-i dt/2 H[rho(psi_n), B(t_n)]) psi_n
 *        psi~ = T(-i dt/2 H[rho(psi_n), B(t_n)]) phi
 *        psi_{n+1} = T(-i dt/2 H[rho(psi~), B(t_n + dt)]) phi
 *
 * Units: Hartree atomic units.
 *
 * Memory layout of a set of states ("psi"), device memory owned by the caller:
 *   psi[i][s][ix][iy][iz], i < nstates, s = 0 (up) / 1 (down), iz fastest;
 *   interleaved complex: complex128 (double re, im) when precision = NCT_FP64,
 *   complex64 (float re, im) when precision = NCT_FP32_MIXED.
 *   Grid point r = (ix hx, iy hy, iz hz), h_d = cell[d] / n[d].
 *   Normalisation: dV sum_r sum_s |psi_i(r,s)|^2 = 1, dV = hx hy hz.
 * Real fields ("[4][N]") are double, index [k][ix][iy][iz], N = nx ny nz.
 *
 * Ownership: every device pointer passed in stays owned by the caller; the
 * library allocates its own workspace in nct_create_system and frees it in
 * nct_destroy_system.
 *
 * Streams: all work is enqueued on params.stream (a hipStream_t; NULL means
 * the default stream); some passes run on the library's own streams, ordered
 * against params.stream by events.  Calls return once the work is enqueued,
 * except calls that write host memory (totals_host, obs_host, dLdB_host,
 * dLdtheta_host), which synchronise the stream before returning.
 *
 * Errors: every call returns an nct_status; no exception crosses the ABI.
 * NCT_ERR_ARG is returned before any work is enqueued and leaves every output
 * untouched.  After NCT_ERR_HIP or NCT_ERR_NONFINITE the contents of psi
 * outputs are unspecified.  nct_last_error(sys) returns a text description of
 * the last failure on that system (nct_last_error(NULL) for failures of
 * nct_create_system).  One system must not be used by two host threads at once.
 */
#ifndef NCT_H
#define NCT_H

#ifdef __cplusplus
extern "C" {
#endif

typedef struct nct_system nct_system;

typedef enum {
  NCT_OK = 0,
  NCT_ERR_ARG = 1,          /* invalid argument; nothing was done */
  NCT_ERR_UNSUPPORTED = 2,  /* grid size or option not built into this library */
  NCT_ERR_OOM = 3,          /* device allocation failed */
  NCT_ERR_HIP = 4,          /* a HIP runtime call or kernel launch failed */
  NCT_ERR_NONFINITE = 5,    /* a non-finite density or energy was produced */
  NCT_ERR_STATE = 6         /* call out of sequence (e.g. no tape recorded) */
} nct_status;

enum { NCT_FP64 = 0, NCT_FP32_MIXED = 1 };

/* One Kleinman-Bylander channel (l, j = twoj/2): projector radial form
 * r^l exp(-r^2 / 2 rc^2), cut at r_sphere and normalised by its continuum
 * radial integral; 'energy' is the KB energy E_lj (Eq. Vps with the
 * denominator absorbed).  The channel expands to twoj+1 projectors
 * (m_j = -j..j) built from the spinor harmonics of the spin-orbit section,
 * read with m = m_j - 1/2 for j = l + 1/2 and m = m_j + 1/2 for j = l - 1/2. */
typedef struct {
  int l;          /* 0, 1 or 2 */
  int twoj;       /* 2l+1 or 2l-1 (>= 1) */
  double energy;  /* Hartree */
  double rc;      /* bohr */
} nct_channel;

/* Circularly polarised Gaussian pulse:
 * B(t) = A exp(-(t-t0)^2 / 2 tau^2) [cos(omega (t-t0) + phase) e1 + sin(omega (t-t0) + phase) e2] */
typedef struct {
  double A, omega, t0, tau, phase;
  double e1[3], e2[3];
} nct_pulse;

/* External field B_ext(t) = B0 + sum of pulses (atomic units of field; the
 * Zeeman energy is mu_B B = B/2 Hartree).  Spin Zeeman coupling only. */
typedef struct {
  double B0[3];
  int npulses;
  const nct_pulse *pulses;   /* host [npulses]; copied by nct_set_potentials */
} nct_bfield;

typedef struct {
  int n[3];                   /* grid; each n[d] in {8,12,16,24,32,48,64,96}; (n[1],n[2]) must be a built pair */
  double cell[3];             /* orthorhombic periodic cell edges (bohr) */
  int nstates;                /* S >= 1 */
  const double *occ;          /* host [S] occupations, or NULL for all 1 */
  int natoms;                 /* >= 0 */
  const double *positions;    /* host [natoms][3] (bohr) */
  int nchannels;              /* projector channels per atom (0: no nonlocal term) */
  const nct_channel *channels;/* host [nchannels], the same table for every atom */
  double r_sphere;            /* projector sphere radius (bohr), < half the smallest cell edge */
  int xc;                     /* 0: none; 1: Slater exchange; 2: Slater exchange + PW92 correlation
                                 (LSDA); both locally collinear */
  int hartree;                /* 0: none; 1: FFT Poisson */
  double m_threshold;         /* |m| below which b_xc = 0 (bohr^-3) */
  double dt;                  /* time step (a.u.) */
  int taylor_order;           /* 1..16 */
  int precision;              /* NCT_FP64 or NCT_FP32_MIXED */
  int tape_steps;             /* steps the adjoint tape can hold (0: recompute mode only) */
  int overlap;                /* nonzero: run the Taylor stages of two halves of the states on two
                                 internal streams so their passes overlap (off by default: the
                                 per-kernel timings then measure overlapping kernels) */
  void *stream;               /* hipStream_t or NULL */
} nct_params;

/* Build a system (the problem of Eq. TDSDFT for two-component spinor states, Sec. 3.1): copies
 * the parameters, builds FFT tables and the projector tables of every atom (Eqs. Vps, Vps-soc),
 * and allocates all device workspace.  External potential starts at zero, B_ext at zero, fields
 * self-consistent.
 * Errors: NCT_ERR_ARG (a parameter out of range; *out untouched), NCT_ERR_UNSUPPORTED (a grid
 * size or plane pair not built, more than 32 projectors per atom), NCT_ERR_OOM, NCT_ERR_HIP. */
nct_status nct_create_system(const nct_params *params, nct_system **out);

/* Free every resource of the system (synchronises its stream). NULL is a no-op. */
void nct_destroy_system(nct_system *sys);

/* Text of the last error on sys, or of the last nct_create_system failure when sys is NULL. */
const char *nct_last_error(const nct_system *sys);

/* Uniform electric pulse (Sec. 4.7; the magnetic component of the light is neglected):
 * E(t) = A pol cos(omega t + phase) exp(-(t - t0)^2 / 2 tau^2), atomic units of field. */
typedef struct {
  double A, omega, t0, tau, phase;
  double pol[3];
} nct_laser_pulse;

/* Set the uniform electric field E(t) = sum of the given pulses, acting on the charge in the
 * length gauge: the local potential gains v_E(r, t) = E(t).(r - c) (potential energy of a charge
 * -1), r = (ix hx, iy hy, iz hz), c = cell / 2.  The sawtooth jumps on the cell faces, so this
 * describes an isolated system whose density vanishes there.  E is evaluated like B_ext: at t_n
 * for H_n and at t_n + dt for H~.  int v_E n enters E_loc of the observables, and the fields
 * returned by nct_get_fields include v_E(t).  Like B_ext it is not applied while the fields are
 * frozen (nct_set_potentials with fields_dev).
 *   pulses  host [npulses] (copied); npulses = 0 (pulses may be NULL) removes the field.
 * Errors: NCT_ERR_ARG if npulses < 0, npulses > 0 with pulses NULL, or a pulse has tau <= 0 or
 * a non-finite parameter. */
nct_status nct_set_laser(nct_system *sys, int npulses, const nct_laser_pulse *pulses);

/* Atomic data of the initial spin-density matrix (initialisation algorithm of Sec. 3.2): the
 * atom's charge Z (electrons) spread as a Gaussian of width sigma (bohr) and its magnetic moment
 * (mu_B, |moment| <= Z). */
typedef struct {
  double Z;
  double sigma;
  double moment[3];
} nct_atom_density;

/* Initial spin-density matrix (Sec. 3.2, DMInitialization): every grid point belongs to its
 * nearest atom (Voronoi partition with the minimum-image distance d, ties to the lowest index);
 * there n = Z (2 pi sigma^2)^(-3/2) exp(-d^2 / 2 sigma^2), the local polarisation vector is
 * m = moment / Z (the atom's moment per electron), and
 * rho_v = n {(1 + m_z)/2, (1 - m_z)/2, m_x/2, -m_y/2} (Eq. density4).
 *   atoms        host [params.natoms], in the order of params.positions;
 *   rho_v_dev    device double [4][N] receives rho_v, or NULL;
 *   update_fields nonzero: the system's fields become those of this density (self-consistent
 *                mode only), e.g. to start nct_ground_state from it.
 * Synchronises the stream.  Errors: NCT_ERR_ARG (no atoms, NULL atoms, Z or sigma not positive,
 * |moment| > Z), NCT_ERR_STATE (update_fields with frozen fields). */
nct_status nct_dm_initialization(nct_system *sys, const nct_atom_density *atoms, double *rho_v_dev,
                                 int update_fields);

/* Ground state by self-consistent imaginary-time propagation (the paper does not specify its
 * solver): psi is first orthonormalised, then every iteration forms T_K(-tau H[rho]) psi (the
 * Taylor polynomial of exp(-tau H) of order params.taylor_order, through the same kernels as
 * the real-time step), orthonormalises it (Cholesky of the state overlap: the overlap
 * dV Psi^H Psi and the triangular change of basis Psi L^-H run on the matrix cores with FP64
 * accumulation in either precision, the S x S factorisation on the host; with k-points, within
 * each run of consecutive states that share one Bloch vector)
 * and recomputes rho and the fields from it.  keep_fields nonzero: the first iteration uses the
 * system's current fields (e.g. from nct_dm_initialization); 0: those of psi's own density.
 * With frozen fields they stay frozen.  energies_host, if non-NULL, receives [niter] total
 * energies (the E_total of nct_step's observables).  B_ext is taken at t = 0.  tau must keep
 * tau |H| within the stability range of the Taylor polynomial (|T_4(-x)| < 1 for x < 2.78).
 * Synchronises the stream.  Errors: NCT_ERR_ARG (niter < 0, tau not positive), NCT_ERR_NONFINITE
 * (states linearly dependent, or a non-finite energy), NCT_ERR_UNSUPPORTED (more than 4096
 * states, or the states of one Bloch vector not consecutive). */
nct_status nct_ground_state(nct_system *sys, void *psi_dev, int niter, double tau, int keep_fields,
                            double *energies_host);

/* Gauge of the laser set by nct_set_laser.
 *   NCT_GAUGE_LENGTH (default): v_E = E(t).(r - c) as described there (isolated systems);
 *   NCT_GAUGE_VELOCITY: for periodic systems; every state's kinetic momentum is shifted by the
 *     vector potential A(t) = -int_0^t E dt' (evaluated like B_ext: t_n for H_n, t_n + dt for
 *     H~): kinetic factor 1/2 |G + k + A|^2 and projector phases exp(+/- i (k + A).d), no scalar
 *     potential and no E.D term in E_loc.
 * Errors: NCT_ERR_ARG for any other value. */
enum { NCT_GAUGE_LENGTH = 0, NCT_GAUGE_VELOCITY = 1 };
nct_status nct_set_laser_gauge(nct_system *sys, int gauge);

/* k-point sampling (the state index i = (n, k) of Eq. KSDFT; Sec. 5 runs 8 k-points of a bcc
 * supercell).  kvec host double [nstates][3]: the Bloch vector of each state (bohr^-1, copied);
 * the states then hold the periodic parts u_i of psi_i = exp(i k_i.r) u_i: the kinetic factor
 * becomes 1/2 |G + k_i|^2 and the projector rows carry exp(i k_i.d) on projection and
 * exp(-i k_i.d) on scatter (d the grid point's displacement from the atom).  The k-point weights
 * enter through params.occ (f_i w_k).  States of one k-point are expected consecutive (the
 * ground-state solver orthonormalises each such run).  NULL returns to Gamma only.
 * Synchronises the stream.
 * Errors: NCT_ERR_ARG for a non-finite component. */
nct_status nct_set_kpoints(nct_system *sys, const double *kvec);

/* Set the potentials of Eq. (HNC-SDFT) and the external field of the Zeeman term
 * (Eq. zeeman_potential):
 *   v_ext_dev  device double [N]: external local potential v_ext(r) (copied), or NULL to keep;
 *   b          host: B_ext(t) description (copied), or NULL to keep;
 *   fields_dev device double [4][N] {v, b_x, b_y, b_z}: if non-NULL, the total local fields
 *              are frozen to these values (no density update, no B_ext added) until
 *              nct_set_potentials is called again with fields_dev = NULL, which returns the
 *              system to self-consistent fields. */
nct_status nct_set_potentials(nct_system *sys, const double *v_ext_dev, const nct_bfield *b,
                              const double *fields_dev);

/* Spin density of psi (Eq. density4; n and m from it by Eqs. rho1-3), and optionally the fields
 * of Eq. (HNC-SDFT) that follow from it (Hartree, Eq. KSpot; exchange-correlation, Eqs. LC+ALDA2,
 * LC+ALDA):
 *   rho_v_dev    device double [4][N] {rho_uu, rho_dd, Re rho_ud, Im rho_ud}, or NULL;
 *   totals_host  host double[4] {N_e, M_x, M_y, M_z} (integrated), or NULL (synchronises);
 *   update_fields  nonzero: recompute v_H and the exchange fields from this density and keep
 *                  them as the system's current fields (self-consistent mode only).
 *   t is used only to report the fields; B_ext(t) is applied when H is applied. */
nct_status nct_density_magnetization(nct_system *sys, const void *psi_dev, double t,
                                     double *rho_v_dev, double *totals_host, int update_fields);

/* Allocation-free variant of nct_density_magnetization, for callers that cannot allocate device
 * memory during the call (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  Same arguments, results and synchronisation as nct_density_magnetization; it calls
 * no hipMalloc, hipFree or allocating library routine.  The temporaries of its kernels (Poisson
 * work, the fields output when update_fields is 0, block partial sums and totals) live in a static
 * device array of NCT_STATIC_SCRATCH_BYTES (32 MiB) that the library holds on every device it runs
 * on until the process ends: it takes 48 N bytes plus a little, which admits grids up to about
 * 690,000 points (64 x 96 x 96, not 96^3).  That array is shared by every system on the device and keeps the last
 * call's contents: calls that overlap on one device (two host threads, or work on two streams not
 * ordered by events) race.
 * Errors: as nct_density_magnetization, plus NCT_ERR_UNSUPPORTED (before any work) when the grid
 * needs more than the array holds, and NCT_ERR_HIP if the array's address could not be looked up
 * when the system was created. */
nct_status nct_density_magnetization_static(nct_system *sys, const void *psi_dev, double t,
                                            double *rho_v_dev, double *totals_host, int update_fields);

/* Current total local fields at time t into device double [4][N] {v, b_x, b_y, b_z}
 * (v = v_ext + v_E(t) + v_H + vbar_xc, b = b_xc + mu_B B_ext(t); v_E is zero without a laser). */
nct_status nct_get_fields(nct_system *sys, double t, double *fields_dev);

/* hpsi = H psi: the spinor Kohn-Sham Hamiltonian of Eqs. (TDSDFT) and (HNC-SDFT) with the
 * pseudopotential of Eqs. (Vps), (Vps-soc): -1/2 nabla^2 + [v + b.sigma] + V_NL, with the current
 * fields, B_ext(t) and v_E(t).  psi and hpsi are distinct device buffers of the psi layout above
 * (caller-owned; hpsi is overwritten).
 * Errors: NCT_ERR_ARG (NULL or identical buffers), NCT_ERR_STATE (no fields yet: call
 * nct_density_magnetization with update_fields, or freeze fields with nct_set_potentials). */
nct_status nct_apply_hamiltonian(nct_system *sys, const void *psi_dev, void *hpsi_dev, double t);

/* Advance psi in place by nsteps steps of Eq. (TDSDFT) from time t0, each one enforced
 * time-reversal-symmetry step (the paper names no propagator; see the top of this file).  The
 * fields of the first step are computed from psi itself.  obs_host, if non-NULL, receives [nsteps][13] doubles after each
 * step: t, N_e, M_x, M_y, M_z, E_total, E_kin, E_loc, E_NL, E_H, E_xc, E_Z,
 * max_i |<psi_i|psi_i> - 1|, with
 *   E = sum_i f_i <psi_i|T|psi_i> + int (v_ext + v_E(t)) n + sum_i f_i sum_p E_p |C_p,i|^2
 *       + 1/2 int v_H n + int e_xc + mu_B B.M  (e_xc: exchange, plus PW92 correlation if xc = 2).
 * tape nonzero: record what nct_backward_step needs for each of these steps (requires
 * nsteps <= params.tape_steps); the record of step k of this call has tape_index k.
 * Returns NCT_ERR_NONFINITE if N_e became non-finite. */
nct_status nct_step(nct_system *sys, void *psi_dev, double t0, int nsteps, double *obs_host,
                    int tape);

/* Per-step watchdog of nct_step.  Every self-consistent step reduces the electron count
 * N_e = sum_i f_i <psi_i|psi_i> with its fields; nct_step keeps that value for every step of the
 * call on the device and, once the call's work is done, returns NCT_ERR_NONFINITE (naming the
 * first failing step) if it is not finite or if |N_e(step) - N_e(start)| / |N_e(start)| exceeds
 * max_rel_drift (default 1e-3; <= 0 checks finiteness only).  A non-finite value anywhere in a
 * state makes N_e non-finite.  With frozen fields only the final state is checked.
 * Errors: NCT_ERR_ARG if max_rel_drift is NaN. */
nct_status nct_set_watchdog(nct_system *sys, double max_rel_drift);

/* lam = 2 dV f_i (w . sigma) psi_i: the adjoint seed 2 dL/dpsi* of L = w . M(t) with
 * M = int m dV.  psi and lam have the psi layout; w is host double[3]. */
nct_status nct_magnetization_seed(nct_system *sys, const void *psi_dev, const double *w,
                                  void *lam_dev);

/* Reverse-mode (adjoint) of one step of nct_step, n -> n+1: the transpose of the step's
 * linearisation (the paper has no adjoint; this is the derivative of the discrete step of
 * Eq. TDSDFT as nct_step computes it, used for gradients of M(T) with respect to the pulse
 * parameters of B_ext).  With lam = 2 dL/dpsi* (so that
 * dL = Re sum lam^* dpsi), given lam_{n+1} returns lam_n, including the response of the
 * Hartree and exchange(-correlation) fields to the density at psi_n and psi~.  The forward quantities come
 * from tape record tape_index of the last taped nct_step, or, when tape_index < 0, are
 * recomputed from psi_n_dev (device, psi layout) at time t_n.
 *   dLdB_host      host double[6]: dL/dB_ext(t_n) (3) and dL/dB_ext(t_n + dt) (3);
 *   dLdtheta_host  host double[2*npulses]: dL/d(A_k) then dL/d(omega_k) are ADDED to it
 *                  (accumulate over steps), or NULL.
 * lam_np1_dev and lam_n_dev may be the same buffer.  Every xc setting is covered (the PW92
 * correlation response by forward-mode derivatives of its potentials).  A laser (nct_set_laser)
 * is re-applied in the reverse stages at the forward times, in either gauge. */
nct_status nct_backward_step(nct_system *sys, int tape_index, const void *psi_n_dev, double t_n,
                             const void *lam_np1_dev, void *lam_n_dev, double *dLdB_host,
                             double *dLdtheta_host);

/* Kernel classes for the timing facility below. */
enum {
  NCT_K_PLANE_STAGE = 0,  /* fused plane pass of one H application / Taylor stage */
  NCT_K_XPASS = 1,        /* column pass along x (kinetic multiplier) */
  NCT_K_PLANE_FWD = 2,    /* forward yz transform of the input states */
  NCT_K_DENSITY = 3,      /* spin density matrix reduction */
  NCT_K_FIELDS = 4,       /* Poisson solve, exchange, field totals */
  NCT_K_PROJ = 5,         /* projector contraction + scatter (MFMA) */
  NCT_K_OBS = 6,          /* observables (energy pass, row assembly) */
  NCT_K_ADJOINT = 7,      /* adjoint-only kernels (pair reductions, density back-propagation) */
  NCT_K_ORTH = 8,         /* ground-state orthonormalisation (overlap and change of basis, MFMA) */
  NCT_K_COUNT = 9
};

/* Profiling aid.  nct_set_timing(sys, mask) resets the counters and, for every kernel class k
 * with bit k of mask set, records a pair of HIP events on each launch of that class (attached to
 * the dispatch, on the stream it runs on); mask = 0 stops, mask = -1 records every class.
 * nct_get_timing synchronises the stream and returns for kernel class kclass the summed
 * duration in milliseconds, the number of launches, and the algorithmic bytes and flops of
 * those launches (compulsory HBM traffic and useful arithmetic of the launch's definition,
 * not counters).  Outputs may be NULL. */
nct_status nct_set_timing(nct_system *sys, int enable);
/* Record only one launch in every 'every' launches of each enabled class (default 1: all).  The
 * events ride on the kernel dispatch, which costs the stream ~10 us per recorded launch; sampling
 * with a stride coprime to the launches per step still visits every stage of the step.
 * Errors: NCT_ERR_ARG if every < 1. */
nct_status nct_set_timing_sample(nct_system *sys, int every);
nct_status nct_get_timing(nct_system *sys, int kclass, double *ms, long long *launches,
                          double *bytes, double *flops);

/* Library build string (architecture, precisions, grid sizes built). */
const char *nct_version(void);

#ifdef __cplusplus
}
#endif
#endif /* NCT_H */
