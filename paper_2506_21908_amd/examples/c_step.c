/* A plain C client of libnct (no Python, no torch): a 16^3 cell with one atom carrying the
 * 18 KB+SOC projectors (s, p1/2, p3/2, d3/2, d5/2), a Gaussian local well, self-consistent
 * exchange + Hartree and a static B_ext; four spinor states advanced by 20 ETRS steps.
 * Device memory comes from the HIP runtime directly.  Exit status 0 when the electron number and
 * every state's norm stay within 1e-6 (the fourth-order Taylor exponential is unitary to that
 * order at this dt) and the total energy within 1e-3 relative (ETRS drift, second order in dt).
 * With a path argument the [20][13] observables are also written there as raw doubles.
 *
 * Build (what paper_2506_21908_amd/build.py does):
 *   gcc -O2 -std=c99 -D__HIP_PLATFORM_AMD__ -I include -I $ROCM/include c_step.c -o c_step \
 *       -L paper_2506_21908_amd -lnct -L $ROCM/lib -lamdhip64 -lm -Wl,-rpath,<both lib dirs> */
#include <hip/hip_runtime_api.h>
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

#include "nct.h"

#define CHECK(call)                                                                   \
  do {                                                                                \
    nct_status st_ = (call);                                                          \
    if (st_ != NCT_OK) {                                                              \
      fprintf(stderr, "%s failed: %s\n", #call, nct_last_error(sys));                 \
      return 1;                                                                       \
    }                                                                                 \
  } while (0)

int main(int argc, char** argv) {
  const int n = 16, S = 4, NSTEPS = 20;
  const double L = 8.0, h = L / n, dV = h * h * h;
  const size_t N = (size_t)n * n * n;
  nct_system* sys = NULL;

  nct_channel ch[5] = {{0, 1, 1.0, 0.7}, {1, 1, 0.45, 0.7}, {1, 3, 0.525, 0.7},
                       {2, 3, -0.33, 0.7}, {2, 5, -0.28, 0.7}};
  double pos[3] = {4.1, 3.9, 4.0};
  nct_params p = {0};
  p.n[0] = p.n[1] = p.n[2] = n;
  p.cell[0] = p.cell[1] = p.cell[2] = L;
  p.nstates = S;
  p.natoms = 1;
  p.positions = pos;
  p.nchannels = 5;
  p.channels = ch;
  p.r_sphere = 2.5;
  p.xc = 1;
  p.hartree = 1;
  p.m_threshold = 1e-12;
  p.dt = 0.05;
  p.taylor_order = 4;
  p.precision = NCT_FP64;
  CHECK(nct_create_system(&p, &sys));
  printf("%s\n", nct_version());

  /* Gaussian well at the atom and a static field */
  double* vext = (double*)malloc(N * sizeof(double));
  for (int x = 0; x < n; ++x)
    for (int y = 0; y < n; ++y)
      for (int z = 0; z < n; ++z) {
        const double dx = x * h - pos[0], dy = y * h - pos[1], dz = z * h - pos[2];
        vext[((size_t)x * n + y) * n + z] = -2.0 * exp(-(dx * dx + dy * dy + dz * dz) / 2.0);
      }
  double* vext_d = NULL;
  if (hipMalloc((void**)&vext_d, N * sizeof(double)) != hipSuccess) return 1;
  if (hipMemcpy(vext_d, vext, N * sizeof(double), hipMemcpyHostToDevice) != hipSuccess) return 1;
  nct_bfield b = {{0.0, 0.0, 0.02}, 0, NULL};
  CHECK(nct_set_potentials(sys, vext_d, &b, NULL));

  /* states: Gaussian-weighted spinors with different spin directions, each normalised */
  const size_t per = 2 * N;
  double* psi = (double*)malloc((size_t)S * per * 2 * sizeof(double));
  for (int i = 0; i < S; ++i) {
    const double th = 0.5 + 0.4 * i, ph = 0.7 * i;
    const double cu = cos(0.5 * th), su = sin(0.5 * th);
    double norm = 0.0;
    for (size_t e = 0; e < N; ++e) {
      const int x = (int)(e / (n * n)), y = (int)(e / n % n), z = (int)(e % n);
      const double dx = x * h - pos[0], dy = y * h - pos[1], dz = z * h - pos[2];
      const double g = exp(-(dx * dx + dy * dy + dz * dz) / (2.0 * (1.2 + 0.3 * i)));
      const double k = 2.0 * 3.14159265358979323846 / L * (i % 2);
      double* up = psi + ((size_t)i * per + e) * 2;
      double* dn = psi + ((size_t)i * per + N + e) * 2;
      up[0] = g * cu * cos(k * x * h);
      up[1] = g * cu * sin(k * x * h);
      dn[0] = g * su * cos(k * x * h + ph);
      dn[1] = g * su * sin(k * x * h + ph);
      norm += (up[0] * up[0] + up[1] * up[1] + dn[0] * dn[0] + dn[1] * dn[1]) * dV;
    }
    const double s = 1.0 / sqrt(norm);
    for (size_t c = 0; c < per * 2; ++c) psi[(size_t)i * per * 2 + c] *= s;
  }
  void* psi_d = NULL;
  const size_t bytes = (size_t)S * per * 2 * sizeof(double);
  if (hipMalloc(&psi_d, bytes) != hipSuccess) return 1;
  if (hipMemcpy(psi_d, psi, bytes, hipMemcpyHostToDevice) != hipSuccess) return 1;

  double obs[NSTEPS * 13];
  CHECK(nct_step(sys, psi_d, 0.0, NSTEPS, obs, 0));
  const double n0 = obs[1], e0 = obs[5];
  double dn = 0.0, de = 0.0;
  for (int k = 0; k < NSTEPS; ++k) {
    dn = fmax(dn, fabs(obs[13 * k + 1] - n0));
    de = fmax(de, fabs(obs[13 * k + 5] - e0));
  }
  printf("c_step: %d states, %d steps: N_e %.12f (max drift %.2e), E %.10f (max drift %.2e), "
         "M = (%.6f, %.6f, %.6f)\n",
         S, NSTEPS, n0, dn, e0, de, obs[13 * (NSTEPS - 1) + 2], obs[13 * (NSTEPS - 1) + 3],
         obs[13 * (NSTEPS - 1) + 4]);
  nct_destroy_system(sys);
  (void)hipFree(psi_d);
  (void)hipFree(vext_d);
  free(psi);
  free(vext);
  double dnorm = 0.0;
  for (int k = 0; k < NSTEPS; ++k) dnorm = fmax(dnorm, obs[13 * k + 12]);
  if (argc > 1) {
    FILE* f = fopen(argv[1], "wb");
    if (!f || fwrite(obs, sizeof(double), 13 * NSTEPS, f) != (size_t)(13 * NSTEPS)) return 1;
    fclose(f);
  }
  if (!(fabs(n0 - 4.0) < 1e-6 && dn < 1e-6 && dnorm < 1e-6 && de < 1e-3 * fabs(e0))) {
    fprintf(stderr, "c_step: conservation check failed\n");
    return 1;
  }
  return 0;
}
