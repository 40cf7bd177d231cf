// Host-side projector tables of the Kleinman-Bylander + spin-orbit nonlocal term (Eqs. Vps,
// Vps-soc and the spinor harmonics of the spin-orbit section): the grid points inside each atom's
// sphere ("sphere rows"), the projector values on them, and the per-plane row ranges the plane
// pass walks.  Plain C++ (no HIP): the library uploads the result, and a CPU test builds it under
// AddressSanitizer / UndefinedBehaviorSanitizer for every projector shape the tests use.
#pragma once
#include <algorithm>
#include <cmath>
#include <complex>
#include <string>
#include <vector>

#include "../../include/nct.h"

namespace nct {
namespace tables {

constexpr double kPi = 3.14159265358979323846;

// complex spherical harmonics with the Condon-Shortley phase, l <= 2, at the unit vector (x, y, z)
inline std::complex<double> ylm(int l, int m, double x, double y, double z) {
  using C = std::complex<double>;
  if (std::abs(m) > l) return C(0, 0);
  const double pi = kPi;
  if (l == 0) return C(0.5 / std::sqrt(pi), 0);
  if (l == 1) {
    if (m == 0) return C(std::sqrt(3.0 / (4 * pi)) * z, 0);
    return -double(m) * std::sqrt(3.0 / (8 * pi)) * C(x, m * y);
  }
  if (l == 2) {
    if (m == 0) return C(std::sqrt(5.0 / (16 * pi)) * (3 * z * z - 1), 0);
    if (std::abs(m) == 1) return -double(m) * std::sqrt(15.0 / (8 * pi)) * z * C(x, m * y);
    const double sgn = m > 0 ? 1.0 : -1.0;
    const C u(x, sgn * y);
    return std::sqrt(15.0 / (32 * pi)) * u * u;
  }
  return C(0, 0);
}

// Gauss-Legendre nodes/weights on [-1,1]
inline void gauss_legendre(int n, std::vector<double>& xs, std::vector<double>& ws) {
  xs.assign(n, 0);
  ws.assign(n, 0);
  for (int i = 0; i < (n + 1) / 2; ++i) {
    double x = std::cos(kPi * (i + 0.75) / (n + 0.5));
    for (int it = 0; it < 100; ++it) {
      double p0 = 1, p1 = x;
      for (int k = 2; k <= n; ++k) {
        double p2 = ((2 * k - 1) * x * p1 - (k - 1) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      const double dp = n * (x * p1 - p0) / (x * x - 1);
      const double dx = p1 / dp;
      x -= dx;
      if (std::fabs(dx) < 1e-16) break;
    }
    double p0 = 1, p1 = x;
    for (int k = 2; k <= n; ++k) {
      double p2 = ((2 * k - 1) * x * p1 - (k - 1) * p0) / k;
      p0 = p1;
      p1 = p2;
    }
    const double dp = n * (x * p1 - p0) / (x * x - 1);
    xs[i] = -x;
    xs[n - 1 - i] = x;
    ws[i] = ws[n - 1 - i] = 2.0 / ((1 - x * x) * dp * dp);
  }
}

// 24-point Gauss-Legendre rule on [-1, 1], built once (thread-safe static initialisation)
struct GLRule {
  std::vector<double> x, w;
  explicit GLRule(int n) { gauss_legendre(n, x, w); }
};
inline const GLRule& gl24() {
  static const GLRule rule(24);
  return rule;
}

// sqrt( int_0^rs (r^l e^{-r^2/2rc^2})^2 r^2 dr ), composite Gauss-Legendre
inline double radial_norm(int l, double rc, double rs) {
  const std::vector<double>& xs = gl24().x;
  const std::vector<double>& ws = gl24().w;
  const int panels = 16;
  double acc = 0.0;
  for (int p = 0; p < panels; ++p) {
    const double a = rs * p / panels, b = rs * (p + 1) / panels;
    for (size_t q = 0; q < xs.size(); ++q) {
      const double r = 0.5 * (a + b) + 0.5 * (b - a) * xs[q];
      const double f = std::pow(r, l) * std::exp(-r * r / (2 * rc * rc));
      acc += 0.5 * (b - a) * ws[q] * f * f * r * r;
    }
  }
  return std::sqrt(acc);
}

// Spinor harmonic coefficients: Phi = c_up Y_l^{m_up} chi_up + c_dn Y_l^{m_dn} chi_dn
inline void spinor_coeffs(int l, int twoj, int twomj, double& cu, int& mu, double& cd, int& md) {
  const double mj = 0.5 * twomj;
  mu = (twomj - 1) / 2;  // twomj is odd: exact division, m_up = m_j - 1/2
  md = (twomj + 1) / 2;  // m_dn = m_j + 1/2
  if (twoj == 2 * l + 1) {
    cu = std::sqrt((l + mj + 0.5) / (2 * l + 1));
    cd = std::sqrt((l - mj + 0.5) / (2 * l + 1));
  } else {
    cu = std::sqrt((l - mj + 0.5) / (2 * l + 1));
    cd = -std::sqrt((l + mj + 0.5) / (2 * l + 1));
  }
}


// Tables of one system.  Sphere rows of all atoms are numbered J = 0..Jtot-1; atom a owns rows
// [row_off[a], row_off[a+1]) in increasing flat grid index (ix NY + iy) NZ + iz, so the rows of
// one x-plane form one contiguous range per atom; ranges [pr_begin[r], pr_end[r]) for
// r in [pr_off[x], pr_off[x+1]) list them plane by plane (atoms with no row on the plane have no
// range there).
struct ProjectorTables {
  int natoms = 0;
  int P = 0;            // projectors per atom (sum over channels of 2j + 1)
  int PP = 0;           // P padded to a multiple of 16 (the MFMA tile)
  int Jtot = 0;         // total sphere rows
  int max_kchunks = 1;  // max over atoms of ceil(2 rows / 64), at least 1
  int max_rowtiles = 1; // max over atoms of ceil(2 rows / 16), at least 1
  std::vector<int> row_off;                   // [natoms + 1]
  std::vector<int> pidx;                      // [Jtot] in-plane index iy NZ + iz
  std::vector<int> ix_of_row;                 // [Jtot] plane of each row
  std::vector<int> pr_off;                    // [NX + 1]
  std::vector<int> pr_begin, pr_end;          // [nranges]
  std::vector<std::complex<double>> beta;     // [Jtot][2][PP]: beta_p(r, s), zero beyond P
  std::vector<double> disp;                   // [Jtot][3] minimum-image displacement r - R_a
  std::vector<double> energy;                 // [natoms][PP] KB energy E_p, zero beyond P
};

// Builds the tables for grid n, cell, the atoms and the channel table shared by every atom.
// Returns an empty string on success, else the reason (nothing else is reported).
// Requirements: n[d] >= 1, cell[d] > 0, 0 < r_sphere < half the smallest cell edge (so that the
// minimum image is the only image inside the sphere), channels with 0 <= l <= 2,
// twoj = 2l +/- 1 >= 1, rc > 0, and at most 32 projectors per atom.
inline std::string build_projector_tables(const int n[3], const double cell[3], int natoms,
                                          const double* positions, int nchannels,
                                          const nct_channel* channels, double r_sphere,
                                          ProjectorTables& out) {
  out = ProjectorTables{};
  if (natoms <= 0 || nchannels <= 0) return "";
  if (!positions || !channels) return "null positions or channels";
  for (int d = 0; d < 3; ++d)
    if (n[d] < 1 || !(cell[d] > 0.0)) return "bad grid or cell";
  const double mincell = std::min(cell[0], std::min(cell[1], cell[2]));
  if (!(r_sphere > 0.0) || !(r_sphere < 0.5 * mincell)) return "r_sphere must be in (0, cell/2)";
  int P = 0;
  for (int c = 0; c < nchannels; ++c) {
    const nct_channel& ch = channels[c];
    if (ch.l < 0 || ch.l > 2 || (ch.twoj != 2 * ch.l + 1 && ch.twoj != 2 * ch.l - 1) || !(ch.rc > 0.0))
      return "bad channel";
    P += ch.twoj + 1;
  }
  if (P > 32) return "at most 32 projectors per atom";
  const int PP = ((P + 15) / 16) * 16;
  const int NX = n[0], NY = n[1], NZ = n[2];
  const double h[3] = {cell[0] / NX, cell[1] / NY, cell[2] / NZ};
  out.natoms = natoms;
  out.P = P;
  out.PP = PP;
  out.row_off.assign(size_t(natoms) + 1, 0);
  out.energy.assign(size_t(natoms) * PP, 0.0);
  std::vector<double> rnorm(nchannels);
  for (int c = 0; c < nchannels; ++c) rnorm[c] = radial_norm(channels[c].l, channels[c].rc, r_sphere);
  int maxk = 0, maxrt = 0;
  for (int a = 0; a < natoms; ++a) {
    const double* R0 = positions + 3 * size_t(a);
    int pcount = 0;
    for (int c = 0; c < nchannels; ++c)
      for (int twomj = -channels[c].twoj; twomj <= channels[c].twoj; twomj += 2)
        out.energy[size_t(a) * PP + pcount++] = channels[c].energy;
    int cnt = 0;
    for (int ix = 0; ix < NX; ++ix)
      for (int iy = 0; iy < NY; ++iy)
        for (int iz = 0; iz < NZ; ++iz) {
          double d[3] = {ix * h[0] - R0[0], iy * h[1] - R0[1], iz * h[2] - R0[2]};
          for (int k = 0; k < 3; ++k) d[k] -= cell[k] * std::nearbyint(d[k] / cell[k]);
          const double dist = std::sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
          if (!(dist < r_sphere)) continue;
          double u[3] = {0, 0, 1};
          if (dist > 0) {
            u[0] = d[0] / dist;
            u[1] = d[1] / dist;
            u[2] = d[2] / dist;
          }
          out.pidx.push_back(iy * NZ + iz);
          out.ix_of_row.push_back(ix);
          for (int k = 0; k < 3; ++k) out.disp.push_back(d[k]);
          const size_t base = out.beta.size();
          out.beta.resize(base + 2 * size_t(PP), std::complex<double>(0.0, 0.0));
          int p = 0;
          for (int c = 0; c < nchannels; ++c) {
            const nct_channel& ch = channels[c];
            const double f = std::pow(dist, ch.l) * std::exp(-dist * dist / (2 * ch.rc * ch.rc)) / rnorm[c];
            for (int twomj = -ch.twoj; twomj <= ch.twoj; twomj += 2) {
              double cu, cd;
              int mu, md;
              spinor_coeffs(ch.l, ch.twoj, twomj, cu, mu, cd, md);
              out.beta[base + p] = f * cu * ylm(ch.l, mu, u[0], u[1], u[2]);
              out.beta[base + PP + p] = f * cd * ylm(ch.l, md, u[0], u[1], u[2]);
              ++p;
            }
          }
          ++cnt;
        }
    out.row_off[a + 1] = out.row_off[a] + cnt;
    maxk = std::max(maxk, (2 * cnt + 63) / 64);
    maxrt = std::max(maxrt, (2 * cnt + 15) / 16);
  }
  out.Jtot = out.row_off[natoms];
  out.max_kchunks = std::max(maxk, 1);
  out.max_rowtiles = std::max(maxrt, 1);
  // plane -> one range per atom with rows on that plane; an atom's rows are in increasing flat
  // index, so its rows on plane x are consecutive: find them by binary search on ix_of_row
  out.pr_off.assign(size_t(NX) + 1, 0);
  for (int x = 0; x < NX; ++x) {
    for (int a = 0; a < natoms; ++a) {
      const int* first = out.ix_of_row.data() + out.row_off[a];
      const int* last = out.ix_of_row.data() + out.row_off[a + 1];
      const int* b = std::lower_bound(first, last, x);
      const int* e = std::upper_bound(b, last, x);
      if (b != e) {
        out.pr_begin.push_back(int(b - out.ix_of_row.data()));
        out.pr_end.push_back(int(e - out.ix_of_row.data()));
      }
    }
    out.pr_off[x + 1] = int(out.pr_begin.size());
  }
  return "";
}

}  // namespace tables
}  // namespace nct
