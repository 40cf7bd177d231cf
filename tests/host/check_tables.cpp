// CPU check of the host projector tables (paper_2506_21908_amd/csrc/nct_tables.hpp), built with
// AddressSanitizer and UndefinedBehaviorSanitizer by tests/test_host_tables.py.  For every case it
// checks, against a brute-force search over the periodic images, that each atom's sphere rows
// are exactly the grid points within r_sphere, that the rows are in increasing flat index, that
// every index the kernels use is in bounds, and that the per-plane ranges cover each atom's rows of
// that plane exactly once.  Prints "ok <cases>" and returns 0, or names the first failure.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <random>
#include <set>
#include <vector>

#include "../../paper_2506_21908_amd/csrc/nct_tables.hpp"

namespace {

int g_fail = 0;
#define CHECK(cond, ...)                                  \
  do {                                                    \
    if (!(cond)) {                                        \
      std::printf("FAIL %s:%d: ", __FILE__, __LINE__);    \
      std::printf(__VA_ARGS__);                           \
      std::printf("\n");                                  \
      ++g_fail;                                           \
      return;                                             \
    }                                                     \
  } while (0)

std::vector<nct_channel> kb18() {
  // s, p1/2, p3/2, d3/2, d5/2: 2 + 2 + 4 + 4 + 6 = 18 projectors
  return {{0, 1, 1.0, 0.7}, {1, 1, 0.45, 0.7}, {1, 3, 0.525, 0.7}, {2, 3, -0.375, 0.7}, {2, 5, -0.25, 0.7}};
}

// brute force: grid points whose distance to some periodic image of R (within 4 cells) is below rs
std::set<long> sphere_points(const int n[3], const double cell[3], const double* R, double rs) {
  std::set<long> pts;
  const double h[3] = {cell[0] / n[0], cell[1] / n[1], cell[2] / n[2]};
  for (int ix = 0; ix < n[0]; ++ix)
    for (int iy = 0; iy < n[1]; ++iy)
      for (int iz = 0; iz < n[2]; ++iz) {
        double best = 1e300;
        for (int a = -4; a <= 4; ++a)
          for (int b = -4; b <= 4; ++b)
            for (int c = -4; c <= 4; ++c) {
              const double dx = ix * h[0] - (R[0] + a * cell[0]);
              const double dy = iy * h[1] - (R[1] + b * cell[1]);
              const double dz = iz * h[2] - (R[2] + c * cell[2]);
              best = std::min(best, std::sqrt(dx * dx + dy * dy + dz * dz));
            }
        if (best < rs) pts.insert((long(ix) * n[1] + iy) * n[2] + iz);
      }
  return pts;
}

void check_case(const char* name, const int n[3], const double cell[3], const std::vector<double>& pos,
                const std::vector<nct_channel>& ch, double rs, bool brute) {
  const int natoms = int(pos.size() / 3);
  nct::tables::ProjectorTables t;
  const std::string why = nct::tables::build_projector_tables(n, cell, natoms, pos.data(), int(ch.size()),
                                                              ch.data(), rs, t);
  CHECK(why.empty(), "%s: builder refused: %s", name, why.c_str());
  const int NX = n[0], NYZ = n[1] * n[2];
  int P = 0;
  for (const auto& c : ch) P += c.twoj + 1;
  CHECK(t.P == P && t.PP % 16 == 0 && t.PP >= P && t.PP - P < 16, "%s: P %d PP %d", name, t.P, t.PP);
  CHECK(int(t.row_off.size()) == natoms + 1 && t.row_off[0] == 0 && t.row_off[natoms] == t.Jtot,
        "%s: row_off ends", name);
  CHECK(int(t.pidx.size()) == t.Jtot && int(t.ix_of_row.size()) == t.Jtot, "%s: row arrays", name);
  CHECK(t.beta.size() == size_t(t.Jtot) * 2 * t.PP, "%s: beta size", name);
  CHECK(t.disp.size() == size_t(t.Jtot) * 3, "%s: disp size", name);
  CHECK(t.energy.size() == size_t(natoms) * t.PP, "%s: energy size", name);
  int maxk = 1, maxrt = 1;
  for (int a = 0; a < natoms; ++a) {
    const int b = t.row_off[a], e = t.row_off[a + 1];
    CHECK(b <= e, "%s: atom %d rows decrease", name, a);
    maxk = std::max(maxk, (2 * (e - b) + 63) / 64);
    maxrt = std::max(maxrt, (2 * (e - b) + 15) / 16);
    long prev = -1;
    std::set<long> got;
    for (int J = b; J < e; ++J) {
      CHECK(t.pidx[J] >= 0 && t.pidx[J] < NYZ, "%s: pidx out of range at row %d", name, J);
      CHECK(t.ix_of_row[J] >= 0 && t.ix_of_row[J] < NX, "%s: plane out of range at row %d", name, J);
      const long flat = long(t.ix_of_row[J]) * NYZ + t.pidx[J];
      CHECK(flat > prev, "%s: atom %d rows not in increasing flat index", name, a);
      prev = flat;
      got.insert(flat);
      const double* d = &t.disp[size_t(J) * 3];
      CHECK(std::sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]) < rs, "%s: row %d outside the sphere", name, J);
      for (int k = 0; k < 2 * t.PP; ++k)
        CHECK(std::isfinite(t.beta[size_t(J) * 2 * t.PP + k].real()) &&
                  std::isfinite(t.beta[size_t(J) * 2 * t.PP + k].imag()), "%s: non-finite beta", name);
      for (int s = 0; s < 2; ++s)
        for (int p = P; p < t.PP; ++p)
          CHECK(t.beta[size_t(J) * 2 * t.PP + s * t.PP + p] == std::complex<double>(0.0, 0.0),
                "%s: padding column %d not zero", name, p);
    }
    if (brute) {
      const std::set<long> ref = sphere_points(n, cell, &pos[3 * size_t(a)], rs);
      CHECK(got == ref, "%s: atom %d has %zu rows, brute force %zu points", name, a, got.size(), ref.size());
    }
    for (int p = 0; p < t.PP; ++p) CHECK(std::isfinite(t.energy[size_t(a) * t.PP + p]), "%s: energy", name);
    for (int p = P; p < t.PP; ++p) CHECK(t.energy[size_t(a) * t.PP + p] == 0.0, "%s: energy padding", name);
  }
  CHECK(t.max_kchunks == maxk && t.max_rowtiles == maxrt, "%s: chunk counts %d/%d vs %d/%d", name,
        t.max_kchunks, t.max_rowtiles, maxk, maxrt);
  // plane ranges
  CHECK(int(t.pr_off.size()) == NX + 1 && t.pr_off[0] == 0, "%s: pr_off size", name);
  CHECK(t.pr_begin.size() == t.pr_end.size() && int(t.pr_begin.size()) == t.pr_off[NX], "%s: range count", name);
  std::vector<int> seen(t.Jtot, 0);
  for (int x = 0; x < NX; ++x) {
    CHECK(t.pr_off[x] <= t.pr_off[x + 1], "%s: pr_off decreases at %d", name, x);
    for (int r = t.pr_off[x]; r < t.pr_off[x + 1]; ++r) {
      const int b = t.pr_begin[r], e = t.pr_end[r];
      CHECK(0 <= b && b < e && e <= t.Jtot, "%s: range %d [%d, %d) of plane %d", name, r, b, e, x);
      int owner = -1;
      for (int a = 0; a < natoms; ++a)
        if (t.row_off[a] <= b && b < t.row_off[a + 1]) owner = a;
      CHECK(owner >= 0 && e <= t.row_off[owner + 1], "%s: range %d crosses atoms", name, r);
      for (int J = b; J < e; ++J) {
        CHECK(t.ix_of_row[J] == x, "%s: row %d of range %d is on plane %d, not %d", name, J, r, t.ix_of_row[J], x);
        ++seen[J];
      }
    }
  }
  for (int J = 0; J < t.Jtot; ++J) CHECK(seen[J] == 1, "%s: row %d covered %d times", name, J, seen[J]);
}

void run_case(const char* name, int nx, int ny, int nz, double Lx, double Ly, double Lz, int natoms,
              unsigned seed, double rs = 2.5, bool brute = true, const std::vector<double>* fixed = nullptr) {
  const int n[3] = {nx, ny, nz};
  const double cell[3] = {Lx, Ly, Lz};
  std::vector<double> pos;
  if (fixed) {
    pos = *fixed;
  } else {
    std::mt19937_64 g(seed);
    std::uniform_real_distribution<double> u(0.0, 1.0);
    for (int a = 0; a < natoms; ++a) {
      pos.push_back(u(g) * Lx);
      pos.push_back(u(g) * Ly);
      pos.push_back(u(g) * Lz);
    }
  }
  check_case(name, n, cell, pos, kb18(), rs, brute);
}

}  // namespace

int main() {
  int cases = 0;
  // the projector shapes of the tests and workloads (grid, cell, atoms)
  run_case("8^3", 8, 8, 8, 6.0, 6.0, 6.0, 1, 1), ++cases;
  run_case("12x16x12", 12, 16, 12, 6.5, 8.0, 6.5, 1, 2), ++cases;
  run_case("12x16x12 x3", 12, 16, 12, 6.0, 8.0, 6.0, 3, 3), ++cases;
  run_case("16^3 x2", 16, 16, 16, 8.0, 8.0, 8.0, 2, 4), ++cases;
  run_case("16x12x16 x2", 16, 12, 16, 8.0, 6.0, 8.0, 2, 5), ++cases;
  run_case("16^3 reduced", 16, 16, 16, 6.72, 6.72, 6.72, 2, 6), ++cases;
  run_case("24^3 x3", 24, 24, 24, 12.0, 12.0, 12.0, 3, 7), ++cases;
  run_case("32^3 x2", 32, 32, 32, 13.44, 13.44, 13.44, 2, 8), ++cases;
  run_case("48^3 x4", 48, 48, 48, 20.0, 20.0, 20.0, 4, 9), ++cases;
  run_case("64^3 x16", 64, 64, 64, 26.88, 26.88, 26.88, 16, 10, 2.5, false), ++cases;
  run_case("96^3 x32", 96, 96, 96, 40.32, 40.32, 40.32, 32, 11, 2.5, false), ++cases;
  // edge cases: an atom on a grid point (dist = 0), on the cell corner (its sphere wraps in every
  // direction), outside [0, L) (negative and beyond L), two atoms on the same point, a sphere
  // smaller than the grid spacing around an off-grid point (no rows at all), and a sphere just
  // below half the cell
  const std::vector<double> corner = {0.0, 0.0, 0.0, 3.0, 3.0, 3.0};
  run_case("grid point and corner", 16, 16, 16, 8.0, 8.0, 8.0, 2, 0, 2.5, true, &corner), ++cases;
  const std::vector<double> outside = {-1.3, 9.7, 4.2, 17.9, -8.1, 0.01};
  run_case("outside the cell", 16, 16, 16, 8.0, 8.0, 8.0, 2, 0, 2.5, true, &outside), ++cases;
  const std::vector<double> same = {2.0, 2.0, 2.0, 2.0, 2.0, 2.0};
  run_case("coincident atoms", 12, 12, 12, 6.0, 6.0, 6.0, 2, 0, 2.0, true, &same), ++cases;
  const std::vector<double> empty = {0.25, 0.25, 0.25, 3.0, 3.0, 3.0};
  run_case("empty sphere", 8, 8, 8, 8.0, 8.0, 8.0, 2, 0, 0.3, true, &empty), ++cases;
  run_case("large sphere", 8, 12, 16, 6.0, 7.0, 9.0, 2, 12, 2.99, true), ++cases;
  // the builder refuses what the kernels cannot take
  {
    const int n[3] = {8, 8, 8};
    const double cell[3] = {6.0, 6.0, 6.0};
    const double p[3] = {1.0, 1.0, 1.0};
    const auto ch = kb18();
    nct::tables::ProjectorTables t;
    if (nct::tables::build_projector_tables(n, cell, 1, p, int(ch.size()), ch.data(), 3.0, t).empty()) {
      std::printf("FAIL: r_sphere = cell/2 accepted\n");
      ++g_fail;
    }
    std::vector<nct_channel> big(6, nct_channel{2, 5, 0.1, 0.7});  // 36 projectors
    if (nct::tables::build_projector_tables(n, cell, 1, p, int(big.size()), big.data(), 2.0, t).empty()) {
      std::printf("FAIL: 36 projectors accepted\n");
      ++g_fail;
    }
    ++cases;
  }
  if (g_fail) return 1;
  std::printf("ok %d\n", cases);
  return 0;
}
