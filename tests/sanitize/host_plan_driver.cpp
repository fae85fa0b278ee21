// Exercises the library's host plan builder (tree, traversal, marks, operator
// tables, Fourier layout) on clouds of several shapes and sizes, including the
// degenerate ones, so that a build with AddressSanitizer and
// UndefinedBehaviorSanitizer sees every table the device path uploads.
// Test infrastructure: built and run only by tests/test_host_sanitizers.py.
#include <cmath>
#include <cstdio>
#include <random>
#include <vector>

#include "../../paper_2202_04894_amd/csrc/plan.hpp"

namespace {

std::vector<double> cloud(int kind, int64_t n, unsigned seed) {
  std::mt19937_64 g(seed);
  std::normal_distribution<double> nd;
  std::uniform_real_distribution<double> ud(-1.0, 1.0);
  std::vector<double> x(3 * n);
  for (int64_t i = 0; i < n; ++i) {
    double p[3] = {nd(g), nd(g), nd(g)};
    if (kind == 0) {  // sphere
      const double r = std::sqrt(p[0] * p[0] + p[1] * p[1] + p[2] * p[2]);
      for (double& v : p) v /= r;
    } else if (kind == 1) {  // volume
      for (double& v : p) v = ud(g);
    } else if (kind == 2) {  // cube surface
      for (double& v : p) v = ud(g);
      p[i % 3] = (i % 2) ? 1.0 : -1.0;
    } else {  // every point at one place
      p[0] = 0.25;
      p[1] = -0.5;
      p[2] = 0.125;
    }
    for (int d = 0; d < 3; ++d) x[3 * i + d] = p[d];
  }
  return x;
}

int64_t run(int kind, int64_t n, int64_t ny, const defmm::BuildParams& prm) {
  std::vector<double> X = cloud(kind, n, 11u + (unsigned)n);
  std::vector<double> Y = cloud(kind == 3 ? 3 : 1, ny, 29u + (unsigned)ny);
  defmm::HostPlan hp;
  defmm::build_host_plan(hp, X.data(), n, prm.same_points ? nullptr : Y.data(), prm.same_points ? n : ny, prm);
  return (int64_t)hp.m2l.size() + (int64_t)hp.runs.size() + (int64_t)hp.wi_blk.size();
}

}  // namespace

int main() {
  int64_t sum = 0;
  for (int L : {2, 4, 5, 6, 8}) {
    defmm::FourierLayout F = defmm::make_fourier_layout(L, defmm::m2l_slices(L), defmm::fourier_cap(L));
    sum += F.row;
  }
  struct Case { int kind; int64_t n, ny; int L, ncrit; double eta, hf, kappa; int e0; bool same, screened, compress; };
  const Case cases[] = {
      {0, 3000, 0, 4, 16, 1.0, 2.0, 40.0, 0, true, false, false},
      {0, 20000, 0, 5, 64, 0.35, 0.75, 128.0, 1, true, false, false},
      {1, 4000, 0, 6, 20, 0.7, 2.0, 25.0, 0, true, false, true},
      {2, 6000, 0, 3, 8, 0.5, 1.0, 60.0, 2, true, false, false},
      {0, 3000, 2500, 4, 12, 1.0, 1.0, 30.0, 0, false, false, false},
      {0, 5000, 0, 5, 24, 0.5, 2.0, 40.0, 0, true, true, false},
      {3, 500, 0, 4, 16, 1.0, 2.0, 5.0, 0, true, false, false},
      {0, 1, 0, 5, 64, 1.0, 2.0, 5.0, 0, true, false, false},
      {0, 0, 0, 5, 64, 1.0, 2.0, 5.0, 0, true, false, false},
      {1, 2000, 0, 3, 1, 1.0, 2.0, 0.0, 0, true, false, false},
  };
  for (const Case& c : cases) {
    defmm::BuildParams prm;
    prm.L = c.L;
    prm.ncrit = c.ncrit;
    prm.eta = c.eta;
    prm.hf_threshold = c.hf;
    prm.kappa = c.kappa;
    prm.dir_refine = c.e0;
    prm.same_points = c.same;
    prm.screened = c.screened;
    prm.compress_spectra = c.compress;
    sum += run(c.kind, c.n, c.ny, prm);
  }
  std::printf("host plan driver: ok (%lld)\n", (long long)sum);
  return 0;
}
