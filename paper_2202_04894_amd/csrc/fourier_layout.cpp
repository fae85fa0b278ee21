// Storage order of the Fourier-domain rows (spectra, M~, L~) and the
// hyperoctahedral symmetry of the M2L spectra (Sec. 4.3).
//
// The kernel G depends on |z| only, so for every signed permutation R of the
// three axes (48 of them) the circulant column of eq. CirculantKernel obeys
// c_{R delta}[j] = c_delta[R^-1 j], and its DFT D_{R delta}[xi] =
// D_delta[R^-1 xi] (indices taken mod P = 2L-1, on representatives in
// [-(L-1), L-1]).  One spectrum per canonical offset (sorted absolute
// components) therefore serves every offset of its class, read through one
// index permutation.
//
// Layout.  Frequencies are stored in pairs (xi, -xi); R maps a pair onto a
// pair (R is linear), so a lane that owns the pair of xi finds D_delta[R^-1 xi]
// and D_delta[-R^-1 xi] side by side in the canonical row, possibly swapped.
// The pairs are grouped by their orbit under the 48 symmetries and the orbits
// are packed into `slices` slices of `cap` pairs (first fit, largest orbit
// first), so each symmetry permutes pairs inside a slice: the frequency slices
// that the M2L kernels assign to XCDs stay closed under the permutation.
#include <algorithm>
#include <array>
#include <cstdlib>
#include <map>
#include <stdexcept>
#include <string>

#include "plan.hpp"

namespace defmm {

namespace {

// The six permutations of (0, 1, 2); symmetry code = 8 * permutation + signs.
constexpr int kPerm[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};

// w = R^-1 v for the symmetry (R v)_i = s_i v_{pi(i)}: w_{pi(i)} = s_i v_i.
std::array<int, 3> apply_inverse(int code, const std::array<int, 3>& v) {
  const int* pi = kPerm[code >> 3];
  std::array<int, 3> w{};
  for (int i = 0; i < 3; ++i) w[pi[i]] = ((code >> i) & 1) ? -v[i] : v[i];
  return w;
}

bool positive(const std::array<int, 3>& v) {  // first nonzero component > 0 (zero counts as positive)
  for (int i = 0; i < 3; ++i)
    if (v[i] != 0) return v[i] > 0;
  return true;
}

}  // namespace

int canonical_offset(const int32_t d[3], int32_t d0[3]) {
  int a[3] = {std::abs(d[0]), std::abs(d[1]), std::abs(d[2])};
  int order[3] = {0, 1, 2};
  std::stable_sort(order, order + 3, [&](int x, int y) { return a[x] < a[y]; });
  int pi[3];
  for (int k = 0; k < 3; ++k) {
    d0[k] = a[order[k]];
    pi[order[k]] = k;
  }
  int p = 0;
  while (!(kPerm[p][0] == pi[0] && kPerm[p][1] == pi[1] && kPerm[p][2] == pi[2])) ++p;
  int signs = (d[0] < 0 ? 1 : 0) | (d[1] < 0 ? 2 : 0) | (d[2] < 0 ? 4 : 0);
  return 8 * p + signs;
}

FourierLayout make_fourier_layout(int L, int slices, int cap) {
  if (L < 2 || slices < 1 || cap < 1 || cap > 64) throw std::invalid_argument("fourier layout: bad sizes");
  const int P = 2 * L - 1, n = L - 1;
  auto flat = [&](const std::array<int, 3>& v) {
    return ((v[0] + P) % P) + P * (((v[1] + P) % P) + P * ((v[2] + P) % P));
  };
  // pair representatives grouped by orbit (key: sorted absolute values)
  std::map<std::array<int, 3>, std::vector<std::array<int, 3>>> orbits;
  for (int z = -n; z <= n; ++z)
    for (int y = -n; y <= n; ++y)
      for (int x = -n; x <= n; ++x) {
        std::array<int, 3> v{x, y, z};
        if (!positive(v)) continue;
        std::array<int, 3> k{std::abs(x), std::abs(y), std::abs(z)};
        std::sort(k.begin(), k.end());
        orbits[k].push_back(v);
      }
  std::vector<std::vector<std::array<int, 3>>> orb;
  for (auto& kv : orbits) {
    std::sort(kv.second.begin(), kv.second.end(),
              [&](const std::array<int, 3>& a, const std::array<int, 3>& b) { return flat(a) < flat(b); });
    orb.push_back(kv.second);
  }
  std::stable_sort(orb.begin(), orb.end(), [](const auto& a, const auto& b) { return a.size() > b.size(); });
  std::vector<std::vector<int>> bin(slices);
  std::vector<int> fill(slices, 0);
  for (int o = 0; o < (int)orb.size(); ++o) {
    int s = 0;
    while (s < slices && fill[s] + (int)orb[o].size() > cap) ++s;
    if (s == slices) throw std::runtime_error("fourier layout: orbits do not fit the slices");
    bin[s].push_back(o);
    fill[s] += (int)orb[o].size();
  }
  FourierLayout F;
  F.L = L;
  F.slices = slices;
  F.cap = cap;
  F.row = 2 * slices * cap;
  F.freq.assign(F.row, -1);
  F.perm.assign((size_t)slices * 48 * 64, 0);
  std::map<std::array<int, 3>, int> where;  // frequency -> storage position
  for (int s = 0; s < slices; ++s) {
    int k = 0;
    for (int o : bin[s])
      for (const auto& v : orb[o]) {
        const int p = 2 * (s * cap + k);
        F.freq[p] = flat(v);
        where[v] = p;
        const std::array<int, 3> m{-v[0], -v[1], -v[2]};
        if (m != v) {
          F.freq[p + 1] = flat(m);
          where[m] = p + 1;
        }
        ++k;
      }
  }
  for (int s = 0; s < slices; ++s)
    for (int code = 0; code < 48; ++code) {
      uint8_t* row = &F.perm[((size_t)s * 48 + code) * 64];
      for (int k = 0; k < 64; ++k) row[k] = (uint8_t)(k < cap ? k : 0);
      for (int k = 0; k < cap; ++k) {
        const int p = 2 * (s * cap + k);
        if (F.freq[p] < 0) continue;
        const int f = F.freq[p];
        std::array<int, 3> v{f % P, (f / P) % P, f / (P * P)};
        for (int& c : v)
          if (c > n) c -= P;
        const int q = where.at(apply_inverse(code, v));
        const int kq = q / 2 - s * cap;
        if (kq < 0 || kq >= cap) throw std::logic_error("fourier layout: orbit left its slice");
        row[k] = (uint8_t)(kq | ((q & 1) << 7));
      }
    }
  return F;
}

}  // namespace defmm
