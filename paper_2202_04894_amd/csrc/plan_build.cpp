// Host-side plan builder: bounding cube, Morton sort, Ncrit tree (Sec. 4.2.1),
// level-synchronous dual tree traversal (Alg. 1 with the MAC of
// eq. macdirref), best directions and blank passes (Alg. 2, Alg. 3), and the
// flat operator tables the device kernels read.
//
// Floating-point decisions (MAC thresholds, regime tests, direction choice)
// are written with the same operations in the same order as the paper's
// definitions so that the lists are reproducible bit for bit; this file must
// be compiled without floating-point contraction.
#include <algorithm>
#include <array>
#include <climits>
#include <cmath>
#include <cstring>
#include <map>
#include <numeric>
#include <stdexcept>
#include <tuple>
#include <thread>
#include <unordered_map>

#include "plan.hpp"

namespace defmm {

namespace {

template <class F>
void parallel_chunks(int64_t n, int64_t min_chunk, F&& f) {
  unsigned hw = std::thread::hardware_concurrency();
  int64_t nt = std::max<int64_t>(1, std::min<int64_t>(hw ? hw : 4, 32));
  nt = std::min<int64_t>(nt, std::max<int64_t>(1, n / std::max<int64_t>(1, min_chunk)));
  if (nt <= 1) {
    f(0, n, 0);
    return;
  }
  std::vector<std::thread> th;
  for (int64_t t = 0; t < nt; ++t) {
    int64_t b = n * t / nt, e = n * (t + 1) / nt;
    th.emplace_back([&, b, e, t] { f(b, e, (int)t); });
  }
  for (auto& x : th) x.join();
}

uint64_t spread_bits(uint64_t v) {
  // bit b of v -> bit 3b
  v &= 0x1fffffull;
  v = (v | (v << 32)) & 0x1f00000000ffffull;
  v = (v | (v << 16)) & 0x1f0000ff0000ffull;
  v = (v | (v << 8)) & 0x100f00f00f00f00full;
  v = (v | (v << 4)) & 0x10c30c30c30c30c3ull;
  v = (v | (v << 2)) & 0x1249249249249249ull;
  return v;
}

int64_t quantise(double x, double o, double D) {
  if (!(D > 0.0)) return 0;
  double s = std::floor((x - o) / D * (double)(1 << kKeyBits));
  if (s < 0.0) s = 0.0;
  if (s > (double)((1 << kKeyBits) - 1)) s = (double)((1 << kKeyBits) - 1);
  return (int64_t)s;
}

// Stable LSD radix sort of (key, index) by key; indices start in caller order.
void radix_sort(std::vector<uint64_t>& key, std::vector<int32_t>& idx) {
  size_t n = key.size();
  std::vector<uint64_t> k2(n);
  std::vector<int32_t> i2(n);
  for (int pass = 0; pass < 8; ++pass) {
    int sh = 8 * pass;
    size_t cnt[257] = {0};
    for (size_t i = 0; i < n; ++i) cnt[((key[i] >> sh) & 255) + 1]++;
    if (cnt[1] == n) continue;  // all digits zero in this pass
    bool skip = false;
    for (int d = 0; d < 256; ++d)
      if (cnt[d + 1] == n) skip = true;
    if (skip) continue;
    for (int d = 0; d < 256; ++d) cnt[d + 1] += cnt[d];
    for (size_t i = 0; i < n; ++i) {
      size_t pos = cnt[(key[i] >> sh) & 255]++;
      k2[pos] = key[i];
      i2[pos] = idx[i];
    }
    key.swap(k2);
    idx.swap(i2);
  }
}

void build_tree(Tree& T, const double* pts, int64_t n, const double* origin, double D, int ncrit) {
  T.n = n;
  std::vector<uint64_t> key(n);
  std::vector<int32_t> idx(n);
  parallel_chunks(n, 1 << 16, [&](int64_t b, int64_t e, int) {
    for (int64_t i = b; i < e; ++i) {
      uint64_t qx = (uint64_t)quantise(pts[3 * i + 0], origin[0], D);
      uint64_t qy = (uint64_t)quantise(pts[3 * i + 1], origin[1], D);
      uint64_t qz = (uint64_t)quantise(pts[3 * i + 2], origin[2], D);
      key[i] = spread_bits(qx) | (spread_bits(qy) << 1) | (spread_bits(qz) << 2);
      idx[i] = (int32_t)i;
    }
  });
  radix_sort(key, idx);
  T.key = std::move(key);
  T.perm = std::move(idx);
  T.soa.resize(3 * n);
  for (int64_t i = 0; i < n; ++i)
    for (int d = 0; d < 3; ++d) T.soa[d * n + i] = pts[3 * (int64_t)T.perm[i] + d];
  // level 0: the root
  T.level = {0};
  T.first = {0};
  T.count = {(int32_t)n};
  T.parent = {-1};
  T.ijk = {0, 0, 0};
  T.leaf = {0};
  T.child0 = {0};
  T.nchild = {0};
  T.lev_start = {0, 1};
  for (int lev = 0;; ++lev) {
    int64_t b = T.lev_start[lev], e = T.lev_start[lev + 1];
    for (int64_t c = b; c < e; ++c) {
      if (T.count[c] > ncrit && lev < kMaxLevel) {
        T.leaf[c] = 0;
        T.child0[c] = (int32_t)T.level.size();
        int sh = 3 * (kKeyBits - lev - 1);
        int64_t i = T.first[c], end = (int64_t)T.first[c] + T.count[c];
        while (i < end) {
          uint64_t dg = (T.key[i] >> sh) & 7ull;
          int64_t j = i;
          while (j < end && ((T.key[j] >> sh) & 7ull) == dg) ++j;
          T.level.push_back(lev + 1);
          T.first.push_back((int32_t)i);
          T.count.push_back((int32_t)(j - i));
          T.parent.push_back((int32_t)c);
          T.ijk.push_back(2 * T.ijk[3 * c + 0] + (int32_t)(dg & 1));
          T.ijk.push_back(2 * T.ijk[3 * c + 1] + (int32_t)((dg >> 1) & 1));
          T.ijk.push_back(2 * T.ijk[3 * c + 2] + (int32_t)((dg >> 2) & 1));
          T.leaf.push_back(0);
          T.child0.push_back(0);
          T.nchild.push_back(0);
          T.nchild[c]++;
          i = j;
        }
      } else {
        T.leaf[c] = 1;
      }
    }
    T.lev_start.push_back((int64_t)T.level.size());
    if (T.lev_start[lev + 2] == T.lev_start[lev + 1]) {
      T.nlevels = lev + 1;
      T.lev_start.pop_back();
      break;
    }
  }
}

// Flat open-addressing map (level, delta) -> offset id.
struct OffsetMap {
  std::vector<int32_t> slot;
  std::vector<Offset>* offs;
  uint64_t mask = 0;
  explicit OffsetMap(std::vector<Offset>* o) : offs(o) { rehash(1 << 12); }
  static uint64_t hash(int32_t l, const int32_t* d) {
    uint64_t h = 0x9e3779b97f4a7c15ull * (uint64_t)(uint32_t)l;
    for (int k = 0; k < 3; ++k) h = (h ^ (uint64_t)(uint32_t)d[k]) * 0xff51afd7ed558ccdull;
    return h ^ (h >> 31);
  }
  void rehash(size_t cap) {
    slot.assign(cap, -1);
    mask = cap - 1;
    for (size_t i = 0; i < offs->size(); ++i) {
      uint64_t h = hash((*offs)[i].level, (*offs)[i].d) & mask;
      while (slot[h] >= 0) h = (h + 1) & mask;
      slot[h] = (int32_t)i;
    }
  }
  int32_t get(int32_t l, const int32_t* d) {
    if (offs->size() * 2 >= slot.size()) rehash(slot.size() * 2);
    uint64_t h = hash(l, d) & mask;
    while (slot[h] >= 0) {
      const Offset& o = (*offs)[slot[h]];
      if (o.level == l && o.d[0] == d[0] && o.d[1] == d[1] && o.d[2] == d[2]) return slot[h];
      h = (h + 1) & mask;
    }
    Offset o;
    o.level = l;
    o.d[0] = d[0];
    o.d[1] = d[1];
    o.d[2] = d[2];
    o.dir = -1;
    offs->push_back(o);
    slot[h] = (int32_t)(offs->size() - 1);
    return slot[h];
  }
};

}  // namespace

int64_t num_directions(int E) { return 6ll << (2 * E); }

// Direction tree (Sec. 4.1.2, Sec. 2.1), built by splitting patches: every face
// patch of level E-1 splits into its four quarter patches at level E.  Scaled by
// 2^E, a patch centre has the face coordinate +-2^E and odd free coordinates;
// splitting maps a free coordinate k of the father to 2k-1 and 2k+1 (k = 0 at
// E = 0).  The direction is the integer vector n over |n|: every quantity before
// the square root is an exact integer in FP64 up to E = 25.  Index
// face*4^E + i*2^E + j (faces +x,-x,+y,-y,+z,-z; i, j along the two free axes in
// increasing order), father = the patch (i/2, j/2) of the same face at E-1.
void make_directions(int E, double* dirs, int64_t* father) {
  std::vector<int64_t> k(1, 0);
  for (int e = 1; e <= E; ++e) {
    std::vector<int64_t> split(2 * k.size());
    for (size_t i = 0; i < k.size(); ++i) {
      split[2 * i] = 2 * k[i] - 1;
      split[2 * i + 1] = 2 * k[i] + 1;
    }
    k.swap(split);
  }
  const int64_t side = (int64_t)k.size();
  for (int face = 0; face < 6; ++face) {
    const int axis = face / 2;
    const int64_t lead = (face % 2 == 0) ? side : -side;
    const int f0 = axis == 0 ? 1 : 0, f1 = axis == 2 ? 1 : 2;
    for (int64_t i = 0; i < side; ++i)
      for (int64_t j = 0; j < side; ++j) {
        int64_t n[3];
        n[axis] = lead;
        n[f0] = k[i];
        n[f1] = k[j];
        const double len = std::sqrt((double)(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]));
        const int64_t u = (face * side + i) * side + j;
        for (int d = 0; d < 3; ++d) dirs[3 * u + d] = (double)n[d] / len;
        father[u] = E == 0 ? -1 : (face * (side / 2) + i / 2) * (side / 2) + j / 2;
      }
  }
}

int64_t Tree::find_exp(int32_t c, int32_t u) const {
  const int32_t* b = exp_dir.data() + exp_begin[c];
  const int32_t* e = exp_dir.data() + exp_begin[c + 1];
  const int32_t* it = std::lower_bound(b, e, u);
  if (it == e || *it != u) return -1;
  return exp_begin[c] + (it - b);
}

int dir_level(const HostPlan& hp, int l) { return hp.lstar - l + hp.prm.dir_refine; }

namespace {

int32_t best_direction(const HostPlan& hp, int E, const int32_t* d) {
  const double* V = hp.dirs.data() + 3 * hp.dir_off[E];
  int64_t n = num_directions(E);
  double dd[3] = {(double)d[0], (double)d[1], (double)d[2]};
  double best = -1e300;
  for (int64_t u = 0; u < n; ++u) {
    double s = V[3 * u] * dd[0] + V[3 * u + 1] * dd[1] + V[3 * u + 2] * dd[2];
    if (s > best) best = s;
  }
  double tol = 1e-12 * std::sqrt(dd[0] * dd[0] + dd[1] * dd[1] + dd[2] * dd[2]);
  for (int64_t u = 0; u < n; ++u) {
    double s = V[3 * u] * dd[0] + V[3 * u + 1] * dd[1] + V[3 * u + 2] * dd[2];
    if (s >= best - tol) return (int32_t)u;
  }
  return 0;
}

// Dual tree traversal, one level at a time: the frontier holds same-level
// pairs; admissible -> M2L, else a leaf -> P2P, else all pairs of sons.
void traverse(HostPlan& hp) {
  const Tree& X = hp.tx;
  const Tree& Y = *hp.ty;
  std::vector<std::pair<int32_t, int32_t>> front = {{0, 0}};
  OffsetMap omap(&hp.offsets);
  for (int lev = 0; !front.empty(); ++lev) {
    int64_t nf = (int64_t)front.size();
    int64_t nchunk = std::min<int64_t>(64, std::max<int64_t>(1, nf / 4096));
    struct Out {
      std::vector<std::pair<int32_t, int32_t>> m2l, p2p, next;
      std::vector<int32_t> dl;
    };
    std::vector<Out> out(nchunk);
    parallel_chunks(nchunk, 1, [&](int64_t cb, int64_t ce, int) {
      for (int64_t ch = cb; ch < ce; ++ch) {
        Out& o = out[ch];
        int64_t b = nf * ch / nchunk, e = nf * (ch + 1) / nchunk;
        for (int64_t i = b; i < e; ++i) {
          int32_t t = front[i].first, s = front[i].second;
          int32_t d[3];
          int64_t n2 = 0;
          for (int k = 0; k < 3; ++k) {
            d[k] = X.ijk[3 * t + k] - Y.ijk[3 * s + k];
            int64_t a = d[k] < 0 ? -(int64_t)d[k] : (int64_t)d[k];
            int64_t nk = a - 1 > 0 ? a - 1 : 0;
            n2 += nk * nk;
          }
          if ((double)n2 >= hp.thr[lev]) {
            o.m2l.push_back({t, s});
            o.dl.insert(o.dl.end(), d, d + 3);
          } else if (X.leaf[t] || Y.leaf[s]) {
            o.p2p.push_back({t, s});
          } else {
            for (int a = 0; a < X.nchild[t]; ++a)
              for (int c = 0; c < Y.nchild[s]; ++c) o.next.push_back({X.child0[t] + a, Y.child0[s] + c});
          }
        }
      }
    });
    std::vector<std::pair<int32_t, int32_t>> next;
    size_t nn = 0;
    for (auto& o : out) nn += o.next.size();
    next.reserve(nn);
    for (auto& o : out) {
      for (size_t i = 0; i < o.m2l.size(); ++i) {
        HostPlan::M2L m;
        m.t = o.m2l[i].first;
        m.s = o.m2l[i].second;
        m.off = omap.get(lev, &o.dl[3 * i]);
        hp.m2l.push_back(m);
      }
      for (auto& pr : o.p2p) {
        hp.p2p_t.push_back(pr.first);
        hp.p2p_s.push_back(pr.second);
      }
      next.insert(next.end(), o.next.begin(), o.next.end());
      o = Out();
    }
    front.swap(next);
  }
}

// Marks of Alg. 2 on one tree, then the blank downward pass of Alg. 3
// (a low-frequency son of a marked cell carries the non-directional mark).
void mark_tree(HostPlan& hp, Tree& T, const std::vector<uint64_t>& own) {
  int64_t nc = T.ncells();
  std::vector<std::vector<int32_t>> marks(nc);
  for (uint64_t m : own) marks[m >> 32].push_back((int32_t)(m & 0xffffffffu) - 1);
  for (int l = 0; l < T.nlevels; ++l) {
    for (int64_t c = T.lev_start[l]; c < T.lev_start[l + 1]; ++c) {
      auto& mk = marks[c];
      std::sort(mk.begin(), mk.end());
      mk.erase(std::unique(mk.begin(), mk.end()), mk.end());
      if (mk.empty() || T.leaf[c]) continue;
      for (int a = 0; a < T.nchild[c]; ++a) {
        auto& cm = marks[T.child0[c] + a];
        if (hp.hf[l + 1]) {
          const int64_t* fa = hp.father_flat.data() + hp.dir_off[dir_level(hp, l)];
          for (int32_t u : mk) cm.push_back((int32_t)fa[u]);
        } else {
          cm.push_back(-1);
        }
      }
    }
  }
  T.exp_begin.assign(nc + 1, 0);
  for (int64_t c = 0; c < nc; ++c) T.exp_begin[c + 1] = T.exp_begin[c] + (int64_t)marks[c].size();
  int64_t ne = T.exp_begin[nc];
  T.exp_dir.resize(ne);
  T.exp_cell.resize(ne);
  T.exp_u.assign(3 * ne, 0.0);
  for (int64_t c = 0; c < nc; ++c) {
    for (size_t k = 0; k < marks[c].size(); ++k) {
      int64_t e = T.exp_begin[c] + (int64_t)k;
      int32_t u = marks[c][k];
      T.exp_dir[e] = u;
      T.exp_cell[e] = (int32_t)c;
      if (u >= 0) {
        const double* v = hp.dirs.data() + 3 * (hp.dir_off[dir_level(hp, T.level[c])] + u);
        for (int d = 0; d < 3; ++d) T.exp_u[3 * e + d] = v[d];
      }
    }
  }
}

}  // namespace

void build_tables(HostPlan& hp) {
  Tree& X = hp.tx;
  Tree& Y = *hp.ty;
  // canonical spectra: offsets of one level related by a signed permutation
  // share the spectrum of their sorted absolute offset (Sec. 4.3)
  {
    std::map<std::array<int32_t, 4>, int32_t> cid;
    hp.canon.clear();
    hp.off_spec.resize(hp.offsets.size());
    hp.compressed = hp.prm.compress_spectra ||
                    (double)hp.offsets.size() * fourier_row(hp.prm.L) * 16.0 > kMaxSpectraBytes ||
                    hp.offsets.size() >= (size_t(1) << 22);
    for (size_t i = 0; i < hp.offsets.size(); ++i) {
      const Offset& o = hp.offsets[i];
      int32_t d0[3];
      const int code = canonical_offset(o.d, d0);
      const std::array<int32_t, 4> key{o.level, d0[0], d0[1], d0[2]};
      auto it = cid.find(key);
      if (it == cid.end()) {
        it = cid.emplace(key, (int32_t)hp.canon.size()).first;
        hp.canon.push_back(Offset{o.level, {d0[0], d0[1], d0[2]}, -1});
      }
      hp.off_spec[i] = hp.compressed ? (it->second << 6) | code : (int32_t)(i << 6);
    }
    if (hp.canon.size() >= (size_t(1) << 22)) throw std::runtime_error("too many distinct spectra");
  }
  // P2M: every expansion of a source leaf
  for (int64_t e = 0; e < Y.nexp(); ++e)
    if (Y.leaf[Y.exp_cell[e]]) hp.p2m_exp.push_back((int32_t)e);
  // M2M, fathers level by level
  hp.m2m_par.assign(Y.nlevels, {});
  hp.m2m_child.assign(Y.nlevels, {});
  hp.m2m_oct.assign(Y.nlevels, {});
  for (int l = 0; l + 1 < Y.nlevels; ++l) {
    for (int64_t c = Y.lev_start[l]; c < Y.lev_start[l + 1]; ++c) {
      if (Y.leaf[c]) continue;
      for (int64_t e = Y.exp_begin[c]; e < Y.exp_begin[c + 1]; ++e) {
        int32_t v = Y.exp_dir[e];
        int32_t u = -1;
        if (hp.hf[l + 1]) u = (int32_t)hp.father_flat[hp.dir_off[dir_level(hp, l)] + v];
        hp.m2m_par[l].push_back((int32_t)e);
        for (int k = 0; k < 8; ++k) {
          if (k < Y.nchild[c]) {
            int32_t cc = Y.child0[c] + k;
            int64_t ce = Y.find_exp(cc, u);
            if (ce < 0) throw std::runtime_error("internal: missing son expansion");
            int oct = (Y.ijk[3 * cc] - 2 * Y.ijk[3 * c]) | ((Y.ijk[3 * cc + 1] - 2 * Y.ijk[3 * c + 1]) << 1) |
                      ((Y.ijk[3 * cc + 2] - 2 * Y.ijk[3 * c + 2]) << 2);
            hp.m2m_child[l].push_back((int32_t)ce);
            hp.m2m_oct[l].push_back((int8_t)oct);
          } else {
            hp.m2m_child[l].push_back(-1);
            hp.m2m_oct[l].push_back(0);
          }
        }
      }
    }
  }
  // M2L grouped by target expansion
  int64_t nm = (int64_t)hp.m2l.size();
  std::vector<int32_t> te(nm), se(nm);
  parallel_chunks(nm, 1 << 14, [&](int64_t b, int64_t e, int) {
    for (int64_t i = b; i < e; ++i) {
      const auto& m = hp.m2l[i];
      int32_t u = hp.offsets[m.off].dir;
      int64_t a = X.find_exp(m.t, u), c = Y.find_exp(m.s, u);
      if (a < 0 || c < 0) throw std::runtime_error("internal: missing M2L expansion");
      te[i] = (int32_t)a;
      se[i] = (int32_t)c;
    }
  });
  std::vector<int32_t> row(Y.nexp(), -1);
  for (int64_t i = 0; i < nm; ++i) row[se[i]] = 0;
  for (int64_t e = 0; e < Y.nexp(); ++e)
    if (row[e] == 0) {
      row[e] = (int32_t)hp.m2f_exp.size();
      hp.m2f_exp.push_back((int32_t)e);
    }
  // targets ordered by (level, direction, Morton cell): neighbouring work
  // shares sources and spectra; inside a target, sources in Morton order.
  // Counting sort of the pairs by target rank, then each target's pairs by
  // source expansion.
  std::vector<int32_t> rank(X.nexp(), -1), tl;
  for (int64_t i = 0; i < nm; ++i)
    if (rank[te[i]] < 0) {
      rank[te[i]] = 0;
      tl.push_back(te[i]);
    }
  std::sort(tl.begin(), tl.end(), [&](int32_t a, int32_t b) {
    int32_t ca = X.exp_cell[a], cb = X.exp_cell[b];
    return std::make_tuple(X.level[ca], X.exp_dir[a], ca) < std::make_tuple(X.level[cb], X.exp_dir[b], cb);
  });
  for (size_t r = 0; r < tl.size(); ++r) rank[tl[r]] = (int32_t)r;
  std::vector<int64_t> tpos(tl.size() + 1, 0);
  for (int64_t i = 0; i < nm; ++i) tpos[rank[te[i]] + 1]++;
  for (size_t r = 0; r < tl.size(); ++r) tpos[r + 1] += tpos[r];
  std::vector<int64_t> order(nm);
  {
    std::vector<int64_t> fill(tpos.begin(), tpos.end() - 1);
    for (int64_t i = 0; i < nm; ++i) order[fill[rank[te[i]]]++] = i;
  }
  parallel_chunks((int64_t)tl.size(), 256, [&](int64_t b, int64_t e, int) {
    for (int64_t r = b; r < e; ++r)
      std::sort(order.begin() + tpos[r], order.begin() + tpos[r + 1],
                [&](int64_t x, int64_t y) { return se[x] < se[y]; });
  });
  hp.m2l_src.resize(nm);
  hp.m2l_off.resize(nm);
  for (int64_t k = 0; k < nm; ++k) {
    int64_t i = order[k];
    if (k == 0 || te[i] != te[order[k - 1]]) {
      hp.m2l_tgt.push_back(te[i]);
      hp.m2l_begin.push_back((int32_t)k);
    }
    hp.m2l_src[k] = row[se[i]];
    hp.m2l_off[k] = hp.m2l[i].off;
  }
  hp.m2l_begin.push_back((int32_t)nm);
  // groups of <= kRunTargets targets sharing level and direction, merged by source
  {
    int64_t nt = (int64_t)hp.m2l_tgt.size();
    std::vector<int64_t> g0;  // first target of each group
    for (int64_t t0 = 0; t0 < nt;) {
      int32_t c0 = X.exp_cell[hp.m2l_tgt[t0]];
      int lv = X.level[c0], dr = X.exp_dir[hp.m2l_tgt[t0]];
      int64_t t1 = t0 + 1;
      while (t1 < nt && t1 - t0 < kRunTargets && X.level[X.exp_cell[hp.m2l_tgt[t1]]] == lv &&
             X.exp_dir[hp.m2l_tgt[t1]] == dr)
        ++t1;
      g0.push_back(t0);
      t0 = t1;
    }
    const int64_t ng = (int64_t)g0.size();
    g0.push_back(nt);
    // groups in chunks on the host threads, runs concatenated in group order
    const int64_t nch = std::max<int64_t>(1, std::min<int64_t>(64, ng / 512));
    std::vector<std::vector<int32_t>> chunk_runs(nch), chunk_nrun(nch);
    parallel_chunks(nch, 1, [&](int64_t cb, int64_t ce, int) {
      std::vector<std::pair<int32_t, int64_t>> ent;  // (source row, tloc * 2^32 + spectrum code)
      for (int64_t ch = cb; ch < ce; ++ch) {
        for (int64_t g = ng * ch / nch; g < ng * (ch + 1) / nch; ++g) {
          ent.clear();
          for (int64_t t = g0[g]; t < g0[g + 1]; ++t)
            for (int32_t k = hp.m2l_begin[t]; k < hp.m2l_begin[t + 1]; ++k)
              ent.push_back({hp.m2l_src[k], ((t - g0[g]) << 32) | (int64_t)(uint32_t)hp.off_spec[hp.m2l_off[k]]});
          std::sort(ent.begin(), ent.end());
          int32_t nr = 0;
          for (size_t a = 0; a < ent.size();) {
            size_t b = a;
            int32_t rec[1 + kRunTargets];
            rec[0] = ent[a].first;
            for (int q = 1; q < 1 + kRunTargets; ++q) rec[q] = -1;
            while (b < ent.size() && ent[b].first == ent[a].first) {
              rec[1 + (ent[b].second >> 32)] = (int32_t)(ent[b].second & 0xffffffffll);
              ++b;
            }
            chunk_runs[ch].insert(chunk_runs[ch].end(), rec, rec + 1 + kRunTargets);
            ++nr;
            a = b;
          }
          chunk_nrun[ch].push_back(nr);
        }
      }
    });
    hp.grp_tfirst.resize(ng);
    hp.grp_tcount.resize(ng);
    hp.grp_run_begin.resize(ng + 1);
    int64_t g = 0, run = 0;
    for (int64_t ch = 0; ch < nch; ++ch) {
      for (int32_t nr : chunk_nrun[ch]) {
        hp.grp_tfirst[g] = (int32_t)g0[g];
        hp.grp_tcount[g] = (int32_t)(g0[g + 1] - g0[g]);
        hp.grp_run_begin[g] = (int32_t)run;
        run += nr;
        ++g;
      }
      hp.runs.insert(hp.runs.end(), chunk_runs[ch].begin(), chunk_runs[ch].end());
      std::vector<int32_t>().swap(chunk_runs[ch]);
    }
    hp.grp_run_begin[ng] = (int32_t)run;
  }
  hp.m2l_level_tgt.assign(X.nlevels + 1, 0);
  for (int32_t e : hp.m2l_tgt) hp.m2l_level_tgt[X.level[X.exp_cell[e]] + 1]++;
  for (int l = 0; l < X.nlevels; ++l) hp.m2l_level_tgt[l + 1] += hp.m2l_level_tgt[l];
  // per-level ranges of groups and of Fourier rows (both are level-major)
  {
    int nl = std::max(X.nlevels, Y.nlevels);
    hp.lvl_grp.assign(nl + 1, 0);
    for (int32_t t0 : hp.grp_tfirst) hp.lvl_grp[X.level[X.exp_cell[hp.m2l_tgt[t0]]] + 1]++;
    hp.lvl_m2f.assign(nl + 1, 0);
    for (int32_t e : hp.m2f_exp) hp.lvl_m2f[Y.level[Y.exp_cell[e]] + 1]++;
    for (int l = 0; l < nl; ++l) {
      hp.lvl_grp[l + 1] += hp.lvl_grp[l];
      hp.lvl_m2f[l + 1] += hp.lvl_m2f[l];
    }
    if ((int)hp.m2l_level_tgt.size() < nl + 1) hp.m2l_level_tgt.resize(nl + 1, hp.m2l_level_tgt.back());
    // dense M2L tables, offset-major per level (only when the M2L mode may use
    // them, and only for the levels whose matrices and products fit)
    hp.dns_off_begin.assign(1, 0);
    hp.dns_pair_begin.assign(1, 0);
    hp.dns_tile_begin.assign(1, 0);
    std::vector<int32_t> local(hp.prm.dense_tables ? hp.offsets.size() : 0, -1);
    size_t dense_used = 0;
    for (int l = 0; l < nl; ++l) {
      int32_t tb = hp.m2l_level_tgt[l], te = hp.m2l_level_tgt[l + 1];
      int32_t kb = hp.m2l_begin[tb], ke = hp.m2l_begin[te];
      std::vector<int32_t> offs;
      if (hp.prm.dense_tables) {
        int64_t noff = 0;
        for (int32_t k = kb; k < ke; ++k)
          if (local[hp.m2l_off[k]] != -2 - l) {
            local[hp.m2l_off[k]] = -2 - l;
            ++noff;
          }
        if (dense_level_fits(hp.prm.L, (size_t)hp.prm.csize, noff, ke - kb, dense_used)) {
          for (int32_t k = kb; k < ke; ++k) offs.push_back(hp.m2l_off[k]);
          std::sort(offs.begin(), offs.end());
          offs.erase(std::unique(offs.begin(), offs.end()), offs.end());
          dense_used += (size_t)noff * dense_pad(hp.prm.L) * dense_pad(hp.prm.L) * (size_t)hp.prm.csize;
        }
      }
      if (offs.empty()) {
        hp.dns_off_begin.push_back((int32_t)hp.dns_off.size());
        hp.dns_pair_begin.push_back((int32_t)hp.dns_src.size());
        hp.dns_tile_begin.push_back((int32_t)hp.dns_tile_off.size());
        continue;
      }
      for (size_t i = 0; i < offs.size(); ++i) local[offs[i]] = (int32_t)i;
      std::vector<std::pair<int32_t, int32_t>> pr;  // (local offset, CSR position)
      for (int32_t k = kb; k < ke; ++k) pr.push_back({local[hp.m2l_off[k]], k});
      std::sort(pr.begin(), pr.end());
      int32_t pbase = (int32_t)hp.dns_src.size();
      for (size_t i = 0; i < pr.size(); ++i) {
        hp.dns_src.push_back(hp.m2f_exp[hp.m2l_src[pr[i].second]]);
        hp.dns_slot.push_back(pr[i].second - kb);
      }
      for (size_t i = 0; i < pr.size();) {
        size_t j = i;
        while (j < pr.size() && pr[j].first == pr[i].first && j - i < 16) ++j;
        hp.dns_tile_off.push_back(pr[i].first);
        hp.dns_tile_first.push_back(pbase + (int32_t)i);
        hp.dns_tile_cnt.push_back((int32_t)(j - i));
        i = j;
      }
      hp.dns_off.insert(hp.dns_off.end(), offs.begin(), offs.end());
      hp.dns_off_begin.push_back((int32_t)hp.dns_off.size());
      hp.dns_pair_begin.push_back((int32_t)hp.dns_src.size());
      hp.dns_tile_begin.push_back((int32_t)hp.dns_tile_off.size());
    }
  }
  // L2L, sons level by level
  hp.l2l_ch.assign(X.nlevels, {});
  hp.l2l_begin.assign(X.nlevels, {});
  hp.l2l_par.assign(X.nlevels, {});
  hp.l2l_oct.assign(X.nlevels, {});
  for (int l = 0; l + 1 < X.nlevels; ++l) {
    // the father's expansions keyed by the son direction they feed (Father(v),
    // or -1 for a low-frequency son), in expansion order within a key
    std::vector<std::pair<int32_t, int32_t>> feed;
    int32_t fed = -1;
    for (int64_t c = X.lev_start[l + 1]; c < X.lev_start[l + 2]; ++c) {
      int32_t p = X.parent[c];
      int oct = (X.ijk[3 * c] - 2 * X.ijk[3 * p]) | ((X.ijk[3 * c + 1] - 2 * X.ijk[3 * p + 1]) << 1) |
                ((X.ijk[3 * c + 2] - 2 * X.ijk[3 * p + 2]) << 2);
      if (p != fed) {
        feed.clear();
        for (int64_t pe = X.exp_begin[p]; pe < X.exp_begin[p + 1]; ++pe) {
          int32_t fv = -1;
          if (hp.hf[l + 1]) fv = (int32_t)hp.father_flat[hp.dir_off[dir_level(hp, l)] + X.exp_dir[pe]];
          feed.push_back({fv, (int32_t)pe});
        }
        std::sort(feed.begin(), feed.end());
        fed = p;
      }
      for (int64_t e = X.exp_begin[c]; e < X.exp_begin[c + 1]; ++e) {
        int32_t u = X.exp_dir[e];
        size_t before = hp.l2l_par[l].size();
        auto it = std::lower_bound(feed.begin(), feed.end(), std::make_pair(u, (int32_t)INT32_MIN));
        for (; it != feed.end() && it->first == u; ++it) {
          hp.l2l_par[l].push_back(it->second);
          hp.l2l_oct[l].push_back((int8_t)oct);
        }
        if (hp.l2l_par[l].size() != before) {
          hp.l2l_ch[l].push_back((int32_t)e);
          hp.l2l_begin[l].push_back((int32_t)before);
        }
      }
    }
    hp.l2l_begin[l].push_back((int32_t)hp.l2l_par[l].size());
  }
  // L2P work items: target leaves holding expansions, in chunks of points
  for (int64_t c = 0; c < X.ncells(); ++c) {
    if (!X.leaf[c] || X.exp_begin[c + 1] == X.exp_begin[c]) continue;
    for (int32_t f = 0; f < X.count[c]; f += kL2PChunk) {
      hp.l2p_cell.push_back((int32_t)c);
      hp.l2p_first.push_back(X.first[c] + f);
      hp.l2p_count.push_back(std::min(kL2PChunk, X.count[c] - f));
    }
  }
  // P2P: push pairs with a non-leaf target down to its leaves, then group by
  // target leaf, split into blocks of points and balanced work items.
  int64_t np = (int64_t)hp.p2p_t.size();
  std::vector<std::pair<int32_t, int32_t>> lp;
  lp.reserve(np);
  std::vector<int32_t> stack;
  for (int64_t i = 0; i < np; ++i) {
    int32_t t = hp.p2p_t[i], s = hp.p2p_s[i];
    if (X.leaf[t]) {
      lp.push_back({t, s});
      continue;
    }
    stack.assign(1, t);
    while (!stack.empty()) {
      int32_t c = stack.back();
      stack.pop_back();
      if (X.leaf[c]) {
        lp.push_back({c, s});
      } else {
        for (int a = X.nchild[c] - 1; a >= 0; --a) stack.push_back(X.child0[c] + a);
      }
    }
  }
  std::sort(lp.begin(), lp.end(), [&](const auto& a, const auto& b) {
    if (a.first != b.first) return a.first < b.first;
    return Y.first[a.second] < Y.first[b.second];
  });
  hp.p2p_point_pairs = 0;
  for (size_t i = 0; i < lp.size();) {
    size_t j = i;
    while (j < lp.size() && lp[j].first == lp[i].first) ++j;
    int32_t t = lp[i].first;
    // merge adjacent source ranges
    std::vector<std::pair<int32_t, int32_t>> ranges;
    for (size_t k = i; k < j; ++k) {
      int32_t f = Y.first[lp[k].second], n = Y.count[lp[k].second];
      if (!ranges.empty() && ranges.back().first + ranges.back().second == f)
        ranges.back().second += n;
      else
        ranges.push_back({f, n});
    }
    int64_t total = 0;
    for (auto& r : ranges) total += r.second;
    for (int32_t bf = 0; bf < X.count[t]; bf += kP2PBlock) {
      int32_t bc = std::min(kP2PBlock, X.count[t] - bf);
      hp.blk_first.push_back(X.first[t] + bf);
      hp.blk_count.push_back(bc);
      hp.blk_wi_begin.push_back((int32_t)hp.wi_blk.size());
      hp.p2p_point_pairs += total * bc;
      int32_t blk = (int32_t)hp.blk_first.size() - 1;
      int64_t acc = kP2PChunk;  // forces a new work item first
      int nseg = 0;
      for (auto& r : ranges) {
        for (int32_t off = 0; off < r.second;) {
          if (acc >= kP2PChunk || nseg >= kMaxSegPerItem) {
            hp.wi_blk.push_back(blk);
            hp.wi_seg_begin.push_back((int32_t)hp.seg_first.size());
            acc = 0;
            nseg = 0;
          }
          ++nseg;
          int32_t take = (int32_t)std::min<int64_t>(r.second - off, kP2PChunk - acc);
          hp.seg_first.push_back(r.first + off);
          hp.seg_count.push_back(take);
          acc += take;
          off += take;
        }
      }
    }
    i = j;
  }
  hp.blk_wi_begin.push_back((int32_t)hp.wi_blk.size());
  hp.wi_seg_begin.push_back((int32_t)hp.seg_first.size());
}

void set_geometry(HostPlan& hp, const double* lo, const double* hi, bool any) {
  double D = 0.0;
  if (any) {
    for (int d = 0; d < 3; ++d) D = std::fmax(D, hi[d] - lo[d]);
    for (int d = 0; d < 3; ++d) hp.origin[d] = 0.5 * (lo[d] + hi[d]) - 0.5 * D;
  }
  hp.D = D;
  hp.tau = 1e-12 * D;
}

void set_regimes(HostPlan& hp) {
  hp.lstar = -1;
  for (int l = 0; l <= kMaxLevel; ++l) {
    double w = std::ldexp(hp.D, -(l + 1));
    // the screened kernel does not oscillate: the plain MAC at every level
    const double kw = hp.prm.screened ? 0.0 : hp.prm.kappa * w;
    hp.hf[l] = (kw > hp.prm.hf_threshold) ? 1 : 0;
    if (hp.hf[l]) hp.lstar = l;
    double a = std::fmax(kw, 2.0) / (2.0 * hp.prm.eta);
    hp.thr[l] = a * a;
  }
}

void make_direction_tables(HostPlan& hp) {
  int Emax = -1;
  for (const Offset& o : hp.offsets)
    if (hp.hf[o.level]) Emax = std::max(Emax, dir_level(hp, o.level));
  hp.dir_off.assign(std::max(Emax + 1, 1), -1);
  int64_t tot = 0;
  for (int E = 0; E <= Emax; ++E) {
    hp.dir_off[E] = tot;
    tot += num_directions(E);
  }
  hp.dirs.resize(3 * tot);
  hp.father_flat.resize(tot);
  for (int E = 0; E <= Emax; ++E)
    make_directions(E, hp.dirs.data() + 3 * hp.dir_off[E], hp.father_flat.data() + hp.dir_off[E]);
}

void set_expansion_directions(HostPlan& hp, Tree& T) {
  T.exp_u.assign(3 * T.nexp(), 0.0);
  for (int64_t e = 0; e < T.nexp(); ++e) {
    int32_t u = T.exp_dir[e];
    if (u < 0) continue;
    const double* v = hp.dirs.data() + 3 * (hp.dir_off[dir_level(hp, T.level[T.exp_cell[e]])] + u);
    for (int d = 0; d < 3; ++d) T.exp_u[3 * e + d] = v[d];
  }
}

void build_host_plan(HostPlan& hp, const double* X, int64_t nx, const double* Y, int64_t ny,
                     const BuildParams& prm) {
  hp.prm = prm;
  const double* Yp = prm.same_points ? X : Y;
  if (prm.same_points) ny = nx;
  double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
  for (int64_t i = 0; i < nx; ++i)
    for (int d = 0; d < 3; ++d) {
      lo[d] = std::fmin(lo[d], X[3 * i + d]);
      hi[d] = std::fmax(hi[d], X[3 * i + d]);
    }
  if (!prm.same_points)
    for (int64_t i = 0; i < ny; ++i)
      for (int d = 0; d < 3; ++d) {
        lo[d] = std::fmin(lo[d], Yp[3 * i + d]);
        hi[d] = std::fmax(hi[d], Yp[3 * i + d]);
      }
  set_geometry(hp, lo, hi, nx + (prm.same_points ? 0 : ny) > 0);
  build_tree(hp.tx, X, nx, hp.origin, hp.D, prm.ncrit);
  if (prm.same_points) {
    hp.ty = &hp.tx;
  } else {
    build_tree(hp.ty_own, Yp, ny, hp.origin, hp.D, prm.ncrit);
    hp.ty = &hp.ty_own;
  }
  set_regimes(hp);
  if (nx > 0 && ny > 0) traverse(hp);
  // directions up to the finest level any M2L needs
  make_direction_tables(hp);
  parallel_chunks((int64_t)hp.offsets.size(), 64, [&](int64_t b, int64_t e, int) {
    for (int64_t i = b; i < e; ++i) {
      Offset& o = hp.offsets[i];
      if (hp.hf[o.level]) o.dir = best_direction(hp, dir_level(hp, o.level), o.d);
    }
  });
  // marks
  std::vector<uint64_t> mx, my;
  mx.reserve(hp.m2l.size());
  my.reserve(hp.m2l.size());
  for (const auto& m : hp.m2l) {
    uint64_t u = (uint64_t)(uint32_t)(hp.offsets[m.off].dir + 1);
    mx.push_back(((uint64_t)(uint32_t)m.t << 32) | u);
    my.push_back(((uint64_t)(uint32_t)m.s << 32) | u);
  }
  if (prm.same_points) {
    mx.insert(mx.end(), my.begin(), my.end());
    my.clear();
  }
  std::sort(mx.begin(), mx.end());
  mx.erase(std::unique(mx.begin(), mx.end()), mx.end());
  mark_tree(hp, hp.tx, mx);
  if (!prm.same_points) {
    std::sort(my.begin(), my.end());
    my.erase(std::unique(my.begin(), my.end()), my.end());
    mark_tree(hp, hp.ty_own, my);
  }
  build_tables(hp);
}

}  // namespace defmm
