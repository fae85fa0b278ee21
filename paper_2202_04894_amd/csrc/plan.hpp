// Internal plan structures of libdefmm: the host-side build of the tree,
// traversal lists, marks and operator tables, and the device mirror the
// matvec kernels read.  Not part of the C ABI.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

namespace defmm {

constexpr int kKeyBits = 21;   // Morton key bits per dimension
constexpr int kMaxLevel = 21;  // cells at this level are always leaves
constexpr int kP2PBlock = 64;  // target points per P2P block
constexpr int kP2PChunk = 2048;  // source points per P2P work item (balance)
constexpr int kL2PChunk = 256;   // target points per L2P work item
constexpr int kMaxSegPerItem = 64;  // source segments per P2P work item (one wave-wide scan)
constexpr int kRunTargets = 8;     // targets per M2L group (a run record holds 1 + this many words)
constexpr double kMaxSpectraBytes = 8.0 * (1ull << 30);  // per-offset spectra beyond this are compressed

// Dense M2L: L^3 padded to a multiple of 16 (the MFMA tile edge).
constexpr int dense_pad(int L) { return ((L * L * L + 15) / 16) * 16; }

// Whether a level may run the dense M2L: its noff matrices (dense_pad(L)^2
// complex of cs bytes each) fit 2 GiB and what is left of 8 GiB after the
// matrices of the dense levels below (used), and one product per pair
// (npairs x L^3 complex, the workspace's slots) fits 8 GiB.
inline bool dense_level_fits(int L, size_t cs, int64_t noff, int64_t npairs, size_t used) {
  const size_t mat = (size_t)noff * dense_pad(L) * dense_pad(L) * cs;
  const size_t slots = (size_t)npairs * (size_t)(L * L * L) * cs;
  return noff > 0 && mat <= (2ull << 30) && used + mat <= (8ull << 30) && slots <= (8ull << 30);
}

// Frequency slices of the M2L kernels and the Fourier-domain row:
// frequencies stored as (xi, -xi) pairs, grouped into m2l_slices(L) slices of
// fourier_cap(L) pairs, each slice closed under the 48 symmetries of the
// spectra.  A wave's lane owns one pair of a slice, so 64-pair slices keep
// every lane of a load busy; the counts are the fewest slices into which
// make_fourier_layout's packing of the symmetry orbits fits (95 % full at
// L >= 5).
constexpr int m2l_slices(int L) {
  return L <= 3 ? 1 : L == 4 ? 3 : L == 5 ? 6 : L == 6 ? 11 : L == 7 ? 18 : 28;
}
constexpr int fourier_cap(int L) { return L == 2 ? 14 : 64; }
constexpr int fourier_row(int L) { return 2 * m2l_slices(L) * fourier_cap(L); }

struct BuildParams {
  int L = 5;
  int ncrit = 64;
  double eta = 1.0;
  double hf_threshold = 2.0;
  int dir_refine = 0;
  bool same_points = false;
  double kappa = 0.0;
  bool dense_tables = true;  // build the dense M2L index tables (the M2L mode may use them)
  int csize = 8;             // bytes of one complex value of the matvec (8: complex64, 16: complex128)
  bool compress_spectra = false;  // one spectrum per symmetry class (also forced past kMaxSpectraBytes)
  bool screened = false;  // G = exp(-kappa r)/(4 pi r): no oscillation, every level low-frequency
};

// One 2^d-tree over a point set, level-major, Morton order inside a level.
struct Tree {
  int64_t n = 0;
  std::vector<int32_t> perm;   // sorted position -> caller index
  std::vector<double> soa;     // sorted coordinates, x[n] y[n] z[n]
  std::vector<uint64_t> key;   // sorted Morton keys
  int nlevels = 0;
  std::vector<int64_t> lev_start;  // nlevels + 1
  std::vector<int32_t> level, first, count, leaf, child0, nchild, parent;
  std::vector<int32_t> ijk;        // 3 per cell
  // marks = effective expansions (cell, direction), sorted per cell; -1 = none
  std::vector<int64_t> exp_begin;  // ncells + 1
  std::vector<int32_t> exp_dir, exp_cell;
  std::vector<double> exp_u;       // 3 per expansion, zero vector for -1
  int64_t ncells() const { return (int64_t)level.size(); }
  int64_t nexp() const { return (int64_t)exp_dir.size(); }
  int64_t find_exp(int32_t c, int32_t u) const;
};

struct Offset {  // one distinct (level, delta) M2L offset
  int32_t level, d[3], dir;
};

// Storage order of the Fourier-domain rows and the permutation tables that
// read a canonical spectrum for any offset of its symmetry class.
struct FourierLayout {
  int L = 0, slices = 0, cap = 0, row = 0;  // row = 2 * slices * cap entries
  std::vector<int32_t> freq;  // [row]: frequency kx + P ky + P^2 kz stored there, -1 = padding (zero)
  std::vector<uint8_t> perm;  // [slices][48][64]: lane k of a slice, symmetry code r: pair (perm & 127), swapped if perm & 128
};
FourierLayout make_fourier_layout(int L, int slices, int cap);
// Canonical offset d0 (sorted absolute components) and the symmetry code r
// with d = R_r d0, (R_r v)_i = s_i v_{pi(i)}; r = 8 * (index of pi) + sign bits.
int canonical_offset(const int32_t d[3], int32_t d0[3]);

// Everything the matvec needs, built on the host.
struct HostPlan {
  BuildParams prm;
  double D = 0.0, origin[3] = {0, 0, 0}, tau = 0.0;
  Tree tx, ty_own;
  Tree* ty = nullptr;
  int lstar = -1;
  int hf[kMaxLevel + 2] = {0};
  double thr[kMaxLevel + 2] = {0};
  // direction sets per direction level, flattened
  std::vector<double> dirs;
  std::vector<int64_t> dir_off;  // per direction level E: offset (in directions), -1 if absent
  std::vector<int64_t> father_flat;  // per direction (flattened): father index at E-1
  // traversal output
  struct M2L { int32_t t, s, off; };
  std::vector<M2L> m2l;
  std::vector<Offset> offsets;
  // spectra: compressed, one per canonical (level, sorted |delta|) and per
  // offset id the code (canonical id << 6) | symmetry code; otherwise one per
  // offset id and the code (offset id << 6)
  bool compressed = false;
  std::vector<Offset> canon;
  std::vector<int32_t> off_spec;
  std::vector<int32_t> p2p_t, p2p_s;
  int64_t p2p_point_pairs = 0;

  // ---- operator tables (device mirror in DevicePlan) ----
  // P2M: source-leaf expansions
  std::vector<int32_t> p2m_exp;
  // M2M per level l (parents at l): parent expansions and 8 (child exp, octant) slots
  std::vector<std::vector<int32_t>> m2m_par, m2m_child;  // child: 8 per parent, -1 empty
  std::vector<std::vector<int8_t>> m2m_oct;
  // M2F: source expansions used by M2L, mapped to rows of the Fourier table
  std::vector<int32_t> m2f_exp;
  // M2L: target expansions with interactions, CSR of (Fourier row, offset id)
  std::vector<int32_t> m2l_tgt, m2l_begin;  // begin: ntgt + 1
  std::vector<int32_t> m2l_level_tgt;       // per level l: first target of level l (nlevels + 1)
  // M2L source runs: targets grouped by <= kRunTargets (same level and
  // direction, consecutive); per group the pairs are merged by source into runs
  // of 1 + kRunTargets int32: Fourier row of the source, then the spectrum code
  // for each of the group's targets (-1 where that target has no pair with
  // this source).
  std::vector<int32_t> grp_tfirst, grp_tcount, grp_run_begin;  // run CSR: ngrp + 1
  std::vector<int32_t> runs;
  std::vector<int32_t> lvl_grp, lvl_m2f;  // per level: group range, Fourier-row range (nlevels + 1)
  // Dense M2L per level: the level's distinct offsets (global ids), its pairs
  // in offset-major order (source expansion, position in the target CSR
  // relative to the level's first pair) and tiles of <= 16 pairs sharing an
  // offset (level-local offset index, first pair, count).
  std::vector<int32_t> dns_off_begin, dns_off;
  std::vector<int32_t> dns_pair_begin, dns_src, dns_slot;
  std::vector<int32_t> dns_tile_begin, dns_tile_off, dns_tile_first, dns_tile_cnt;
  std::vector<int32_t> m2l_src, m2l_off;
  // L2L per level l (children at l+1): child expansions, CSR of (parent exp, octant)
  std::vector<std::vector<int32_t>> l2l_ch, l2l_begin, l2l_par;
  std::vector<std::vector<int8_t>> l2l_oct;
  // L2P work items: (leaf, first point, count <= kL2PChunk)
  std::vector<int32_t> l2p_cell, l2p_first, l2p_count;
  // P2P: target blocks, work items with source segments
  std::vector<int32_t> blk_first, blk_count, blk_wi_begin;  // blocks; wi CSR (nblk + 1)
  std::vector<int32_t> wi_blk, wi_seg_begin;                 // work items; seg CSR (nwi + 1)
  std::vector<int32_t> seg_first, seg_count;
};

// Builds the whole host plan; throws std::runtime_error / std::bad_alloc.
void build_host_plan(HostPlan& hp, const double* X, int64_t nx, const double* Y, int64_t ny,
                     const BuildParams& prm);

// Stages shared by the host builder and the device builder.
// Bounding cube from the coordinate extremes (any = at least one point).
void set_geometry(HostPlan& hp, const double* lo, const double* hi, bool any);
// Per level: high-frequency flag, squared MAC threshold, deepest HF level.
void set_regimes(HostPlan& hp);
// Direction sets up to the finest level any M2L offset needs (offsets set).
void make_direction_tables(HostPlan& hp);
// Unit direction of each expansion (exp_dir, exp_cell and directions set).
void set_expansion_directions(HostPlan& hp, Tree& T);
// Direction level (refinement E) of tree level l.
int dir_level(const HostPlan& hp, int l);
// Operator tables from the trees, lists, offsets and marks.
void build_tables(HostPlan& hp);

int64_t num_directions(int E);
void make_directions(int E, double* dirs, int64_t* father);

}  // namespace defmm
