// Device mirror of the plan and the per-matvec workspace.  Internal.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <memory>
#include <string>
#include <vector>

#include "plan.hpp"

namespace defmm {


// Pass indices for timing and work accounting.
enum Pass {
  kPassSetup = 0,   // charge gather, zeroing
  kPassP2M = 1,
  kPassM2M = 2,
  kPassM2F = 3,
  kPassM2L = 4,     // Hadamard accumulate (+ F2L when fused)
  kPassL2L = 5,
  kPassP2P = 6,
  kPassP2PRed = 7,
  kPassL2P = 8,
  kPassScatter = 9,
  kPassF2L = 10,    // separate F2L when the M2L runs frequency-sliced
  kPassM2LDense = 11,  // dense MFMA M2L (levels that run it) and its per-target sum
  kNumPasses = 12
};

struct DevTree {
  int64_t n = 0, ncells = 0, nexp = 0;
  int nlevels = 0;
  double* soa = nullptr;      // 3n sorted coordinates (x | y | z)
  int32_t* perm = nullptr;    // sorted -> caller
  int32_t* level = nullptr;
  int32_t* ijk = nullptr;     // 3 per cell
  int32_t* first = nullptr;
  int32_t* count = nullptr;
  int32_t* exp_begin = nullptr;  // ncells + 1
  int32_t* exp_cell = nullptr;
  double* exp_u = nullptr;       // 3 per expansion
};

// Words per M2L source-run record in the device table (one 64-byte scalar load).
constexpr int kRunWords = 16;

// Runs per batch of the source-run M2L kernel: two when a run's loads are
// 16 bytes per lane (complex64 pairs), one for complex128.
template <typename R>
constexpr int m2l_run_batch() { return sizeof(R) == 4 ? 2 : 1; }

struct LevelTable {  // per-level operator table on the device
  int64_t n = 0;     // number of work items
  int32_t* a = nullptr;
  int32_t* b = nullptr;
  int32_t* c = nullptr;
  int8_t* oct = nullptr;
  // the pencil kernels' work: items of one cell taken two at a time when a half
  // wave holds an expansion (L^2 <= 32), else one at a time (-1 = no second)
  int32_t* pair = nullptr;
  int64_t npair = 0;
  // L2L by families (complex64 pencil path): kFamWords words per family, the
  // son expansions of one father cell fed by the same father expansions, and
  // the families taken two at a time (same father cell) as `pair` is
  int32_t* fam = nullptr;
  int32_t* fpair = nullptr;
  int64_t nfpair = 0;
};

// An L2L family record: [0] first of its father expansions in the level's
// parent list, [1] their number, [2 + o] the son expansion at octant o or -1.
constexpr int kFamWords = 16;
// Largest order the family L2L serves (measured faster than the kernel per
// son expansion at L = 5 and 6; four sons' sums in registers at a time: 128
// VGPRs at L = 5, four waves per SIMD, 140 at L = 6, three).
constexpr int kL2LFamilyMaxL = 6;

struct DevPlan {
  HostPlan host;   // kept for introspection and stats
  int L = 5, precision = 1;
  int m2l_variant = 2;  // default for new workspaces (see Workspace::m2l_variant)
  int num_cu = 256;           // compute units of the device (hipDeviceProp)
  int p2p_waves_per_cu = 2;   // default for new workspaces (see Workspace::p2p_waves)
  double kappa = 0.0, D = 0.0, origin[3] = {0, 0, 0}, tau = 0.0;
  bool screened = false;  // kernel exp(-kappa r)/(4 pi r) instead of exp(i kappa r)/(4 pi r)
  DevTree tx, ty;
  bool same = false;
  bool host_only = false;  // built by defmm_plan_inspect_create: no device data
  int64_t nx = 0, ny = 0;
  // tables
  int32_t* p2m_exp = nullptr;
  int64_t n_p2m = 0;
  int32_t* p2m_leaf = nullptr;  // source leaves holding expansions (P2M per leaf)
  uint8_t* has_m2l = nullptr;   // per local expansion: 1 if it is an M2L target
  int32_t* zero_exp = nullptr;  // local expansions written by neither M2L nor L2L
  int64_t n_zero_exp = 0;
  int64_t n_p2m_leaf = 0;
  std::vector<LevelTable> m2m;  // a = parent exps, b = 8 child exps per parent, oct = 8 per parent
  int32_t* m2f_exp = nullptr;
  int64_t n_m2f = 0;
  int32_t *m2l_tgt = nullptr, *m2l_begin = nullptr;
  int32_t* m2l_pair = nullptr;  // per entry: (Fourier-domain multipole row, spectrum id)
  int64_t n_m2l_tgt = 0, n_m2l = 0;
  std::vector<int64_t> m2l_level_tgt;  // target range per level (host copy)
  // M2L source runs as the kernel reads them: kRunWords words per record
  // (source row, 8 spectrum codes or -1, padding), each group's runs padded to a
  // multiple of m2l_run_batch with target-less records, two batches more at
  // the end; grp_run_begin counts records of this padded table
  int32_t *grp_tfirst = nullptr, *grp_tcount = nullptr, *grp_run_begin = nullptr, *runs = nullptr;
  int64_t n_grp = 0;
  std::vector<int64_t> lvl_grp, lvl_m2f;  // per level: group range, Fourier-row range
  // dense M2L (per level; K tables only where they fit, see dense_ok)
  int32_t *dns_src = nullptr, *dns_slot = nullptr, *dns_tile_off = nullptr, *dns_tile_first = nullptr,
          *dns_tile_cnt = nullptr;
  std::vector<int64_t> dns_off_begin, dns_pair_begin, dns_tile_begin;
  std::vector<void*> dense_K;        // per level: n_off_l x dense_pad^2 complex (transposed), or null
  std::vector<char> dense_ok;        // per level: K built
  int64_t dense_slots_max = 0;       // max pairs of a dense-capable level
  int m2l_mode = 1;                  // defmm_m2l_mode the plan was built with
  std::vector<LevelTable> l2l;  // a = child exps, b = CSR begin (n+1), c = parent exps, oct
  int32_t *l2p_cell = nullptr, *l2p_first = nullptr, *l2p_count = nullptr;
  int64_t n_l2p = 0;
  int32_t *blk_first = nullptr, *blk_count = nullptr, *blk_wi_begin = nullptr;
  int64_t nblk = 0;
  int32_t *wi_blk = nullptr, *wi_seg_begin = nullptr;
  int64_t nwi = 0;
  int32_t *seg_first = nullptr, *seg_count = nullptr;
  void* spectra = nullptr;  // n_spec x fourier_row(L) complex (plan precision), scaled by 1/P^3; compressed
                            // (sym): n_spec canonical spectra x 2 rows (layout order, pair members exchanged)
  int64_t n_spec = 0;
  bool sym = false;
  int32_t* freq = nullptr;  // Fourier layout: frequency at each row position (-1 = padding)
  int32_t live_pairs = 0;   // entry pairs of a row up to the last one holding a frequency
  uint8_t* perm = nullptr;  // Fourier layout: [slices][48][64] pair permutation per symmetry code
  std::vector<void*> allocs;
  size_t resident_bytes = 0;
  ~DevPlan();
};

struct Workspace {
  DevPlan* plan = nullptr;
  void* qs = nullptr;    // sorted charges
  void* ps = nullptr;    // sorted potentials
  void* M = nullptr;     // multipoles, ty.nexp x L^3
  void* Lx = nullptr;    // locals, tx.nexp x L^3
  void* Mt = nullptr;    // Fourier-domain multipoles, n_m2f x P^3
  void* Lt = nullptr;    // Fourier-domain locals, n_m2l_tgt x P^3 (sliced M2L only)
  void* part = nullptr;  // P2P partial sums, nwi x 64
  int* queue = nullptr;  // 8 work-queue heads of the persistent P2P
  size_t bytes = 0;
  hipStream_t side = nullptr;   // near-field stream (default priority), forked per matvec
  int overlap = 2;  // 0: in sequence; 1: near field forked after the gather; 2: forked after M2F
  int p2p_waves = 2;     // persistent near-field workgroups (one wave) per CU when overlapped
  int m2l_variant = 2;   // 0: fused per target, 1: sliced per target, 2: sliced per group of 8 (source runs)
  int fourier_items = 0;  // M2F/F2L expansions per workgroup: 1, 2 or 4 (capped to what fits LDS), 0 = default
  int pencil_updown = 1;  // P2M, M2M and L2L: 1 = per leaf / pencil kernels (default), 0 = a workgroup per expansion
  std::vector<char> dense_level;  // per level: use the dense MFMA M2L
  void* slots = nullptr;          // dense M2L per-pair results, dense_slots_max x L^3
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  bool timing = false;
  std::vector<hipEvent_t> ev_pool;
  size_t ev_used = 0;
  struct Rec { int pass; size_t a, b; };
  std::vector<Rec> pending;
  double pass_ms[kNumPasses] = {0};
  int64_t pass_calls[kNumPasses] = {0};
  // captured matvec (defmm_matvec_graph): valid for the recorded q and p and
  // the execution choices at capture; any change of those recaptures
  hipGraph_t graph = nullptr;
  hipGraphExec_t graph_exec = nullptr;
  const void* graph_q = nullptr;
  void* graph_p = nullptr;
  bool graph_stale = true;
  // recorded after every replay; waited on before the executable is destroyed,
  // so a recapture or the workspace's end never frees a graph still running
  hipEvent_t graph_done = nullptr;
  bool graph_launched = false;
  void drop_graph();
  ~Workspace();
};

// Kernel launchers (kernels.hip).
hipError_t compute_spectra(DevPlan& P, const int32_t* d_lev, const int32_t* d_delta, hipStream_t s);
hipError_t compute_dense_K(DevPlan& P, int level, const int32_t* d_delta, hipStream_t s);
hipError_t run_matvec(DevPlan& P, Workspace& W, const void* q, void* p, hipStream_t s);

}  // namespace defmm
