// C ABI of libdefmm.so (include/defmm.h): argument checks, plan upload,
// workspaces, matvec dispatch, introspection and per-pass timing.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdlib>
#include <algorithm>
#include <cstring>
#include <vector>
#include <mutex>
#include <new>
#include <stdexcept>
#include <string>
#include <tuple>

#include "../../include/defmm.h"
#include "build_device.hpp"
#include "device.hpp"

using namespace defmm;

struct defmm_plan {
  DevPlan impl;
};
struct defmm_workspace {
  Workspace impl;
};

namespace {

thread_local std::string g_err;

defmm_status fail(defmm_status s, const std::string& m) {
  g_err = m;
  return s;
}

struct HipError : std::runtime_error {
  hipError_t code;
  HipError(hipError_t c, const char* what) : std::runtime_error(std::string(what) + ": " + hipGetErrorString(c)), code(c) {}
};

void check(hipError_t e, const char* what) {
  if (e != hipSuccess) throw HipError(e, what);
}

void* dalloc(DevPlan& P, size_t bytes) {
  if (bytes == 0) return nullptr;
  void* p = nullptr;
  check(hipMalloc(&p, bytes), "hipMalloc");
  P.allocs.push_back(p);
  P.resident_bytes += bytes;
  return p;
}

template <class T>
T* upload(DevPlan& P, const std::vector<T>& v) {
  if (v.empty()) return nullptr;
  T* d = (T*)dalloc(P, v.size() * sizeof(T));
  check(hipMemcpy(d, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice), "hipMemcpy");
  return d;
}

template <class T>
std::vector<int32_t> to_i32(const std::vector<T>& v) {
  return std::vector<int32_t>(v.begin(), v.end());
}

void upload_tree(DevPlan& P, DevTree& d, const Tree& t) {
  d.n = t.n;
  d.ncells = t.ncells();
  d.nexp = t.nexp();
  d.nlevels = t.nlevels;
  d.soa = upload(P, t.soa);
  d.perm = upload(P, t.perm);
  d.level = upload(P, t.level);
  d.ijk = upload(P, t.ijk);
  d.first = upload(P, t.first);
  d.count = upload(P, t.count);
  d.exp_begin = upload(P, to_i32(t.exp_begin));
  d.exp_cell = upload(P, t.exp_cell);
  d.exp_u = upload(P, t.exp_u);
}

size_t csize(const DevPlan& P) { return P.precision == 0 ? 16 : 8; }

// Expansions per wave of the pencil M2M/L2L kernels (the device side's
// pencil_epw): two when a half wave holds the L^2 pencils of one expansion.
int pencil_epw_host(int L) { return L * L <= 32 ? 2 : 1; }

// L2L families of son level l + 1: the son items (son expansion, CSR range of
// its father expansions) of one father cell that the same father expansions
// feed (one son direction, or the only expansion of a low-frequency son),
// found by (father cell, first father expansion); at most one son per octant.
// Families in father-cell order, kFamWords words each; fcell the father cell
// of each.  False if a family would hold two sons of one octant (not built).
bool l2l_families(const HostPlan& H, size_t l, std::vector<int32_t>& fam, std::vector<int32_t>& fcell) {
  const auto& ch = H.l2l_ch[l];
  const auto& bg = H.l2l_begin[l];
  const auto& pa = H.l2l_par[l];
  const auto& oc = H.l2l_oct[l];
  const int64_t n = (int64_t)ch.size();
  std::vector<std::tuple<int32_t, int32_t, int32_t>> key(n);  // (father cell, first father exp, item)
  for (int64_t i = 0; i < n; ++i)
    key[i] = {H.tx.parent[H.tx.exp_cell[ch[i]]], pa[bg[i]], (int32_t)i};
  std::sort(key.begin(), key.end());
  for (int64_t a = 0; a < n;) {
    int64_t b = a;
    const int32_t i0 = std::get<2>(key[a]);
    int32_t rec[kFamWords];
    for (int q = 0; q < kFamWords; ++q) rec[q] = q < 2 ? 0 : -1;
    rec[0] = bg[i0];
    rec[1] = bg[i0 + 1] - bg[i0];
    while (b < n && std::get<0>(key[b]) == std::get<0>(key[a]) && std::get<1>(key[b]) == std::get<1>(key[a])) {
      const int32_t i = std::get<2>(key[b]);
      if (bg[i + 1] - bg[i] != rec[1]) return false;
      const int o = oc[bg[i]];
      if (o < 0 || o > 7 || rec[2 + o] >= 0) return false;
      rec[2 + o] = ch[i];
      ++b;
    }
    fam.insert(fam.end(), rec, rec + kFamWords);
    fcell.push_back(std::get<0>(key[a]));
    a = b;
  }
  return true;
}

// Work list of the pencil kernels from the cell of each item (items of a cell
// consecutive): pairs of items of the same cell, (i, -1) for a lone one; with
// one expansion per wave, every item alone.
std::vector<int32_t> pencil_pairs(const std::vector<int32_t>& cell, int L) {
  std::vector<int32_t> out;
  const int64_t n = (int64_t)cell.size();
  if (pencil_epw_host(L) == 1) {
    for (int64_t i = 0; i < n; ++i) out.push_back((int32_t)i);
    return out;
  }
  for (int64_t i = 0; i < n;) {
    out.push_back((int32_t)i);
    if (i + 1 < n && cell[i + 1] == cell[i]) {
      out.push_back((int32_t)(i + 1));
      i += 2;
    } else {
      out.push_back(-1);
      i += 1;
    }
  }
  return out;
}


}  // namespace

namespace defmm {
DevPlan::~DevPlan() {
  for (void* p : allocs) hipFree(p);
}
void Workspace::drop_graph() {
  if (graph_launched && graph_done) (void)hipEventSynchronize(graph_done);
  graph_launched = false;
  if (graph_exec) (void)hipGraphExecDestroy(graph_exec);
  if (graph) (void)hipGraphDestroy(graph);
  graph_exec = nullptr;
  graph = nullptr;
  graph_stale = true;
}
Workspace::~Workspace() {
  drop_graph();
  for (void* p : {qs, ps, M, Lx, Mt, Lt, part, (void*)queue, slots})
    if (p) hipFree(p);
  for (hipEvent_t e : ev_pool) hipEventDestroy(e);
  if (ev_fork) hipEventDestroy(ev_fork);
  if (ev_join) hipEventDestroy(ev_join);
  if (graph_done) hipEventDestroy(graph_done);
  if (side) hipStreamDestroy(side);
}
}  // namespace defmm

extern "C" {

const char* defmm_status_string(defmm_status s) {
  switch (s) {
    case DEFMM_OK: return "ok";
    case DEFMM_ERR_INVALID_ARG: return "invalid argument";
    case DEFMM_ERR_OUT_OF_MEMORY: return "out of memory";
    case DEFMM_ERR_DEVICE: return "device error";
    case DEFMM_ERR_UNSUPPORTED: return "unsupported";
  }
  return "unknown status";
}

const char* defmm_last_error(void) { return g_err.c_str(); }

defmm_status defmm_default_params(defmm_params* out) {
  if (!out) return fail(DEFMM_ERR_INVALID_ARG, "out is NULL");
  out->order_L = 5;
  out->ncrit = 64;
  out->eta = 1.0;
  out->hf_threshold = 2.0;
  out->dir_refine = 0;
  out->precision = DEFMM_C64;
  out->m2l_mode = DEFMM_M2L_FFT;
  out->flags = 0;
  return DEFMM_OK;
}

static defmm_status validate(const double* X, int64_t nx, const double* Y, int64_t ny, double kappa,
                             const defmm_params* prm, defmm_plan** out) {
  if (!out || !prm) return fail(DEFMM_ERR_INVALID_ARG, "out or prm is NULL");
  *out = nullptr;
  bool same = (prm->flags & DEFMM_SAME_POINTS) != 0;
  if (nx < 0 || ny < 0) return fail(DEFMM_ERR_INVALID_ARG, "negative point count");
  if (nx > 0x7fffffffll || ny > 0x7fffffffll) return fail(DEFMM_ERR_UNSUPPORTED, "more than 2^31-1 points");
  if ((nx > 0 && !X) || (!same && ny > 0 && !Y)) return fail(DEFMM_ERR_INVALID_ARG, "point array is NULL");
  if (prm->order_L < 2 || prm->order_L > 8) return fail(DEFMM_ERR_INVALID_ARG, "order_L outside 2..8");
  if (prm->ncrit < 1) return fail(DEFMM_ERR_INVALID_ARG, "ncrit < 1");
  if (!(kappa >= 0.0) || !std::isfinite(kappa)) return fail(DEFMM_ERR_INVALID_ARG, "kappa < 0 or not finite");
  if (!(prm->eta > 0.0) || !std::isfinite(prm->eta)) return fail(DEFMM_ERR_INVALID_ARG, "eta <= 0");
  if (!(prm->hf_threshold >= 0.0)) return fail(DEFMM_ERR_INVALID_ARG, "hf_threshold < 0");
  if (prm->dir_refine < 0 || prm->dir_refine > 4) return fail(DEFMM_ERR_INVALID_ARG, "dir_refine outside 0..4");
  if (prm->precision != DEFMM_C64 && prm->precision != DEFMM_C128)
    return fail(DEFMM_ERR_INVALID_ARG, "unknown precision");
  if (prm->m2l_mode != DEFMM_M2L_AUTO && prm->m2l_mode != DEFMM_M2L_FFT && prm->m2l_mode != DEFMM_M2L_DENSE)
    return fail(DEFMM_ERR_INVALID_ARG, "unknown m2l_mode");
  if (prm->flags & ~(DEFMM_SAME_POINTS | DEFMM_COMPRESS_SPECTRA | DEFMM_YUKAWA))
    return fail(DEFMM_ERR_INVALID_ARG, "unknown flag bits");
  return DEFMM_OK;
}

// Host half of plan creation: copies the points, checks them and builds the
// host plan.  Throws on allocation/device errors; returns a status for bad input.
// Builds the plan's trees, lists, marks and operator tables: on the device
// (HIP kernels, stream s) from device coordinates, or entirely on the host
// from host coordinates (inspection plans).  Throws on allocation/device
// errors; returns a status for bad input.
static defmm_status plan_build(defmm_plan* plan, const double* X, int64_t nx, const double* Y, int64_t ny,
                               double kappa, const defmm_params* prm, bool host_pointers, hipStream_t s) {
  bool same = (prm->flags & DEFMM_SAME_POINTS) != 0;
  DevPlan& P = plan->impl;
  BuildParams bp;
  bp.L = prm->order_L;
  bp.ncrit = prm->ncrit;
  bp.eta = prm->eta;
  bp.hf_threshold = prm->hf_threshold;
  bp.dir_refine = prm->dir_refine;
  bp.same_points = same;
  bp.kappa = kappa;
  bp.dense_tables = prm->m2l_mode != DEFMM_M2L_FFT;
  bp.csize = prm->precision == DEFMM_C128 ? 16 : 8;
  bp.compress_spectra = (prm->flags & DEFMM_COMPRESS_SPECTRA) != 0;
  bp.screened = (prm->flags & DEFMM_YUKAWA) != 0;
  if (host_pointers) {
    for (int64_t i = 0; i < 3 * nx; ++i)
      if (!std::isfinite(X[i])) return fail(DEFMM_ERR_INVALID_ARG, "non-finite coordinate in X");
    if (!same)
      for (int64_t i = 0; i < 3 * ny; ++i)
        if (!std::isfinite(Y[i])) return fail(DEFMM_ERR_INVALID_ARG, "non-finite coordinate in Y");
    build_host_plan(P.host, X, nx, same ? nullptr : Y, ny, bp);
  } else if (!build_device_plan(P.host, X, nx, same ? nullptr : Y, ny, bp, s)) {
    return fail(DEFMM_ERR_INVALID_ARG, "non-finite coordinate in X or Y");
  }
  const HostPlan& H = P.host;
  P.L = bp.L;
  P.precision = prm->precision;
  P.kappa = kappa;
  P.screened = bp.screened;
  P.D = H.D;
  for (int d = 0; d < 3; ++d) P.origin[d] = H.origin[d];
  P.tau = H.tau;
  P.same = same;
  P.nx = nx;
  P.ny = ny;
  return DEFMM_OK;
}

defmm_status defmm_plan_inspect_create(const double* X, int64_t nx, const double* Y, int64_t ny, double kappa,
                                       const defmm_params* prm, defmm_plan** out) {
  defmm_status st = validate(X, nx, Y, ny, kappa, prm, out);
  if (st != DEFMM_OK) return st;
  if (prm->flags & DEFMM_SAME_POINTS) ny = nx;
  defmm_plan* plan = nullptr;
  try {
    plan = new defmm_plan();
    plan->impl.host_only = true;
    st = plan_build(plan, X, nx, Y, ny, kappa, prm, true, nullptr);
    if (st != DEFMM_OK) {
      delete plan;
      return st;
    }
    *out = plan;
    return DEFMM_OK;
  } catch (const std::bad_alloc&) {
    delete plan;
    return fail(DEFMM_ERR_OUT_OF_MEMORY, "host allocation failed");
  } catch (const std::exception& e) {
    delete plan;
    return fail(DEFMM_ERR_DEVICE, e.what());
  }
}

defmm_status defmm_plan_create(const double* X, int64_t nx, const double* Y, int64_t ny, double kappa,
                               const defmm_params* prm, void* hip_stream, defmm_plan** out) {
  defmm_status st = validate(X, nx, Y, ny, kappa, prm, out);
  if (st != DEFMM_OK) return st;
  bool same = (prm->flags & DEFMM_SAME_POINTS) != 0;
  if (same) ny = nx;
  hipStream_t s = (hipStream_t)hip_stream;
  defmm_plan* plan = nullptr;
  try {
    plan = new defmm_plan();
    st = plan_build(plan, X, nx, Y, ny, kappa, prm, false, s);
    if (st != DEFMM_OK) {
      delete plan;
      return st;
    }
    DevPlan& P = plan->impl;
    HostPlan& H = P.host;
    upload_tree(P, P.tx, H.tx);
    if (same) P.ty = P.tx;
    else upload_tree(P, P.ty, H.ty_own);
    P.p2m_exp = upload(P, H.p2m_exp);
    P.n_p2m = (int64_t)H.p2m_exp.size();
    {
      std::vector<int32_t> lv;
      for (int32_t e : H.p2m_exp) {
        const int32_t c = H.ty->exp_cell[e];
        if (lv.empty() || lv.back() != c) lv.push_back(c);
      }
      P.p2m_leaf = upload(P, lv);
      P.n_p2m_leaf = (int64_t)lv.size();
    }
    P.m2m.resize(H.m2m_par.size());
    for (size_t l = 0; l < H.m2m_par.size(); ++l) {
      P.m2m[l].n = (int64_t)H.m2m_par[l].size();
      P.m2m[l].a = upload(P, H.m2m_par[l]);
      P.m2m[l].b = upload(P, H.m2m_child[l]);
      P.m2m[l].oct = upload(P, H.m2m_oct[l]);
      std::vector<int32_t> cell(H.m2m_par[l].size());
      for (size_t i = 0; i < cell.size(); ++i) cell[i] = H.ty->exp_cell[H.m2m_par[l][i]];
      std::vector<int32_t> pr = pencil_pairs(cell, P.L);
      P.m2m[l].npair = (int64_t)pr.size() / pencil_epw_host(P.L);
      P.m2m[l].pair = upload(P, pr);
    }
    P.m2f_exp = upload(P, H.m2f_exp);
    P.n_m2f = (int64_t)H.m2f_exp.size();
    P.m2l_tgt = upload(P, H.m2l_tgt);
    P.m2l_begin = upload(P, H.m2l_begin);
    {
      std::vector<int32_t> pr(2 * H.m2l_src.size());
      for (size_t k = 0; k < H.m2l_src.size(); ++k) {
        pr[2 * k] = H.m2l_src[k];
        pr[2 * k + 1] = H.off_spec[H.m2l_off[k]];
      }
      P.m2l_pair = upload(P, pr);
    }
    P.n_m2l_tgt = (int64_t)H.m2l_tgt.size();
    {
      std::vector<uint8_t> fl((size_t)std::max<int64_t>(H.tx.nexp(), 1), 0);
      for (int32_t e : H.m2l_tgt) fl[e] = 1;
      P.has_m2l = upload(P, fl);
      // local expansions no M2L and no L2L writes (cells marked only as M2L
      // sources, with no father expansion feeding them): cleared every matvec
      std::vector<uint8_t> fed(fl.begin(), fl.end());
      for (const auto& v : H.l2l_ch)
        for (int32_t e : v) fed[e] = 1;
      std::vector<int32_t> z;
      for (int64_t e = 0; e < H.tx.nexp(); ++e)
        if (!fed[e]) z.push_back((int32_t)e);
      P.zero_exp = upload(P, z);
      P.n_zero_exp = (int64_t)z.size();
    }
    P.m2l_level_tgt.assign(H.m2l_level_tgt.begin(), H.m2l_level_tgt.end());
    P.grp_tfirst = upload(P, H.grp_tfirst);
    P.grp_tcount = upload(P, H.grp_tcount);
    {
      // device layout of the runs: kRunWords words per record, each group padded
      // to a multiple of the kernel's batch with target-less records (the
      // group's first source again), two batches of them more at the end (the
      // kernel reads records one batch and source words two batches ahead)
      const int U = P.precision == 0 ? m2l_run_batch<double>() : m2l_run_batch<float>();
      const int64_t ng = (int64_t)H.grp_tfirst.size();
      std::vector<int32_t> rb(ng + 1, 0), rr;
      constexpr int RQ = 1 + kRunTargets;  // words of a host record
      static_assert(RQ <= kRunWords, "run record too long");
      static_assert(kRunTargets == 8, "k_m2l_runs reads 8 target codes per record");
      rr.reserve((H.runs.size() / RQ + ng + 2 * U) * kRunWords);
      auto push = [&](const int32_t* rec) {
        for (int q = 0; q < kRunWords; ++q) rr.push_back(q < RQ ? rec[q] : 0);
      };
      int32_t dummy[RQ];
      for (int64_t gi = 0; gi < ng; ++gi) {
        rb[gi] = (int32_t)(rr.size() / kRunWords);
        const int64_t a = H.grp_run_begin[gi], e = H.grp_run_begin[gi + 1];
        for (int64_t k = a; k < e; ++k) push(&H.runs[RQ * k]);
        dummy[0] = e > a ? H.runs[RQ * a] : 0;
        for (int q = 1; q < RQ; ++q) dummy[q] = -1;
        for (int64_t k = e - a; k % U != 0; ++k) push(dummy);
      }
      rb[ng] = (int32_t)(rr.size() / kRunWords);
      dummy[0] = 0;
      for (int k = 0; k < 2 * U; ++k) push(dummy);
      if ((int64_t)rr.size() / kRunWords > INT32_MAX) throw std::runtime_error("M2L run table too large");
      P.grp_run_begin = upload(P, rb);
      P.runs = upload(P, rr);
    }
    P.n_grp = (int64_t)H.grp_tfirst.size();
    P.lvl_grp.assign(H.lvl_grp.begin(), H.lvl_grp.end());
    P.lvl_m2f.assign(H.lvl_m2f.begin(), H.lvl_m2f.end());
    P.m2l_level_tgt.assign(H.m2l_level_tgt.begin(), H.m2l_level_tgt.end());
    // dense M2L tables: index lists always, K matrices where they fit
    P.dns_src = upload(P, H.dns_src);
    P.dns_slot = upload(P, H.dns_slot);
    P.dns_tile_off = upload(P, H.dns_tile_off);
    P.dns_tile_first = upload(P, H.dns_tile_first);
    P.dns_tile_cnt = upload(P, H.dns_tile_cnt);
    P.dns_off_begin.assign(H.dns_off_begin.begin(), H.dns_off_begin.end());
    P.dns_pair_begin.assign(H.dns_pair_begin.begin(), H.dns_pair_begin.end());
    P.dns_tile_begin.assign(H.dns_tile_begin.begin(), H.dns_tile_begin.end());
    {
      int nl = (int)P.lvl_m2f.size() - 1;
      P.dense_K.assign(nl, nullptr);
      P.dense_ok.assign(nl, 0);
      P.m2l_mode = prm->m2l_mode;
      if (prm->m2l_mode != DEFMM_M2L_FFT) {
        // the builder packed tables only for the levels whose matrices and
        // per-pair products fit (dense_level_fits)
        const size_t per_off = (size_t)dense_pad(P.L) * dense_pad(P.L) * csize(P);
        for (int l = 0; l < nl; ++l) {
          int64_t noff = P.dns_off_begin[l + 1] - P.dns_off_begin[l];
          if (noff == 0) continue;
          const size_t bytes = (size_t)noff * per_off;
          std::vector<int32_t> dl(3 * noff);
          for (int64_t i = 0; i < noff; ++i)
            for (int d = 0; d < 3; ++d) dl[3 * i + d] = H.offsets[H.dns_off[P.dns_off_begin[l] + i]].d[d];
          P.dense_K[l] = dalloc(P, bytes);
          int32_t* ddl = upload(P, dl);
          check(compute_dense_K(P, l, ddl, s), "dense K launch");
          P.dense_ok[l] = 1;
          P.dense_slots_max = std::max<int64_t>(P.dense_slots_max, P.dns_pair_begin[l + 1] - P.dns_pair_begin[l]);
        }
        check(hipStreamSynchronize(s), "dense K");
      }
    }
    {
      int dev = 0;
      hipDeviceProp_t prop;
      if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess &&
          prop.multiProcessorCount > 0)
        P.num_cu = prop.multiProcessorCount;
      P.p2p_waves_per_cu = 2;
    }

    P.n_m2l = (int64_t)H.m2l_src.size();
    P.l2l.resize(H.l2l_ch.size());
    for (size_t l = 0; l < H.l2l_ch.size(); ++l) {
      P.l2l[l].n = (int64_t)H.l2l_ch[l].size();
      if (P.l2l[l].n == 0) continue;
      P.l2l[l].a = upload(P, H.l2l_ch[l]);
      P.l2l[l].b = upload(P, H.l2l_begin[l]);
      P.l2l[l].c = upload(P, H.l2l_par[l]);
      P.l2l[l].oct = upload(P, H.l2l_oct[l]);
      std::vector<int32_t> cell(H.l2l_ch[l].size());
      for (size_t i = 0; i < cell.size(); ++i) cell[i] = H.tx.exp_cell[H.l2l_ch[l][i]];
      std::vector<int32_t> pr = pencil_pairs(cell, P.L);
      P.l2l[l].npair = (int64_t)pr.size() / pencil_epw_host(P.L);
      P.l2l[l].pair = upload(P, pr);
      std::vector<int32_t> fam, fcell;
      if (P.L <= kL2LFamilyMaxL && l2l_families(H, l, fam, fcell)) {
        std::vector<int32_t> fp = pencil_pairs(fcell, P.L);
        P.l2l[l].nfpair = (int64_t)fp.size() / pencil_epw_host(P.L);
        P.l2l[l].fpair = upload(P, fp);
        P.l2l[l].fam = upload(P, fam);
      }
    }
    P.l2p_cell = upload(P, H.l2p_cell);
    P.l2p_first = upload(P, H.l2p_first);
    P.l2p_count = upload(P, H.l2p_count);
    P.n_l2p = (int64_t)H.l2p_cell.size();
    P.blk_first = upload(P, H.blk_first);
    P.blk_count = upload(P, H.blk_count);
    P.blk_wi_begin = upload(P, H.blk_wi_begin);
    P.nblk = (int64_t)H.blk_first.size();
    P.wi_blk = upload(P, H.wi_blk);
    P.wi_seg_begin = upload(P, H.wi_seg_begin);
    P.nwi = (int64_t)H.wi_blk.size();
    P.seg_first = upload(P, H.seg_first);
    P.seg_count = upload(P, H.seg_count);
    // Fourier layout and the spectra, computed on the device in FP64: one per
    // distinct (level, delta), or, compressed, one per canonical (level,
    // sorted |delta|) in two rows (layout order, pair members exchanged)
    {
      FourierLayout F = make_fourier_layout(P.L, m2l_slices(P.L), fourier_cap(P.L));
      if (F.row != fourier_row(P.L)) throw std::logic_error("fourier layout: row length mismatch");
      P.freq = upload(P, F.freq);
      P.live_pairs = 0;
      for (size_t i = 0; i < F.freq.size(); ++i)
        if (F.freq[i] >= 0) P.live_pairs = (int32_t)(i / 2 + 1);
      P.perm = upload(P, F.perm);
    }
    P.sym = H.compressed;
    const std::vector<Offset>& spec = P.sym ? H.canon : H.offsets;
    P.n_spec = (int64_t)spec.size();
    if (P.n_spec > 0) {
      P.spectra = dalloc(P, (size_t)(P.sym ? 2 : 1) * P.n_spec * fourier_row(P.L) * csize(P));
      std::vector<int32_t> lev(P.n_spec), dl(3 * P.n_spec);
      for (int64_t i = 0; i < P.n_spec; ++i) {
        lev[i] = spec[i].level;
        for (int d = 0; d < 3; ++d) dl[3 * i + d] = spec[i].d[d];
      }
      int32_t* dlev = upload(P, lev);
      int32_t* ddl = upload(P, dl);
      check(compute_spectra(P, dlev, ddl, s), "spectra launch");
      check(hipStreamSynchronize(s), "spectra");
    }
    *out = plan;
    return DEFMM_OK;
  } catch (const HipError& e) {
    delete plan;
    if (e.code == hipErrorOutOfMemory) return fail(DEFMM_ERR_OUT_OF_MEMORY, e.what());
    return fail(DEFMM_ERR_DEVICE, e.what());
  } catch (const std::bad_alloc&) {
    delete plan;
    return fail(DEFMM_ERR_OUT_OF_MEMORY, "host allocation failed");
  } catch (const std::exception& e) {
    delete plan;
    return fail(DEFMM_ERR_DEVICE, e.what());
  }
}

// Device bytes of one workspace: exactly the buffers workspace creation
// allocates (charges, potentials, expansions, Fourier rows, near-field
// partials, dense-M2L slots, work counters).
static size_t workspace_bytes(const DevPlan& P) {
  size_t cs = csize(P);
  int L3 = P.L * P.L * P.L, P3 = fourier_row(P.L);
  return cs * ((size_t)P.ny + (size_t)P.nx + (size_t)P.ty.nexp * L3 + (size_t)P.tx.nexp * L3 +
               (size_t)P.n_m2f * P3 + (size_t)P.nwi * 64 + (size_t)P.n_m2l_tgt * P3 +
               (size_t)P.dense_slots_max * L3) +
         8 * sizeof(int);
}

defmm_status defmm_plan_footprint(const defmm_plan* plan, size_t* resident, size_t* ws) {
  if (!plan) return fail(DEFMM_ERR_INVALID_ARG, "plan is NULL");
  if (resident) *resident = plan->impl.resident_bytes;
  if (ws) *ws = workspace_bytes(plan->impl);
  return DEFMM_OK;
}

defmm_status defmm_plan_stats(const defmm_plan* plan, defmm_stats* out) {
  if (!plan || !out) return fail(DEFMM_ERR_INVALID_ARG, "NULL argument");
  const DevPlan& P = plan->impl;
  const HostPlan& H = P.host;
  std::memset(out, 0, sizeof(*out));
  out->levels = H.tx.nlevels;
  int hfl = 0;
  for (int l = 0; l < H.tx.nlevels; ++l) hfl += H.hf[l];
  out->hf_levels = hfl;
  out->cells = H.tx.ncells() + (P.same ? 0 : H.ty->ncells());
  int64_t leaves = 0;
  for (int64_t c = 0; c < H.tx.ncells(); ++c) leaves += H.tx.leaf[c];
  if (!P.same)
    for (int64_t c = 0; c < H.ty->ncells(); ++c) leaves += H.ty->leaf[c];
  out->leaves = leaves;
  out->m2l_pairs = (int64_t)H.m2l.size();
  out->p2p_cell_pairs = (int64_t)H.p2p_t.size();
  out->p2p_point_pairs = H.p2p_point_pairs;
  out->eff_expansions = H.tx.nexp() + (P.same ? 0 : H.ty->nexp());
  out->m2l_expansions = (int64_t)H.m2f_exp.size() + (int64_t)H.m2l_tgt.size();
  out->unique_offsets = (int64_t)H.offsets.size();
  out->spectra = (int64_t)(H.compressed ? H.canon.size() : H.offsets.size());
  out->compressed_spectra = H.compressed ? 1 : 0;
  for (int l = 0; l < 32; ++l)
    out->m2l_mode_per_level[l] =
        (l < (int)P.dense_ok.size() && P.dense_ok[l]) ? DEFMM_M2L_DENSE : DEFMM_M2L_FFT;
  return DEFMM_OK;
}

defmm_status defmm_workspace_create(defmm_plan* plan, defmm_workspace** out) {
  if (!plan || !out) return fail(DEFMM_ERR_INVALID_ARG, "NULL argument");
  *out = nullptr;
  DevPlan& P = plan->impl;
  if (P.host_only) return fail(DEFMM_ERR_INVALID_ARG, "plan was built for inspection only");
  defmm_workspace* ws = new (std::nothrow) defmm_workspace();
  if (!ws) return fail(DEFMM_ERR_OUT_OF_MEMORY, "host allocation failed");
  Workspace& W = ws->impl;
  W.plan = &P;
  W.m2l_variant = P.m2l_variant;
  W.p2p_waves = P.p2p_waves_per_cu;
  W.dense_level.assign(P.dense_ok.size(), 0);
  if (P.m2l_mode == DEFMM_M2L_DENSE)
    for (size_t l = 0; l < P.dense_ok.size(); ++l) W.dense_level[l] = P.dense_ok[l];
  size_t cs = csize(P);
  int L3 = P.L * P.L * P.L, P3 = fourier_row(P.L);
  struct {
    void** p;
    size_t n;
  } bufs[] = {{&W.qs, cs * (size_t)P.ny},
              {&W.ps, cs * (size_t)P.nx},
              {&W.M, cs * (size_t)P.ty.nexp * L3},
              {&W.Lx, cs * (size_t)P.tx.nexp * L3},
              {&W.Mt, cs * (size_t)P.n_m2f * P3},
              {&W.Lt, cs * (size_t)P.n_m2l_tgt * P3},
              {&W.part, cs * (size_t)P.nwi * 64},
              {(void**)&W.queue, 8 * sizeof(int)},
              {&W.slots, cs * (size_t)P.dense_slots_max * L3}};
  for (auto& b : bufs) {
    if (b.n == 0) continue;
    hipError_t e = hipMalloc(b.p, b.n);
    if (e != hipSuccess) {
      delete ws;
      return fail(e == hipErrorOutOfMemory ? DEFMM_ERR_OUT_OF_MEMORY : DEFMM_ERR_DEVICE,
                  std::string("workspace hipMalloc: ") + hipGetErrorString(e));
    }
    W.bytes += b.n;
  }
  {
    hipError_t e = hipStreamCreateWithFlags(&W.side, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&W.ev_fork, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&W.ev_join, hipEventDisableTiming);
    if (e != hipSuccess) {
      delete ws;
      return fail(DEFMM_ERR_DEVICE, std::string("workspace stream/events: ") + hipGetErrorString(e));
    }
  }
  *out = ws;
  return DEFMM_OK;
}

defmm_status defmm_matvec(defmm_plan* plan, defmm_workspace* ws, const void* q, void* p, void* hip_stream) {
  if (!plan || !ws) return fail(DEFMM_ERR_INVALID_ARG, "plan or workspace is NULL");
  DevPlan& P = plan->impl;
  if (P.host_only) return fail(DEFMM_ERR_INVALID_ARG, "plan was built for inspection only");
  if (ws->impl.plan != &P) return fail(DEFMM_ERR_INVALID_ARG, "workspace belongs to another plan");
  if ((P.ny > 0 && !q) || (P.nx > 0 && !p)) return fail(DEFMM_ERR_INVALID_ARG, "q or p is NULL");
  hipError_t e = run_matvec(P, ws->impl, q, p, (hipStream_t)hip_stream);
  if (e != hipSuccess) return fail(DEFMM_ERR_DEVICE, std::string("matvec launch: ") + hipGetErrorString(e));
  return DEFMM_OK;
}

defmm_status defmm_matvec_graph(defmm_plan* plan, defmm_workspace* ws, const void* q, void* p, void* hip_stream) {
  if (!plan || !ws) return fail(DEFMM_ERR_INVALID_ARG, "plan or workspace is NULL");
  DevPlan& P = plan->impl;
  Workspace& W = ws->impl;
  if (P.host_only) return fail(DEFMM_ERR_INVALID_ARG, "plan was built for inspection only");
  if (W.plan != &P) return fail(DEFMM_ERR_INVALID_ARG, "workspace belongs to another plan");
  if ((P.ny > 0 && !q) || (P.nx > 0 && !p)) return fail(DEFMM_ERR_INVALID_ARG, "q or p is NULL");
  if (!hip_stream) return fail(DEFMM_ERR_INVALID_ARG, "graph mode needs a created stream, not the null stream");
  if (W.timing) return fail(DEFMM_ERR_INVALID_ARG, "per-pass timing is on: use defmm_matvec");
  hipStream_t s = (hipStream_t)hip_stream;
  if (W.graph_stale || W.graph_q != q || W.graph_p != p || !W.graph_exec) {
    W.drop_graph();
    hipError_t e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return fail(DEFMM_ERR_DEVICE, std::string("begin capture: ") + hipGetErrorString(e));
    hipError_t er = run_matvec(P, W, q, p, s);
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(s, &g);
    if (er != hipSuccess || e != hipSuccess) {
      if (g) (void)hipGraphDestroy(g);
      return fail(DEFMM_ERR_DEVICE, std::string("capture: ") + hipGetErrorString(er != hipSuccess ? er : e));
    }
    W.graph = g;
    e = hipGraphInstantiate(&W.graph_exec, g, nullptr, nullptr, 0);
    if (e != hipSuccess) {
      W.drop_graph();
      return fail(DEFMM_ERR_DEVICE, std::string("graph instantiate: ") + hipGetErrorString(e));
    }
    W.graph_q = q;
    W.graph_p = p;
    W.graph_stale = false;
  }
  hipError_t e = hipGraphLaunch(W.graph_exec, s);
  if (e != hipSuccess) return fail(DEFMM_ERR_DEVICE, std::string("graph launch: ") + hipGetErrorString(e));
  if (!W.graph_done) {
    e = hipEventCreateWithFlags(&W.graph_done, hipEventDisableTiming);
    if (e != hipSuccess) {
      W.graph_done = nullptr;
      (void)hipStreamSynchronize(s);  // no event to wait on later: wait now
      return fail(DEFMM_ERR_DEVICE, std::string("graph event: ") + hipGetErrorString(e));
    }
  }
  e = hipEventRecord(W.graph_done, s);
  if (e != hipSuccess) {
    (void)hipStreamSynchronize(s);
    return fail(DEFMM_ERR_DEVICE, std::string("graph event record: ") + hipGetErrorString(e));
  }
  W.graph_launched = true;
  return DEFMM_OK;
}

}  // extern "C"

// ---- Allocation-free matvec ---------------------------------------------
// For callers that cannot allocate device memory (HIP graph capture, tight
// serving loops): the workspace arrays live in one file-scope device array of
// kNoAllocScratchBytes per GPU, which every call on that GPU shares.  Its
// device address comes from hipGetSymbolAddress, taken once per device on the
// first call with that device current; host code never uses the array's name
// as an address.
namespace {
constexpr size_t kNoAllocScratchBytes = size_t(64) << 20;
constexpr int kNoAllocMaxDevices = 64;
}  // namespace

static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

namespace {
std::once_flag g_scratch_once[kNoAllocMaxDevices];
void* g_scratch_ptr[kNoAllocMaxDevices];
hipError_t g_scratch_err[kNoAllocMaxDevices];

size_t round256(size_t n) { return (n + 255) & ~size_t(255); }

// Workspace arrays of the allocation-free matvec, in scratch order: sorted
// charges and potentials, multipoles, locals, Fourier-domain multipoles and
// locals, near-field partial sums, the near field's 8 work-queue heads.
void noalloc_layout(const DevPlan& P, size_t sizes[8]) {
  const size_t cs = csize(P);
  const size_t L3 = (size_t)P.L * P.L * P.L, R = (size_t)fourier_row(P.L);
  sizes[0] = cs * (size_t)P.ny;
  sizes[1] = cs * (size_t)P.nx;
  sizes[2] = cs * (size_t)P.ty.nexp * L3;
  sizes[3] = cs * (size_t)P.tx.nexp * L3;
  sizes[4] = cs * (size_t)P.n_m2f * R;
  sizes[5] = cs * (size_t)P.n_m2l_tgt * R;
  sizes[6] = cs * (size_t)P.nwi * 64;
  sizes[7] = 8 * sizeof(int);
}

// A workspace whose arrays point into the scratch: it owns nothing, so its
// destructor (which frees what a workspace owns) must find every pointer null.
struct BorrowedWorkspace {
  Workspace W;
  ~BorrowedWorkspace() {
    W.qs = W.ps = W.M = W.Lx = W.Mt = W.Lt = W.part = W.slots = nullptr;
    W.queue = nullptr;
  }
};
}  // namespace

extern "C" {

size_t defmm_matvec_noalloc_capacity(void) { return kNoAllocScratchBytes; }

defmm_status defmm_matvec_noalloc(defmm_plan* plan, const void* q, void* p, void* hip_stream) {
  if (!plan) return fail(DEFMM_ERR_INVALID_ARG, "plan is NULL");
  DevPlan& P = plan->impl;
  if (P.host_only) return fail(DEFMM_ERR_INVALID_ARG, "plan was built for inspection only");
  if ((P.ny > 0 && !q) || (P.nx > 0 && !p)) return fail(DEFMM_ERR_INVALID_ARG, "q or p is NULL");
  size_t sizes[8], need = 0;
  noalloc_layout(P, sizes);
  for (size_t b : sizes) need += round256(b);
  if (need > kNoAllocScratchBytes)
    return fail(DEFMM_ERR_INVALID_ARG, "plan needs " + std::to_string(need) +
                                           " bytes of workspace; the allocation-free matvec holds " +
                                           std::to_string(kNoAllocScratchBytes) + ": use defmm_matvec");
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return fail(DEFMM_ERR_DEVICE, std::string("hipGetDevice: ") + hipGetErrorString(e));
  if (dev < 0 || dev >= kNoAllocMaxDevices) return fail(DEFMM_ERR_UNSUPPORTED, "device index out of range");
  std::call_once(g_scratch_once[dev], [dev] {
    g_scratch_err[dev] = hipGetSymbolAddress(&g_scratch_ptr[dev], HIP_SYMBOL(scratch));
  });
  if (g_scratch_err[dev] != hipSuccess || !g_scratch_ptr[dev])
    return fail(DEFMM_ERR_DEVICE, std::string("scratch address: ") + hipGetErrorString(g_scratch_err[dev]));
  unsigned char* base = (unsigned char*)g_scratch_ptr[dev];
  BorrowedWorkspace B;
  Workspace& W = B.W;
  void** slot[7] = {&W.qs, &W.ps, &W.M, &W.Lx, &W.Mt, &W.Lt, &W.part};
  size_t off = 0;
  for (int i = 0; i < 7; ++i) {
    *slot[i] = sizes[i] ? (void*)(base + off) : nullptr;
    off += round256(sizes[i]);
  }
  W.queue = (int*)(base + off);
  W.plan = &P;
  W.overlap = 0;  // one stream: no side stream or events to create
  W.m2l_variant = P.m2l_variant;
  W.p2p_waves = P.p2p_waves_per_cu;
  e = run_matvec(P, W, q, p, (hipStream_t)hip_stream);
  if (e != hipSuccess) return fail(DEFMM_ERR_DEVICE, std::string("matvec launch: ") + hipGetErrorString(e));
  return DEFMM_OK;
}

defmm_status defmm_workspace_destroy(defmm_workspace* ws) {
  delete ws;
  return DEFMM_OK;
}

defmm_status defmm_plan_destroy(defmm_plan* plan) {
  delete plan;
  return DEFMM_OK;
}

defmm_status defmm_plan_geometry(const defmm_plan* plan, double* D, double* origin3) {
  if (!plan) return fail(DEFMM_ERR_INVALID_ARG, "plan is NULL");
  if (D) *D = plan->impl.D;
  if (origin3)
    for (int d = 0; d < 3; ++d) origin3[d] = plan->impl.origin[d];
  return DEFMM_OK;
}

defmm_status defmm_plan_export_tree(const defmm_plan* plan, int32_t which, int64_t* n, int32_t* level,
                                    int32_t* ijk, int32_t* first, int32_t* count, int32_t* is_leaf,
                                    int32_t* perm) {
  if (!plan || !n || (which != 0 && which != 1)) return fail(DEFMM_ERR_INVALID_ARG, "bad argument");
  const HostPlan& H = plan->impl.host;
  const Tree& T = which == 0 ? H.tx : *H.ty;
  *n = T.ncells();
  if (level) std::memcpy(level, T.level.data(), T.level.size() * 4);
  if (ijk) std::memcpy(ijk, T.ijk.data(), T.ijk.size() * 4);
  if (first) std::memcpy(first, T.first.data(), T.first.size() * 4);
  if (count) std::memcpy(count, T.count.data(), T.count.size() * 4);
  if (is_leaf) std::memcpy(is_leaf, T.leaf.data(), T.leaf.size() * 4);
  if (perm) std::memcpy(perm, T.perm.data(), T.perm.size() * 4);
  return DEFMM_OK;
}

defmm_status defmm_plan_export_m2l(const defmm_plan* plan, int64_t* n, int32_t* level, int32_t* t, int32_t* s,
                                   int32_t* delta, int32_t* dir) {
  if (!plan || !n) return fail(DEFMM_ERR_INVALID_ARG, "bad argument");
  const HostPlan& H = plan->impl.host;
  *n = (int64_t)H.m2l.size();
  if (level || t || s || delta || dir)
    for (size_t i = 0; i < H.m2l.size(); ++i) {
      const Offset& o = H.offsets[H.m2l[i].off];
      if (level) level[i] = o.level;
      if (t) t[i] = H.m2l[i].t;
      if (s) s[i] = H.m2l[i].s;
      if (delta)
        for (int d = 0; d < 3; ++d) delta[3 * i + d] = o.d[d];
      if (dir) dir[i] = o.dir;
    }
  return DEFMM_OK;
}

defmm_status defmm_plan_export_p2p(const defmm_plan* plan, int64_t* n, int32_t* t, int32_t* s) {
  if (!plan || !n) return fail(DEFMM_ERR_INVALID_ARG, "bad argument");
  const HostPlan& H = plan->impl.host;
  *n = (int64_t)H.p2p_t.size();
  if (t) std::memcpy(t, H.p2p_t.data(), H.p2p_t.size() * 4);
  if (s) std::memcpy(s, H.p2p_s.data(), H.p2p_s.size() * 4);
  return DEFMM_OK;
}

defmm_status defmm_plan_export_marks(const defmm_plan* plan, int32_t which, int64_t* n, int32_t* cell,
                                     int32_t* dir) {
  if (!plan || !n || (which != 0 && which != 1)) return fail(DEFMM_ERR_INVALID_ARG, "bad argument");
  const HostPlan& H = plan->impl.host;
  const Tree& T = which == 0 ? H.tx : *H.ty;
  *n = T.nexp();
  if (cell) std::memcpy(cell, T.exp_cell.data(), T.exp_cell.size() * 4);
  if (dir) std::memcpy(dir, T.exp_dir.data(), T.exp_dir.size() * 4);
  return DEFMM_OK;
}

defmm_status defmm_workspace_export_expansions(defmm_workspace* ws, int32_t which, int32_t kind, int64_t* n,
                                               int32_t* cell, int32_t* dir, void* values) {
  if (!ws || !n || (which != 0 && which != 1) || (kind != 0 && kind != 1))
    return fail(DEFMM_ERR_INVALID_ARG, "bad argument");
  const DevPlan& P = *ws->impl.plan;
  const Tree& T = which == 0 ? P.host.tx : *P.host.ty;
  *n = T.nexp();
  if (cell) std::memcpy(cell, T.exp_cell.data(), T.exp_cell.size() * 4);
  if (dir) std::memcpy(dir, T.exp_dir.data(), T.exp_dir.size() * 4);
  if (values && T.nexp() > 0) {
    // multipoles live on the source tree, locals on the target tree
    bool ok = (kind == 0) ? (which == 1 || P.same) : (which == 0 || P.same);
    if (!ok) return fail(DEFMM_ERR_INVALID_ARG, "this tree holds no such expansions");
    const void* src = kind == 0 ? ws->impl.M : ws->impl.Lx;
    size_t bytes = (size_t)T.nexp() * P.L * P.L * P.L * csize(P);
    hipError_t e = hipDeviceSynchronize();
    if (e == hipSuccess) e = hipMemcpy(values, src, bytes, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return fail(DEFMM_ERR_DEVICE, hipGetErrorString(e));
  }
  return DEFMM_OK;
}

defmm_status defmm_workspace_set_timing(defmm_workspace* ws, int32_t enable) {
  if (!ws) return fail(DEFMM_ERR_INVALID_ARG, "workspace is NULL");
  ws->impl.timing = enable != 0;
  return DEFMM_OK;
}

defmm_status defmm_workspace_set_overlap(defmm_workspace* ws, int32_t enable) {
  if (!ws) return fail(DEFMM_ERR_INVALID_ARG, "workspace is NULL");
  ws->impl.overlap = enable == 2 ? 2 : (enable != 0 ? 1 : 0);
  ws->impl.graph_stale = true;
  return DEFMM_OK;
}

defmm_status defmm_workspace_get_tuning(const defmm_workspace* ws, defmm_tuning* out) {
  if (!ws || !out) return fail(DEFMM_ERR_INVALID_ARG, "NULL argument");
  out->overlap = ws->impl.overlap;
  out->p2p_waves_per_cu = ws->impl.p2p_waves;
  out->m2l_variant = ws->impl.m2l_variant;
  out->updown_variant = ws->impl.pencil_updown;
  out->fourier_items = ws->impl.fourier_items;
  out->dense_levels = 0;
  for (size_t l = 0; l < ws->impl.dense_level.size() && l < 32; ++l)
    if (ws->impl.dense_level[l]) out->dense_levels |= 1u << l;
  out->ms = 0.0;
  return DEFMM_OK;
}

defmm_status defmm_workspace_set_tuning(defmm_workspace* ws, const defmm_tuning* t) {
  if (!ws || !t) return fail(DEFMM_ERR_INVALID_ARG, "NULL argument");
  if (t->p2p_waves_per_cu < 1 || t->p2p_waves_per_cu > 32 || t->m2l_variant < 0 || t->m2l_variant > 2 ||
      t->overlap < 0 || t->overlap > 2 || t->updown_variant < 0 || t->updown_variant > 1 ||
      !(t->fourier_items == 0 || t->fourier_items == 1 || t->fourier_items == 2 || t->fourier_items == 4))
    return fail(DEFMM_ERR_INVALID_ARG, "tuning out of range");
  ws->impl.graph_stale = true;
  ws->impl.overlap = t->overlap;
  ws->impl.p2p_waves = t->p2p_waves_per_cu;
  ws->impl.m2l_variant = t->m2l_variant;
  ws->impl.pencil_updown = t->updown_variant;
  ws->impl.fourier_items = t->fourier_items;
  const DevPlan& P = *ws->impl.plan;
  for (size_t l = 0; l < ws->impl.dense_level.size(); ++l)
    ws->impl.dense_level[l] = (l < 32 && (t->dense_levels >> l) & 1u && P.dense_ok[l]) ? 1 : 0;
  return DEFMM_OK;
}

defmm_status defmm_workspace_autotune(defmm_plan* plan, defmm_workspace* ws, const void* q, void* p,
                                      void* hip_stream, int32_t reps, defmm_tuning* chosen) {
  if (!plan || !ws) return fail(DEFMM_ERR_INVALID_ARG, "plan or workspace is NULL");
  DevPlan& P = plan->impl;
  Workspace& W = ws->impl;
  if (P.host_only || W.plan != &P) return fail(DEFMM_ERR_INVALID_ARG, "workspace/plan mismatch");
  if ((P.ny > 0 && !q) || (P.nx > 0 && !p)) return fail(DEFMM_ERR_INVALID_ARG, "q or p is NULL");
  if (reps < 1) reps = 3;
  hipStream_t s = (hipStream_t)hip_stream;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
    return fail(DEFMM_ERR_DEVICE, "autotune events");
  bool timing = W.timing;
  W.timing = false;
  W.graph_stale = true;
  auto apply = [&](const defmm_tuning& t) {
    W.overlap = t.overlap;
    W.p2p_waves = t.p2p_waves_per_cu;
    W.m2l_variant = t.m2l_variant;
    W.pencil_updown = t.updown_variant;
    W.fourier_items = t.fourier_items;
    for (size_t l = 0; l < W.dense_level.size(); ++l)
      W.dense_level[l] = (l < 32 && (t.dense_levels >> l) & 1u && P.dense_ok[l]) ? 1 : 0;
  };
  auto measure = [&](const defmm_tuning& t, double* ms) -> hipError_t {
    apply(t);
    hipError_t e = run_matvec(P, W, q, p, s);  // warm-up
    std::vector<double> v;
    for (int r = 0; r < reps && e == hipSuccess; ++r) {
      e = hipEventRecord(e0, s);
      if (e == hipSuccess) e = run_matvec(P, W, q, p, s);
      if (e == hipSuccess) e = hipEventRecord(e1, s);
      if (e == hipSuccess) e = hipEventSynchronize(e1);
      float f = 0.f;
      if (e == hipSuccess) e = hipEventElapsedTime(&f, e0, e1);
      v.push_back(f);
    }
    if (e == hipSuccess) {
      std::sort(v.begin(), v.end());
      *ms = v[v.size() / 2];
    }
    return e;
  };
  defmm_tuning best{0, 8, 2, 0u, 1, 0, 1e30};
  hipError_t err = hipSuccess;
  // M2L variant, timed with every pass in sequence
  for (int var : {2, 1}) {
    defmm_tuning t{0, 8, var, 0u, 1, 0, 0.0};
    err = measure(t, &t.ms);
    if (err != hipSuccess) break;
    if (t.ms < best.ms) best = t;
  }
  // M2M/L2L kernels
  if (err == hipSuccess) {
    defmm_tuning t{0, 8, best.m2l_variant, 0u, 0, 0, 0.0};
    err = measure(t, &t.ms);
    if (err == hipSuccess && t.ms < best.ms) best = t;
  }
  // M2F/F2L expansions per workgroup
  for (int gi : {1, 2, 4}) {
    if (err != hipSuccess) break;
    defmm_tuning t{0, 8, best.m2l_variant, 0u, best.updown_variant, gi, 0.0};
    err = measure(t, &t.ms);
    if (err == hipSuccess && t.ms < best.ms) best = t;
  }
  // per level: dense MFMA M2L instead of the Fourier path where it is faster
  for (size_t l = 0; l < P.dense_ok.size() && l < 32 && err == hipSuccess; ++l) {
    if (!P.dense_ok[l]) continue;
    defmm_tuning t{0, 8, best.m2l_variant, best.dense_levels | (1u << l), best.updown_variant, best.fourier_items,
                   0.0};
    err = measure(t, &t.ms);
    if (err != hipSuccess) break;
    if (t.ms < best.ms) best = t;
  }
  // near field overlapped with the far field, forked early or after M2F,
  // with a few wave budgets
  for (int ov : {1, 2})
    for (int w : {2, 3, 4, 6}) {
      if (err != hipSuccess) break;
      defmm_tuning t{ov, w, best.m2l_variant, best.dense_levels, best.updown_variant, best.fourier_items, 0.0};
      err = measure(t, &t.ms);
      if (err != hipSuccess) break;
      if (t.ms < best.ms) best = t;
    }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  W.timing = timing;
  if (err != hipSuccess) return fail(DEFMM_ERR_DEVICE, std::string("autotune: ") + hipGetErrorString(err));
  apply(best);
  if (chosen) *chosen = best;
  return DEFMM_OK;
}

defmm_status defmm_workspace_pass_times(defmm_workspace* ws, double* pass_ms, int64_t* calls) {
  if (!ws) return fail(DEFMM_ERR_INVALID_ARG, "workspace is NULL");
  Workspace& W = ws->impl;
  for (const auto& r : W.pending) {
    hipError_t e = hipEventSynchronize(W.ev_pool[r.b]);
    if (e != hipSuccess) return fail(DEFMM_ERR_DEVICE, hipGetErrorString(e));
    float ms = 0.f;
    e = hipEventElapsedTime(&ms, W.ev_pool[r.a], W.ev_pool[r.b]);
    if (e != hipSuccess) return fail(DEFMM_ERR_DEVICE, hipGetErrorString(e));
    W.pass_ms[r.pass] += ms;
    W.pass_calls[r.pass] += 1;
  }
  W.pending.clear();
  W.ev_used = 0;
  for (int i = 0; i < kNumPasses; ++i) {
    if (pass_ms) pass_ms[i] = W.pass_ms[i];
    if (calls) calls[i] = W.pass_calls[i];
    W.pass_ms[i] = 0;
    W.pass_calls[i] = 0;
  }
  return DEFMM_OK;
}

defmm_status defmm_fourier_layout(int32_t L, int32_t* slices, int32_t* cap, int32_t* row, int32_t* freq,
                                  uint8_t* perm) {
  if (L < 2 || L > 8 || !slices || !cap || !row) return fail(DEFMM_ERR_INVALID_ARG, "bad layout query");
  try {
    FourierLayout F = make_fourier_layout(L, m2l_slices(L), fourier_cap(L));
    *slices = F.slices;
    *cap = F.cap;
    *row = F.row;
    if (freq) std::memcpy(freq, F.freq.data(), F.freq.size() * sizeof(int32_t));
    if (perm) std::memcpy(perm, F.perm.data(), F.perm.size());
    return DEFMM_OK;
  } catch (const std::exception& e) {
    return fail(DEFMM_ERR_DEVICE, e.what());
  }
}

defmm_status defmm_directions(int32_t E, int64_t* n, double* dirs, int64_t* father) {
  if (E < 0 || E > 12 || !n) return fail(DEFMM_ERR_INVALID_ARG, "bad direction level");
  *n = num_directions(E);
  if (!dirs && !father) return DEFMM_OK;
  try {
    std::vector<double> d(3 * (size_t)*n);
    std::vector<int64_t> f((size_t)*n);
    make_directions(E, d.data(), f.data());
    if (dirs) std::memcpy(dirs, d.data(), d.size() * sizeof(double));
    if (father) std::memcpy(father, f.data(), f.size() * sizeof(int64_t));
    return DEFMM_OK;
  } catch (const std::exception& e) {
    return fail(DEFMM_ERR_OUT_OF_MEMORY, e.what());
  }
}

defmm_status defmm_canonical_offset(const int32_t* d, int32_t* d0, int32_t* code) {
  if (!d || !d0 || !code) return fail(DEFMM_ERR_INVALID_ARG, "NULL argument");
  *code = canonical_offset(d, d0);
  return DEFMM_OK;
}

const char* defmm_pass_name(int32_t i) {
  static const char* names[kNumPasses] = {"setup", "p2m", "m2m", "m2f", "m2l", "l2l", "p2p", "p2p_reduce",
                                          "l2p", "scatter", "f2l", "m2l_dense"};
  if (i < 0 || i >= kNumPasses) return "";
  return names[i];
}

defmm_status defmm_workspace_pass_work(const defmm_workspace* ws, double* bytes, double* flops) {
  if (!ws) return fail(DEFMM_ERR_INVALID_ARG, "workspace is NULL");
  const Workspace& W = ws->impl;
  const DevPlan& P = *W.plan;
  const HostPlan& H = P.host;
  double cs = (double)csize(P);
  double L = P.L, Pp = 2 * P.L - 1, L3 = L * L * L, P3 = Pp * Pp * Pp;
  double b[kNumPasses] = {0}, f[kNumPasses] = {0};
  b[kPassSetup] = (double)P.ny * (2 * cs + 4) +
                  cs * ((W.pencil_updown ? (double)P.n_zero_exp : (double)H.tx.nexp()) * L3 + (double)P.nx);
  double npts = 0;
  for (int32_t e : H.p2m_exp) npts += H.ty->count[H.ty->exp_cell[e]];
  b[kPassP2M] = npts * (24 + cs) + (double)P.n_p2m * cs * L3;
  f[kPassP2M] = npts * L3 * 8;
  // M2M: each son expansion that feeds a father read once (one feeds every
  // father direction it serves), each father written once
  double nm2m = 0, nm2m_child = 0, nm2m_son = 0;
  {
    std::vector<uint8_t> seen((size_t)std::max<int64_t>(H.ty->nexp(), 1), 0);
    for (const auto& v : H.m2m_par) nm2m += (double)v.size();
    for (const auto& v : H.m2m_child)
      for (int32_t c : v)
        if (c >= 0) {
          nm2m_child += 1;
          if (!seen[c]) {
            seen[c] = 1;
            nm2m_son += 1;
          }
        }
  }
  b[kPassM2M] = (nm2m + nm2m_son) * cs * L3;
  f[kPassM2M] = nm2m_child * 8 * (3 * L3 * L + 2 * L3);
  const double f2l_per_tgt = 8 * (Pp * Pp * L * Pp + Pp * L * L * Pp + L3 * Pp);
  const double m2f_per_row = 8 * (Pp * L * L * L + Pp * Pp * L * L + P3 * L);
  const int nlev = (int)H.lvl_m2f.size() - 1;
  std::vector<double> n_spec(nlev > 0 ? nlev : 0, 0.0);
  for (const Offset& o : (P.sym ? H.canon : H.offsets))
    if (o.level >= 0 && o.level < nlev) n_spec[o.level] += 1;
  for (int l = 0; l < nlev; ++l) {
    const double n_src = (double)(H.lvl_m2f[l + 1] - H.lvl_m2f[l]);
    const int64_t tb = H.m2l_level_tgt[l], te = H.m2l_level_tgt[l + 1];
    const double n_tgt = (double)(te - tb);
    const double n_pair = (double)(H.m2l_begin[te] - H.m2l_begin[tb]);
    const bool dense = l < (int)W.dense_level.size() && W.dense_level[l] && P.dense_ok[l];
    if (dense) {
      const double n_off = (double)(H.dns_off_begin[l + 1] - H.dns_off_begin[l]);
      b[kPassM2LDense] += n_off * L3 * L3 * cs + (n_src + n_tgt) * L3 * cs;
      f[kPassM2LDense] += n_pair * 8 * L3 * L3;
      continue;
    }
    b[kPassM2F] += n_src * cs * (L3 + P3);
    f[kPassM2F] += n_src * m2f_per_row;
    // Hadamard: each spectrum and each source row read once, each target row
    // written once (the per-pair operand stream, 2 cs P^3 per pair, is what
    // the caches must serve beyond that)
    if (W.m2l_variant == 0) {
      b[kPassM2L] += (n_spec[l] + n_src) * cs * P3 + n_tgt * cs * L3;
      f[kPassM2L] += n_pair * 8 * P3 + n_tgt * f2l_per_tgt;
    } else {
      b[kPassM2L] += (n_spec[l] + n_src + n_tgt) * cs * P3;
      f[kPassM2L] += n_pair * 8 * P3;
      b[kPassF2L] += n_tgt * cs * (P3 + L3);
      f[kPassF2L] += n_tgt * f2l_per_tgt;
    }
  }
  // L2L: each father expansion that feeds a son read once, each son read and
  // written once
  double nl2l = 0, nl2l_par = 0;
  {
    std::vector<uint8_t> seen((size_t)std::max<int64_t>(H.tx.nexp(), 1), 0);
    for (const auto& v : H.l2l_par) {
      nl2l += (double)v.size();
      for (int32_t e : v)
        if (!seen[e]) {
          seen[e] = 1;
          nl2l_par += 1;
        }
    }
  }
  double nl2l_ch = 0;
  for (const auto& v : H.l2l_ch) nl2l_ch += (double)v.size();
  b[kPassL2L] = (nl2l_par + 2 * nl2l_ch) * cs * L3;
  f[kPassL2L] = nl2l * 8 * (3 * L3 * L + 3 * L3);
  // per pair: 3 differences, 5 for r^2, rsqrt, r, kappa r, then sin, cos, 2 scalings
  // and a complex multiply-add (8), or, screened, exp, 1 scaling and a real-by-
  // complex multiply-add (4)
  f[kPassP2P] = (P.screened ? 17.0 : 23.0) * (double)H.p2p_point_pairs;
  double nwi = (double)H.wi_blk.size();
  b[kPassP2P] = nwi * 64 * cs;
  b[kPassP2PRed] = nwi * 64 * cs + (double)P.nx * cs;
  double nl2p_pts = 0, nl2p_exp = 0;
  for (size_t i = 0; i < H.l2p_cell.size(); ++i) {
    int c = H.l2p_cell[i];
    double ne = (double)(H.tx.exp_begin[c + 1] - H.tx.exp_begin[c]);
    nl2p_pts += H.l2p_count[i];
    nl2p_exp += ne;
    f[kPassL2P] += (double)H.l2p_count[i] * ne * 8 * (L3 + L * L + L);
  }
  b[kPassL2P] = nl2p_pts * (24 + 2 * cs) + nl2p_exp * cs * L3;
  b[kPassScatter] = (double)P.nx * (2 * cs + 4);
  for (int i = 0; i < kNumPasses; ++i) {
    if (bytes) bytes[i] = b[i];
    if (flops) flops[i] = f[i];
  }
  return DEFMM_OK;
}

}  // extern "C"
