// Device-side plan builder.  The steps that touch every point or every pair
// of cells run as HIP kernels on the plan's stream:
//   * bounding cube (block min/max reduction) and the finiteness check;
//   * Morton keys (21 bits per dimension) and a stable radix sort of
//     (key, caller index) pairs;
//   * the Ncrit tree (Sec. 4.2.1), one level at a time: a point opens a new
//     cell where its next octant digit changes inside a non-leaf cell, cells
//     are numbered by a scan over those heads;
//   * the dual tree traversal (Alg. 1 with the MAC of eq. macdirref), one
//     level at a time over a frontier of same-level cell pairs, compacted by
//     scans so the lists come out in frontier order;
//   * the distinct (level, offset) M2L spectra of each level (sort + unique)
//     and the best direction of each (Sec. 4.1.2, argmax of <v, offset>,
//     ties to the lowest index);
//   * the marks of Alg. 2 and the blank downward pass of Alg. 3 on per-level
//     (cell, direction) flag arrays.
// Trees, lists, offsets and marks are then copied to the host once, where
// the operator tables are packed.  Every decision uses the same arithmetic
// as the definitions (FP64, no contraction), so the lists are identical to
// the host builder's.
#pragma clang fp contract(off)

#include <hip/hip_runtime.h>

#include <rocprim/device/device_radix_sort.hpp>
#include <rocprim/device/device_scan.hpp>
#include <rocprim/device/device_select.hpp>

#include <algorithm>
#include <cmath>
#include <new>
#include <stdexcept>
#include <string>
#include <vector>

#include "build_device.hpp"

namespace defmm {

namespace {

void chk(hipError_t e, const char* what) {
  if (e == hipErrorOutOfMemory) throw std::bad_alloc();
  if (e != hipSuccess) throw std::runtime_error(std::string("device builder: ") + what + ": " + hipGetErrorString(e));
}

// Stream of the build in progress: the builder's temporaries are allocated
// and freed in stream order on it (no device-wide synchronisation, so a
// build does not stall other streams' work).
thread_local hipStream_t g_stream = nullptr;

// Owning device array (stream-ordered on the build stream).
template <class T>
struct DVec {
  T* p = nullptr;
  size_t n = 0;
  DVec() = default;
  explicit DVec(size_t k) { resize(k); }
  DVec(const DVec&) = delete;
  DVec& operator=(const DVec&) = delete;
  DVec(DVec&& o) noexcept : p(o.p), n(o.n) {
    o.p = nullptr;
    o.n = 0;
  }
  DVec& operator=(DVec&& o) noexcept {
    std::swap(p, o.p);
    std::swap(n, o.n);
    return *this;
  }
  ~DVec() {
    if (p) (void)hipFreeAsync(p, g_stream);
  }
  void resize(size_t k) {
    if (p) (void)hipFreeAsync(p, g_stream);
    p = nullptr;
    n = k;
    if (k) chk(hipMallocAsync((void**)&p, k * sizeof(T), g_stream), "allocation");
  }
};

template <class T>
void to_host(std::vector<T>& h, const T* d, size_t n, hipStream_t s) {
  h.resize(n);
  if (n) chk(hipMemcpyAsync(h.data(), d, n * sizeof(T), hipMemcpyDeviceToHost, s), "download");
  chk(hipStreamSynchronize(s), "download");
}

template <class T>
void to_device(DVec<T>& d, const std::vector<T>& h, hipStream_t s) {
  d.resize(h.size());
  if (!h.empty()) chk(hipMemcpyAsync(d.p, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice, s), "upload");
}

template <class T>
T read_one(const T* d, hipStream_t s) {
  T v{};
  chk(hipMemcpyAsync(&v, d, sizeof(T), hipMemcpyDeviceToHost, s), "read");
  chk(hipStreamSynchronize(s), "read");
  return v;
}

// Scratch for rocPRIM's device algorithms, grown on demand.
struct Temp {
  DVec<unsigned char> buf;
  // never null: rocPRIM takes a null pointer as a size query
  void* get(size_t bytes) {
    if (bytes > buf.n || !buf.p) buf.resize(std::max(bytes, (size_t)1 << 20));
    return buf.p;
  }
};

// Exclusive prefix sum of n values into out[0..n]; returns the total.
template <class T>
T scan_total(Temp& tmp, const T* in, T* out, int64_t n, hipStream_t s) {
  if (n == 0) return 0;
  size_t bytes = 0;
  chk(rocprim::exclusive_scan(nullptr, bytes, in, out, (T)0, (size_t)n, rocprim::plus<T>(), s), "scan size");
  chk(rocprim::exclusive_scan(tmp.get(bytes), bytes, in, out, (T)0, (size_t)n, rocprim::plus<T>(), s), "scan");
  T a = read_one(out + n - 1, s), b = read_one(in + n - 1, s);
  return a + b;
}

inline unsigned grid_for(int64_t n, int bs) { return (unsigned)std::max<int64_t>(1, (n + bs - 1) / bs); }

// ------------------------------------------------------------------ bounding cube
constexpr int kBoxBlocks = 1024;

__global__ __launch_bounds__(256) void k_bbox(const double* __restrict__ X, int64_t n, double* __restrict__ part) {
  __shared__ double lo[3][256], hi[3][256];
  __shared__ int bad[256];
  double l[3] = {1e300, 1e300, 1e300}, h[3] = {-1e300, -1e300, -1e300};
  int nb = 0;
  for (int64_t i = blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
    for (int d = 0; d < 3; ++d) {
      double v = X[3 * i + d];
      if (!isfinite(v)) nb = 1;
      l[d] = fmin(l[d], v);
      h[d] = fmax(h[d], v);
    }
  for (int d = 0; d < 3; ++d) {
    lo[d][threadIdx.x] = l[d];
    hi[d][threadIdx.x] = h[d];
  }
  bad[threadIdx.x] = nb;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      for (int d = 0; d < 3; ++d) {
        lo[d][threadIdx.x] = fmin(lo[d][threadIdx.x], lo[d][threadIdx.x + w]);
        hi[d][threadIdx.x] = fmax(hi[d][threadIdx.x], hi[d][threadIdx.x + w]);
      }
      bad[threadIdx.x] |= bad[threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    for (int d = 0; d < 3; ++d) {
      part[7 * blockIdx.x + d] = lo[d][0];
      part[7 * blockIdx.x + 3 + d] = hi[d][0];
    }
    part[7 * blockIdx.x + 6] = bad[0] ? 1.0 : 0.0;
  }
}

// Folds the points into lo/hi; returns false if any coordinate is not finite.
bool bbox(const double* X, int64_t n, double* lo, double* hi, hipStream_t s) {
  if (n == 0) return true;
  int nb = (int)std::min<int64_t>(kBoxBlocks, (n + 255) / 256);
  DVec<double> part(7 * (size_t)nb);
  hipLaunchKernelGGL(k_bbox, dim3(nb), dim3(256), 0, s, X, n, part.p);
  chk(hipGetLastError(), "bbox launch");
  std::vector<double> h;
  to_host(h, part.p, part.n, s);
  bool ok = true;
  for (int b = 0; b < nb; ++b) {
    for (int d = 0; d < 3; ++d) {
      lo[d] = std::fmin(lo[d], h[7 * b + d]);
      hi[d] = std::fmax(hi[d], h[7 * b + 3 + d]);
    }
    if (h[7 * b + 6] != 0.0) ok = false;
  }
  return ok;
}

// ------------------------------------------------------------------ Morton keys
__device__ __forceinline__ uint64_t spread3(uint64_t v) {
  v &= 0x1fffffull;
  v = (v | (v << 32)) & 0x1f00000000ffffull;
  v = (v | (v << 16)) & 0x1f0000ff0000ffull;
  v = (v | (v << 8)) & 0x100f00f00f00f00full;
  v = (v | (v << 4)) & 0x10c30c30c30c30c3ull;
  v = (v | (v << 2)) & 0x1249249249249249ull;
  return v;
}

__device__ __forceinline__ uint64_t quant(double x, double o, double D) {
  if (!(D > 0.0)) return 0;
  double q = floor((x - o) / D * (double)(1 << kKeyBits));
  if (q < 0.0) q = 0.0;
  if (q > (double)((1 << kKeyBits) - 1)) q = (double)((1 << kKeyBits) - 1);
  return (uint64_t)q;
}

__global__ __launch_bounds__(256) void k_morton(const double* __restrict__ X, int64_t n, double o0, double o1,
                                                double o2, double D, uint64_t* __restrict__ key,
                                                int32_t* __restrict__ idx) {
  int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  key[i] = spread3(quant(X[3 * i], o0, D)) | (spread3(quant(X[3 * i + 1], o1, D)) << 1) |
           (spread3(quant(X[3 * i + 2], o2, D)) << 2);
  idx[i] = (int32_t)i;
}

__global__ __launch_bounds__(256) void k_soa(const double* __restrict__ X, int64_t n,
                                             const int32_t* __restrict__ perm, double* __restrict__ soa) {
  int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  int64_t j = perm[i];
  for (int d = 0; d < 3; ++d) soa[d * n + i] = X[3 * j + d];
}

// ------------------------------------------------------------------ tree levels
// Cells of the current level, local ids.
__global__ __launch_bounds__(256) void k_leaf(int64_t m, const int32_t* __restrict__ count, int ncrit, int lev,
                                              int32_t* __restrict__ leaf) {
  int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (c >= m) return;
  leaf[c] = (count[c] > ncrit && lev < kMaxLevel) ? 0 : 1;
}

// head[i] = 1 where point i opens a son of its (non-leaf) cell.
__global__ __launch_bounds__(256) void k_heads(int64_t n, const uint64_t* __restrict__ key,
                                               const int32_t* __restrict__ cell_of,
                                               const int32_t* __restrict__ first, const int32_t* __restrict__ leaf,
                                               int sh, int32_t* __restrict__ head) {
  int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  int32_t c = cell_of[i];
  int h = 0;
  if (c >= 0 && !leaf[c]) {
    if (i == first[c]) h = 1;
    else h = (((key[i] >> sh) & 7ull) != ((key[i - 1] >> sh) & 7ull)) ? 1 : 0;
  }
  head[i] = h;
}

__global__ __launch_bounds__(256) void k_new_cells(int64_t n, const uint64_t* __restrict__ key,
                                                   const int32_t* __restrict__ cell_of,
                                                   const int32_t* __restrict__ head,
                                                   const int32_t* __restrict__ hpos,
                                                   const int32_t* __restrict__ ijk, int sh,
                                                   int32_t* __restrict__ nfirst, int32_t* __restrict__ nparent,
                                                   int32_t* __restrict__ nijk) {
  int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n || !head[i]) return;
  int32_t r = hpos[i], c = cell_of[i];
  uint64_t dg = (key[i] >> sh) & 7ull;
  nfirst[r] = (int32_t)i;
  nparent[r] = c;
  nijk[3 * r] = 2 * ijk[3 * c] + (int32_t)(dg & 1);
  nijk[3 * r + 1] = 2 * ijk[3 * c + 1] + (int32_t)((dg >> 1) & 1);
  nijk[3 * r + 2] = 2 * ijk[3 * c + 2] + (int32_t)((dg >> 2) & 1);
}

// Son counts, and for the last son of each father: its first son and number of sons.
__global__ __launch_bounds__(256) void k_son_counts(int64_t m, const int32_t* __restrict__ nfirst,
                                                    const int32_t* __restrict__ nparent,
                                                    const int32_t* __restrict__ first,
                                                    const int32_t* __restrict__ count,
                                                    const int32_t* __restrict__ hpos, int64_t next_base,
                                                    int32_t* __restrict__ ncount, int32_t* __restrict__ child0,
                                                    int32_t* __restrict__ nchild) {
  int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (r >= m) return;
  int32_t p = nparent[r];
  bool last = (r + 1 == m) || nparent[r + 1] != p;
  int32_t end = last ? first[p] + count[p] : nfirst[r + 1];
  ncount[r] = end - nfirst[r];
  if (last) {
    int32_t r0 = hpos[first[p]];
    child0[p] = (int32_t)(next_base + r0);
    nchild[p] = (int32_t)(r - r0 + 1);
  }
}

__global__ __launch_bounds__(256) void k_cell_of(int64_t n, const int32_t* __restrict__ head,
                                                 const int32_t* __restrict__ hpos, const int32_t* __restrict__ leaf,
                                                 int32_t* __restrict__ cell_of) {
  int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  int32_t c = cell_of[i];
  // a point stays active while its cell splits; it then belongs to the son
  // opened by the last head at or before it
  cell_of[i] = (c >= 0 && !leaf[c]) ? hpos[i] + head[i] - 1 : -1;
}

void build_tree_device(Tree& T, const double* X, int64_t n, const double* origin, double D, int ncrit,
                       hipStream_t s, Temp& tmp) {
  T.n = n;
  DVec<uint64_t> k0(n), k1(n);
  DVec<int32_t> i0(n), i1(n);
  if (n > 0) {
    hipLaunchKernelGGL(k_morton, dim3(grid_for(n, 256)), dim3(256), 0, s, X, n, origin[0], origin[1], origin[2], D,
                       k0.p, i0.p);
    chk(hipGetLastError(), "morton launch");
    size_t bytes = 0;
    chk(rocprim::radix_sort_pairs(nullptr, bytes, k0.p, k1.p, i0.p, i1.p, (size_t)n, 0u, 3u * kKeyBits, s),
        "sort size");
    chk(rocprim::radix_sort_pairs(tmp.get(bytes), bytes, k0.p, k1.p, i0.p, i1.p, (size_t)n, 0u, 3u * kKeyBits, s),
        "sort");
  }
  const uint64_t* key = k1.p;
  to_host(T.key, key, n, s);
  to_host(T.perm, i1.p, n, s);
  {
    DVec<double> soa(3 * (size_t)n);
    if (n > 0) {
      hipLaunchKernelGGL(k_soa, dim3(grid_for(n, 256)), dim3(256), 0, s, X, n, i1.p, soa.p);
      chk(hipGetLastError(), "soa launch");
    }
    to_host(T.soa, soa.p, soa.n, s);
  }
  k0 = DVec<uint64_t>();
  i0 = DVec<int32_t>();
  // level 0: the root, every point in it
  T.level = {0};
  T.first = {0};
  T.count = {(int32_t)n};
  T.parent = {-1};
  T.ijk = {0, 0, 0};
  T.leaf = {0};
  T.child0 = {0};
  T.nchild = {0};
  T.lev_start = {0, 1};
  DVec<int32_t> cell_of(n), head(n), hpos(n);
  if (n > 0) chk(hipMemsetAsync(cell_of.p, 0, n * sizeof(int32_t), s), "cell_of");
  DVec<int32_t> first, count, ijk, leaf;
  std::vector<int32_t> h_first = {0}, h_count = {(int32_t)n}, h_ijk = {0, 0, 0};
  to_device(first, h_first, s);
  to_device(count, h_count, s);
  to_device(ijk, h_ijk, s);
  for (int lev = 0;; ++lev) {
    const int64_t base = T.lev_start[lev], m = T.lev_start[lev + 1] - base;
    leaf.resize(m);
    hipLaunchKernelGGL(k_leaf, dim3(grid_for(m, 256)), dim3(256), 0, s, m, count.p, ncrit, lev, leaf.p);
    chk(hipGetLastError(), "leaf launch");
    int64_t nn = 0;
    const int sh = 3 * (kKeyBits - lev - 1);
    if (n > 0 && lev < kMaxLevel) {
      hipLaunchKernelGGL(k_heads, dim3(grid_for(n, 256)), dim3(256), 0, s, n, key, cell_of.p, first.p, leaf.p, sh,
                         head.p);
      chk(hipGetLastError(), "heads launch");
      nn = scan_total<int32_t>(tmp, head.p, hpos.p, n, s);
    }
    DVec<int32_t> child0(m), nchild(m);
    if (m > 0) {
      chk(hipMemsetAsync(child0.p, 0, m * sizeof(int32_t), s), "child0");
      chk(hipMemsetAsync(nchild.p, 0, m * sizeof(int32_t), s), "nchild");
    }
    DVec<int32_t> nfirst(nn), nparent(nn), nijk(3 * nn), ncount(nn);
    if (nn > 0) {
      hipLaunchKernelGGL(k_new_cells, dim3(grid_for(n, 256)), dim3(256), 0, s, n, key, cell_of.p, head.p, hpos.p,
                         ijk.p, sh, nfirst.p, nparent.p, nijk.p);
      chk(hipGetLastError(), "cells launch");
      hipLaunchKernelGGL(k_son_counts, dim3(grid_for(nn, 256)), dim3(256), 0, s, nn, nfirst.p, nparent.p, first.p,
                         count.p, hpos.p, base + m, ncount.p, child0.p, nchild.p);
      chk(hipGetLastError(), "son counts launch");
      hipLaunchKernelGGL(k_cell_of, dim3(grid_for(n, 256)), dim3(256), 0, s, n, head.p, hpos.p, leaf.p, cell_of.p);
      chk(hipGetLastError(), "cell_of launch");
    }
    // this level is final: leaf, child0, nchild
    std::vector<int32_t> h_leaf, h_c0, h_nc;
    to_host(h_leaf, leaf.p, m, s);
    to_host(h_c0, child0.p, m, s);
    to_host(h_nc, nchild.p, m, s);
    for (int64_t c = 0; c < m; ++c) {
      T.leaf[base + c] = h_leaf[c];
      T.child0[base + c] = h_c0[c];
      T.nchild[base + c] = h_nc[c];
    }
    if (nn == 0) {
      T.nlevels = lev + 1;
      break;
    }
    std::vector<int32_t> hf_, hp_, hc_, hi_;
    to_host(hf_, nfirst.p, nn, s);
    to_host(hp_, nparent.p, nn, s);
    to_host(hc_, ncount.p, nn, s);
    to_host(hi_, nijk.p, 3 * nn, s);
    for (int64_t r = 0; r < nn; ++r) {
      T.level.push_back(lev + 1);
      T.first.push_back(hf_[r]);
      T.count.push_back(hc_[r]);
      T.parent.push_back((int32_t)(base + hp_[r]));
      T.ijk.insert(T.ijk.end(), {hi_[3 * r], hi_[3 * r + 1], hi_[3 * r + 2]});
      T.leaf.push_back(0);
      T.child0.push_back(0);
      T.nchild.push_back(0);
    }
    T.lev_start.push_back(base + m + nn);
    first = std::move(nfirst);
    count = std::move(ncount);
    ijk = std::move(nijk);
  }
}

// ------------------------------------------------------------------ traversal
struct DevCells {  // per-cell arrays of one tree, global ids
  DVec<int32_t> ijk, leaf, child0, nchild;
};

void upload_cells(DevCells& d, const Tree& T, hipStream_t s) {
  to_device(d.ijk, T.ijk, s);
  to_device(d.leaf, T.leaf, s);
  to_device(d.child0, T.child0, s);
  to_device(d.nchild, T.nchild, s);
}

// 0: admissible (M2L), 1: near with a leaf (P2P), 2: split into all pairs of sons.
__global__ __launch_bounds__(256) void k_classify(int64_t nf, const int2* __restrict__ front,
                                                  const int32_t* __restrict__ xijk, const int32_t* __restrict__ xleaf,
                                                  const int32_t* __restrict__ xnch,
                                                  const int32_t* __restrict__ yijk, const int32_t* __restrict__ yleaf,
                                                  const int32_t* __restrict__ ynch, double thr,
                                                  int32_t* __restrict__ is_m2l, int32_t* __restrict__ is_p2p,
                                                  int64_t* __restrict__ n_next) {
  int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= nf) return;
  int32_t t = front[i].x, s = front[i].y;
  int64_t n2 = 0;
  for (int k = 0; k < 3; ++k) {
    int32_t d = xijk[3 * t + k] - yijk[3 * s + k];
    int64_t a = d < 0 ? -(int64_t)d : (int64_t)d;
    int64_t nk = a - 1 > 0 ? a - 1 : 0;
    n2 += nk * nk;
  }
  int m = 0, p = 0;
  int64_t nx = 0;
  if ((double)n2 >= thr) m = 1;
  else if (xleaf[t] || yleaf[s]) p = 1;
  else nx = (int64_t)xnch[t] * ynch[s];
  is_m2l[i] = m;
  is_p2p[i] = p;
  n_next[i] = nx;
}

constexpr int kOffBits = 21;  // per dimension in an offset key; |offset| < 2^20
constexpr int32_t kOffBias = 1 << (kOffBits - 1);

__global__ __launch_bounds__(256) void k_emit(int64_t nf, const int2* __restrict__ front,
                                              const int32_t* __restrict__ xijk, const int32_t* __restrict__ xch0,
                                              const int32_t* __restrict__ xnch, const int32_t* __restrict__ yijk,
                                              const int32_t* __restrict__ ych0, const int32_t* __restrict__ ynch,
                                              const int32_t* __restrict__ is_m2l, const int32_t* __restrict__ m_pos,
                                              const int32_t* __restrict__ is_p2p, const int32_t* __restrict__ p_pos,
                                              const int64_t* __restrict__ n_next, const int64_t* __restrict__ x_pos,
                                              int2* __restrict__ m2l, uint64_t* __restrict__ mkey,
                                              int2* __restrict__ p2p, int2* __restrict__ next,
                                              int32_t* __restrict__ overflow) {
  int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= nf) return;
  int32_t t = front[i].x, s = front[i].y;
  if (is_m2l[i]) {
    int32_t r = m_pos[i];
    m2l[r] = make_int2(t, s);
    uint64_t k = 0;
    for (int d = 0; d < 3; ++d) {
      int32_t v = xijk[3 * t + d] - yijk[3 * s + d];
      if (v <= -kOffBias || v >= kOffBias) overflow[0] = 1;
      k = (k << kOffBits) | (uint64_t)(uint32_t)((v + kOffBias) & ((1 << kOffBits) - 1));
    }
    mkey[r] = k;
  } else if (is_p2p[i]) {
    p2p[p_pos[i]] = make_int2(t, s);
  } else if (n_next[i] > 0) {
    int64_t q = x_pos[i];
    int32_t nc = ynch[s];
    for (int a = 0; a < xnch[t]; ++a)
      for (int c = 0; c < nc; ++c) next[q++] = make_int2(xch0[t] + a, ych0[s] + c);
  }
}

// Offset id of each M2L pair of the level: base + rank of its key among the
// level's distinct keys (sorted).
__global__ __launch_bounds__(256) void k_offset_ids(int64_t m, const uint64_t* __restrict__ mkey,
                                                    const uint64_t* __restrict__ uniq, int64_t nu, int32_t base,
                                                    int32_t* __restrict__ ids) {
  int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= m) return;
  uint64_t k = mkey[i];
  int64_t lo = 0, hi = nu;
  while (lo < hi) {
    int64_t mid = (lo + hi) / 2;
    if (uniq[mid] < k) lo = mid + 1;
    else hi = mid;
  }
  ids[i] = base + (int32_t)lo;
}

struct LevelPairs {  // M2L pairs of one level, kept on the device for the marks
  int lev = 0;
  int64_t m = 0;
  DVec<int2> ts;
  DVec<int32_t> off;
};

void traverse_device(HostPlan& hp, const DevCells& X, const DevCells& Y, hipStream_t s, Temp& tmp,
                     std::vector<LevelPairs>& keep) {
  DVec<int2> front(1);
  {
    std::vector<int2> root = {make_int2(0, 0)};
    to_device(front, root, s);
  }
  int64_t nf = 1;
  DVec<int32_t> overflow(1);
  chk(hipMemsetAsync(overflow.p, 0, sizeof(int32_t), s), "overflow flag");
  for (int lev = 0; nf > 0; ++lev) {
    if (lev > kMaxLevel) throw std::runtime_error("device builder: traversal deeper than the tree");
    DVec<int32_t> is_m(nf), m_pos(nf), is_p(nf), p_pos(nf);
    DVec<int64_t> n_next(nf), x_pos(nf);
    hipLaunchKernelGGL(k_classify, dim3(grid_for(nf, 256)), dim3(256), 0, s, nf, front.p, X.ijk.p, X.leaf.p,
                       X.nchild.p, Y.ijk.p, Y.leaf.p, Y.nchild.p, hp.thr[lev], is_m.p, is_p.p, n_next.p);
    chk(hipGetLastError(), "classify launch");
    const int64_t nm = scan_total<int32_t>(tmp, is_m.p, m_pos.p, nf, s);
    const int64_t np = scan_total<int32_t>(tmp, is_p.p, p_pos.p, nf, s);
    const int64_t nn = scan_total<int64_t>(tmp, n_next.p, x_pos.p, nf, s);
    if (nn > (int64_t)INT32_MAX) throw std::runtime_error("device builder: traversal frontier too large");
    LevelPairs lp;
    lp.lev = lev;
    lp.m = nm;
    lp.ts.resize(nm);
    DVec<uint64_t> mkey(nm);
    DVec<int2> p2p(np), next(nn);
    hipLaunchKernelGGL(k_emit, dim3(grid_for(nf, 256)), dim3(256), 0, s, nf, front.p, X.ijk.p, X.child0.p,
                       X.nchild.p, Y.ijk.p, Y.child0.p, Y.nchild.p, is_m.p, m_pos.p, is_p.p, p_pos.p, n_next.p,
                       x_pos.p, lp.ts.p, mkey.p, p2p.p, next.p, overflow.p);
    chk(hipGetLastError(), "emit launch");
    if (read_one(overflow.p, s)) throw std::runtime_error("device builder: M2L offset beyond 2^20 cells");
    if (nm > 0) {
      // distinct offsets of this level, ids in key order
      DVec<uint64_t> sorted(nm), uniq(nm);
      DVec<int64_t> nu_d(1);
      size_t bytes = 0;
      chk(rocprim::radix_sort_keys(nullptr, bytes, mkey.p, sorted.p, (size_t)nm, 0u, 3u * kOffBits, s), "key sort");
      chk(rocprim::radix_sort_keys(tmp.get(bytes), bytes, mkey.p, sorted.p, (size_t)nm, 0u, 3u * kOffBits, s),
          "key sort");
      bytes = 0;
      chk(rocprim::unique(nullptr, bytes, sorted.p, uniq.p, nu_d.p, (size_t)nm, rocprim::equal_to<uint64_t>(), s),
          "unique size");
      chk(rocprim::unique(tmp.get(bytes), bytes, sorted.p, uniq.p, nu_d.p, (size_t)nm, rocprim::equal_to<uint64_t>(),
                          s),
          "unique");
      const int64_t nu = read_one(nu_d.p, s);
      const int32_t base = (int32_t)hp.offsets.size();
      lp.off.resize(nm);
      hipLaunchKernelGGL(k_offset_ids, dim3(grid_for(nm, 256)), dim3(256), 0, s, nm, mkey.p, uniq.p, nu, base,
                         lp.off.p);
      chk(hipGetLastError(), "offset ids launch");
      std::vector<uint64_t> hu;
      to_host(hu, uniq.p, nu, s);
      for (uint64_t k : hu) {
        Offset o;
        o.level = lev;
        for (int d = 2; d >= 0; --d) {
          o.d[d] = (int32_t)(k & ((1u << kOffBits) - 1)) - kOffBias;
          k >>= kOffBits;
        }
        o.dir = -1;
        hp.offsets.push_back(o);
      }
      std::vector<int2> hts;
      std::vector<int32_t> hoff;
      to_host(hts, lp.ts.p, nm, s);
      to_host(hoff, lp.off.p, nm, s);
      for (int64_t i = 0; i < nm; ++i) hp.m2l.push_back({hts[i].x, hts[i].y, hoff[i]});
    }
    if (np > 0) {
      std::vector<int2> hp2;
      to_host(hp2, p2p.p, np, s);
      for (const int2& v : hp2) {
        hp.p2p_t.push_back(v.x);
        hp.p2p_s.push_back(v.y);
      }
    }
    if (nm > 0) keep.push_back(std::move(lp));
    front = std::move(next);
    nf = nn;
  }
}

// ------------------------------------------------------------------ directions
// Best direction of each offset of a high-frequency level: the maximum of
// <v, offset> over the level's directions, and among the directions within
// 1e-12 |offset| of it the lowest index.
__global__ __launch_bounds__(256) void k_best_dir(int64_t n, const int32_t* __restrict__ od,
                                                  const int64_t* __restrict__ vbase, const int64_t* __restrict__ nv,
                                                  const double* __restrict__ dirs, int32_t* __restrict__ out) {
  int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  if (nv[i] <= 0) {
    out[i] = -1;
    return;
  }
  const double dd[3] = {(double)od[3 * i], (double)od[3 * i + 1], (double)od[3 * i + 2]};
  const double* V = dirs + 3 * vbase[i];
  double best = -1e300;
  for (int64_t u = 0; u < nv[i]; ++u) {
    double sc = V[3 * u] * dd[0] + V[3 * u + 1] * dd[1] + V[3 * u + 2] * dd[2];
    if (sc > best) best = sc;
  }
  double tol = 1e-12 * sqrt(dd[0] * dd[0] + dd[1] * dd[1] + dd[2] * dd[2]);
  int32_t r = 0;
  for (int64_t u = 0; u < nv[i]; ++u) {
    double sc = V[3 * u] * dd[0] + V[3 * u + 1] * dd[1] + V[3 * u + 2] * dd[2];
    if (sc >= best - tol) {
      r = (int32_t)u;
      break;
    }
  }
  out[i] = r;
}

void best_directions_device(HostPlan& hp, hipStream_t s) {
  const int64_t n = (int64_t)hp.offsets.size();
  if (n == 0) return;
  std::vector<int32_t> od(3 * n);
  std::vector<int64_t> vb(n, 0), nv(n, 0);
  for (int64_t i = 0; i < n; ++i) {
    const Offset& o = hp.offsets[i];
    for (int d = 0; d < 3; ++d) od[3 * i + d] = o.d[d];
    if (hp.hf[o.level]) {
      int E = dir_level(hp, o.level);
      vb[i] = hp.dir_off[E];
      nv[i] = num_directions(E);
    }
  }
  DVec<int32_t> d_od, d_out(n);
  DVec<int64_t> d_vb, d_nv;
  DVec<double> d_dirs;
  to_device(d_od, od, s);
  to_device(d_vb, vb, s);
  to_device(d_nv, nv, s);
  to_device(d_dirs, hp.dirs, s);
  hipLaunchKernelGGL(k_best_dir, dim3(grid_for(n, 256)), dim3(256), 0, s, n, d_od.p, d_vb.p, d_nv.p, d_dirs.p,
                     d_out.p);
  chk(hipGetLastError(), "best direction launch");
  std::vector<int32_t> h;
  to_host(h, d_out.p, n, s);
  for (int64_t i = 0; i < n; ++i) hp.offsets[i].dir = h[i];
}

// ------------------------------------------------------------------ marks
// Per level l of a tree: a flag per (cell, direction), nd(l) = number of
// directions of an HF level or 1 (the non-directional mark) for an LF level.
struct MarkLevels {
  std::vector<DVec<unsigned char>> flag;
  std::vector<int64_t> nd;
};

__global__ __launch_bounds__(256) void k_mark_own(int64_t m, const int2* __restrict__ ts,
                                                  const int32_t* __restrict__ off,
                                                  const int32_t* __restrict__ off_dir, int side, int64_t base,
                                                  int64_t nd, unsigned char* __restrict__ flag) {
  int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= m) return;
  int32_t c = side == 0 ? ts[i].x : ts[i].y;
  int32_t u = off_dir[off[i]];
  flag[(c - base) * nd + (u < 0 ? 0 : u)] = 1;
}

// Blank downward pass: every son of a marked non-leaf cell gets Father(u)
// (directional son level) or the non-directional mark.
__global__ __launch_bounds__(256) void k_mark_down(int64_t m, int64_t nd, const unsigned char* __restrict__ flag,
                                                   int64_t base, const int32_t* __restrict__ leaf,
                                                   const int32_t* __restrict__ child0,
                                                   const int32_t* __restrict__ nchild, int64_t next_base,
                                                   int64_t nd_next, int son_hf, const int64_t* __restrict__ father,
                                                   unsigned char* __restrict__ next_flag) {
  int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= m * nd || !flag[i]) return;
  int64_t c = i / nd, u = i % nd;
  if (leaf[base + c]) return;
  int64_t v = son_hf ? father[u] : 0;
  if (v < 0 || v >= nd_next) return;
  for (int a = 0; a < nchild[base + c]; ++a) next_flag[(child0[base + c] + a - next_base) * nd_next + v] = 1;
}

__global__ __launch_bounds__(256) void k_mark_count(int64_t m, int64_t nd, const unsigned char* __restrict__ flag,
                                                    int64_t* __restrict__ cnt) {
  int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (c >= m) return;
  int64_t k = 0;
  for (int64_t u = 0; u < nd; ++u) k += flag[c * nd + u];
  cnt[c] = k;
}

__global__ __launch_bounds__(256) void k_mark_write(int64_t m, int64_t nd, int hf,
                                                    const unsigned char* __restrict__ flag, int64_t base,
                                                    const int64_t* __restrict__ pos, int32_t* __restrict__ edir,
                                                    int32_t* __restrict__ ecell) {
  int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (c >= m) return;
  int64_t q = pos[c];
  for (int64_t u = 0; u < nd; ++u)
    if (flag[c * nd + u]) {
      edir[q] = hf ? (int32_t)u : -1;
      ecell[q] = (int32_t)(base + c);
      ++q;
    }
}

void marks_device(HostPlan& hp, Tree& T, const DevCells& C, const std::vector<LevelPairs>& pairs, int side,
                  bool both_sides, hipStream_t s, Temp& tmp) {
  const int nl = T.nlevels;
  MarkLevels mk;
  mk.flag.resize(nl);
  mk.nd.assign(nl, 0);
  int lmin = nl;
  for (const LevelPairs& lp : pairs) lmin = std::min(lmin, lp.lev);
  for (int l = lmin; l < nl; ++l) {
    mk.nd[l] = hp.hf[l] ? num_directions(dir_level(hp, l)) : 1;
    const int64_t m = T.lev_start[l + 1] - T.lev_start[l];
    mk.flag[l].resize((size_t)(m * mk.nd[l]));
    if (mk.flag[l].n) chk(hipMemsetAsync(mk.flag[l].p, 0, mk.flag[l].n, s), "flags");
  }
  std::vector<int32_t> odir(hp.offsets.size());
  for (size_t i = 0; i < odir.size(); ++i) odir[i] = hp.offsets[i].dir;
  DVec<int32_t> d_odir;
  to_device(d_odir, odir, s);
  for (const LevelPairs& lp : pairs) {
    const int l = lp.lev;
    if (l >= nl) throw std::runtime_error("device builder: M2L level beyond the tree");
    for (int sd = 0; sd < 2; ++sd) {
      if (!both_sides && sd != side) continue;
      hipLaunchKernelGGL(k_mark_own, dim3(grid_for(lp.m, 256)), dim3(256), 0, s, lp.m, lp.ts.p, lp.off.p, d_odir.p,
                         sd, T.lev_start[l], mk.nd[l], mk.flag[l].p);
      chk(hipGetLastError(), "mark launch");
    }
  }
  DVec<int64_t> d_father;
  to_device(d_father, hp.father_flat, s);
  for (int l = lmin; l + 1 < nl; ++l) {
    const int64_t m = T.lev_start[l + 1] - T.lev_start[l];
    const int64_t tot = m * mk.nd[l];
    if (tot == 0) continue;
    const int64_t* fa = hp.hf[l + 1] ? d_father.p + hp.dir_off[dir_level(hp, l)] : nullptr;
    hipLaunchKernelGGL(k_mark_down, dim3(grid_for(tot, 256)), dim3(256), 0, s, m, mk.nd[l], mk.flag[l].p,
                       T.lev_start[l], C.leaf.p, C.child0.p, C.nchild.p, T.lev_start[l + 1], mk.nd[l + 1],
                       hp.hf[l + 1], fa, mk.flag[l + 1].p);
    chk(hipGetLastError(), "mark down launch");
  }
  const int64_t nc = T.ncells();
  DVec<int64_t> cnt(nc), pos(nc);
  if (nc > 0) chk(hipMemsetAsync(cnt.p, 0, nc * sizeof(int64_t), s), "mark counts");
  for (int l = lmin; l < nl; ++l) {
    const int64_t m = T.lev_start[l + 1] - T.lev_start[l];
    if (m == 0) continue;
    hipLaunchKernelGGL(k_mark_count, dim3(grid_for(m, 256)), dim3(256), 0, s, m, mk.nd[l], mk.flag[l].p,
                       cnt.p + T.lev_start[l]);
    chk(hipGetLastError(), "mark count launch");
  }
  const int64_t ne = scan_total<int64_t>(tmp, cnt.p, pos.p, nc, s);
  DVec<int32_t> edir(ne), ecell(ne);
  for (int l = lmin; l < nl; ++l) {
    const int64_t m = T.lev_start[l + 1] - T.lev_start[l];
    if (m == 0) continue;
    hipLaunchKernelGGL(k_mark_write, dim3(grid_for(m, 256)), dim3(256), 0, s, m, mk.nd[l], hp.hf[l], mk.flag[l].p,
                       T.lev_start[l], pos.p + T.lev_start[l], edir.p, ecell.p);
    chk(hipGetLastError(), "mark write launch");
  }
  std::vector<int64_t> hpos;
  to_host(hpos, pos.p, nc, s);
  T.exp_begin.assign(nc + 1, 0);
  for (int64_t c = 0; c < nc; ++c) T.exp_begin[c] = hpos[c];
  T.exp_begin[nc] = ne;
  to_host(T.exp_dir, edir.p, ne, s);
  to_host(T.exp_cell, ecell.p, ne, s);
  set_expansion_directions(hp, T);
}

}  // namespace

bool build_device_plan(HostPlan& hp, const double* X, int64_t nx, const double* Y, int64_t ny,
                       const BuildParams& prm, hipStream_t s) {
  hp.prm = prm;
  const double* Yp = prm.same_points ? X : Y;
  if (prm.same_points) ny = nx;
  struct StreamScope {
    hipStream_t prev;
    explicit StreamScope(hipStream_t st) : prev(g_stream) { g_stream = st; }
    ~StreamScope() {
      (void)hipStreamSynchronize(g_stream);
      g_stream = prev;
    }
  } scope(s);
  Temp tmp;
  double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
  bool ok = bbox(X, nx, lo, hi, s);
  if (!prm.same_points) ok = bbox(Yp, ny, lo, hi, s) && ok;
  if (!ok) return false;
  set_geometry(hp, lo, hi, nx + (prm.same_points ? 0 : ny) > 0);
  build_tree_device(hp.tx, X, nx, hp.origin, hp.D, prm.ncrit, s, tmp);
  if (prm.same_points) {
    hp.ty = &hp.tx;
  } else {
    build_tree_device(hp.ty_own, Yp, ny, hp.origin, hp.D, prm.ncrit, s, tmp);
    hp.ty = &hp.ty_own;
  }
  set_regimes(hp);
  DevCells cx, cy;
  upload_cells(cx, hp.tx, s);
  if (!prm.same_points) upload_cells(cy, hp.ty_own, s);
  const DevCells& CY = prm.same_points ? cx : cy;
  std::vector<LevelPairs> pairs;
  if (nx > 0 && ny > 0) traverse_device(hp, cx, CY, s, tmp, pairs);
  make_direction_tables(hp);
  best_directions_device(hp, s);
  if (prm.same_points) {
    marks_device(hp, hp.tx, cx, pairs, 0, true, s, tmp);
  } else {
    marks_device(hp, hp.tx, cx, pairs, 0, false, s, tmp);
    marks_device(hp, hp.ty_own, cy, pairs, 1, false, s, tmp);
  }
  pairs.clear();
  build_tables(hp);
  return true;
}

}  // namespace defmm
