// HIP kernels of the defmm matvec for gfx950 (wave64) and their launchers.
//
// One matvec (Sec. 2.2 operators, Sec. 4.1.1 Fourier-domain M2L):
//   gather q -> P2M (source leaves) -> M2M (sons to fathers, level by level)
//   -> M2F (pruned 3D DFT of each zero-padded multipole grid)
//   -> M2L: per target expansion, Hadamard accumulate over its interaction
//      list, then F2L (pruned inverse DFT, restricted to the L^3 grid)
//   -> L2L (fathers to sons) -> P2P (near field) + L2P -> scatter p.
// Every output element is owned by one thread: no atomics, results are
// bitwise reproducible run to run.
//
// Precision: R = float (complex64 path) or double (complex128 path).  Phase
// arguments kappa*<d,u> are formed in FP64 from differences of points of the
// same cell and reduced modulo 2 pi in FP64 before a float sincos.
#include <hip/hip_runtime.h>

#include <cmath>
#include <algorithm>
#include <cstdio>
#include <type_traits>

#include "device.hpp"

namespace defmm {

template <typename R>
struct C2 {
  R x, y;
};

// two adjacent complex entries, moved as one 16- or 32-byte access
template <typename R>
struct alignas(2 * sizeof(C2<R>)) C2x2 {
  C2<R> a, b;
};

template <typename R>
__device__ __forceinline__ C2<R> cmul(C2<R> a, C2<R> b) {
  return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}

template <typename R>
__device__ __forceinline__ void cfma(C2<R>& acc, C2<R> a, C2<R> b) {
  acc.x = fma(a.x, b.x, fma(-a.y, b.y, acc.x));
  acc.y = fma(a.x, b.y, fma(a.y, b.x, acc.y));
}

// acc += a * w for a real weight w (two multiply-adds, not four).
template <typename R>
__device__ __forceinline__ void cfma_r(C2<R>& acc, C2<R> a, R w) {
  acc.x = fma(a.x, w, acc.x);
  acc.y = fma(a.y, w, acc.y);
}

template <typename R>
__device__ __forceinline__ C2<R> cscale(C2<R> a, R s) {
  return {a.x * s, a.y * s};
}

// sin and cos of 2 pi t for t in turns, FP64: reduction to the nearest
// quarter turn q/4 (g = t - q/4 in [-1/8, 1/8], exact), x = 2 pi g, the Taylor
// series of sin x to x^17 and of cos x to x^18 (truncation below 1e-19 for
// |x| <= pi/4), then the rotation by q quarter turns.
__device__ __forceinline__ void sincos_turns(double t, double& s, double& c) {
  constexpr double S[9] = {1.0, -1.0 / 6.0, 1.0 / 120.0, -1.0 / 5040.0, 1.0 / 362880.0, -1.0 / 39916800.0,
                           1.0 / 6227020800.0, -1.0 / 1307674368000.0, 1.0 / 355687428096000.0};
  constexpr double C[10] = {1.0, -1.0 / 2.0, 1.0 / 24.0, -1.0 / 720.0, 1.0 / 40320.0, -1.0 / 3628800.0,
                            1.0 / 479001600.0, -1.0 / 87178291200.0, 1.0 / 20922789888000.0,
                            -1.0 / 6402373705728000.0};
  const double q = rint(4.0 * t);
  const double x = (t - 0.25 * q) * 6.283185307179586477;
  const double x2 = x * x;
  double ps = S[8], pc = C[9];
#pragma unroll
  for (int k = 7; k >= 0; --k) ps = fma(ps, x2, S[k]);
#pragma unroll
  for (int k = 8; k >= 0; --k) pc = fma(pc, x2, C[k]);
  const double sn = ps * x;
  const int qi = (int)((long long)q & 3);
  s = (qi & 1) ? pc : sn;
  c = (qi & 1) ? -sn : pc;
  if (qi & 2) {
    s = -s;
    c = -c;
  }
}

// exp(i a) for an FP64 argument a (radians), through turns t = a / (2 pi):
// sincos_turns (complex128), or t reduced in FP64 to its fraction of a turn
// and passed to v_sin_f32 / v_cos_f32, which take turns (complex64).
template <typename R>
__device__ __forceinline__ C2<R> expi(double a);

template <>
__device__ __forceinline__ C2<double> expi<double>(double a) {
  double s, c;
  sincos_turns(a * 0.15915494309189533577, s, c);
  return {c, s};
}

template <>
__device__ __forceinline__ C2<float> expi<float>(double a) {
  const double t = a * 0.15915494309189533577;
  const float f = (float)(t - rint(t));
  return {__builtin_amdgcn_cosf(f), __builtin_amdgcn_sinf(f)};
}

// exp(i 2 pi t) from FP64 turns t, reduced in FP64 (the phases of P2M, M2M
// and L2L, whose arguments are formed in turns).
template <typename R>
__device__ __forceinline__ C2<R> expi_turns(double t);
template <>
__device__ __forceinline__ C2<float> expi_turns<float>(double t) {
  const float f = (float)(t - rint(t));
  return {__builtin_amdgcn_cosf(f), __builtin_amdgcn_sinf(f)};
}
template <>
__device__ __forceinline__ C2<double> expi_turns<double>(double t) {
  double s, c;
  sincos_turns(t, s, c);
  return {c, s};
}

// 1 / prod_{j != m} (m - j) for the L equispaced nodes: the constant factor
// of the Lagrange basis polynomial of node m (computed in FP64 at compile time).
template <int L>
struct LagrangeScale {
  double c[L];
  constexpr LagrangeScale() : c() {
    for (int m = 0; m < L; ++m) {
      double d = 1.0;
      for (int j = 0; j < L; ++j)
        if (j != m) d *= (double)(m - j);
      c[m] = 1.0 / d;
    }
  }
};

// Lagrange basis on the L equispaced nodes j/(L-1) of [0,1] (Sec. 2.3):
// l_m(t) = c_m prod_{j != m} (s - j), s = (L-1) t, with c_m a compile-time
// constant (no division at run time).
template <typename R, int L>
__device__ __forceinline__ void lagrange(R t, R* w) {
  constexpr LagrangeScale<L> C{};
  R s = t * (R)(L - 1);
#pragma unroll
  for (int m = 0; m < L; ++m) {
    R v = (R)C.c[m];
#pragma unroll
    for (int j = 0; j < L; ++j)
      if (j != m) v *= (s - (R)j);
    w[m] = v;
  }
}

constexpr int round64(int x) { return ((x + 63) / 64) * 64; }

// Row stride of the Fourier-domain arrays (spectra, M~, L~): fourier_row(L),
// in the order of the Fourier layout; padding entries hold zeros (spectra,
// M~) or are never read back (L~).

// XCD-aware block order: the hardware deals consecutive workgroups to the 8
// XCDs round-robin; remap so each XCD walks a contiguous range of items and
// neighbours in Morton order share that XCD's L2.
__device__ __forceinline__ int64_t xcd_item(int64_t n) {
  int64_t nper = (n + 7) / 8;
  int64_t b = blockIdx.x;
  return (b % 8) * nper + b / 8;
}

static inline unsigned xcd_grid(int64_t n) { return (unsigned)(8 * ((n + 7) / 8)); }

// Persistent M2F grid: 4 workgroups per CU (what the LDS holds at 4
// expansions per workgroup, and the registers at fewer), a multiple of 8, no
// more than the chunks need.
static inline unsigned fourier_grid(int64_t nchunk, int num_cu) {
  return xcd_grid(std::min<int64_t>(nchunk, (int64_t)num_cu * 4));
}

// Work item (slice, i) of nsl frequency slices x n items, in slice-major
// order through xcd_item: each XCD walks a contiguous share of the list, so
// its L2 holds one slice (two at a share boundary) of the rows its items
// touch.  Launch xcd_grid(nsl * n) blocks; false for the padding blocks.
__device__ __forceinline__ bool slice_item(int nsl, int64_t n, int& slice, int64_t& i) {
  const int64_t w = xcd_item((int64_t)nsl * n);
  if (w >= (int64_t)nsl * n) return false;
  slice = (int)(w / n);
  i = w % n;
  return true;
}

// Persistent XCD-aware walk over n items: with a grid that is a multiple of
// 8, block b runs on XCD b % 8 and takes items first, first + step, ... < end
// of that XCD's contiguous share.
struct XcdWalk {
  int64_t first, end, step;
};
__device__ __forceinline__ XcdWalk xcd_walk(int64_t n) {
  const int64_t nper = (n + 7) / 8, x = blockIdx.x % 8;
  return {x * nper + blockIdx.x / 8, min(n, (x + 1) * nper), (int64_t)(gridDim.x / 8)};
}

struct TreeView {
  int64_t n;
  const double* soa;
  const int32_t* level;
  const int32_t* ijk;
  const int32_t* first;
  const int32_t* count;
  const int32_t* exp_begin;
  const int32_t* exp_cell;
  const double* exp_u;
};

static TreeView view(const DevTree& t) {
  return {t.n, t.soa, t.level, t.ijk, t.first, t.count, t.exp_begin, t.exp_cell, t.exp_u};
}

struct Geo {
  double kappa, D, ox, oy, oz;
};

// ------------------------------------------------------------------ elementwise
template <typename R>
__global__ void k_gather(int64_t n, const int32_t* __restrict__ perm, const C2<R>* __restrict__ q,
                         C2<R>* __restrict__ qs) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) qs[i] = q[perm[i]];
}

template <typename R>
__global__ void k_scatter(int64_t n, const int32_t* __restrict__ perm, const C2<R>* __restrict__ ps,
                          C2<R>* __restrict__ p) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[perm[i]] = ps[i];
}

template <typename R>
__global__ void k_zero(int64_t n, C2<R>* __restrict__ a) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) a[i] = {(R)0, (R)0};
}

// Clears rows of LEN values: row rows[i] of a, for i < n.  A workgroup clears
// kZeroRowsPerBlock consecutive rows of the list, consecutive threads on
// consecutive values (a row's index divides by a compile-time length).
constexpr int kZeroRowsPerBlock = 8;
template <typename R, int LEN>
__global__ __launch_bounds__(256) void k_zero_rows(int64_t n, const int32_t* __restrict__ rows,
                                                   C2<R>* __restrict__ a) {
  const int64_t r0 = (int64_t)blockIdx.x * kZeroRowsPerBlock;
  for (int k = threadIdx.x; k < kZeroRowsPerBlock * LEN; k += 256) {
    const int q = k / LEN, c = k - q * LEN;
    if (r0 + q < n) a[(int64_t)rows[r0 + q] * LEN + c] = {(R)0, (R)0};
  }
}

// ------------------------------------------------------------------ spectra
// The kernel G(r) in FP64: exp(i kappa r) / (4 pi r), or, screened,
// exp(-kappa r) / (4 pi r).
__device__ __forceinline__ C2<double> kernel_fp64(double r, double kappa, int screened) {
  const double g = 1.0 / (4.0 * M_PI * r);
  if (screened) return {exp(-kappa * r) * g, 0.0};
  double s, c;
  sincos(kappa * r, &s, &c);
  return {c * g, s * g};
}

// Fourier-domain M2L diagonal (eq. FourierDiagonal) for each canonical
// (level, delta): the kernel on the (2L-1)^3 difference grid (eq.
// CirculantKernel), a 3D DFT in FP64, scaled by 1/P^3 so that F2L is a plain
// inverse sum, in the order of the Fourier layout (freq).  With nrow = 2
// (compressed spectra) a second row holds the two members of every pair
// exchanged, so that a permuted read never swaps values after the load.
template <typename R, int L>
__global__ __launch_bounds__(256) void k_spectra(int64_t n, const int32_t* __restrict__ lev,
                                                 const int32_t* __restrict__ delta, double kappa, int screened,
                                                 double D, const int32_t* __restrict__ freq, int nrow,
                                                 C2<R>* __restrict__ S) {
  constexpr int P = 2 * L - 1, P3 = P * P * P;
  __shared__ C2<double> a[P3];
  __shared__ C2<double> W[P];
  int64_t o = blockIdx.x;
  if (o >= n) return;
  int tid = threadIdx.x;
  double h = ldexp(D, -lev[o]);
  double dx = delta[3 * o], dy = delta[3 * o + 1], dz = delta[3 * o + 2];
  if (tid < P) {
    double s, c;
    sincospi(-2.0 * (double)tid / (double)P, &s, &c);
    W[tid] = {c, s};
  }
  for (int i = tid; i < P3; i += blockDim.x) {
    int m0 = i % P, m1 = (i / P) % P, m2 = i / (P * P);
    int j0 = m0 <= L - 1 ? m0 : m0 - P;
    int j1 = m1 <= L - 1 ? m1 : m1 - P;
    int j2 = m2 <= L - 1 ? m2 : m2 - P;
    double z0 = h * dx + (h / (double)(L - 1)) * (double)j0;
    double z1 = h * dy + (h / (double)(L - 1)) * (double)j1;
    double z2 = h * dz + (h / (double)(L - 1)) * (double)j2;
    a[i] = kernel_fp64(sqrt(z0 * z0 + z1 * z1 + z2 * z2), kappa, screened);
  }
  __syncthreads();
  const int stride[3] = {1, P, P * P};
#pragma unroll 1
  for (int d = 0; d < 3; ++d) {
    for (int line = tid; line < P * P; line += blockDim.x) {
      int base;
      if (d == 0) base = line * P;
      else if (d == 1) base = (line % P) + (line / P) * P * P;
      else base = line;
      C2<double> in[P];
#pragma unroll
      for (int m = 0; m < P; ++m) in[m] = a[base + m * stride[d]];
#pragma unroll
      for (int k = 0; k < P; ++k) {
        C2<double> acc = {0.0, 0.0};
#pragma unroll
        for (int m = 0; m < P; ++m) cfma(acc, in[m], W[(k * m) % P]);
        a[base + k * stride[d]] = acc;
      }
    }
    __syncthreads();
  }
  const double scale = 1.0 / (double)P3;
  for (int p = tid; p < nrow * fourier_row(L); p += blockDim.x) {
    const int q = p < fourier_row(L) ? p : (p - fourier_row(L)) ^ 1;
    const int f = freq[q];
    S[nrow * o * fourier_row(L) + p] = f >= 0 ? C2<R>{(R)(a[f].x * scale), (R)(a[f].y * scale)} : C2<R>{(R)0, (R)0};
  }
}

// ------------------------------------------------------------------ P2M
// M^u(y_r) = exp(ik<y_r - a, u>) sum_y S_r(y) exp(-ik<y - a, u>) q(y): the
// phases split at the cell corner a, one thread per node r.
template <typename R, int L>
__global__ __launch_bounds__(round64(L* L* L)) void k_p2m(int64_t n, const int32_t* __restrict__ exps,
                                                         TreeView T, Geo g, const C2<R>* __restrict__ qs,
                                                         C2<R>* __restrict__ M) {
  constexpr int L3 = L * L * L, PT = 64;
  __shared__ R w[PT][3][L];
  __shared__ C2<R> qq[PT];
  int64_t item = blockIdx.x;
  if (item >= n) return;
  int e = exps[item];
  int c = T.exp_cell[e];
  double h = ldexp(g.D, -T.level[c]);
  double ax = g.ox + h * T.ijk[3 * c], ay = g.oy + h * T.ijk[3 * c + 1], az = g.oz + h * T.ijk[3 * c + 2];
  double ux = T.exp_u[3 * e], uy = T.exp_u[3 * e + 1], uz = T.exp_u[3 * e + 2];
  int first = T.first[c], cnt = T.count[c];
  int tid = threadIdx.x;
  int rx = tid % L, ry = (tid / L) % L, rz = tid / (L * L);
  C2<R> acc = {(R)0, (R)0};
  for (int base = 0; base < cnt; base += PT) {
    int j = base + tid;
    if (tid < PT && j < cnt) {
      int64_t pi = first + j;
      double d0 = T.soa[pi] - ax, d1 = T.soa[T.n + pi] - ay, d2 = T.soa[2 * T.n + pi] - az;
      lagrange<R, L>((R)(d0 / h), w[tid][0]);
      lagrange<R, L>((R)(d1 / h), w[tid][1]);
      lagrange<R, L>((R)(d2 / h), w[tid][2]);
      qq[tid] = cmul(qs[pi], expi<R>(-g.kappa * (ux * d0 + uy * d1 + uz * d2)));
    }
    __syncthreads();
    int m = min(PT, cnt - base);
    if (tid < L3)
      for (int k = 0; k < m; ++k) cfma_r(acc, qq[k], w[k][0][rx] * w[k][1][ry] * w[k][2][rz]);
    __syncthreads();
  }
  if (tid < L3) {
    double arg = g.kappa * h / (double)(L - 1) * (ux * rx + uy * ry + uz * rz);
    M[(int64_t)e * L3 + tid] = cmul(acc, expi<R>(arg));
  }
}

// P2M per leaf: the workgroup of a source leaf computes, for a chunk of up to
// PT points, the weights S_r(y) once (one per node and point, held in
// registers) and then serves every expansion u of the leaf:
// M^u(y_r) = exp(ik<y_r - a, u>) sum_y S_r(y) [exp(-ik<y - a, u>) q(y)].
template <typename R, int L>
__global__ __launch_bounds__(round64(L* L* L)) void k_p2m_leaf(int64_t n, const int32_t* __restrict__ leaf,
                                                              TreeView T, Geo g, const C2<R>* __restrict__ qs,
                                                              C2<R>* __restrict__ M) {
  constexpr int L3 = L * L * L, PT = sizeof(R) == 4 ? 64 : 32;
  constexpr double inv2pi = 0.15915494309189533577;
  __shared__ R w[PT][3][L];
  __shared__ double dd[PT][3];
  __shared__ C2<R> qv[PT];
  __shared__ C2<R> qq[PT];
  const int64_t item = blockIdx.x;
  if (item >= n) return;
  const int c = leaf[item];
  const double h = ldexp(g.D, -T.level[c]);
  const double ax = g.ox + h * T.ijk[3 * c], ay = g.oy + h * T.ijk[3 * c + 1], az = g.oz + h * T.ijk[3 * c + 2];
  const int first = T.first[c], cnt = T.count[c];
  const int e0 = T.exp_begin[c], e1 = T.exp_begin[c + 1];
  const int tid = threadIdx.x;
  const int tn = tid < L3 ? tid : L3 - 1;  // padding threads read a valid node
  const int rx = tn % L, ry = (tn / L) % L, rz = tn / (L * L);
  const int nch = (cnt + PT - 1) / PT;
  R W[PT];
  int m = 0;
  auto load_chunk = [&](int ch) {
    __syncthreads();
    const int j = ch * PT + tid;
    if (tid < PT && j < cnt) {
      const int64_t pi = first + j;
      const double d0 = T.soa[pi] - ax, d1 = T.soa[T.n + pi] - ay, d2 = T.soa[2 * T.n + pi] - az;
      lagrange<R, L>((R)(d0 / h), w[tid][0]);
      lagrange<R, L>((R)(d1 / h), w[tid][1]);
      lagrange<R, L>((R)(d2 / h), w[tid][2]);
      dd[tid][0] = d0;
      dd[tid][1] = d1;
      dd[tid][2] = d2;
      qv[tid] = qs[pi];
    }
    __syncthreads();
    m = min(PT, cnt - ch * PT);
#pragma unroll
    for (int k = 0; k < PT; ++k) W[k] = k < m ? w[k][0][rx] * w[k][1][ry] * w[k][2][rz] : (R)0;
  };
  if (nch == 1) load_chunk(0);
  for (int e = e0; e < e1; ++e) {
    const double ux = T.exp_u[3 * e], uy = T.exp_u[3 * e + 1], uz = T.exp_u[3 * e + 2];
    const double ku = g.kappa * inv2pi;
    C2<R> acc = {(R)0, (R)0};
    for (int ch = 0; ch < nch; ++ch) {
      if (nch > 1) load_chunk(ch);
      // entries past the chunk's points are zero
      if (tid < PT)
        qq[tid] = tid < m ? cmul(qv[tid], expi_turns<R>(-ku * (ux * dd[tid][0] + uy * dd[tid][1] + uz * dd[tid][2])))
                          : C2<R>{(R)0, (R)0};
      __syncthreads();
      // the chunk's points in blocks of 8, skipping the empty blocks (m is
      // uniform; leaves hold 18 points on average)
#pragma unroll
      for (int kb = 0; kb < PT; kb += 8) {
        if (kb >= m) break;
#pragma unroll
        for (int k = kb; k < kb + 8; ++k) cfma_r(acc, qq[k], W[k]);
      }
      __syncthreads();
    }
    if (tid < L3) {
      const double t = g.kappa * h / (double)(L - 1) * inv2pi * (ux * rx + uy * ry + uz * rz);
      M[(int64_t)e * L3 + tid] = cmul(acc, expi_turns<R>(t));
    }
  }
}

// Interpolation matrices between a cell and its sons (Sec. 5.2, tensorised
// M2M/L2L): A[b][l][r] = l_l((b + r/(L-1))/2), b = son half along an axis.
template <typename R, int L>
__device__ __forceinline__ void son_matrices(R (*A)[L][L]) {
  int tid = threadIdx.x;
  if (tid < 2 * L) {
    int b = tid / L, r = tid % L;
    R w[L];
    lagrange<R, L>(((R)b + (R)r / (R)(L - 1)) * (R)0.5, w);
#pragma unroll
    for (int l = 0; l < L; ++l) A[b][l][r] = w[l];
  }
}

// ------------------------------------------------------------------ pencil M2M / L2L
// Son matrices as compile-time constants: a[b][l][r] = l_l((b + r/(L-1))/2),
// the Lagrange basis of the father's nodes at the son's nodes (b = the son's
// half along the axis), in FP64.
template <int L>
struct SonMatrices {
  double a[2][L][L];
  constexpr SonMatrices() : a() {
    for (int b = 0; b < 2; ++b)
      for (int r = 0; r < L; ++r) {
        const double s = ((double)b + (double)r / (double)(L - 1)) * 0.5 * (double)(L - 1);
        for (int l = 0; l < L; ++l) {
          double v = 1.0;
          for (int j = 0; j < L; ++j)
            if (j != l) v *= (s - (double)j) / (double)(l - j);
          a[b][l][r] = v;
        }
      }
  }
};

// out[l] = sum_r w(l, r) in[r] along one axis with the son matrix of half B:
// w = a[B][l][r] (son to father, M2M) or a[B][r][l] (father to son, L2L).
// Zero weights (a node shared by father and son) are skipped at compile time.
template <typename R, int L, int B, bool TR>
__device__ __forceinline__ void son_mode(const C2<R> (&in)[L], C2<R> (&out)[L]) {
  constexpr SonMatrices<L> S{};
#pragma unroll
  for (int l = 0; l < L; ++l) {
    C2<R> acc = {(R)0, (R)0};
#pragma unroll
    for (int r = 0; r < L; ++r) {
      const R w = (R)(TR ? S.a[B][r][l] : S.a[B][l][r]);
      if (w != (R)0) cfma_r(acc, in[r], w);
    }
    out[l] = acc;
  }
}

template <typename R, int L, bool TR>
__device__ __forceinline__ void son_mode_b(int b, const C2<R> (&in)[L], C2<R> (&out)[L]) {
  if (b) son_mode<R, L, 1, TR>(in, out);
  else son_mode<R, L, 0, TR>(in, out);
}

// exp(i 2 pi (t0 + l dt)) for l < N: both turns reduced in FP64, the run by
// repeated rotation (N - 1 complex products in R), as along one pencil of a
// cell's nodes.
template <typename R, int N>
__device__ __forceinline__ void phase_run(double t0, double dt, C2<R> (&ph)[N]) {
  ph[0] = expi_turns<R>(t0);
  if constexpr (N > 1) {
    const C2<R> st = expi_turns<R>(dt);
#pragma unroll
    for (int l = 1; l < N; ++l) ph[l] = cmul(ph[l - 1], st);
  }
}

// Expansions (of one cell) per wave in the pencil kernels: two when a half
// wave holds the L^2 pencils of one expansion.
template <int L>
constexpr int pencil_epw() { return L * L <= 32 ? 2 : 1; }

// M2M by pencils (Sec. 5.2, eq. dlefturight, one father cell's expansions
// sharing a wave).  A wave serves up to two expansions v of one father cell;
// lane p < L^2 of a half holds pencil p.  For each son: the son's expansion
// Father(v) as x-pencils (r_y, r_z), the son-node phases exp(-i kappa <y'_r -
// a_s, v>) with FP64 arguments, and three mode products with the son matrices
// (x-, y- and z-pencils, exchanged through LDS), summed over sons; a mode
// matrix depends only on the son's half along its axis, so the sum is taken
// factor by factor (the x-mode results of sons differing only in x before
// their common y-mode product, and so on: 14 mode products for 8 sons instead
// of 24); then the father-node phases exp(i kappa <y_l - a_s, v>).
// Along a pencil the phases are one FP64-reduced turn and its step rotated
// L - 1 times (phase_run).
// Both expansions of a wave share the father cell, so its sons and their
// octants (which choose the matrices) are the same for every lane.
template <typename R, int L>
__global__ __launch_bounds__(64) void k_m2m_p(int64_t npair, const int32_t* __restrict__ pairs,
                                              const int32_t* __restrict__ par, const int32_t* __restrict__ child,
                                              const int8_t* __restrict__ oct, TreeView T, Geo g,
                                              C2<R>* __restrict__ M) {
  constexpr int L2 = L * L, L3 = L2 * L, EPW = pencil_epw<L>(), HW = 64 / EPW;
  __shared__ C2<R> st[EPW][L3];
  const int64_t w = blockIdx.x;
  if (w >= npair) return;
  const int lane = threadIdx.x, hf = lane / HW, p = lane % HW;
  const int item0 = pairs[EPW * w];
  const int item = EPW == 2 ? pairs[EPW * w + hf] : item0;
  const bool on = item >= 0 && p < L2;
  const int it = item >= 0 ? item : item0;
  const int pe = par[it];
  const int c = T.exp_cell[pe];
  const double h = ldexp(g.D, -T.level[c]), hc = 0.5 * h;
  const double v0 = T.exp_u[3 * pe], v1 = T.exp_u[3 * pe + 1], v2 = T.exp_u[3 * pe + 2];
  // turns per unit of son-node index along each axis, kappa hc v_d / ((L-1) 2 pi)
  constexpr double inv2pi = 0.15915494309189533577;
  const double ks = g.kappa * hc * inv2pi;
  const int a0 = p % L, a1 = (p / L) % L;  // (first, second) pencil coordinates
  C2<R> acc[L];
#pragma unroll
  for (int l = 0; l < L; ++l) acc[l] = {(R)0, (R)0};
  C2<R>* stg = st[hf];
  // the sons by octant o = bx + 2 by + 4 bz: whether present (the same for
  // both expansions of the wave) and this half's son expansion
  bool pres[8];
  int se[8];
  {
    int ce0s[8], ces[8], os[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      ce0s[k] = child[(int64_t)item0 * 8 + k];
      ces[k] = child[(int64_t)it * 8 + k];
      os[k] = oct[(int64_t)item0 * 8 + k];
    }
#pragma unroll
    for (int o = 0; o < 8; ++o) {
      pres[o] = false;
      se[o] = -1;
#pragma unroll
      for (int k = 0; k < 8; ++k)
        if (ce0s[k] >= 0 && os[k] == o) {
          pres[o] = true;
          se[o] = ces[k];
        }
    }
  }
  // each son's pencil is loaded one son ahead, sons in octant order
  C2<R> nv[L];
  auto load_after = [&](int o0) {  // the pencil of the first present son at octant >= o0
    int e = -1;
#pragma unroll
    for (int o = 7; o >= 0; --o)
      if (o >= o0 && pres[o]) e = se[o];
    if (on && e >= 0) {
#pragma unroll
      for (int r = 0; r < L; ++r) nv[r] = M[(int64_t)e * L3 + p * L + r];
    }
  };
  load_after(0);
  // Sum factorisation over the sons: the x-mode products of the two sons that
  // differ only in bx are summed before their common y-mode product, and the
  // y-mode results of the two halves by before their common z-mode product.
#pragma unroll
  for (int bz = 0; bz < 2; ++bz) {
    if (!(pres[4 * bz] || pres[4 * bz + 1] || pres[4 * bz + 2] || pres[4 * bz + 3])) continue;
    C2<R> ysum[L];
#pragma unroll
    for (int l = 0; l < L; ++l) ysum[l] = {(R)0, (R)0};
#pragma unroll
    for (int by = 0; by < 2; ++by) {
      const int ob = 2 * by + 4 * bz;
      if (!(pres[ob] || pres[ob + 1])) continue;
      C2<R> xsum[L], in[L], out[L];
#pragma unroll
      for (int l = 0; l < L; ++l) xsum[l] = {(R)0, (R)0};
#pragma unroll
      for (int bx = 0; bx < 2; ++bx) {
        const int o = ob + bx;
        if (!pres[o]) continue;
#pragma unroll
        for (int r = 0; r < L; ++r) in[r] = {(R)0, (R)0};
        if (on) {
          // x-pencil (r_y, r_z) = (a0, a1) of the son, times exp(-i kappa <y'_r - a_s, v>)
          const double t0 = -ks * (v0 * bx + v1 * (by + (double)a0 / (L - 1)) + v2 * (bz + (double)a1 / (L - 1)));
          C2<R> ph[L];
          phase_run<R, L>(t0, -ks * v0 / (L - 1), ph);
#pragma unroll
          for (int r = 0; r < L; ++r) in[r] = cmul(nv[r], ph[r]);
        }
        load_after(o + 1);
        if (bx) son_mode<R, L, 1, false>(in, out);
        else son_mode<R, L, 0, false>(in, out);
#pragma unroll
        for (int l = 0; l < L; ++l) {
          xsum[l].x += out[l].x;
          xsum[l].y += out[l].y;
        }
      }
      __syncthreads();
      if (on) {  // x-pencil (r_y, r_z) -> stage [l_x][r_z][r_y]
#pragma unroll
        for (int l = 0; l < L; ++l) stg[(l + L * a1) * L + a0] = xsum[l];
      }
      __syncthreads();
      if (on) {  // y-pencil (l_x, r_z) = (a0, a1)
#pragma unroll
        for (int r = 0; r < L; ++r) in[r] = stg[p * L + r];
      }
      if (by) son_mode<R, L, 1, false>(in, out);
      else son_mode<R, L, 0, false>(in, out);
#pragma unroll
      for (int l = 0; l < L; ++l) {
        ysum[l].x += out[l].x;
        ysum[l].y += out[l].y;
      }
    }
    C2<R> in[L], out[L];
    __syncthreads();
    if (on) {  // -> stage [l_x][l_y][r_z]
#pragma unroll
      for (int l = 0; l < L; ++l) stg[(a0 + L * l) * L + a1] = ysum[l];
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < L; ++r) in[r] = {(R)0, (R)0};
    if (on) {  // z-pencil (l_x, l_y) = (a0, a1)
#pragma unroll
      for (int r = 0; r < L; ++r) in[r] = stg[p * L + r];
    }
    if (bz) son_mode<R, L, 1, false>(in, out);
    else son_mode<R, L, 0, false>(in, out);
#pragma unroll
    for (int l = 0; l < L; ++l) {
      acc[l].x += out[l].x;
      acc[l].y += out[l].y;
    }
  }
  if (on) {
    // father-node phases exp(i kappa h <l, v> / (L-1)), z-pencil (l_x, l_y)
    const double kf = g.kappa * h / (L - 1) * inv2pi;
    C2<R> ph[L];
    phase_run<R, L>(kf * (v0 * a0 + v1 * a1), kf * v2, ph);
    C2<R>* dst = M + (int64_t)pe * L3 + p;
#pragma unroll
    for (int l = 0; l < L; ++l) dst[L2 * l] = cmul(acc[l], ph[l]);
  }
}

// L2L by pencils, the transpose of k_m2m_p: a wave serves up to two local
// expansions u of one son cell; for each father expansion v feeding u
// (Father(v) = u, or every one for a low-frequency son): the father's values
// as x-pencils, the father-node phases exp(-i kappa <x_k - a_t, v>), three
// mode products with the transposed son matrices, the son-node phases
// exp(i kappa <x'_h - a_t, v>), summed over fathers; then added to the son's
// values.  The two expansions may have different numbers of fathers.
template <typename R, int L>
__global__ __launch_bounds__(64) void k_l2l_p(int64_t npair, const int32_t* __restrict__ pairs,
                                              const int32_t* __restrict__ ch, const int32_t* __restrict__ begin,
                                              const int32_t* __restrict__ par, const int8_t* __restrict__ oct,
                                              const uint8_t* __restrict__ has_m2l, TreeView T, Geo g,
                                              C2<R>* __restrict__ Lx) {
  constexpr int L2 = L * L, L3 = L2 * L, EPW = pencil_epw<L>(), HW = 64 / EPW;
  __shared__ C2<R> st[EPW][L3];
  const int64_t w = blockIdx.x;
  if (w >= npair) return;
  const int lane = threadIdx.x, hf = lane / HW, p = lane % HW;
  const int item0 = pairs[EPW * w];
  const int item1 = EPW == 2 ? pairs[EPW * w + 1] : -1;
  const int item = hf == 0 ? item0 : item1;
  const bool on = item >= 0 && p < L2;
  const int it = item >= 0 ? item : item0;
  const int ce = ch[it];
  const int c = T.exp_cell[ce];
  const double hcs = ldexp(g.D, -T.level[c]), hp = 2.0 * hcs;
  constexpr double inv2pi = 0.15915494309189533577;
  const int a0 = p % L, a1 = (p / L) % L;
  const int k0 = begin[it], k1 = begin[it + 1];
  const int n0 = begin[item0 + 1] - begin[item0];
  const int n1 = item1 >= 0 ? begin[item1 + 1] - begin[item1] : 0;
  const int nmax = n0 > n1 ? n0 : n1;
  const int o = oct[begin[item0]];  // the son's octant: the same for every father of the wave
  const int bx = o & 1, by = (o >> 1) & 1, bz = (o >> 2) & 1;
  C2<R> acc[L];
#pragma unroll
  for (int l = 0; l < L; ++l) acc[l] = {(R)0, (R)0};
  C2<R>* stg = st[hf];
  for (int k = 0; k < nmax; ++k) {
    const bool act = on && k0 + k < k1;
    const int pe = par[act ? k0 + k : k0];
    const double v0 = T.exp_u[3 * pe], v1 = T.exp_u[3 * pe + 1], v2 = T.exp_u[3 * pe + 2];
    C2<R> in[L], out[L];
#pragma unroll
    for (int r = 0; r < L; ++r) in[r] = {(R)0, (R)0};
    if (act) {
      // x-pencil (k_y, k_z) of the father, times exp(-i kappa hp <k, v> / (L-1))
      const C2<R>* src = Lx + (int64_t)pe * L3 + p * L;
      const double kf = g.kappa * hp / (L - 1) * inv2pi;
      C2<R> ph[L];
      phase_run<R, L>(-kf * (v1 * a0 + v2 * a1), -kf * v0, ph);
#pragma unroll
      for (int r = 0; r < L; ++r) in[r] = cmul(src[r], ph[r]);
    }
    son_mode_b<R, L, true>(bx, in, out);
    __syncthreads();
    if (act) {
#pragma unroll
      for (int l = 0; l < L; ++l) stg[(l + L * a1) * L + a0] = out[l];
    }
    __syncthreads();
    if (act) {
#pragma unroll
      for (int r = 0; r < L; ++r) in[r] = stg[p * L + r];
    }
    son_mode_b<R, L, true>(by, in, out);
    __syncthreads();
    if (act) {
#pragma unroll
      for (int l = 0; l < L; ++l) stg[(a0 + L * l) * L + a1] = out[l];
    }
    __syncthreads();
    if (act) {
#pragma unroll
      for (int r = 0; r < L; ++r) in[r] = stg[p * L + r];
      son_mode_b<R, L, true>(bz, in, out);
      // son-node phases exp(i kappa hc <b + h / (L-1), v>), z-pencil (h_x, h_y)
      const double ks = g.kappa * hcs * inv2pi;
      C2<R> ph[L];
      phase_run<R, L>(ks * (v0 * (bx + (double)a0 / (L - 1)) + v1 * (by + (double)a1 / (L - 1)) + v2 * bz),
                      ks * v2 / (L - 1), ph);
#pragma unroll
      for (int l = 0; l < L; ++l) cfma(acc[l], out[l], ph[l]);
    }
  }
  if (on) {
    // added to what M2L wrote (an M2L target), else the son's only contribution:
    // the local expansions are not cleared before the matvec
    C2<R>* dst = Lx + (int64_t)ce * L3 + p;
    const bool add = has_m2l[ce] != 0;
#pragma unroll
    for (int l = 0; l < L; ++l) {
      const C2<R> cur = add ? dst[L2 * l] : C2<R>{(R)0, (R)0};
      dst[L2 * l] = {cur.x + acc[l].x, cur.y + acc[l].y};
    }
  }
}

// L2L by families (the complex64 pencil path): a half wave serves one family,
// the son expansions u_o (octant o) of one father cell that the same father
// expansions v feed, and takes each v once for all of them in each of two
// passes (one per son half bx, whose four sons' sums stay in registers).  Per
// v and pass: the father's values as x-pencils times the father-node phases,
// then the mode products with the transposed son matrices shared between
// sons: the x-mode product of the half, one y-mode product per by, one z-mode
// product per son (14 for 8 sons instead of 24), each son's result times its
// son-node phases exp(i kappa <x'_h - a_t, v>) added to the son's sum.  Both
// families of a wave have the same father cell; the branches over octants
// follow the union of their sons, so they are uniform.
template <typename R, int L>
__global__ __launch_bounds__(64) void k_l2l_f(int64_t npair, const int32_t* __restrict__ pairs,
                                              const int32_t* __restrict__ fam, const int32_t* __restrict__ par,
                                              const uint8_t* __restrict__ has_m2l, TreeView T, Geo g,
                                              C2<R>* __restrict__ Lx) {
  constexpr int L2 = L * L, L3 = L2 * L, EPW = pencil_epw<L>(), HW = 64 / EPW;
  __shared__ C2<R> sx[EPW][L3];     // the x-mode result, [l_x][k_z][k_y]
  __shared__ C2<R> sy[EPW][2][L3];  // y-mode results by by, [l_x][l_y][k_z]
  const int64_t w = blockIdx.x;
  if (w >= npair) return;
  const int lane = threadIdx.x, hf = lane / HW, p = lane % HW;
  const int item0 = pairs[EPW * w];
  const int item1 = EPW == 2 ? pairs[EPW * w + 1] : -1;
  int rec0[10], rec1[10];
#pragma unroll
  for (int q = 0; q < 10; ++q) {
    rec0[q] = fam[(int64_t)item0 * kFamWords + q];
    rec1[q] = item1 >= 0 ? fam[(int64_t)item1 * kFamWords + q] : (q < 2 ? 0 : -1);
  }
  const bool mine = hf == 0 || item1 >= 0;
  const bool on = mine && p < L2;
  const int vb = hf == 0 ? rec0[0] : rec1[0];
  const int vn = mine ? (hf == 0 ? rec0[1] : rec1[1]) : 0;
  const int nmax = rec0[1] > rec1[1] ? rec0[1] : rec1[1];
  bool pres[8];
  int se[8];
#pragma unroll
  for (int o = 0; o < 8; ++o) {
    pres[o] = rec0[2 + o] >= 0 || rec1[2 + o] >= 0;
    se[o] = mine ? (hf == 0 ? rec0[2 + o] : rec1[2 + o]) : -1;
  }
  bool need_y[4], need_x[2];
#pragma unroll
  for (int q = 0; q < 4; ++q) need_y[q] = pres[q] || pres[q + 4];
  need_x[0] = need_y[0] || need_y[2];
  need_x[1] = need_y[1] || need_y[3];
  // the father cell (of every v of both families) and the sons' level
  const int cf = T.exp_cell[par[rec0[0]]];
  const double hp = ldexp(g.D, -T.level[cf]), hcs = 0.5 * hp;
  constexpr double inv2pi = 0.15915494309189533577;
  const double kf = g.kappa * hp / (L - 1) * inv2pi, ks = g.kappa * hcs * inv2pi;
  const int a0 = p % L, a1 = (p / L) % L;
  // the sons in two passes over the fathers, one per half bx: a pass holds
  // the sums of its four sons in registers
#pragma unroll
  for (int bx = 0; bx < 2; ++bx) {
    if (!need_x[bx]) continue;
    C2<R> acc[4][L];  // son bx + 2 q, q = by + 2 bz
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int l = 0; l < L; ++l) acc[q][l] = {(R)0, (R)0};
    // the father expansions one ahead (their indices two ahead)
    auto pe_at = [&](int j) { return par[on && j < vn ? vb + j : rec0[0]]; };
    int pe_n = pe_at(0);
    double nv0 = 0, nv1 = 0, nv2 = 0;
    C2<R> nraw[L];
    auto fetch = [&](int pe, bool a) {
      nv0 = T.exp_u[3 * pe];
      nv1 = T.exp_u[3 * pe + 1];
      nv2 = T.exp_u[3 * pe + 2];
      if (a) {
        const C2<R>* src = Lx + (int64_t)pe * L3 + p * L;
#pragma unroll
        for (int r = 0; r < L; ++r) nraw[r] = src[r];
      }
    };
    fetch(pe_n, on && 0 < vn);
    pe_n = pe_at(1);
    for (int k = 0; k < nmax; ++k) {
      const bool act = on && k < vn;
      const double v0 = nv0, v1 = nv1, v2 = nv2;
      C2<R> in[L], out[L];
#pragma unroll
      for (int r = 0; r < L; ++r) in[r] = act ? nraw[r] : C2<R>{(R)0, (R)0};
      if (k + 1 < nmax) {
        fetch(pe_n, on && k + 1 < vn);
        pe_n = pe_at(k + 2);
      }
      if (act) {
        // x-pencil (k_y, k_z) of the father, times exp(-i kappa hp <k, v> / (L-1))
        C2<R> ph[L];
        phase_run<R, L>(-kf * (v1 * a0 + v2 * a1), -kf * v0, ph);
#pragma unroll
        for (int r = 0; r < L; ++r) in[r] = cmul(in[r], ph[r]);
      }
      // the son-node phases exp(i kappa hc <b + h / (L-1), v>) as
      // exp(i kappa hc <h / (L-1), v>) (ph0, along the z-pencil) times
      // exp(i kappa hc v_d) for each axis d whose half b_d is 1, the latter
      // applied to the mode product of that axis (scalars commute with them)
      const C2<R> cx = expi_turns<R>(ks * v0), cy = expi_turns<R>(ks * v1), cz = expi_turns<R>(ks * v2);
      if (bx) son_mode<R, L, 1, true>(in, out);
      else son_mode<R, L, 0, true>(in, out);
      __syncthreads();
      if (act) {
#pragma unroll
        for (int l = 0; l < L; ++l) sx[hf][(l + L * a1) * L + a0] = bx ? cmul(out[l], cx) : out[l];
      }
      __syncthreads();
      if (act) {  // y-pencil (l_x, k_z) = (a0, a1)
#pragma unroll
        for (int r = 0; r < L; ++r) in[r] = sx[hf][p * L + r];
      }
#pragma unroll
      for (int by = 0; by < 2; ++by) {
        if (!need_y[bx + 2 * by]) continue;
        if (by) son_mode<R, L, 1, true>(in, out);
        else son_mode<R, L, 0, true>(in, out);
        if (act) {
#pragma unroll
          for (int l = 0; l < L; ++l) sy[hf][by][(a0 + L * l) * L + a1] = by ? cmul(out[l], cy) : out[l];
        }
      }
      __syncthreads();
      C2<R> ph0[L];
      phase_run<R, L>(ks * (v0 * a0 + v1 * a1) / (L - 1), ks * v2 / (L - 1), ph0);
#pragma unroll
      for (int by = 0; by < 2; ++by) {
        if (!need_y[bx + 2 * by]) continue;
        if (act) {  // z-pencil (l_x, l_y) = (a0, a1)
#pragma unroll
          for (int r = 0; r < L; ++r) in[r] = sy[hf][by][p * L + r];
        }
#pragma unroll
        for (int bz = 0; bz < 2; ++bz) {
          const int o = bx + 2 * by + 4 * bz;
          if (!pres[o]) continue;
          if (bz) son_mode<R, L, 1, true>(in, out);
          else son_mode<R, L, 0, true>(in, out);
          if (act && se[o] >= 0) {
#pragma unroll
            for (int l = 0; l < L; ++l) cfma(acc[by + 2 * bz][l], bz ? cmul(out[l], cz) : out[l], ph0[l]);
          }
        }
      }
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int o = bx + 2 * q;
      if (!pres[o]) continue;
      if (on && se[o] >= 0) {
        // added to what M2L wrote (an M2L target), else the son's only contribution
        C2<R>* dst = Lx + (int64_t)se[o] * L3 + p;
        const bool add = has_m2l[se[o]] != 0;
#pragma unroll
        for (int l = 0; l < L; ++l) {
          const C2<R> cur = add ? dst[L2 * l] : C2<R>{(R)0, (R)0};
          dst[L2 * l] = {cur.x + acc[q][l].x, cur.y + acc[q][l].y};
        }
      }
    }
  }
}

// ------------------------------------------------------------------ M2M
// M_s^v(y_l) = D0 (x)A_b (D1 M_{s'}) summed over sons (eq. dlefturight):
// D1 = exp(-ik<y'_r - a_s, v>), three mode products with the real son
// matrices (Sec. 5.2.3), D0 = exp(ik<y_l - a_s, v>).  One thread per node.
template <typename R, int L>
__global__ __launch_bounds__(round64(L* L* L)) void k_m2m(int64_t n, const int32_t* __restrict__ par,
                                                         const int32_t* __restrict__ child,
                                                         const int8_t* __restrict__ oct, TreeView T, Geo g,
                                                         C2<R>* __restrict__ M) {
  constexpr int L3 = L * L * L;
  __shared__ R A[2][L][L];
  __shared__ C2<R> ph[3][L];
  __shared__ C2<R> b0[L3], b1[L3];
  int64_t item = blockIdx.x;
  if (item >= n) return;
  int pe = par[item];
  int c = T.exp_cell[pe];
  double h = ldexp(g.D, -T.level[c]), hc = 0.5 * h;
  double v[3] = {T.exp_u[3 * pe], T.exp_u[3 * pe + 1], T.exp_u[3 * pe + 2]};
  int tid = threadIdx.x;
  int lx = tid % L, ly = (tid / L) % L, lz = tid / (L * L);
  son_matrices<R, L>(A);
  // every son's value at this thread's node, loaded before the first product
  // so that the eight loads are in flight together
  C2<R> sv[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    const int ce = child[item * 8 + k];
    sv[k] = (ce >= 0 && tid < L3) ? M[(int64_t)ce * L3 + tid] : C2<R>{(R)0, (R)0};
  }
  C2<R> acc = {(R)0, (R)0};
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    int ce = child[item * 8 + k];
    if (ce < 0) break;
    int o = oct[item * 8 + k];
    int b[3] = {o & 1, (o >> 1) & 1, (o >> 2) & 1};
    __syncthreads();
    if (tid < 3 * L) {
      int d = tid / L, r = tid % L;
      ph[d][r] = expi<R>(-g.kappa * hc * v[d] * ((double)b[d] + (double)r / (double)(L - 1)));
    }
    __syncthreads();
    if (tid < L3) b0[tid] = cmul(cmul(sv[k], ph[0][lx]), cmul(ph[1][ly], ph[2][lz]));
    __syncthreads();
    if (tid < L3) {
      C2<R> s = {(R)0, (R)0};
#pragma unroll
      for (int r = 0; r < L; ++r) cfma_r(s, b0[r + L * ly + L * L * lz], A[b[0]][lx][r]);
      b1[tid] = s;
    }
    __syncthreads();
    if (tid < L3) {
      C2<R> s = {(R)0, (R)0};
#pragma unroll
      for (int r = 0; r < L; ++r) cfma_r(s, b1[lx + L * r + L * L * lz], A[b[1]][ly][r]);
      b0[tid] = s;
    }
    __syncthreads();
    if (tid < L3) {
#pragma unroll
      for (int r = 0; r < L; ++r) cfma_r(acc, b0[lx + L * ly + L * L * r], A[b[2]][lz][r]);
    }
  }
  if (tid < L3) {
    double arg = g.kappa * h / (double)(L - 1) * (v[0] * lx + v[1] * ly + v[2] * lz);
    M[(int64_t)pe * L3 + tid] = cmul(acc, expi<R>(arg));
  }
}

// ------------------------------------------------------------------ M2F / F2L
// The DFT twiddles e^{2 pi i k / P} as compile-time constants: cosine and sine
// of the angle reduced to [-pi, pi], by their Taylor series (40 terms, far below
// FP64 rounding for |x| <= pi).
struct Twiddles {
  double c[16], s[16];
  constexpr explicit Twiddles(int P) : c(), s() {
    for (int k = 0; k < P; ++k) {
      const int kk = 2 * k > P ? k - P : k;
      const double x = 6.283185307179586476925286766559 * (double)kk / (double)P, x2 = x * x;
      double term = x, sn = 0.0;
      for (int n = 1; n < 40; n += 2) {
        sn += term;
        term *= -x2 / (double)((n + 1) * (n + 2));
      }
      double cs = 0.0;
      term = 1.0;
      for (int n = 0; n < 40; n += 2) {
        cs += term;
        term *= -x2 / (double)((n + 1) * (n + 2));
      }
      c[k] = cs;
      s[k] = sn;
    }
  }
};

// y[k] = sum_{a < NIN} x[a] w^{a k} for k < NOUT, w = e^{SIGN 2 pi i / 3}: a
// length-3 DFT on a prefix of its inputs, for a prefix of its outputs, with
// w = -1/2 + SIGN i sqrt(3)/2 (two constants instead of a complex product).
template <typename R, int SIGN, int NIN, int NOUT>
__device__ __forceinline__ void dft3(const C2<R> (&x)[3], C2<R> (&y)[3]) {
  static_assert(NIN >= 1 && NIN <= 3 && NOUT >= 1 && NOUT <= 3, "length-3 DFT");
  constexpr R h = (R)0.5, r3 = (R)(SIGN * 0.86602540378443864676372317075294);
  if constexpr (NIN == 1) {
#pragma unroll
    for (int k = 0; k < NOUT; ++k) y[k] = x[0];
  } else if constexpr (NIN == 2) {
    y[0] = {x[0].x + x[1].x, x[0].y + x[1].y};
    const C2<R> t = {fma(-h, x[1].x, x[0].x), fma(-h, x[1].y, x[0].y)};
    if constexpr (NOUT > 1) y[1] = {fma(-r3, x[1].y, t.x), fma(r3, x[1].x, t.y)};
    if constexpr (NOUT > 2) y[2] = {fma(r3, x[1].y, t.x), fma(-r3, x[1].x, t.y)};
  } else {
    const C2<R> sm = {x[1].x + x[2].x, x[1].y + x[2].y};
    y[0] = {x[0].x + sm.x, x[0].y + sm.y};
    if constexpr (NOUT > 1) {
      const C2<R> d = {x[1].x - x[2].x, x[1].y - x[2].y};
      const C2<R> t = {fma(-h, sm.x, x[0].x), fma(-h, sm.y, x[0].y)};
      y[1] = {fma(-r3, d.y, t.x), fma(r3, d.x, t.y)};
      if constexpr (NOUT > 2) y[2] = {fma(r3, d.y, t.x), fma(-r3, d.x, t.y)};
    }
  }
}

// The pencil DFT of length 9 as 3 x 3 (Cooley-Tukey): with m = 3a + b and
// k = k1 + 3 k2, out[k] = sum_b w9^{b k} sum_a in[3a + b] w3^{a k1}, where
// w9^{b k} = w9^{b k1} w3^{b k2}: three length-3 DFTs over a (on the inputs
// present), the twiddles w9^{b k1}, then three length-3 DFTs over b (for the
// outputs asked for).  About 2.3x fewer operations than the direct sums.
template <typename R, int NI, int NO, int SIGN>
__device__ __forceinline__ void dft9(const C2<R> (&in)[NI], C2<R> (&out)[NO]) {
  static_assert(NI >= 3 && NI <= 9 && NO >= 3 && NO <= 9, "length-9 pencil");
  constexpr Twiddles T(9);
  C2<R> z[3][3];  // z[b][k1]
#pragma unroll
  for (int b = 0; b < 3; ++b) {
    C2<R> x[3], y[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) x[a] = 3 * a + b < NI ? in[3 * a + b < NI ? 3 * a + b : 0] : C2<R>{(R)0, (R)0};
    if (b == 0) dft3<R, SIGN, (NI + 2) / 3, 3>(x, y);
    else if (b == 1) dft3<R, SIGN, (NI + 1) / 3, 3>(x, y);
    else dft3<R, SIGN, NI / 3, 3>(x, y);
#pragma unroll
    for (int k1 = 0; k1 < 3; ++k1) {
      if (b * k1 == 0) {
        z[b][k1] = y[k1];
      } else {
        const R c = (R)T.c[b * k1], sn = (R)(SIGN * T.s[b * k1]);
        z[b][k1] = {fma(y[k1].x, c, -y[k1].y * sn), fma(y[k1].x, sn, y[k1].y * c)};
      }
    }
  }
#pragma unroll
  for (int k1 = 0; k1 < 3; ++k1) {
    C2<R> x[3] = {z[0][k1], z[1][k1], z[2][k1]}, y[3];
    if (k1 == 0) dft3<R, SIGN, 3, (NO + 2) / 3>(x, y);
    else if (k1 == 1) dft3<R, SIGN, 3, (NO + 1) / 3>(x, y);
    else dft3<R, SIGN, 3, NO / 3>(x, y);
#pragma unroll
    for (int k2 = 0; k2 < 3; ++k2)
      if (k1 + 3 * k2 < NO) out[k1 + 3 * k2 < NO ? k1 + 3 * k2 : 0] = y[k2];
  }
}

// out[k] = sum_m in[m] e^{SIGN 2 pi i k m / P} for k < NO, m < NI: one pencil of
// a separable DFT, twiddles folded in at compile time (P = 9 factored).
template <typename R, int P, int NI, int NO, int SIGN>
__device__ __forceinline__ void dft_pencil(const C2<R> (&in)[NI], C2<R> (&out)[NO]) {
  if constexpr (P == 9 && NI >= 3 && NO >= 3) {
    dft9<R, NI, NO, SIGN>(in, out);
    return;
  }
  constexpr Twiddles T(P);
#pragma unroll
  for (int k = 0; k < NO; ++k) {
    C2<R> acc = in[0];
#pragma unroll
    for (int m = 1; m < NI; ++m) {
      const int km = (k * m) % P;
      const R c = (R)T.c[km], sn = (R)(SIGN * T.s[km]);
      acc.x = fma(in[m].x, c, fma(-in[m].y, sn, acc.x));
      acc.y = fma(in[m].x, sn, fma(in[m].y, c, acc.y));
    }
    out[k] = acc;
  }
}

// Expansions per workgroup of M2F and F2L (each needs a P^3 grid and a P^2 L
// stage in LDS): the default is as many as fit 64 KB, at most 4; a workspace
// may ask for 1, 2 or 4, capped at what fits 96 KB.
template <typename R, int L>
constexpr int fourier_item_bytes() {
  constexpr int P = 2 * L - 1;
  return (P * P * P + P * P * L) * (int)sizeof(C2<R>);
}
template <typename R, int L>
constexpr int fourier_items() {
  constexpr int per = fourier_item_bytes<R, L>();
  return per * 4 <= 65536 ? 4 : per * 2 <= 65536 ? 2 : 1;
}
template <typename R, int L>
constexpr int fourier_items_max() {
  constexpr int per = fourier_item_bytes<R, L>();
  return per * 4 <= 98304 ? 4 : per * 2 <= 98304 ? 2 : 1;
}
template <typename R, int L, int G>
constexpr int fourier_items_capped() {
  return G < fourier_items_max<R, L>() ? G : fourier_items_max<R, L>();
}

// M~ = DFT_P(pad(M)) by pencils: pass x (L^2 pencils of L values -> P), pass y
// (P L pencils), pass z (P^2 pencils), one thread per pencil and G expansions
// per chunk; the P^3 grid is then written in the order of the Fourier layout
// (freq), padding as zeros.  Stage layouts keep consecutive threads on
// consecutive LDS words.  Persistent workgroups walk the chunks (xcd_walk);
// the node values of a thread's next pass-x pencil are loaded while the
// current chunk goes through passes y and z and the store.
template <typename R, int L, int G>
__global__ __launch_bounds__(256) void k_m2f(int64_t n, const int32_t* __restrict__ src,
                                             const int32_t* __restrict__ freq, const C2<R>* __restrict__ M,
                                             C2<R>* __restrict__ Mt) {
  constexpr int P = 2 * L - 1, P3 = P * P * P, L2 = L * L, L3 = L2 * L, NT = 256;
  constexpr int RW = fourier_row(L);
  constexpr int SA = P3 > P * L2 ? P3 : P * L2;  // x-stage, then the full grid
  constexpr int SB = P * P * L;                   // y-stage
  constexpr int NX = (G * L2 + NT - 1) / NT;      // pass-x pencils per thread
  __shared__ C2<R> A[G][SA];
  __shared__ C2<R> B[G][SB];
  __shared__ int32_t fq[RW];
  const int64_t nch = (n + G - 1) / G;
  const XcdWalk wk = xcd_walk(nch);
  if (wk.first >= wk.end) return;
  const int tid = threadIdx.x;
  for (int p = tid; p < RW; p += NT) fq[p] = freq[p];
  C2<R> in_x[NX][L];
  auto load_x = [&](int64_t ch) {
    const int64_t i0 = ch * G;
    const int ng = (int)min((int64_t)G, n - i0);
#pragma unroll
    for (int v = 0; v < NX; ++v) {
      const int w = tid + v * NT;
      if (w < ng * L2) {
        const int g = w / L2, yz = w % L2;
        const C2<R>* m = M + (int64_t)src[i0 + g] * L3 + yz * L;
#pragma unroll
        for (int r = 0; r < L; ++r) in_x[v][r] = m[r];
      }
    }
  };
  load_x(wk.first);
  for (int64_t ch = wk.first; ch < wk.end; ch += wk.step) {
    const int64_t i0 = ch * G;
    const int ng = (int)min((int64_t)G, n - i0);
    // pass x: pencil (ry, rz) of L contiguous values; A[g][xi * L^2 + ry + L rz]
#pragma unroll
    for (int v = 0; v < NX; ++v) {
      const int w = tid + v * NT;
      if (w < ng * L2) {
        const int g = w / L2, yz = w % L2;
        C2<R> out[P];
        dft_pencil<R, P, L, P, -1>(in_x[v], out);
#pragma unroll
        for (int k = 0; k < P; ++k) A[g][k * L2 + yz] = out[k];
      }
    }
    if (ch + wk.step < wk.end) load_x(ch + wk.step);
    __syncthreads();
    // pass y: pencil (rz, xi); B[g][rz + L (xi + P yi)]
    for (int w = tid; w < ng * P * L; w += NT) {
      const int g = w / (P * L), q = w % (P * L), rz = q % L, xi = q / L;
      C2<R> in[L], out[P];
#pragma unroll
      for (int r = 0; r < L; ++r) in[r] = A[g][xi * L2 + r + L * rz];
      dft_pencil<R, P, L, P, -1>(in, out);
#pragma unroll
      for (int k = 0; k < P; ++k) B[g][rz + L * (xi + P * k)] = out[k];
    }
    __syncthreads();
    // pass z: pencil (xi, yi) = xy; A[g][xy + P^2 zi]
    for (int w = tid; w < ng * P * P; w += NT) {
      const int g = w / (P * P), xy = w % (P * P);
      C2<R> in[L], out[P];
#pragma unroll
      for (int r = 0; r < L; ++r) in[r] = B[g][r + L * xy];
      dft_pencil<R, P, L, P, -1>(in, out);
#pragma unroll
      for (int k = 0; k < P; ++k) A[g][xy + P * P * k] = out[k];
    }
    __syncthreads();
    // the G rows are contiguous; stored two entries (16 or 32 bytes) per thread
    constexpr int RW2 = RW / 2, NV = (G * RW2 + NT - 1) / NT;
#pragma unroll
    for (int k = 0; k < NV; ++k) {
      const int w = tid + k * NT;
      if (w < ng * RW2) {
        const int g = w / RW2, p = 2 * (w % RW2);
        const int f0 = fq[p], f1 = fq[p + 1];
        C2x2<R> v;
        v.a = f0 >= 0 ? A[g][f0] : C2<R>{(R)0, (R)0};
        v.b = f1 >= 0 ? A[g][f1] : C2<R>{(R)0, (R)0};
        reinterpret_cast<C2x2<R>*>(Mt + i0 * RW)[w] = v;
      }
    }
    __syncthreads();
  }
}

// ------------------------------------------------------------------ M2L + F2L
// Spectrum entries of the M2L lists are codes (canonical id << 6) | symmetry
// r: the offset's spectrum is the canonical row read through the layout's
// pair permutation for r (D_{R delta}[xi] = D_delta[R^-1 xi], Sec. 4.3).
//
// For one target expansion: L~ = sum over its list of D_{l,delta} (.) M~_s
// (Hadamard products, Sec. 2.3), then F2L = pruned inverse DFT restricted to
// [0,L)^3 (the 1/P^3 is folded into the spectra).  Each thread owns NF row
// positions; the permuted spectrum entries are gathered one by one.
template <typename R, int L>
__global__ __launch_bounds__(256) void k_m2l(int64_t ntgt, const int32_t* __restrict__ tgt,
                                             const int32_t* __restrict__ begin, const int2* __restrict__ pairs,
                                             const int32_t* __restrict__ freq, const uint8_t* __restrict__ perm,
                                             int sym, const C2<R>* __restrict__ Mt, const C2<R>* __restrict__ S,
                                             C2<R>* __restrict__ Lx) {
  constexpr int P = 2 * L - 1, P3 = P * P * P, L3 = L * L * L, RW = fourier_row(L), SL = 2 * fourier_cap(L);
  constexpr int NT = 256, NF = (RW + NT - 1) / NT;
  __shared__ C2<R> A[P3];
  __shared__ C2<R> B1[P * P * L];
  __shared__ C2<R> B2[P * L * L];
  __shared__ C2<R> W[P];
  int64_t i = xcd_item(ntgt);
  if (i >= ntgt) return;
  int tid = threadIdx.x;
  C2<R> acc[NF];
  int pb[NF], qb[NF], sd[NF];
#pragma unroll
  for (int f = 0; f < NF; ++f) {
    acc[f] = {(R)0, (R)0};
    const int p = min(tid + f * NT, RW - 1), sl = p / SL;
    pb[f] = sl * 48 * 64 + (p % SL) / 2;  // perm entry of symmetry 0
    qb[f] = sl * SL;                      // slice start
    sd[f] = p & 1;                        // xi (0) or -xi (1) of the pair
  }
  int kb = begin[i], ke = begin[i + 1];
  for (int k = kb; k < ke; ++k) {
    const int2 pr = pairs[k];
    const C2<R>* ms = Mt + (int64_t)pr.x * RW;
    const C2<R>* ds = S + (int64_t)((sym ? 2 : 1) * (pr.y >> 6)) * RW;
    const int r64 = (pr.y & 63) * 64;
#pragma unroll
    for (int f = 0; f < NF; ++f) {
      int p = tid + f * NT;
      if (p < RW) {
        const int pe = sym ? perm[pb[f] + r64] : (p % SL) / 2;
        cfma(acc[f], ds[qb[f] + 2 * (pe & 127) + (sd[f] ^ (pe >> 7))], ms[p]);
      }
    }
  }
#pragma unroll
  for (int f = 0; f < NF; ++f) {
    int p = tid + f * NT;
    if (p < RW && freq[p] >= 0) A[freq[p]] = acc[f];
  }
  if (tid < P) W[tid] = expi<R>(2.0 * M_PI * (double)tid / (double)P);
  __syncthreads();
  for (int j = tid; j < P * P * L; j += NT) {  // z: (xi, yi, kz)
    int xy = j % (P * P), kz = j / (P * P);
    C2<R> s = {(R)0, (R)0};
#pragma unroll
    for (int m = 0; m < P; ++m) cfma(s, A[xy + P * P * m], W[(m * kz) % P]);
    B1[j] = s;
  }
  __syncthreads();
  for (int j = tid; j < P * L * L; j += NT) {  // y: (xi, ky, kz)
    int xi = j % P, ky = (j / P) % L, kz = j / (P * L);
    C2<R> s = {(R)0, (R)0};
#pragma unroll
    for (int m = 0; m < P; ++m) cfma(s, B1[xi + P * m + P * P * kz], W[(m * ky) % P]);
    B2[j] = s;
  }
  __syncthreads();
  for (int j = tid; j < L3; j += NT) {  // x: (kx, ky, kz)
    int kx = j % L, kyz = j / L;
    C2<R> s = {(R)0, (R)0};
#pragma unroll
    for (int m = 0; m < P; ++m) cfma(s, B2[m + P * kyz], W[(m * kx) % P]);
    Lx[(int64_t)tgt[i] * L3 + j] = s;
  }
}

// M2L Hadamard accumulate, frequency-sliced: the row's frequency pairs are
// split into slices of up to 64 (one per lane) and the (slice, target) items
// are dealt to the XCDs in contiguous slice-major shares (slice_item), so
// each XCD's L2 holds one slice of the spectra and Fourier-domain multipoles
// its targets read.  One wave per workgroup.
// Loads one slice's pair permutations (48 symmetries x 64 lanes, bytes) into
// LDS; the workgroup is one wave.
__device__ __forceinline__ const uint8_t* load_slice_perm(const uint8_t* __restrict__ perm, int slice,
                                                          uint32_t* lds) {
  const uint32_t* src = reinterpret_cast<const uint32_t*>(perm + (size_t)slice * 48 * 64);
  for (int i = threadIdx.x; i < 48 * 16; i += 64) lds[i] = src[i];
  __syncthreads();
  return reinterpret_cast<const uint8_t*>(lds);
}

// The spectrum values of a lane's pair (xi, -xi) for spectrum code e, one
// 16-byte (complex64) load.  Per-offset spectra (SYM false): the lane's own
// pair of row e >> 6.  Compressed spectra: the pair of canonical spectrum
// e >> 6 that the slice's permutation table names for symmetry e & 63, from
// the pair-exchanged row when the symmetry maps xi onto a second member.
template <bool SYM, typename R>
__device__ __forceinline__ C2x2<R> spectrum_pair(const C2<R>* __restrict__ S, int e, int row, int slice_start,
                                                 const uint8_t* pt, int lane, int fl) {
  if constexpr (SYM) {
    const int pe = pt[(e & 63) * 64 + lane];
    return *reinterpret_cast<const C2x2<R>*>(S + (int64_t)(2 * (e >> 6) + (pe >> 7)) * row + slice_start +
                                             2 * (pe & 127));
  } else {
    return *reinterpret_cast<const C2x2<R>*>(S + (int64_t)(e >> 6) * row + fl);
  }
}

template <typename R, int L, int NSL, bool SYM>
__global__ __launch_bounds__(64) void k_m2l_slice(int64_t ntgt, const int32_t* __restrict__ begin,
                                                  const int2* __restrict__ pairs, const uint8_t* __restrict__ perm,
                                                  const C2<R>* __restrict__ Mt, const C2<R>* __restrict__ S,
                                                  C2<R>* __restrict__ Lt) {
  // NSL slices; each XCD walks a contiguous share of the slice-major list
  // (slice_item).  Each lane owns one frequency pair (xi, -xi) of the slice.
  constexpr int P3R = fourier_row(L), SL = P3R / NSL, NP = SL / 2, U = 8;
  static_assert(SL % 2 == 0 && NP <= 64, "a slice holds at most 64 frequency pairs");
  __shared__ uint32_t ptab[48 * 16];
  int slice;
  int64_t i;
  if (!slice_item(NSL, ntgt, slice, i)) return;
  const int lane = threadIdx.x;
  const uint8_t* pt = SYM ? load_slice_perm(perm, slice, ptab) : nullptr;
  const bool ok = lane < NP;
  const int s0 = slice * SL;
  const int fl = ok ? s0 + 2 * lane : s0;
  C2<R> acc0 = {(R)0, (R)0}, acc1 = {(R)0, (R)0};
  int k = begin[i];
  const int ke = begin[i + 1];
  for (; k + U <= ke; k += U) {
    int2 pr[U];
#pragma unroll
    for (int u = 0; u < U; ++u) pr[u] = pairs[k + u];
    C2x2<R> mv[U], dv[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      mv[u] = *reinterpret_cast<const C2x2<R>*>(Mt + (int64_t)pr[u].x * P3R + fl);
      dv[u] = spectrum_pair<SYM>(S, pr[u].y, P3R, s0, pt, lane, fl);
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      cfma(acc0, dv[u].a, mv[u].a);
      cfma(acc1, dv[u].b, mv[u].b);
    }
  }
  for (; k < ke; ++k) {
    const int2 pr = pairs[k];
    const C2x2<R> m = *reinterpret_cast<const C2x2<R>*>(Mt + (int64_t)pr.x * P3R + fl);
    const C2x2<R> d = spectrum_pair<SYM>(S, pr.y, P3R, s0, pt, lane, fl);
    cfma(acc0, d.a, m.a);
    cfma(acc1, d.b, m.b);
  }
  if (ok) *reinterpret_cast<C2x2<R>*>(Lt + i * P3R + fl) = C2x2<R>{acc0, acc1};
}

// Word 3 of a gfx9 buffer descriptor for raw dword access (32-bit data
// format, no swizzle).
constexpr int kBufferWord3 = 0x00020000;

// Two adjacent entries of a row through a buffer descriptor built from the
// row's (uniform) base: the per-lane byte offset is the only vector operand,
// so a batch of loads needs no per-lane 64-bit addresses.  `bytes` bounds the
// offsets (the hardware returns zeros beyond it).
template <typename R>
__device__ __forceinline__ C2x2<R> buffer_pair(const void* base, uint32_t bytes, uint32_t lane_bytes) {
  const __amdgpu_buffer_rsrc_t rs =
      __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)bytes, kBufferWord3);
  if constexpr (sizeof(R) == 4) {
    const auto v = __builtin_amdgcn_raw_buffer_load_b128(rs, (int)lane_bytes, 0, 0);
    C2x2<R> out;
    __builtin_memcpy(&out, &v, sizeof(out));
    return out;
  } else {
    const auto v0 = __builtin_amdgcn_raw_buffer_load_b128(rs, (int)lane_bytes, 0, 0);
    const auto v1 = __builtin_amdgcn_raw_buffer_load_b128(rs, (int)lane_bytes + 16, 0, 0);
    C2x2<R> out;
    __builtin_memcpy(&out.a, &v0, sizeof(out.a));
    __builtin_memcpy(&out.b, &v1, sizeof(out.b));
    return out;
  }
}

template <typename R>
__device__ __forceinline__ C2x2<R> row_pair(const C2<R>* __restrict__ A, uint32_t row, uint32_t row_bytes,
                                            uint32_t lane_bytes) {
  return buffer_pair<R>(reinterpret_cast<const char*>(A) + (uint64_t)row * row_bytes, row_bytes, lane_bytes);
}

// spectrum_pair with the same addressing: per-offset spectra read the lane's
// pair of row e >> 6; compressed spectra the pair the slice's permutation
// table names, in the canonical spectrum's plain or pair-exchanged row.
template <bool SYM, typename R>
__device__ __forceinline__ C2x2<R> spectrum_pair_b(const C2<R>* __restrict__ S, int e, uint32_t row_bytes,
                                                   uint32_t slice_bytes, const uint8_t* pt, int lane,
                                                   uint32_t lane_bytes) {
  if constexpr (SYM) {
    const int pe = pt[(e & 63) * 64 + lane];
    const char* base = reinterpret_cast<const char*>(S) + (uint64_t)(uint32_t)(2 * (e >> 6)) * row_bytes;
    const uint32_t off = (uint32_t)(pe >> 7) * row_bytes + slice_bytes + (uint32_t)(pe & 127) * 2 * sizeof(C2<R>);
    return buffer_pair<R>(base, 2 * row_bytes, off);
  } else {
    return row_pair(S, (uint32_t)(e >> 6), row_bytes, lane_bytes);
  }
}

// Hadamard accumulate over source runs.  A workgroup (one wave) handles one
// group of <= 8 targets sharing level and direction, and one frequency slice
// (slice-major per XCD as in k_m2l_slice).  Each run loads the source's
// Fourier-domain multipole once and the spectrum of every group target that
// interacts with it, so one source load feeds several targets.  Run records
// are 16 words (source row, the 8 targets' spectrum codes or -1, padding), one
// scalar load each; a group's runs are padded to a multiple of the batch, and
// the table carries two batches more at its end, so no record load is
// conditional.  The source rows are loaded one batch ahead (their source
// words two batches ahead): a batch waits only for its spectra, which the
// XCD's L2 mostly holds, while the next batch's source rows, which mostly
// come from beyond it, are in flight.  The two source-row register sets
// alternate (the loop is unrolled by two), so no copy waits for a load.
// All branches depend only on the run records (uniform) and accumulators sit
// at fixed register indices.
template <typename R, int L, int NSL, bool SYM>
__global__ __launch_bounds__(64) void k_m2l_runs(int64_t ngrp, const int32_t* __restrict__ grp_tfirst,
                                                 const int32_t* __restrict__ grp_tcount,
                                                 const int32_t* __restrict__ run_begin, const int32_t* __restrict__ runs,
                                                 const uint8_t* __restrict__ perm, const int32_t* __restrict__ freq,
                                                 const C2<R>* __restrict__ Mt, const C2<R>* __restrict__ S,
                                                 C2<R>* __restrict__ Lt) {
  constexpr int P3R = fourier_row(L), SL = P3R / NSL, NP = SL / 2, G = 8, RS = kRunWords;
  static_assert(SL % 2 == 0 && NP <= 64, "a slice holds at most 64 frequency pairs");
  constexpr int U = m2l_run_batch<R>();  // runs per batch
  constexpr uint32_t RB = P3R * sizeof(C2<R>);  // row bytes
  __shared__ uint32_t ptab[48 * 16];
  int slice;
  int64_t g;
  if (!slice_item(NSL, ngrp, slice, g)) return;
  const int lane = threadIdx.x;
  const uint8_t* pt = SYM ? load_slice_perm(perm, slice, ptab) : nullptr;
  const int s0 = slice * SL;
  const int fl = lane < NP ? s0 + 2 * lane : s0;
  // a pair of padding entries (the row's tail) is neither read nor written:
  // its lane offset lies past every row, where buffer loads return zeros
  // without a memory access
  const bool ok = lane < NP && (freq[fl] >= 0 || freq[fl + 1] >= 0);
  const uint32_t lb = ok ? (uint32_t)fl * sizeof(C2<R>) : RB, sb = (uint32_t)s0 * sizeof(C2<R>);
  C2x2<R> acc[G];
#pragma unroll
  for (int t = 0; t < G; ++t) acc[t] = C2x2<R>{{(R)0, (R)0}, {(R)0, (R)0}};
  int r = run_begin[g];
  const int re = run_begin[g + 1];
  int rec[U][9], src1[U];
  C2x2<R> mA[U], mB[U];
#pragma unroll
  for (int u = 0; u < U; ++u) {
#pragma unroll
    for (int q = 0; q < 9; ++q) rec[u][q] = runs[(int64_t)(r + u) * RS + q];
    src1[u] = runs[(int64_t)(r + U + u) * RS];
  }
#pragma unroll
  for (int u = 0; u < U; ++u) mA[u] = row_pair(Mt, (uint32_t)rec[u][0], RB, lb);
  // one batch: records of the next batch and source words of the one after
  // are fetched, the spectra of this batch and the source rows of the next
  // are loaded, then this batch is accumulated from mc
  auto step = [&](const C2x2<R>(&mc)[U], C2x2<R>(&mn)[U]) {
    int nx[U][9], src2[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
#pragma unroll
      for (int q = 0; q < 9; ++q) nx[u][q] = runs[(int64_t)(r + U + u) * RS + q];
      src2[u] = runs[(int64_t)(r + 2 * U + u) * RS];
    }
    C2x2<R> dv[U][G];
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int t = 0; t < G; ++t) {
        if (rec[u][1 + t] < 0) continue;
        dv[u][t] = spectrum_pair_b<SYM>(S, rec[u][1 + t], RB, sb, pt, lane, lb);
      }
#pragma unroll
    for (int u = 0; u < U; ++u) mn[u] = row_pair(Mt, (uint32_t)src1[u], RB, lb);
#pragma unroll
    for (int u = 0; u < U; ++u) {
#pragma unroll
      for (int t = 0; t < G; ++t) {
        if (rec[u][1 + t] < 0) continue;
        cfma(acc[t].a, dv[u][t].a, mc[u].a);
        cfma(acc[t].b, dv[u][t].b, mc[u].b);
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
#pragma unroll
      for (int q = 0; q < 9; ++q) rec[u][q] = nx[u][q];
      src1[u] = src2[u];
    }
    r += U;
  };
  for (;;) {
    step(mA, mB);
    if (r >= re) break;
    step(mB, mA);
    if (r >= re) break;
  }
  const int64_t tf = grp_tfirst[g];
  const int tc = grp_tcount[g];
#pragma unroll
  for (int t = 0; t < G; ++t)
    if (t < tc && ok) *reinterpret_cast<C2x2<R>*>(Lt + (tf + t) * P3R + fl) = acc[t];
}

// F2L: inverse DFT of each target's accumulated Fourier-domain local
// expansion restricted to [0,L)^3 (the 1/P^3 is folded into the spectra), by
// pencils as in M2F: pass z (P^2 pencils of P values -> L), pass y (P L
// pencils), pass x (L^2 pencils, each writing its L contiguous node values).
// Targets in XCD-aware order, G per workgroup.
template <typename R, int L, int G>
__global__ __launch_bounds__(256) void k_f2l(int64_t ntgt, const int32_t* __restrict__ tgt,
                                             const int32_t* __restrict__ freq, int live_pairs,
                                             const C2<R>* __restrict__ Lt, C2<R>* __restrict__ Lx) {
  constexpr int P = 2 * L - 1, P3 = P * P * P, L2 = L * L, L3 = L2 * L, NT = 256;
  constexpr int RW = fourier_row(L);
  constexpr int SA = P3 > P * L2 ? P3 : P * L2;  // the full grid, then the y-stage output
  constexpr int SB = P * P * L;                   // z-stage output
  __shared__ C2<R> A[G][SA];
  __shared__ C2<R> B[G][SB];
  __shared__ int32_t fq[RW];
  const int64_t nch = (ntgt + G - 1) / G;
  const int64_t ch = xcd_item(nch);
  if (ch >= nch) return;
  const int64_t i0 = ch * G;
  const int ng = (int)min((int64_t)G, ntgt - i0);
  const int tid = threadIdx.x;
  // the G rows are contiguous: every load (two entries per thread) is issued
  // before the first LDS write; the pairs of the row's padding tail (past
  // live_pairs) are not loaded
  constexpr int RW2 = RW / 2, NV = (G * RW2 + NT - 1) / NT;
  C2x2<R> v[NV];
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    const int w = tid + k * NT;
    if (w < ng * RW2 && w % RW2 < live_pairs) v[k] = reinterpret_cast<const C2x2<R>*>(Lt + i0 * RW)[w];
  }
  for (int p = tid; p < RW; p += NT) fq[p] = freq[p];
  __syncthreads();
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    const int w = tid + k * NT;
    if (w < ng * RW2 && w % RW2 < live_pairs) {
      const int g = w / RW2, p = 2 * (w % RW2);
      const int f0 = fq[p], f1 = fq[p + 1];
      if (f0 >= 0) A[g][f0] = v[k].a;
      if (f1 >= 0) A[g][f1] = v[k].b;
    }
  }
  __syncthreads();
  // pass z: pencil xy = (xi, yi) over zi; B[g][kz + L xy]
  for (int w = tid; w < ng * P * P; w += NT) {
    const int g = w / (P * P), xy = w % (P * P);
    C2<R> in[P], out[L];
#pragma unroll
    for (int m = 0; m < P; ++m) in[m] = A[g][xy + P * P * m];
    dft_pencil<R, P, P, L, 1>(in, out);
#pragma unroll
    for (int k = 0; k < L; ++k) B[g][k + L * xy] = out[k];
  }
  __syncthreads();
  // pass y: pencil (kz, xi) over yi; A[g][xi * L^2 + ky + L kz]
  for (int w = tid; w < ng * P * L; w += NT) {
    const int g = w / (P * L), q = w % (P * L), kz = q % L, xi = q / L;
    C2<R> in[P], out[L];
#pragma unroll
    for (int m = 0; m < P; ++m) in[m] = B[g][kz + L * (xi + P * m)];
    dft_pencil<R, P, P, L, 1>(in, out);
#pragma unroll
    for (int k = 0; k < L; ++k) A[g][xi * L2 + k + L * kz] = out[k];
  }
  __syncthreads();
  // pass x: pencil (ky, kz) over xi, L contiguous node values
  for (int w = tid; w < ng * L2; w += NT) {
    const int g = w / L2, yz = w % L2;
    C2<R> in[P], out[L];
#pragma unroll
    for (int m = 0; m < P; ++m) in[m] = A[g][m * L2 + yz];
    dft_pencil<R, P, P, L, 1>(in, out);
    C2<R>* o = Lx + (int64_t)tgt[i0 + g] * L3 + yz * L;
#pragma unroll
    for (int k = 0; k < L; ++k) o[k] = out[k];
  }
}

// ------------------------------------------------------------------ dense M2L
// The alternative M2L (vector stacking of Sec. 4.2.2): all pairs sharing an
// offset share one dense matrix K[k][l] = G(x_k - y_l) (Sec. 2.2, M2L by
// definition), so tiles of 16 such pairs form a product [2L^3 x 2L^3] x
// [2L^3 x 16] in real arithmetic ([Re K, -Im K; Im K, Re K] times [Re M; Im M])
// on the matrix cores.  Results go to one slot per pair and are summed per
// target in list order (deterministic).

// K of each level-local offset, stored transposed (column-major, so the rows
// of an MFMA A-fragment are contiguous), zero-padded to dense_pad(L).
template <typename R, int L>
__global__ __launch_bounds__(256) void k_dense_K(int64_t n, const int32_t* __restrict__ delta, double kappa,
                                                 int screened, double h, C2<R>* __restrict__ Kt) {
  constexpr int L3 = L * L * L, NP = dense_pad(L);
  int64_t o = blockIdx.x;
  if (o >= n) return;
  const double dx = delta[3 * o], dy = delta[3 * o + 1], dz = delta[3 * o + 2];
  const double s = h / (double)(L - 1);
  for (int i = threadIdx.x; i < NP * NP; i += 256) {
    int c = i / NP, r = i % NP;  // Kt[c][r] = K[r][c]
    C2<R> v = {(R)0, (R)0};
    if (r < L3 && c < L3) {
      int rx = r % L, ry = (r / L) % L, rz = r / (L * L);
      int cx = c % L, cy = (c / L) % L, cz = c / (L * L);
      double z0 = h * dx + s * (double)(rx - cx), z1 = h * dy + s * (double)(ry - cy), z2 = h * dz + s * (double)(rz - cz);
      const C2<double> g = kernel_fp64(sqrt(z0 * z0 + z1 * z1 + z2 * z2), kappa, screened);
      v = {(R)g.x, (R)g.y};
    }
    Kt[o * NP * NP + i] = v;
  }
}

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));

template <typename R>
struct Mfma;
template <>
struct Mfma<float> {
  typedef f32x4 acc_t;
  __device__ static acc_t op(float a, float b, acc_t c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
};
template <>
struct Mfma<double> {
  typedef f64x4 acc_t;
  __device__ static acc_t op(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
};

// One wave per tile.  16x16x4 MFMA fragments: A[m][k] in lane m + 16k,
// B[k][n] in lane n + 16k; the result D[m][n] sits in lane n + 16 (m / 4),
// element m % 4 for the f32 instruction and in lane n + 16 (m % 4), element
// m / 4 for the f64 one (both checked on the device).
template <typename R, int L>
__global__ __launch_bounds__(64) void k_m2l_dense(int64_t ntile, const int32_t* __restrict__ t_off,
                                                  const int32_t* __restrict__ t_first,
                                                  const int32_t* __restrict__ t_cnt, const int32_t* __restrict__ src,
                                                  const int32_t* __restrict__ slot, const C2<R>* __restrict__ Kt,
                                                  const C2<R>* __restrict__ M, C2<R>* __restrict__ slots) {
  constexpr int L3 = L * L * L, NP = dense_pad(L), RR = 2 * NP, NT = RR / 16, KS = RR / 4;
  typedef typename Mfma<R>::acc_t acc_t;
  __shared__ R Bm[RR][17];
  const int64_t tile = blockIdx.x;
  if (tile >= ntile) return;
  const int lane = threadIdx.x;
  const int64_t o = t_off[tile];
  const int f = t_first[tile], cnt = t_cnt[tile];
  for (int i = lane; i < 16 * NP; i += 64) {
    int n = i / NP, k = i % NP;
    C2<R> v = {(R)0, (R)0};
    if (n < cnt && k < L3) v = M[(int64_t)src[f + n] * L3 + k];
    Bm[k][n] = v.x;
    Bm[NP + k][n] = v.y;
  }
  __syncthreads();
  acc_t acc[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) acc[t] = acc_t{0, 0, 0, 0};
  const C2<R>* Ko = Kt + o * NP * NP;
  const int mrow = lane % 16, kq = lane / 16;
  for (int st = 0; st < KS; ++st) {
    const int kk = 4 * st + kq;  // real column
    const R b = Bm[kk][mrow];
    const bool ycol = kk >= NP;
    const C2<R>* col = Ko + (int64_t)(ycol ? kk - NP : kk) * NP;
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      const bool imrow = t >= NT / 2;  // real rows NP.. hold imaginary parts
      const int r = (imrow ? t - NT / 2 : t) * 16 + mrow;
      const C2<R> kv = col[r];
      R a;
      if (!imrow) a = ycol ? -kv.y : kv.x;
      else a = ycol ? kv.x : kv.y;
      acc[t] = Mfma<R>::op(a, b, acc[t]);
    }
  }
  const int n = lane % 16;
  if (n < cnt) {
    const int64_t sl = slot[f + n];
    R* out = reinterpret_cast<R*>(slots + sl * L3);
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      const bool imrow = t >= NT / 2;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int m = sizeof(R) == 4 ? 4 * (lane / 16) + j : 4 * j + lane / 16;
        int r = (imrow ? t - NT / 2 : t) * 16 + m;
        if (r < L3) out[2 * r + (imrow ? 1 : 0)] = acc[t][j];
      }
    }
  }
}

// L_t = sum over the target's pairs of the dense slots, in list order.
template <typename R, int L>
__global__ __launch_bounds__(128) void k_dense_reduce(int64_t ntgt, const int32_t* __restrict__ tgt,
                                                      const int32_t* __restrict__ begin, int32_t kbase,
                                                      const C2<R>* __restrict__ slots, C2<R>* __restrict__ Lx) {
  constexpr int L3 = L * L * L;
  int64_t i = blockIdx.x;
  if (i >= ntgt) return;
  for (int k = threadIdx.x; k < L3; k += 128) {
    C2<R> acc = {(R)0, (R)0};
    for (int p = begin[i]; p < begin[i + 1]; ++p) {
      C2<R> v = slots[(int64_t)(p - kbase) * L3 + k];
      acc.x += v.x;
      acc.y += v.y;
    }
    Lx[(int64_t)tgt[i] * L3 + k] = acc;
  }
}

// ------------------------------------------------------------------ L2L
// L_{t'}^u(x'_h) += sum over father expansions v with Father(v) = u of
// exp(ik<x'_h - a_t, v>) (x)A_b^T (exp(-ik<x_k - a_t, v>) L_t^v).
template <typename R, int L>
__global__ __launch_bounds__(round64(L* L* L)) void k_l2l(int64_t n, const int32_t* __restrict__ ch,
                                                         const int32_t* __restrict__ begin,
                                                         const int32_t* __restrict__ par,
                                                         const int8_t* __restrict__ oct, TreeView T, Geo g,
                                                         C2<R>* __restrict__ Lx) {
  constexpr int L3 = L * L * L;
  __shared__ R A[2][L][L];
  __shared__ C2<R> phi[3][L], pho[3][L];
  __shared__ C2<R> b0[L3], b1[L3];
  int64_t item = blockIdx.x;
  if (item >= n) return;
  int ce = ch[item];
  int c = T.exp_cell[ce];
  double hc = ldexp(g.D, -T.level[c]), hp = 2.0 * hc;
  int tid = threadIdx.x;
  int hx = tid % L, hy = (tid / L) % L, hz = tid / (L * L);
  // the son's current values and its first father's, loaded before any work
  const int k0 = begin[item], k1 = begin[item + 1];
  const C2<R> cur = tid < L3 ? Lx[(int64_t)ce * L3 + tid] : C2<R>{(R)0, (R)0};
  C2<R> fv = (tid < L3 && k0 < k1) ? Lx[(int64_t)par[k0] * L3 + tid] : C2<R>{(R)0, (R)0};
  son_matrices<R, L>(A);
  C2<R> acc = {(R)0, (R)0};
  for (int k = k0; k < k1; ++k) {
    int pe = par[k];
    int o = oct[k];
    int b[3] = {o & 1, (o >> 1) & 1, (o >> 2) & 1};
    double v[3] = {T.exp_u[3 * pe], T.exp_u[3 * pe + 1], T.exp_u[3 * pe + 2]};
    __syncthreads();
    if (tid < 3 * L) {
      int d = tid / L, r = tid % L;
      phi[d][r] = expi<R>(-g.kappa * hp * v[d] * ((double)r / (double)(L - 1)));
      pho[d][r] = expi<R>(g.kappa * hc * v[d] * ((double)b[d] + (double)r / (double)(L - 1)));
    }
    __syncthreads();
    if (tid < L3) b0[tid] = cmul(cmul(fv, phi[0][hx]), cmul(phi[1][hy], phi[2][hz]));
    __syncthreads();
    if (tid < L3 && k + 1 < k1) fv = Lx[(int64_t)par[k + 1] * L3 + tid];
    if (tid < L3) {  // (hx, ky, kz)
      C2<R> s = {(R)0, (R)0};
#pragma unroll
      for (int kk = 0; kk < L; ++kk) cfma_r(s, b0[kk + L * hy + L * L * hz], A[b[0]][kk][hx]);
      b1[tid] = s;
    }
    __syncthreads();
    if (tid < L3) {  // (hx, hy, kz)
      C2<R> s = {(R)0, (R)0};
#pragma unroll
      for (int kk = 0; kk < L; ++kk) cfma_r(s, b1[hx + L * kk + L * L * hz], A[b[1]][kk][hy]);
      b0[tid] = s;
    }
    __syncthreads();
    if (tid < L3) {
      C2<R> s = {(R)0, (R)0};
#pragma unroll
      for (int kk = 0; kk < L; ++kk) cfma_r(s, b0[hx + L * hy + L * L * kk], A[b[2]][kk][hz]);
      C2<R> t = cmul(cmul(s, pho[0][hx]), cmul(pho[1][hy], pho[2][hz]));
      acc.x += t.x;
      acc.y += t.y;
    }
  }
  if (tid < L3) Lx[(int64_t)ce * L3 + tid] = {cur.x + acc.x, cur.y + acc.y};
}

// ------------------------------------------------------------------ L2P
// p(x) += sum_u exp(ik<x - a, u>) sum_h S_h(x) exp(-ik<x_h - a, u>) L^u(x_h).
// One wave per work item (a leaf and <= 256 of its points, 64 at a time).
// Leaves hold 18 points on average, so a chunk of m points is replicated:
// with m <= 16 the wave holds 4 replicas of 16 lanes, with m <= 32 two of 32,
// else one; replica q serves expansions q, q + NR, ... of the leaf, one point
// per lane, and the replicas' sums are added at the end.  The interpolation
// weights of a point are computed once; each replica stages its expansion in
// LDS with the node phases (its lanes loading the next one's values while the
// current one is summed).
template <typename R, int L>
__global__ __launch_bounds__(64) void k_l2p(int64_t n, const int32_t* __restrict__ cell,
                                            const int32_t* __restrict__ pfirst, const int32_t* __restrict__ pcount,
                                            TreeView T, Geo g, const C2<R>* __restrict__ Lx,
                                            C2<R>* __restrict__ ps) {
  constexpr int L3 = L * L * L, RMAX = 4, NV = (L3 + 64 / RMAX - 1) / (64 / RMAX);
  __shared__ C2<R> lp[RMAX][L3];
  const int64_t item = blockIdx.x;
  if (item >= n) return;
  const int c = cell[item];
  const double h = ldexp(g.D, -T.level[c]);
  const double ax = g.ox + h * T.ijk[3 * c], ay = g.oy + h * T.ijk[3 * c + 1], az = g.oz + h * T.ijk[3 * c + 2];
  const int first = pfirst[item], cnt = pcount[item];
  const int lane = threadIdx.x;
  const int e0 = T.exp_begin[c], ne = T.exp_begin[c + 1] - e0;
  const double kh = g.kappa * h / (double)(L - 1);
  for (int base = 0; base < cnt; base += 64) {
    const int m = min(64, cnt - base);
    const int nr = m <= 16 ? 4 : m <= 32 ? 2 : 1;  // replicas (uniform)
    const int lpr = 64 / nr, q = lane / lpr, x = lane - q * lpr;
    const bool on = x < m;
    const int j = base + x;
    double d0 = 0, d1 = 0, d2 = 0;
    if (on) {
      const int64_t pi = first + j;
      d0 = T.soa[pi] - ax;
      d1 = T.soa[T.n + pi] - ay;
      d2 = T.soa[2 * T.n + pi] - az;
    }
    R wx[L], wy[L], wz[L];
    lagrange<R, L>((R)(d0 / h), wx);
    lagrange<R, L>((R)(d1 / h), wy);
    lagrange<R, L>((R)(d2 / h), wz);
    C2<R> acc = {(R)0, (R)0};
    // replica q stages nodes x + lpr v of its expansion
    C2<R> nxt[NV];
    double nu0 = 0, nu1 = 0, nu2 = 0;  // the next expansion's direction
    if (q < ne) {
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        const int k = x + lpr * v;
        if (v * lpr < L3 && k < L3) nxt[v] = Lx[(int64_t)(e0 + q) * L3 + k];
      }
      nu0 = T.exp_u[3 * (e0 + q)];
      nu1 = T.exp_u[3 * (e0 + q) + 1];
      nu2 = T.exp_u[3 * (e0 + q) + 2];
    }
    for (int i = 0; i < ne; i += nr) {
      const int e = e0 + i + q;
      const bool has = i + q < ne;
      const double ux = nu0, uy = nu1, uz = nu2;
      __syncthreads();
      if (has) {
#pragma unroll
        for (int v = 0; v < NV; ++v) {
          const int k = x + lpr * v;
          if (v * lpr < L3 && k < L3) {
            const int kx = k % L, ky = (k / L) % L, kz = k / (L * L);
            lp[q][k] = cmul(nxt[v], expi<R>(-kh * (ux * kx + uy * ky + uz * kz)));
          }
        }
      }
      __syncthreads();
      if (i + nr + q < ne) {
#pragma unroll
        for (int v = 0; v < NV; ++v) {
          const int k = x + lpr * v;
          if (v * lpr < L3 && k < L3) nxt[v] = Lx[(int64_t)(e + nr) * L3 + k];
        }
        nu0 = T.exp_u[3 * (e + nr)];
        nu1 = T.exp_u[3 * (e + nr) + 1];
        nu2 = T.exp_u[3 * (e + nr) + 2];
      }
      if (on && has) {
        const C2<R>* l = lp[q];
        C2<R> sz = {(R)0, (R)0};
#pragma unroll
        for (int kz = 0; kz < L; ++kz) {
          C2<R> sy = {(R)0, (R)0};
#pragma unroll
          for (int ky = 0; ky < L; ++ky) {
            C2<R> sx = {(R)0, (R)0};
#pragma unroll
            for (int kx = 0; kx < L; ++kx) cfma_r(sx, l[kx + L * ky + L * L * kz], wx[kx]);
            cfma_r(sy, sx, wy[ky]);
          }
          cfma_r(sz, sy, wz[kz]);
        }
        cfma(acc, sz, expi<R>(g.kappa * (ux * d0 + uy * d1 + uz * d2)));
      }
    }
    // the replicas' sums: lane x collects lanes x + lpr, x + 2 lpr, ...
    for (int o = 32; o >= lpr; o >>= 1) {
      acc.x += __shfl_down(acc.x, o);
      acc.y += __shfl_down(acc.y, o);
    }
    if (on && q == 0) {
      C2<R> cur = ps[first + j];
      ps[first + j] = {cur.x + acc.x, cur.y + acc.y};
    }
    __syncthreads();
  }
}

// ------------------------------------------------------------------ P2P
// Near field (Sec. 2.2 P2P, Sec. 5.3 singular pairs): one work item = one
// block of <= 64 target points of a leaf and a chunk of its source ranges.
// Lanes are (target, sub-stream) pairs; sources are staged through LDS in
// tiles of 256; differences are formed in FP64 (coordinates are FP64), the
// rest in R.  Partial sums per work item are reduced in a fixed order.

// One (target, source) term.  kscale is kappa / (2 pi) for the Helmholtz
// kernel (the phase in turns: v_sin/v_cos on the complex64 path,
// sincos_turns on the complex128 path) and kappa log2(e) for the screened
// one (the exponent for v_exp on the complex64 path; the complex128 path
// takes exp(-kappa r) from kappa).
template <typename R, bool SCREENED>
__device__ __forceinline__ void p2p_pair(C2<R>& acc, double x0, double x1, double x2, double y0, double y1,
                                         double y2, C2<R> q, R kscale, R kappa, R tau2);

template <>
__device__ __forceinline__ void p2p_pair<float, false>(C2<float>& acc, double x0, double x1, double x2, double y0,
                                                       double y1, double y2, C2<float> q, float kap2pi, float,
                                                       float tau2) {
  float dx = (float)(x0 - y0), dy = (float)(x1 - y1), dz = (float)(x2 - y2);
  float r2 = fmaf(dz, dz, fmaf(dy, dy, dx * dx));
  float rinv = __builtin_amdgcn_rsqf(r2);
  rinv = r2 > tau2 ? rinv : 0.0f;
  float r = r2 * rinv;
  float f = __builtin_amdgcn_fractf(r * kap2pi);  // revolutions of kappa r
  float sn = __builtin_amdgcn_sinf(f);             // sin(2 pi f)
  float cs = __builtin_amdgcn_cosf(f);
  float gr = cs * rinv, gi = sn * rinv;
  acc.x = fmaf(gr, q.x, fmaf(-gi, q.y, acc.x));
  acc.y = fmaf(gr, q.y, fmaf(gi, q.x, acc.y));
}

template <>
__device__ __forceinline__ void p2p_pair<float, true>(C2<float>& acc, double x0, double x1, double x2, double y0,
                                                      double y1, double y2, C2<float> q, float klog2e, float,
                                                      float tau2) {
  float dx = (float)(x0 - y0), dy = (float)(x1 - y1), dz = (float)(x2 - y2);
  float r2 = fmaf(dz, dz, fmaf(dy, dy, dx * dx));
  float rinv = __builtin_amdgcn_rsqf(r2);
  rinv = r2 > tau2 ? rinv : 0.0f;
  float r = r2 * rinv;
  float g = __builtin_amdgcn_exp2f(-r * klog2e) * rinv;  // exp(-kappa r) / r
  acc.x = fmaf(g, q.x, acc.x);
  acc.y = fmaf(g, q.y, acc.y);
}

template <>
__device__ __forceinline__ void p2p_pair<double, false>(C2<double>& acc, double x0, double x1, double x2, double y0,
                                                        double y1, double y2, C2<double> q, double kap2pi, double,
                                                        double tau2) {
  double dx = x0 - y0, dy = x1 - y1, dz = x2 - y2;
  double r2 = fma(dz, dz, fma(dy, dy, dx * dx));
  if (r2 > tau2) {
    // 1/r from v_rsq_f64 and two Newton steps, y <- y (3 - r2 y^2) / 2
    double rinv = __builtin_amdgcn_rsq(r2);
    rinv = rinv * fma(-0.5 * r2, rinv * rinv, 1.5);
    rinv = rinv * fma(-0.5 * r2, rinv * rinv, 1.5);
    const double r = r2 * rinv;
    double s, c;
    sincos_turns(r * kap2pi, s, c);  // e^{i kappa r}
    double gr = c * rinv, gi = s * rinv;
    acc.x = fma(gr, q.x, fma(-gi, q.y, acc.x));
    acc.y = fma(gr, q.y, fma(gi, q.x, acc.y));
  }
}

template <>
__device__ __forceinline__ void p2p_pair<double, true>(C2<double>& acc, double x0, double x1, double x2, double y0,
                                                       double y1, double y2, C2<double> q, double, double kappa,
                                                       double tau2) {
  double dx = x0 - y0, dy = x1 - y1, dz = x2 - y2;
  double r2 = fma(dz, dz, fma(dy, dy, dx * dx));
  if (r2 > tau2) {
    double r = sqrt(r2);
    double g = exp(-kappa * r) / r;
    acc.x = fma(g, q.x, acc.x);
    acc.y = fma(g, q.y, acc.y);
  }
}

template <typename R, bool SCREENED>
__device__ __forceinline__ void p2p_item(int64_t w, const int32_t* __restrict__ wi_blk,
                                            const int32_t* __restrict__ wi_seg, const int32_t* __restrict__ seg_first,
                                            const int32_t* __restrict__ seg_count, const int32_t* __restrict__ blk_first,
                                            const int32_t* __restrict__ blk_count, const double* __restrict__ X,
                                            int64_t nx, const double* __restrict__ Y, int64_t ny,
                                            const C2<R>* __restrict__ qs, C2<R>* __restrict__ part, double kappa,
                                            double tau2, double* sx, double* sy, double* sz, C2<R>* sq,
                                            C2<R>* red, int* pre, int* sfirst) {
  // One wave per work item.  Lane = (target pair, sub-stream): each lane owns
  // two targets of the block, so each source read from LDS feeds two
  // independent pair evaluations.
  constexpr int NT = 64;
  const int blk = wi_blk[w];
  const int tf = blk_first[blk], tc = blk_count[blk];
  const int np = (tc + 1) >> 1;  // target pairs
  const int S = NT / np;         // sub-streams
  const int lane = threadIdx.x;
  const int tp = lane % np, sub = lane / np;
  const bool active = sub < S;
  const int ta = 2 * tp, tb = min(2 * tp + 1, tc - 1);
  double xa0 = 0, xa1 = 0, xa2 = 0, xb0 = 0, xb1 = 0, xb2 = 0;
  if (active) {
    xa0 = X[tf + ta];
    xa1 = X[nx + tf + ta];
    xa2 = X[2 * nx + tf + ta];
    xb0 = X[tf + tb];
    xb1 = X[nx + tf + tb];
    xb2 = X[2 * nx + tf + tb];
  }
  // segment prefix sums: one segment per lane, wave-wide inclusive scan
  const int sb = wi_seg[w], ns = wi_seg[w + 1] - sb;
  int len = 0;
  if (lane < ns) {
    len = seg_count[sb + lane];
    sfirst[lane] = seg_first[sb + lane];
  }
  int incl = len;
#pragma unroll
  for (int d = 1; d < NT; d <<= 1) {
    int v = __shfl_up(incl, d, NT);
    if (lane >= d) incl += v;
  }
  pre[lane + 1] = incl;
  if (lane == 0) pre[0] = 0;
  __syncthreads();
  const int total = pre[ns];
  const R inv4pi = (R)(1.0 / (4.0 * M_PI));
  const R kscale = (R)(SCREENED ? kappa * 1.4426950408889634 : kappa / (2.0 * M_PI));  // log2(e), 1/(2 pi)
  auto locate = [&](int pos) {
    int lo = 0, hi = ns - 1;
    while (lo < hi) {
      int mid = (lo + hi + 1) >> 1;
      if (pre[mid] <= pos) lo = mid;
      else hi = mid - 1;
    }
    return sfirst[lo] + (pos - pre[lo]);
  };
  double ry0 = 0, ry1 = 0, ry2 = 0;
  C2<R> rq = {(R)0, (R)0};
  bool valid = lane < total;
  if (valid) {
    int j = locate(lane);
    ry0 = Y[j];
    ry1 = Y[ny + j];
    ry2 = Y[2 * ny + j];
    rq = cscale(qs[j], inv4pi);
  }
  C2<R> acca = {(R)0, (R)0}, accb = {(R)0, (R)0};
  for (int base = 0; base < total; base += NT) {
    if (valid) {
      sx[lane] = ry0;
      sy[lane] = ry1;
      sz[lane] = ry2;
      sq[lane] = rq;
    }
    __syncthreads();
    int npos = base + NT + lane;
    valid = npos < total;
    if (valid) {  // prefetch the next tile while this one is consumed
      int j = locate(npos);
      ry0 = Y[j];
      ry1 = Y[ny + j];
      ry2 = Y[2 * ny + j];
      rq = cscale(qs[j], inv4pi);
    }
    int m = min(NT, total - base);
    if (active) {
#pragma unroll 2
      for (int k = sub; k < m; k += S) {
        double y0 = sx[k], y1 = sy[k], y2 = sz[k];
        C2<R> q = sq[k];
        p2p_pair<R, SCREENED>(acca, xa0, xa1, xa2, y0, y1, y2, q, kscale, (R)kappa, (R)tau2);
        p2p_pair<R, SCREENED>(accb, xb0, xb1, xb2, y0, y1, y2, q, kscale, (R)kappa, (R)tau2);
      }
    }
    __syncthreads();
  }
  red[2 * lane] = acca;
  red[2 * lane + 1] = accb;
  __syncthreads();
  if (lane < tc) {
    const int p = lane >> 1, which = lane & 1;
    C2<R> s = {(R)0, (R)0};
    for (int u = 0; u < S; ++u) {
      C2<R> v = red[2 * (u * np + p) + which];
      s.x += v.x;
      s.y += v.y;
    }
    part[w * 64 + lane] = s;
  }
  __syncthreads();
}

// Persistent near field: a bounded number of one-wave workgroups per CU pull
// work items from 8 queues, queue j covering the j-th eighth of the items
// (workgroup b starts on queue b % 8, which the hardware places on XCD b % 8,
// keeping neighbouring items in one L2), then help the other queues.  The
// free wave slots stay available to the far-field kernels on the other
// stream.  Every workgroup leaves once all queues are drained.
template <typename R, bool SCREENED>
__global__ __launch_bounds__(64) void k_p2p(int64_t nwi, int* __restrict__ queue, const int32_t* __restrict__ wi_blk,
                                            const int32_t* __restrict__ wi_seg, const int32_t* __restrict__ seg_first,
                                            const int32_t* __restrict__ seg_count, const int32_t* __restrict__ blk_first,
                                            const int32_t* __restrict__ blk_count, const double* __restrict__ X,
                                            int64_t nx, const double* __restrict__ Y, int64_t ny,
                                            const C2<R>* __restrict__ qs, C2<R>* __restrict__ part, double kappa,
                                            double tau2) {
  __shared__ double sx[64], sy[64], sz[64];
  __shared__ C2<R> sq[64];
  __shared__ C2<R> red[128];
  __shared__ int pre[65];
  __shared__ int sfirst[64];
  __shared__ int next;
  const int64_t nper = (nwi + 7) / 8;
  const int q0 = (int)(blockIdx.x % 8);
  for (int qq = 0; qq < 8; ++qq) {
    const int qi = (q0 + qq) % 8;
    const int64_t lo = qi * nper, hi = min(nwi, (int64_t)(qi + 1) * nper);
    for (;;) {
      if (threadIdx.x == 0) next = atomicAdd(&queue[qi], 1);
      __syncthreads();
      const int64_t w = lo + next;
      __syncthreads();
      if (w >= hi) break;
      p2p_item<R, SCREENED>(w, wi_blk, wi_seg, seg_first, seg_count, blk_first, blk_count, X, nx, Y, ny, qs, part, kappa,
                  tau2, sx, sy, sz, sq, red, pre, sfirst);
    }
  }
}

__global__ void k_zero_int(int n, int* __restrict__ a) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) a[i] = 0;
}

template <typename R>
__global__ void k_p2p_reduce(int64_t nblk, const int32_t* __restrict__ blk_first,
                             const int32_t* __restrict__ blk_count, const int32_t* __restrict__ blk_wi,
                             const C2<R>* __restrict__ part, C2<R>* __restrict__ ps) {
  int64_t b = blockIdx.x;
  int tid = threadIdx.x;
  if (b >= nblk || tid >= blk_count[b]) return;
  C2<R> s = {(R)0, (R)0};
  for (int w = blk_wi[b]; w < blk_wi[b + 1]; ++w) {
    C2<R> v = part[(int64_t)w * 64 + tid];
    s.x += v.x;
    s.y += v.y;
  }
  ps[blk_first[b] + tid] = s;
}

// ------------------------------------------------------------------ launchers
#define DEFMM_L_SWITCH(Lval, ...)                          \
  switch (Lval) {                                          \
    case 2: { constexpr int LL = 2; __VA_ARGS__; } break;  \
    case 3: { constexpr int LL = 3; __VA_ARGS__; } break;  \
    case 4: { constexpr int LL = 4; __VA_ARGS__; } break;  \
    case 5: { constexpr int LL = 5; __VA_ARGS__; } break;  \
    case 6: { constexpr int LL = 6; __VA_ARGS__; } break;  \
    case 7: { constexpr int LL = 7; __VA_ARGS__; } break;  \
    case 8: { constexpr int LL = 8; __VA_ARGS__; } break;  \
    default: return hipErrorInvalidValue;                  \
  }

template <typename R>
static hipError_t spectra_impl(DevPlan& P, const int32_t* lev, const int32_t* delta, hipStream_t s) {
  if (P.n_spec == 0) return hipSuccess;
  DEFMM_L_SWITCH(P.L, hipLaunchKernelGGL((k_spectra<R, LL>), dim3((unsigned)P.n_spec), dim3(256), 0, s, P.n_spec,
                                         lev, delta, P.kappa, P.screened ? 1 : 0, P.D, P.freq, P.sym ? 2 : 1,
                                         (C2<R>*)P.spectra));
  return hipGetLastError();
}

template <typename R>
static hipError_t dense_K_impl(DevPlan& P, int l, const int32_t* delta, hipStream_t s) {
  int64_t n = P.dns_off_begin[l + 1] - P.dns_off_begin[l];
  if (n == 0) return hipSuccess;
  double h = std::ldexp(P.D, -l);
  DEFMM_L_SWITCH(P.L, hipLaunchKernelGGL((k_dense_K<R, LL>), dim3((unsigned)n), dim3(256), 0, s, n, delta, P.kappa,
                                         P.screened ? 1 : 0, h, (C2<R>*)P.dense_K[l]));
  return hipGetLastError();
}

hipError_t compute_dense_K(DevPlan& P, int level, const int32_t* delta, hipStream_t s) {
  return P.precision == 0 ? dense_K_impl<double>(P, level, delta, s) : dense_K_impl<float>(P, level, delta, s);
}

hipError_t compute_spectra(DevPlan& P, const int32_t* lev, const int32_t* delta, hipStream_t s) {
  return P.precision == 0 ? spectra_impl<double>(P, lev, delta, s) : spectra_impl<float>(P, lev, delta, s);
}

namespace {

struct PassTimer {
  Workspace& W;
  hipStream_t s;
  hipStream_t cur;
  int pass = -1;
  size_t a = 0;
  PassTimer(Workspace& w, hipStream_t st) : W(w), s(st), cur(st) {}
  hipEvent_t next() {
    if (W.ev_used == W.ev_pool.size()) {
      hipEvent_t e;
      if (hipEventCreate(&e) != hipSuccess) return nullptr;
      W.ev_pool.push_back(e);
    }
    return W.ev_pool[W.ev_used++];
  }
  void begin(int p) { begin(p, s); }
  void begin(int p, hipStream_t st) {
    cur = st;
    if (!W.timing) return;
    pass = p;
    a = W.ev_used;
    hipEvent_t e = next();
    if (e) (void)hipEventRecord(e, cur);
  }
  void end() {
    if (!W.timing || pass < 0) return;
    size_t b = W.ev_used;
    hipEvent_t e = next();
    if (e) {
      (void)hipEventRecord(e, cur);
      W.pending.push_back({pass, a, b});
    }
    pass = -1;
  }
};

inline unsigned blocks_for(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

}  // namespace

// Dispatch on the M2F/F2L expansions per workgroup (1, 2 or 4; 0 = the
// default), GG a compile-time constant capped at what fits LDS.
#define DEFMM_G_SWITCH(gv, RR, LLL, ...)                                            \
  do {                                                                              \
    switch (gv) {                                                                   \
      case 1: {                                                                     \
        constexpr int GG = 1;                                                       \
        __VA_ARGS__;                                                                \
        break;                                                                      \
      }                                                                             \
      case 2: {                                                                     \
        constexpr int GG = fourier_items_capped<RR, LLL, 2>();                      \
        __VA_ARGS__;                                                                \
        break;                                                                      \
      }                                                                             \
      case 4: {                                                                     \
        constexpr int GG = fourier_items_capped<RR, LLL, 4>();                      \
        __VA_ARGS__;                                                                \
        break;                                                                      \
      }                                                                             \
      default: {                                                                    \
        constexpr int GG = fourier_items<RR, LLL>();                                \
        __VA_ARGS__;                                                                \
        break;                                                                      \
      }                                                                             \
    }                                                                               \
  } while (0)

template <typename R>
static hipError_t matvec_impl(DevPlan& P, Workspace& W, const void* q, void* p, hipStream_t s) {
  const int L = P.L;
  const int L3 = L * L * L;
  Geo g{P.kappa, P.D, P.origin[0], P.origin[1], P.origin[2]};
  TreeView TX = view(P.tx), TY = view(P.ty);
  C2<R>* qs = (C2<R>*)W.qs;
  C2<R>* ps = (C2<R>*)W.ps;
  C2<R>* M = (C2<R>*)W.M;
  C2<R>* Lx = (C2<R>*)W.Lx;
  C2<R>* Mt = (C2<R>*)W.Mt;
  C2<R>* part = (C2<R>*)W.part;
  const C2<R>* S = (const C2<R>*)P.spectra;
  PassTimer tm(W, s);

  tm.begin(kPassSetup);
  if (P.ny > 0)
    hipLaunchKernelGGL((k_gather<R>), dim3(blocks_for(P.ny, 256)), dim3(256), 0, s, P.ny, P.ty.perm,
                       (const C2<R>*)q, qs);
  // a local expansion is written by its M2L (an M2L target), by L2L, or by
  // neither (cleared here); the node-per-thread L2L adds to what is there, so
  // it needs every one cleared first
  if (P.tx.nexp > 0 && !W.pencil_updown)
    hipLaunchKernelGGL((k_zero<R>), dim3(blocks_for(P.tx.nexp * L3, 256)), dim3(256), 0, s, P.tx.nexp * L3, Lx);
  else if (P.n_zero_exp > 0)
    DEFMM_L_SWITCH(L, hipLaunchKernelGGL((k_zero_rows<R, LL * LL * LL>),
                                          dim3(blocks_for(P.n_zero_exp, kZeroRowsPerBlock)), dim3(256), 0, s,
                                          P.n_zero_exp, P.zero_exp, Lx));
  tm.end();

  // Near field on the workspace's side stream, concurrently with the far
  // field (the ALU-bound P2P overlaps the L2-bound M2L); joined before L2P.
  // Forked after the charge gather (overlap 1) or after M2F (overlap 2, so
  // the short upward-pass kernels do not compete with the persistent P2P).
  hipStream_t s2 = (W.side && W.overlap) ? W.side : s;
  auto launch_near = [&]() -> hipError_t {
    if (s2 != s) {
      hipError_t e = hipEventRecord(W.ev_fork, s);
      if (e == hipSuccess) e = hipStreamWaitEvent(s2, W.ev_fork, 0);
      if (e != hipSuccess) return e;
    }
    if (P.nx > 0) hipLaunchKernelGGL((k_zero<R>), dim3(blocks_for(P.nx, 256)), dim3(256), 0, s2, P.nx, ps);
    tm.begin(kPassP2P, s2);
    if (P.nwi > 0) {
      hipLaunchKernelGGL(k_zero_int, dim3(1), dim3(64), 0, s2, 8, W.queue);
      const int wpc = (s2 != s) ? W.p2p_waves : 8;  // alone: fill every wave slot
      const unsigned nb = (unsigned)std::min<int64_t>(P.nwi, (int64_t)P.num_cu * wpc);
      if (P.screened)
        hipLaunchKernelGGL((k_p2p<R, true>), dim3(nb), dim3(64), 0, s2, P.nwi, W.queue, P.wi_blk, P.wi_seg_begin,
                           P.seg_first, P.seg_count, P.blk_first, P.blk_count, P.tx.soa, P.tx.n, P.ty.soa, P.ty.n,
                           (const C2<R>*)qs, part, P.kappa, P.tau * P.tau);
      else
        hipLaunchKernelGGL((k_p2p<R, false>), dim3(nb), dim3(64), 0, s2, P.nwi, W.queue, P.wi_blk, P.wi_seg_begin,
                           P.seg_first, P.seg_count, P.blk_first, P.blk_count, P.tx.soa, P.tx.n, P.ty.soa, P.ty.n,
                           (const C2<R>*)qs, part, P.kappa, P.tau * P.tau);
    }
    tm.end();
    tm.begin(kPassP2PRed, s2);
    if (P.nblk > 0)
      hipLaunchKernelGGL((k_p2p_reduce<R>), dim3((unsigned)P.nblk), dim3(64), 0, s2, P.nblk, P.blk_first,
                         P.blk_count, P.blk_wi_begin, (const C2<R>*)part, ps);
    tm.end();
    if (s2 != s) return hipEventRecord(W.ev_join, s2);
    return hipSuccess;
  };
  const bool fork_late = s2 != s && W.overlap == 2;
  if (!fork_late) {
    hipError_t e = launch_near();
    if (e != hipSuccess) return e;
  }

  tm.begin(kPassP2M);
  if (P.n_p2m_leaf > 0 && W.pencil_updown) {
    DEFMM_L_SWITCH(L, hipLaunchKernelGGL((k_p2m_leaf<R, LL>), dim3((unsigned)P.n_p2m_leaf),
                                          dim3(round64(LL * LL * LL)), 0, s, P.n_p2m_leaf, P.p2m_leaf, TY, g,
                                          (const C2<R>*)qs, M));
  } else if (P.n_p2m > 0) {
    DEFMM_L_SWITCH(L, hipLaunchKernelGGL((k_p2m<R, LL>), dim3((unsigned)P.n_p2m), dim3(round64(LL * LL * LL)), 0,
                                          s, P.n_p2m, P.p2m_exp, TY, g, (const C2<R>*)qs, M));
  }
  tm.end();

  tm.begin(kPassM2M);
  for (int l = (int)P.m2m.size() - 1; l >= 0; --l) {
    const LevelTable& t = P.m2m[l];
    if (t.n == 0) continue;
    if (W.pencil_updown) {
      DEFMM_L_SWITCH(L, hipLaunchKernelGGL((k_m2m_p<R, LL>), dim3((unsigned)t.npair), dim3(64), 0, s, t.npair,
                                            t.pair, t.a, t.b, t.oct, TY, g, M));
    } else {
      DEFMM_L_SWITCH(L, hipLaunchKernelGGL((k_m2m<R, LL>), dim3((unsigned)t.n), dim3(round64(LL * LL * LL)), 0,
                                            s, t.n, t.a, t.b, t.oct, TY, g, M));
    }
  }
  tm.end();

  // levels whose M2L runs dense skip M2F/F2L; the others use the Fourier path,
  // launched once per maximal range of consecutive Fourier levels (all levels
  // share L, and every table is level-major, so a range is a contiguous slice)
  const int nlev = (int)P.lvl_m2f.size() - 1;
  auto is_dense = [&](int l) {
    return l < (int)W.dense_level.size() && W.dense_level[l] && l < (int)P.dense_ok.size() && P.dense_ok[l];
  };
  int fr_lo[kMaxLevel + 2], fr_hi[kMaxLevel + 2], nfr = 0;
  for (int l = 0; l < nlev;) {
    if (is_dense(l)) {
      ++l;
      continue;
    }
    int e = l;
    while (e < nlev && !is_dense(e)) ++e;
    fr_lo[nfr] = l;
    fr_hi[nfr++] = e;
    l = e;
  }
  const int64_t P3R = fourier_row(L);
  tm.begin(kPassM2F);
  for (int k = 0; k < nfr; ++k) {
    const int64_t rb = P.lvl_m2f[fr_lo[k]], nr = P.lvl_m2f[fr_hi[k]] - rb;
    if (nr == 0) continue;
    DEFMM_L_SWITCH(L, DEFMM_G_SWITCH(W.fourier_items, R, LL, hipLaunchKernelGGL((k_m2f<R, LL, GG>),
                                     dim3(fourier_grid((nr + GG - 1) / GG, P.num_cu)), dim3(256), 0, s, nr,
                                     P.m2f_exp + rb, P.freq, (const C2<R>*)M, Mt + rb * P3R)));
  }
  tm.end();
  if (fork_late) {
    hipError_t e = launch_near();
    if (e != hipSuccess) return e;
  }

  tm.begin(kPassM2LDense);
  for (int l = 0; l < nlev; ++l) {
    const int64_t tb = P.m2l_level_tgt[l], nt = P.m2l_level_tgt[l + 1] - tb;
    if (nt == 0 || !is_dense(l)) continue;
    const int64_t t0 = P.dns_tile_begin[l], ntl = P.dns_tile_begin[l + 1] - t0;
    DEFMM_L_SWITCH(L, hipLaunchKernelGGL((k_m2l_dense<R, LL>), dim3((unsigned)ntl), dim3(64), 0, s, ntl,
                                         P.dns_tile_off + t0, P.dns_tile_first + t0, P.dns_tile_cnt + t0,
                                         P.dns_src, P.dns_slot, (const C2<R>*)P.dense_K[l], (const C2<R>*)M,
                                         (C2<R>*)W.slots));
    DEFMM_L_SWITCH(L, hipLaunchKernelGGL((k_dense_reduce<R, LL>), dim3((unsigned)nt), dim3(128), 0, s, nt,
                                         P.m2l_tgt + tb, P.m2l_begin + tb, P.host.m2l_begin[tb],
                                         (const C2<R>*)W.slots, Lx));
  }
  tm.end();

  tm.begin(kPassM2L);
  C2<R>* Lt = (C2<R>*)W.Lt;
  for (int k = 0; k < nfr; ++k) {
    const int64_t tb = P.m2l_level_tgt[fr_lo[k]], nt = P.m2l_level_tgt[fr_hi[k]] - tb;
    if (nt == 0) continue;
    if (W.m2l_variant == 0) {
      DEFMM_L_SWITCH(L, hipLaunchKernelGGL((k_m2l<R, LL>), dim3(xcd_grid(nt)), dim3(256), 0, s, nt, P.m2l_tgt + tb,
                                           P.m2l_begin + tb, (const int2*)P.m2l_pair, P.freq, P.perm, P.sym ? 1 : 0,
                                           (const C2<R>*)Mt, S, Lx));
    } else if (W.m2l_variant == 2) {
      const int64_t gb = P.lvl_grp[fr_lo[k]], ng = P.lvl_grp[fr_hi[k]] - gb;
      if (P.sym) {
        DEFMM_L_SWITCH(L, hipLaunchKernelGGL((k_m2l_runs<R, LL, m2l_slices(LL), true>),
                                             dim3(xcd_grid(m2l_slices(LL) * ng)), dim3(64), 0, s, ng,
                                             P.grp_tfirst + gb, P.grp_tcount + gb, P.grp_run_begin + gb, P.runs,
                                             P.perm, P.freq, (const C2<R>*)Mt, S, Lt));
      } else {
        DEFMM_L_SWITCH(L, hipLaunchKernelGGL((k_m2l_runs<R, LL, m2l_slices(LL), false>),
                                             dim3(xcd_grid(m2l_slices(LL) * ng)), dim3(64), 0, s, ng,
                                             P.grp_tfirst + gb, P.grp_tcount + gb, P.grp_run_begin + gb, P.runs,
                                             P.perm, P.freq, (const C2<R>*)Mt, S, Lt));
      }
    } else {
      if (P.sym) {
        DEFMM_L_SWITCH(L, hipLaunchKernelGGL((k_m2l_slice<R, LL, m2l_slices(LL), true>),
                                             dim3(xcd_grid(m2l_slices(LL) * nt)), dim3(64), 0, s, nt,
                                             P.m2l_begin + tb, (const int2*)P.m2l_pair, P.perm, (const C2<R>*)Mt, S,
                                             Lt + tb * P3R));
      } else {
        DEFMM_L_SWITCH(L, hipLaunchKernelGGL((k_m2l_slice<R, LL, m2l_slices(LL), false>),
                                             dim3(xcd_grid(m2l_slices(LL) * nt)), dim3(64), 0, s, nt,
                                             P.m2l_begin + tb, (const int2*)P.m2l_pair, P.perm, (const C2<R>*)Mt, S,
                                             Lt + tb * P3R));
      }
    }
  }
  tm.end();
  tm.begin(kPassF2L);
  if (W.m2l_variant != 0)
    for (int k = 0; k < nfr; ++k) {
      const int64_t tb = P.m2l_level_tgt[fr_lo[k]], nt = P.m2l_level_tgt[fr_hi[k]] - tb;
      if (nt == 0) continue;
      DEFMM_L_SWITCH(L, DEFMM_G_SWITCH(W.fourier_items, R, LL, hipLaunchKernelGGL((k_f2l<R, LL, GG>),
                                       dim3(xcd_grid((nt + GG - 1) / GG)), dim3(256), 0, s, nt, P.m2l_tgt + tb,
                                       P.freq, P.live_pairs, (const C2<R>*)(Lt + tb * P3R), Lx)));
    }
  tm.end();

  tm.begin(kPassL2L);
  for (size_t l = 0; l < P.l2l.size(); ++l) {
    const LevelTable& t = P.l2l[l];
    if (t.n == 0) continue;
    if (W.pencil_updown && std::is_same<R, float>::value && t.fam) {
      DEFMM_L_SWITCH(L, hipLaunchKernelGGL((k_l2l_f<float, LL>), dim3((unsigned)t.nfpair), dim3(64), 0, s,
                                            t.nfpair, t.fpair, t.fam, t.c, P.has_m2l, TX, g,
                                            reinterpret_cast<C2<float>*>(Lx)));
    } else if (W.pencil_updown) {
      DEFMM_L_SWITCH(L, hipLaunchKernelGGL((k_l2l_p<R, LL>), dim3((unsigned)t.npair), dim3(64), 0, s, t.npair,
                                            t.pair, t.a, t.b, t.c, t.oct, P.has_m2l, TX, g, Lx));
    } else {
      DEFMM_L_SWITCH(L, hipLaunchKernelGGL((k_l2l<R, LL>), dim3((unsigned)t.n), dim3(round64(LL * LL * LL)), 0,
                                            s, t.n, t.a, t.b, t.c, t.oct, TX, g, Lx));
    }
  }
  tm.end();

  if (s2 != s) {
    hipError_t e = hipStreamWaitEvent(s, W.ev_join, 0);
    if (e != hipSuccess) return e;
  }

  tm.begin(kPassL2P);
  if (P.n_l2p > 0)
    DEFMM_L_SWITCH(L, hipLaunchKernelGGL((k_l2p<R, LL>), dim3((unsigned)P.n_l2p), dim3(64), 0, s, P.n_l2p,
                                          P.l2p_cell, P.l2p_first, P.l2p_count, TX, g, (const C2<R>*)Lx, ps));
  tm.end();

  tm.begin(kPassScatter);
  if (P.nx > 0)
    hipLaunchKernelGGL((k_scatter<R>), dim3(blocks_for(P.nx, 256)), dim3(256), 0, s, P.nx, P.tx.perm,
                       (const C2<R>*)ps, (C2<R>*)p);
  tm.end();
  return hipGetLastError();
}

hipError_t run_matvec(DevPlan& P, Workspace& W, const void* q, void* p, hipStream_t s) {
  return P.precision == 0 ? matvec_impl<double>(P, W, q, p, s) : matvec_impl<float>(P, W, q, p, s);
}

}  // namespace defmm
