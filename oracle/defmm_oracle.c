/*
 * defmm oracle -- TEST INFRASTRUCTURE ONLY.  Nothing in the product path may
 * load or call this file; only the tests, the smoke check and the benchmark's
 * CPU-baseline leg do.
 *
 * A plain FP64 CPU implementation of the directional equispaced-interpolation
 * FMM of Chollet, Claeys, Fortin and Grigori (defmm) and of the direct sum it
 * approximates.  Each step follows the paper's definitions in the paper's
 * order; loops are written the obvious way (no blocking, no tensorisation,
 * no fast transforms).  OpenMP parallelises independent outer loops only.
 *
 * Readings of passages that are silent or ambiguous (kept identical in the
 * GPU library, which is written separately):
 *  - L is the number of nodes per dimension, nodes include both cell faces
 *    (Sec. 2.3 and Lemma 1); the padded length is P = 2L-1.
 *  - DFT convention: D = fftn(c) with exp(-2 pi i), inverse with 1/P^3
 *    (eq. DFTformula up to the normalisation constant).
 *  - w in the MAC (eq. macdirref) is half the cell side; dist(t,s) is the
 *    distance between the two cubes; equality is admissible.
 *  - a level is high-frequency iff kappa*w > hf_threshold (never for the
 *    screened kernel, which does not oscillate).
 *  - directions: projected centres of the faces of the cube (Sec. 4.1.2),
 *    6 * 4^E of them at direction level E, E = 0 at the deepest high-
 *    frequency level, plus dir_refine extra subdivisions.
 *  - best direction (Alg. 2): argmax <v, ctr(t)-ctr(s)>, ties within
 *    1e-12 |delta| go to the smallest index.
 *  - P2P singularity (Sec. 5.3): the term is 0 when |x-y| <= tau = 1e-12 D.
 *
 * Parity: pinned by the CPU tests (direct sum on tiny inputs, polynomial
 * reproduction, circulant-vs-dense M2L, Fourier-domain symmetries, pair
 * coverage, geometric convergence in L).
 */
#include "defmm_oracle.h"

#include <complex.h>
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif
#include <time.h>

typedef double complex cplx;

#define KEYBITS 21
#define MAXLEV 21
#define PI 3.14159265358979323846

static double wall_seconds(void) {
  struct timespec ts;
  clock_gettime(CLOCK_MONOTONIC, &ts);
  return (double)ts.tv_sec + 1e-9 * (double)ts.tv_nsec;
}

/* The kernel G(r), r = |x - y|:
     ORACLE_HELMHOLTZ  exp(i kappa r) / (4 pi r)   (Sec. 1, the paper's kernel);
     ORACLE_YUKAWA     exp(-kappa r) / (4 pi r)    (screened: one of the asymptotically
                       smooth kernels the interpolation framework covers, Sec. 1). */
static cplx kernel_G(double r, double kappa, int kernel) {
  if (kernel == ORACLE_YUKAWA) return exp(-kappa * r) / (4.0 * PI * r);
  return cexp(I * kappa * r) / (4.0 * PI * r);
}

/* ------------------------------------------------------------------ */
/* Direct sum, eq. (fmmsum).                                            */
/* ------------------------------------------------------------------ */
void oracle_direct_sum(const double* X, int64_t nx, const double* Y, int64_t ny,
                       const double* q, double kappa, double tau,
                       const int64_t* targets, int64_t nt, double* p, int32_t kernel) {
  const cplx* qc = (const cplx*)q;
  cplx* pc = (cplx*)p;
  (void)nx;
#pragma omp parallel for schedule(dynamic, 8)
  for (int64_t a = 0; a < nt; ++a) {
    int64_t i = targets ? targets[a] : a;
    cplx acc = 0.0;
    for (int64_t j = 0; j < ny; ++j) {
      double dx = X[3 * i + 0] - Y[3 * j + 0];
      double dy = X[3 * i + 1] - Y[3 * j + 1];
      double dz = X[3 * i + 2] - Y[3 * j + 2];
      double r = sqrt(dx * dx + dy * dy + dz * dz);
      if (r > tau) acc += kernel_G(r, kappa, kernel) * qc[j];
    }
    pc[a] = acc;
  }
}

/* ------------------------------------------------------------------ */
/* Lagrange basis on equispaced nodes j/(L-1), j = 0..L-1 (Sec. 2.3).   */
/* ------------------------------------------------------------------ */
void oracle_lagrange_1d(int32_t L, double t, double* out) {
  for (int m = 0; m < L; ++m) {
    double v = 1.0;
    for (int j = 0; j < L; ++j) {
      if (j == m) continue;
      v *= (t - (double)j / (double)(L - 1)) / ((double)(m - j) / (double)(L - 1));
    }
    out[m] = v;
  }
}

/* S_k(x) for a cell with lower corner alpha and side h: product of 1D bases,
   node k flattened as kx + L ky + L^2 kz (Definition 1). */
static double interp_S(int L, const double* alpha, double h, const double* x, int k) {
  double l1[16];
  double v = 1.0;
  int kk[3] = {k % L, (k / L) % L, k / (L * L)};
  for (int d = 0; d < 3; ++d) {
    oracle_lagrange_1d(L, (x[d] - alpha[d]) / h, l1);
    v *= l1[kk[d]];
  }
  return v;
}

static void node_pos(int L, const double* alpha, double h, int k, double* out) {
  int kk[3] = {k % L, (k / L) % L, k / (L * L)};
  for (int d = 0; d < 3; ++d) out[d] = alpha[d] + h * (double)kk[d] / (double)(L - 1);
}

/* ------------------------------------------------------------------ */
/* Directions (Sec. 4.1.2): projected centres of the face patches of    */
/* the cube, each face split 2^E x 2^E; father = enclosing patch.       */
/* ------------------------------------------------------------------ */
int64_t oracle_directions(int32_t E, double* dirs, int64_t* father) {
  int64_t side = (int64_t)1 << E;
  int64_t n = 6 * side * side;
  if (!dirs) return n;
  for (int f = 0; f < 6; ++f) {
    int a = f / 2;
    double sg = (f % 2 == 0) ? 1.0 : -1.0;
    int b = (a == 0) ? 1 : 0;
    int c = (a == 2) ? 1 : 2;
    for (int64_t i = 0; i < side; ++i)
      for (int64_t j = 0; j < side; ++j) {
        double pnt[3];
        pnt[a] = sg;
        pnt[b] = -1.0 + (double)(2 * i + 1) / (double)side;
        pnt[c] = -1.0 + (double)(2 * j + 1) / (double)side;
        double nr = sqrt(pnt[0] * pnt[0] + pnt[1] * pnt[1] + pnt[2] * pnt[2]);
        int64_t u = (int64_t)f * side * side + i * side + j;
        for (int d = 0; d < 3; ++d) dirs[3 * u + d] = pnt[d] / nr;
        if (father) {
          if (E == 0) father[u] = -1;
          else father[u] = (int64_t)f * (side / 2) * (side / 2) + (i >> 1) * (side / 2) + (j >> 1);
        }
      }
  }
  return n;
}

/* ------------------------------------------------------------------ */
/* DFT on a P^3 grid, index mx + P my + P^2 mz; sign -1 forward.        */
/* The 3D DFT is applied as three 1D DFTs (it factorises by dimension). */
/* ------------------------------------------------------------------ */
void oracle_dft3(int32_t P, const double* in_, double* out_, int32_t sign) {
  const cplx* in = (const cplx*)in_;
  cplx* out = (cplx*)out_;
  int64_t n = (int64_t)P * P * P;
  cplx* a = (cplx*)malloc(sizeof(cplx) * n);
  cplx* b = (cplx*)malloc(sizeof(cplx) * n);
  cplx* w = (cplx*)malloc(sizeof(cplx) * P);
  for (int m = 0; m < P; ++m) w[m] = cexp((double)sign * 2.0 * PI * I * (double)m / (double)P);
  memcpy(a, in, sizeof(cplx) * n);
  int64_t stride[3] = {1, P, (int64_t)P * P};
  for (int d = 0; d < 3; ++d) {
    for (int64_t base = 0; base < n; ++base) {
      int coord = (int)((base / stride[d]) % P);
      if (coord != 0) continue; /* one line per base with coordinate d = 0 */
      for (int k = 0; k < P; ++k) {
        cplx acc = 0.0;
        for (int m = 0; m < P; ++m) acc += a[base + m * stride[d]] * w[(k * m) % P];
        b[base + k * stride[d]] = acc;
      }
    }
    cplx* t = a; a = b; b = t;
  }
  memcpy(out, a, sizeof(cplx) * n);
  free(a); free(b); free(w);
}

/* First column of the circulant embedding (eq. CirculantKernel):
   c[j mod P] = G(h delta + (h/(L-1)) j), j in [-(L-1), L-1]^3. */
static void circulant_column(double kappa, int kernel, double h, int L, const int32_t* delta, cplx* c) {
  int P = 2 * L - 1;
  for (int jz = -(L - 1); jz <= L - 1; ++jz)
    for (int jy = -(L - 1); jy <= L - 1; ++jy)
      for (int jx = -(L - 1); jx <= L - 1; ++jx) {
        double z[3];
        int j[3] = {jx, jy, jz};
        for (int d = 0; d < 3; ++d) z[d] = h * (double)delta[d] + (h / (double)(L - 1)) * (double)j[d];
        double r = sqrt(z[0] * z[0] + z[1] * z[1] + z[2] * z[2]);
        int mx = (jx + P) % P, my = (jy + P) % P, mz = (jz + P) % P;
        c[mx + P * my + P * P * mz] = kernel_G(r, kappa, kernel);
      }
}

/* Diagonal of the Fourier-domain M2L operator (eq. FourierDiagonal). */
void oracle_spectrum(double kappa, double h, int32_t L, const int32_t* delta, double* D, int32_t kernel) {
  int P = 2 * L - 1;
  int64_t n = (int64_t)P * P * P;
  cplx* c = (cplx*)malloc(sizeof(cplx) * n);
  circulant_column(kappa, kernel, h, L, delta, c);
  oracle_dft3(P, (const double*)c, D, -1);
  free(c);
}

/* M2L through the circulant embedding: crop(ifftn(D * fftn(pad(M)))). */
void oracle_m2l_fft(double kappa, double h, int32_t L, const int32_t* delta,
                    const double* M_, double* Lout_, int32_t kernel) {
  const cplx* M = (const cplx*)M_;
  cplx* Lout = (cplx*)Lout_;
  int P = 2 * L - 1;
  int64_t n = (int64_t)P * P * P;
  cplx* D = (cplx*)malloc(sizeof(cplx) * n);
  cplx* pad = (cplx*)calloc(n, sizeof(cplx));
  cplx* Mt = (cplx*)malloc(sizeof(cplx) * n);
  cplx* back = (cplx*)malloc(sizeof(cplx) * n);
  oracle_spectrum(kappa, h, L, delta, (double*)D, kernel);
  for (int k = 0; k < L * L * L; ++k) {
    int kx = k % L, ky = (k / L) % L, kz = k / (L * L);
    pad[kx + P * ky + P * P * kz] = M[k];
  }
  oracle_dft3(P, (const double*)pad, (double*)Mt, -1);
  for (int64_t i = 0; i < n; ++i) Mt[i] *= D[i];
  oracle_dft3(P, (const double*)Mt, (double*)back, +1);
  for (int k = 0; k < L * L * L; ++k) {
    int kx = k % L, ky = (k / L) % L, kz = k / (L * L);
    Lout[k] = back[kx + P * ky + P * P * kz] / (double)n;
  }
  free(D); free(pad); free(Mt); free(back);
}

/* M2L by definition: L(x_k) = sum_l G(x_k - y_l) M(y_l). */
void oracle_m2l_dense(double kappa, double h, int32_t L, const int32_t* delta,
                      const double* M_, double* Lout_, int32_t kernel) {
  const cplx* M = (const cplx*)M_;
  cplx* Lout = (cplx*)Lout_;
  int n = L * L * L;
  for (int k = 0; k < n; ++k) {
    int kk[3] = {k % L, (k / L) % L, k / (L * L)};
    cplx acc = 0.0;
    for (int l = 0; l < n; ++l) {
      int ll[3] = {l % L, (l / L) % L, l / (L * L)};
      double z[3];
      for (int d = 0; d < 3; ++d)
        z[d] = h * (double)delta[d] + (h / (double)(L - 1)) * (double)(kk[d] - ll[d]);
      double r = sqrt(z[0] * z[0] + z[1] * z[1] + z[2] * z[2]);
      acc += kernel_G(r, kappa, kernel) * M[l];
    }
    Lout[k] = acc;
  }
}

/* ------------------------------------------------------------------ */
/* Single-expansion operators (Sec. 2.2).  `u` is a unit direction or   */
/* NULL for the non-directional (low-frequency) form.                   */
/* ------------------------------------------------------------------ */
static double dot_or_zero(const double* u, const double* v) {
  return u ? (u[0] * v[0] + u[1] * v[1] + u[2] * v[2]) : 0.0;
}

/* P2M: M(y_r) = sum_y S_r(y) exp(i kappa <y_r - y, u>) q(y). */
void oracle_p2m(double kappa, int32_t L, const double* alpha, double h, const double* u,
                int64_t n, const double* y, const double* q_, double* M_) {
  const cplx* q = (const cplx*)q_;
  cplx* M = (cplx*)M_;
  int L3 = L * L * L;
  for (int r = 0; r < L3; ++r) {
    double yr[3];
    node_pos(L, alpha, h, r, yr);
    cplx acc = 0.0;
    for (int64_t i = 0; i < n; ++i) {
      double diff[3] = {yr[0] - y[3 * i], yr[1] - y[3 * i + 1], yr[2] - y[3 * i + 2]};
      double ph = kappa * dot_or_zero(u, diff);
      acc += interp_S(L, alpha, h, y + 3 * i, r) * cexp(I * ph) * q[i];
    }
    M[r] = acc;
  }
}

/* M2M, one son: M_s(y_l) += sum_r S_l[s](y'_r) exp(i kappa <y_l - y'_r, v>) M_{s'}(y'_r). */
void oracle_m2m(double kappa, int32_t L, const double* alpha, double h, const double* v,
                const double* calpha, double ch, const double* Mc_, double* M_) {
  const cplx* Mc = (const cplx*)Mc_;
  cplx* M = (cplx*)M_;
  int L3 = L * L * L;
  for (int l = 0; l < L3; ++l) {
    double yl[3];
    node_pos(L, alpha, h, l, yl);
    cplx acc = 0.0;
    for (int r = 0; r < L3; ++r) {
      double yr[3];
      node_pos(L, calpha, ch, r, yr);
      double diff[3] = {yl[0] - yr[0], yl[1] - yr[1], yl[2] - yr[2]};
      double ph = kappa * dot_or_zero(v, diff);
      acc += interp_S(L, alpha, h, yr, l) * cexp(I * ph) * Mc[r];
    }
    M[l] += acc;
  }
}

/* L2L, one father expansion: L_{t'}(x'_h) += sum_k S_k[t](x'_h) exp(i kappa <x'_h - x_k, v>) L_t(x_k). */
void oracle_l2l(double kappa, int32_t L, const double* alpha, double h, const double* v,
                const double* calpha, double ch, const double* Lp_, double* Lc_) {
  const cplx* Lp = (const cplx*)Lp_;
  cplx* Lc = (cplx*)Lc_;
  int L3 = L * L * L;
  for (int hn = 0; hn < L3; ++hn) {
    double xh[3];
    node_pos(L, calpha, ch, hn, xh);
    cplx acc = 0.0;
    for (int k = 0; k < L3; ++k) {
      double xk[3];
      node_pos(L, alpha, h, k, xk);
      double diff[3] = {xh[0] - xk[0], xh[1] - xk[1], xh[2] - xk[2]};
      double ph = kappa * dot_or_zero(v, diff);
      acc += interp_S(L, alpha, h, xh, k) * cexp(I * ph) * Lp[k];
    }
    Lc[hn] += acc;
  }
}

/* L2P: p(x) += sum_h S_h(x) exp(i kappa <x - x_h, u>) L(x_h). */
void oracle_l2p(double kappa, int32_t L, const double* alpha, double h, const double* u,
                const double* Lc_, int64_t n, const double* x, double* p_) {
  const cplx* Lc = (const cplx*)Lc_;
  cplx* p = (cplx*)p_;
  int L3 = L * L * L;
  for (int64_t i = 0; i < n; ++i) {
    cplx acc = 0.0;
    for (int hn = 0; hn < L3; ++hn) {
      double xh[3];
      node_pos(L, alpha, h, hn, xh);
      double diff[3] = {x[3 * i] - xh[0], x[3 * i + 1] - xh[1], x[3 * i + 2] - xh[2]};
      double ph = kappa * dot_or_zero(u, diff);
      acc += interp_S(L, alpha, h, x + 3 * i, hn) * cexp(I * ph) * Lc[hn];
    }
    p[i] += acc;
  }
}

/* ------------------------------------------------------------------ */
/* Trees (Sec. 4.2.1): Morton-sorted points, Ncrit splitting.           */
/* ------------------------------------------------------------------ */
typedef struct {
  int32_t level;
  int64_t ijk[3];
  int64_t first, count;
  int32_t is_leaf;
  int32_t nchild;
  int64_t child[8];
  int64_t parent;
  /* marks (Alg. 2/3) = effective expansions, sorted; -1 = non-directional */
  int32_t nmark, capmark;
  int32_t* mark;
  int64_t exp0; /* index of the first expansion of this cell */
} ocell;

typedef struct {
  int64_t n;
  int64_t* perm;     /* sorted position -> caller index */
  uint64_t* key;     /* sorted Morton keys */
  double* spts;      /* sorted coordinates */
  ocell* cells;
  int64_t ncells, capcells;
  int32_t nlevels;
  int64_t lev_start[MAXLEV + 2];
  int64_t nexp;
} otree;

typedef struct {
  uint64_t key;
  int64_t idx;
} keyidx;

static int cmp_keyidx(const void* a, const void* b) {
  const keyidx* x = (const keyidx*)a;
  const keyidx* y = (const keyidx*)b;
  if (x->key < y->key) return -1;
  if (x->key > y->key) return 1;
  return (x->idx < y->idx) ? -1 : (x->idx > y->idx);
}

static uint64_t spread3(uint64_t v) {
  uint64_t r = 0;
  for (int b = 0; b < KEYBITS; ++b) r |= ((v >> b) & 1ull) << (3 * b);
  return r;
}

static int64_t quantise(double x, double o, double D) {
  if (!(D > 0.0)) return 0;
  double s = floor((x - o) / D * (double)(1 << KEYBITS));
  if (s < 0.0) s = 0.0;
  if (s > (double)((1 << KEYBITS) - 1)) s = (double)((1 << KEYBITS) - 1);
  return (int64_t)s;
}

static void push_cell(otree* T, ocell c) {
  if (T->ncells == T->capcells) {
    T->capcells = T->capcells ? 2 * T->capcells : 1024;
    T->cells = (ocell*)realloc(T->cells, sizeof(ocell) * T->capcells);
  }
  T->cells[T->ncells++] = c;
}

static void build_tree(otree* T, const double* pts, int64_t n, const double* origin, double D, int ncrit) {
  memset(T, 0, sizeof(*T));
  T->n = n;
  T->perm = (int64_t*)malloc(sizeof(int64_t) * (n ? n : 1));
  T->key = (uint64_t*)malloc(sizeof(uint64_t) * (n ? n : 1));
  T->spts = (double*)malloc(sizeof(double) * 3 * (n ? n : 1));
  keyidx* ki = (keyidx*)malloc(sizeof(keyidx) * (n ? n : 1));
  for (int64_t i = 0; i < n; ++i) {
    uint64_t qx = (uint64_t)quantise(pts[3 * i + 0], origin[0], D);
    uint64_t qy = (uint64_t)quantise(pts[3 * i + 1], origin[1], D);
    uint64_t qz = (uint64_t)quantise(pts[3 * i + 2], origin[2], D);
    ki[i].key = spread3(qx) | (spread3(qy) << 1) | (spread3(qz) << 2);
    ki[i].idx = i;
  }
  qsort(ki, (size_t)n, sizeof(keyidx), cmp_keyidx);
  for (int64_t i = 0; i < n; ++i) {
    T->perm[i] = ki[i].idx;
    T->key[i] = ki[i].key;
    for (int d = 0; d < 3; ++d) T->spts[3 * i + d] = pts[3 * ki[i].idx + d];
  }
  free(ki);
  ocell root;
  memset(&root, 0, sizeof(root));
  root.first = 0;
  root.count = n;
  root.parent = -1;
  T->lev_start[0] = 0;
  push_cell(T, root);
  T->lev_start[1] = 1;
  int lev = 0;
  for (;;) {
    int64_t b = T->lev_start[lev], e = T->lev_start[lev + 1];
    for (int64_t ci = b; ci < e; ++ci) {
      ocell* c = &T->cells[ci];
      if (c->count > ncrit && lev < MAXLEV) {
        c->is_leaf = 0;
        int shift = 3 * (KEYBITS - lev - 1);
        int64_t i = c->first, end = c->first + c->count;
        while (i < end) {
          uint64_t digit = (T->key[i] >> shift) & 7ull;
          int64_t j = i;
          while (j < end && ((T->key[j] >> shift) & 7ull) == digit) ++j;
          ocell ch;
          memset(&ch, 0, sizeof(ch));
          ch.level = lev + 1;
          ch.ijk[0] = 2 * T->cells[ci].ijk[0] + (int64_t)(digit & 1);
          ch.ijk[1] = 2 * T->cells[ci].ijk[1] + (int64_t)((digit >> 1) & 1);
          ch.ijk[2] = 2 * T->cells[ci].ijk[2] + (int64_t)((digit >> 2) & 1);
          ch.first = i;
          ch.count = j - i;
          ch.parent = ci;
          int64_t id = T->ncells;
          push_cell(T, ch);
          c = &T->cells[ci]; /* realloc may have moved the array */
          c->child[c->nchild++] = id;
          i = j;
        }
      } else {
        c->is_leaf = 1;
      }
    }
    T->lev_start[lev + 2] = T->ncells;
    if (T->lev_start[lev + 2] == T->lev_start[lev + 1]) {
      T->nlevels = lev + 1;
      break;
    }
    ++lev;
  }
}

static void free_tree(otree* T) {
  for (int64_t i = 0; i < T->ncells; ++i) free(T->cells[i].mark);
  free(T->cells);
  free(T->perm);
  free(T->key);
  free(T->spts);
}

static void add_mark(ocell* c, int32_t u) {
  for (int i = 0; i < c->nmark; ++i)
    if (c->mark[i] == u) return;
  if (c->nmark == c->capmark) {
    c->capmark = c->capmark ? 2 * c->capmark : 4;
    c->mark = (int32_t*)realloc(c->mark, sizeof(int32_t) * c->capmark);
  }
  c->mark[c->nmark++] = u;
}

static int cmp_i32(const void* a, const void* b) {
  int32_t x = *(const int32_t*)a, y = *(const int32_t*)b;
  return (x > y) - (x < y);
}

/* ------------------------------------------------------------------ */
/* (level, delta) memo: best direction and spectrum per M2L matrix      */
/* (Alg. 2 precomputes one matrix and one direction per (level,delta)). */
/* ------------------------------------------------------------------ */
typedef struct {
  int32_t level, d[3];
  int32_t dir;
  cplx* D;
} omemo;

typedef struct {
  int64_t* slot; /* -1 empty, else memo index */
  int64_t cap;
  omemo* m;
  int64_t n, capm;
} omap;

static uint64_t hash4(int32_t l, const int32_t* d) {
  uint64_t h = 1469598103934665603ull;
  int32_t v[4] = {l, d[0], d[1], d[2]};
  for (int i = 0; i < 4; ++i) {
    h ^= (uint64_t)(uint32_t)v[i];
    h *= 1099511628211ull;
  }
  return h ^ (h >> 29);
}

static int64_t map_get(omap* M, int32_t l, const int32_t* d) {
  if (M->n * 2 >= M->cap) {
    int64_t ncap = M->cap ? M->cap * 2 : 4096;
    int64_t* ns = (int64_t*)malloc(sizeof(int64_t) * ncap);
    for (int64_t i = 0; i < ncap; ++i) ns[i] = -1;
    for (int64_t i = 0; i < M->n; ++i) {
      uint64_t h = hash4(M->m[i].level, M->m[i].d) & (uint64_t)(ncap - 1);
      while (ns[h] >= 0) h = (h + 1) & (uint64_t)(ncap - 1);
      ns[h] = i;
    }
    free(M->slot);
    M->slot = ns;
    M->cap = ncap;
  }
  uint64_t h = hash4(l, d) & (uint64_t)(M->cap - 1);
  while (M->slot[h] >= 0) {
    omemo* e = &M->m[M->slot[h]];
    if (e->level == l && e->d[0] == d[0] && e->d[1] == d[1] && e->d[2] == d[2]) return M->slot[h];
    h = (h + 1) & (uint64_t)(M->cap - 1);
  }
  if (M->n == M->capm) {
    M->capm = M->capm ? 2 * M->capm : 4096;
    M->m = (omemo*)realloc(M->m, sizeof(omemo) * M->capm);
  }
  omemo e;
  e.level = l;
  e.d[0] = d[0]; e.d[1] = d[1]; e.d[2] = d[2];
  e.dir = -1;
  e.D = NULL;
  M->m[M->n] = e;
  M->slot[h] = M->n;
  return M->n++;
}

/* ------------------------------------------------------------------ */
/* The FMM state.                                                       */
/* ------------------------------------------------------------------ */
typedef struct {
  int64_t t, s;
  int32_t level, d[3];
  int64_t memo;
} om2l;

typedef struct {
  oracle_params prm;
  double kappa, D, origin[3], tau;
  int same;
  otree tx, ty_own;
  otree* ty; /* == &tx when same points */
  int32_t lstar;
  int32_t hf[MAXLEV + 1];
  double thr[MAXLEV + 1];
  /* directions per direction level, computed on demand */
  double* dirs[32];
  int64_t* father[32];
  int64_t ndirs[32];
  int32_t maxE;
  omap memo;
  om2l* m2l;
  int64_t nm2l, capm2l;
  int64_t* p2p; /* pairs (t,s) */
  int64_t np2p, capp2p;
  /* grouped by target cell */
  int64_t *m2l_off, *m2l_idx;
  int64_t *p2p_off, *p2p_idx;
  /* expansions */
  cplx *Mx, *Lx, *My, *Ly;  /* node values, L^3 per expansion */
  cplx *Mt, *Lt;            /* Fourier-domain values, P^3 per expansion */
} ofmm;

static double level_h(const ofmm* F, int l) { return ldexp(F->D, -l); }

static void need_dirs(ofmm* F, int E) {
  if (F->dirs[E]) return;
  int64_t n = oracle_directions(E, NULL, NULL);
  F->dirs[E] = (double*)malloc(sizeof(double) * 3 * n);
  F->father[E] = (int64_t*)malloc(sizeof(int64_t) * n);
  oracle_directions(E, F->dirs[E], F->father[E]);
  F->ndirs[E] = n;
  if (E > F->maxE) F->maxE = E;
}

static int dir_level(const ofmm* F, int l) { return F->lstar - l + F->prm.dir_refine; }

/* Best direction (Alg. 2): argmin |v - delta/|delta|| = argmax <v, delta>. */
static int32_t best_direction(ofmm* F, int E, const int32_t* d) {
  const double* V = F->dirs[E];
  int64_t n = F->ndirs[E];
  double dd[3] = {(double)d[0], (double)d[1], (double)d[2]};
  double best = -1e300;
  for (int64_t u = 0; u < n; ++u) {
    double s = V[3 * u] * dd[0] + V[3 * u + 1] * dd[1] + V[3 * u + 2] * dd[2];
    if (s > best) best = s;
  }
  double tol = 1e-12 * sqrt(dd[0] * dd[0] + dd[1] * dd[1] + dd[2] * dd[2]);
  for (int64_t u = 0; u < n; ++u) {
    double s = V[3 * u] * dd[0] + V[3 * u + 1] * dd[1] + V[3 * u + 2] * dd[2];
    if (s >= best - tol) return (int32_t)u;
  }
  return 0;
}

static void push_m2l(ofmm* F, int64_t t, int64_t s, int l, const int32_t* d) {
  if (F->nm2l == F->capm2l) {
    F->capm2l = F->capm2l ? 2 * F->capm2l : 4096;
    F->m2l = (om2l*)realloc(F->m2l, sizeof(om2l) * F->capm2l);
  }
  om2l e;
  e.t = t; e.s = s; e.level = l;
  e.d[0] = d[0]; e.d[1] = d[1]; e.d[2] = d[2];
  e.memo = map_get(&F->memo, l, d);
  F->m2l[F->nm2l++] = e;
}

static void push_p2p(ofmm* F, int64_t t, int64_t s) {
  if (F->np2p == F->capp2p) {
    F->capp2p = F->capp2p ? 2 * F->capp2p : 4096;
    F->p2p = (int64_t*)realloc(F->p2p, sizeof(int64_t) * 2 * F->capp2p);
  }
  F->p2p[2 * F->np2p] = t;
  F->p2p[2 * F->np2p + 1] = s;
  F->np2p++;
}

/* Dual tree traversal, Alg. 1: MAC -> M2L; else a leaf -> P2P; else recurse
   over all pairs of sons (both cells split, same level). */
static void dtt(ofmm* F, int64_t ti, int64_t si) {
  const ocell* t = &F->tx.cells[ti];
  const ocell* s = &F->ty->cells[si];
  int32_t d[3];
  int64_t n2 = 0;
  for (int k = 0; k < 3; ++k) {
    d[k] = (int32_t)(t->ijk[k] - s->ijk[k]);
    int64_t a = d[k] < 0 ? -(int64_t)d[k] : (int64_t)d[k];
    int64_t nk = a - 1 > 0 ? a - 1 : 0;
    n2 += nk * nk;
  }
  if ((double)n2 >= F->thr[t->level]) {
    push_m2l(F, ti, si, t->level, d);
    return;
  }
  if (t->is_leaf || s->is_leaf) {
    push_p2p(F, ti, si);
    return;
  }
  for (int a = 0; a < t->nchild; ++a)
    for (int b = 0; b < s->nchild; ++b) dtt(F, F->tx.cells[ti].child[a], F->ty->cells[si].child[b]);
}

/* Blank downward pass (Alg. 3), extended to low-frequency cells, which
   carry one non-directional expansion as soon as the parent has one. */
static void blank_downward(ofmm* F, otree* T) {
  for (int l = 0; l < T->nlevels; ++l) {
    for (int64_t ci = T->lev_start[l]; ci < T->lev_start[l + 1]; ++ci) {
      ocell* c = &T->cells[ci];
      if (c->nmark > 1) qsort(c->mark, (size_t)c->nmark, sizeof(int32_t), cmp_i32);
      if (c->nmark == 0) continue;
      for (int a = 0; a < c->nchild; ++a) {
        ocell* ch = &T->cells[c->child[a]];
        if (F->hf[l + 1]) {
          int E = dir_level(F, l);
          need_dirs(F, E);
          need_dirs(F, E - 1); /* the son's own direction set, which its marks index */
          for (int m = 0; m < c->nmark; ++m) add_mark(ch, (int32_t)F->father[E][c->mark[m]]);
        } else {
          add_mark(ch, -1);
        }
      }
    }
  }
  int64_t e = 0;
  for (int64_t ci = 0; ci < T->ncells; ++ci) {
    T->cells[ci].exp0 = e;
    e += T->cells[ci].nmark;
  }
  T->nexp = e;
}

static int64_t find_exp(const ocell* c, int32_t u) {
  for (int i = 0; i < c->nmark; ++i)
    if (c->mark[i] == u) return c->exp0 + i;
  return -1;
}

static void cell_alpha(const ofmm* F, const ocell* c, double* alpha) {
  double h = level_h(F, c->level);
  for (int d = 0; d < 3; ++d) alpha[d] = F->origin[d] + h * (double)c->ijk[d];
}

static const double* dir_vec(const ofmm* F, int level, int32_t u) {
  if (u < 0) return NULL;
  return F->dirs[dir_level(F, level)] + 3 * (int64_t)u;
}

void* oracle_fmm_create(const double* X, int64_t nx, const double* Y, int64_t ny,
                        int32_t same_points, double kappa, const oracle_params* prm) {
  ofmm* F = (ofmm*)calloc(1, sizeof(ofmm));
  F->prm = *prm;
  F->kappa = kappa;
  F->same = same_points ? 1 : 0;
  /* Bounding cube of X and Y (Sec. 1: D is the side of the smallest box). */
  double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
  for (int64_t i = 0; i < nx; ++i)
    for (int d = 0; d < 3; ++d) {
      lo[d] = fmin(lo[d], X[3 * i + d]);
      hi[d] = fmax(hi[d], X[3 * i + d]);
    }
  for (int64_t i = 0; i < ny; ++i)
    for (int d = 0; d < 3; ++d) {
      lo[d] = fmin(lo[d], Y[3 * i + d]);
      hi[d] = fmax(hi[d], Y[3 * i + d]);
    }
  double D = 0.0;
  if (nx + ny > 0) {
    for (int d = 0; d < 3; ++d) D = fmax(D, hi[d] - lo[d]);
    for (int d = 0; d < 3; ++d) F->origin[d] = 0.5 * (lo[d] + hi[d]) - 0.5 * D;
  }
  F->D = D;
  F->tau = 1e-12 * D;
  build_tree(&F->tx, X, nx, F->origin, D, prm->ncrit);
  if (F->same) {
    F->ty = &F->tx;
  } else {
    build_tree(&F->ty_own, Y, ny, F->origin, D, prm->ncrit);
    F->ty = &F->ty_own;
  }
  /* Regimes and MAC thresholds per level. */
  F->lstar = -1;
  for (int l = 0; l <= MAXLEV; ++l) {
    double w = ldexp(D, -(l + 1));
    /* A screened kernel does not oscillate: every level is low-frequency and
       the MAC is the plain one (kappa w replaced by 0). */
    const double kw = prm->kernel == ORACLE_YUKAWA ? 0.0 : kappa * w;
    F->hf[l] = (kw > prm->hf_threshold) ? 1 : 0;
    if (F->hf[l]) F->lstar = l;
    double a = fmax(kw, 2.0) / (2.0 * prm->eta);
    F->thr[l] = a * a;
  }
  F->maxE = -1;
  if (nx > 0 && ny > 0) dtt(F, 0, 0);
  /* Best direction and spectrum per (level, delta). */
  for (int64_t i = 0; i < F->memo.n; ++i) {
    int l = F->memo.m[i].level;
    if (F->hf[l]) need_dirs(F, dir_level(F, l));
  }
  int L = prm->L, P = 2 * L - 1;
  int64_t P3 = (int64_t)P * P * P;
#pragma omp parallel for schedule(dynamic, 4)
  for (int64_t i = 0; i < F->memo.n; ++i) {
    omemo* e = &F->memo.m[i];
    if (F->hf[e->level]) e->dir = best_direction(F, dir_level(F, e->level), e->d);
    e->D = (cplx*)malloc(sizeof(cplx) * P3);
    oracle_spectrum(kappa, level_h(F, e->level), L, e->d, (double*)e->D, prm->kernel);
  }
  /* Marks (Alg. 2) then the blank downward pass (Alg. 3). */
  for (int64_t i = 0; i < F->nm2l; ++i) {
    om2l* m = &F->m2l[i];
    int32_t u = F->memo.m[m->memo].dir;
    add_mark(&F->tx.cells[m->t], u);
    add_mark(&F->ty->cells[m->s], u);
  }
  blank_downward(F, &F->tx);
  if (!F->same) blank_downward(F, F->ty);
  /* Group M2L and P2P pairs by target cell. */
  int64_t nc = F->tx.ncells;
  F->m2l_off = (int64_t*)calloc(nc + 1, sizeof(int64_t));
  F->p2p_off = (int64_t*)calloc(nc + 1, sizeof(int64_t));
  for (int64_t i = 0; i < F->nm2l; ++i) F->m2l_off[F->m2l[i].t + 1]++;
  for (int64_t i = 0; i < F->np2p; ++i) F->p2p_off[F->p2p[2 * i] + 1]++;
  for (int64_t c = 0; c < nc; ++c) {
    F->m2l_off[c + 1] += F->m2l_off[c];
    F->p2p_off[c + 1] += F->p2p_off[c];
  }
  F->m2l_idx = (int64_t*)malloc(sizeof(int64_t) * (F->nm2l + 1));
  F->p2p_idx = (int64_t*)malloc(sizeof(int64_t) * (F->np2p + 1));
  int64_t* fill = (int64_t*)calloc(nc + 1, sizeof(int64_t));
  for (int64_t i = 0; i < F->nm2l; ++i) {
    int64_t t = F->m2l[i].t;
    F->m2l_idx[F->m2l_off[t] + fill[t]++] = i;
  }
  memset(fill, 0, sizeof(int64_t) * (nc + 1));
  for (int64_t i = 0; i < F->np2p; ++i) {
    int64_t t = F->p2p[2 * i];
    F->p2p_idx[F->p2p_off[t] + fill[t]++] = i;
  }
  free(fill);
  int64_t L3 = (int64_t)L * L * L;
  F->Mx = (cplx*)calloc((size_t)(F->tx.nexp * L3 + 1), sizeof(cplx));
  F->Lx = (cplx*)calloc((size_t)(F->tx.nexp * L3 + 1), sizeof(cplx));
  if (F->same) {
    F->My = F->Mx;
    F->Ly = F->Lx;
  } else {
    F->My = (cplx*)calloc((size_t)(F->ty->nexp * L3 + 1), sizeof(cplx));
    F->Ly = (cplx*)calloc((size_t)(F->ty->nexp * L3 + 1), sizeof(cplx));
  }
  return F;
}

void oracle_fmm_destroy(void* h) {
  ofmm* F = (ofmm*)h;
  if (!F) return;
  for (int64_t i = 0; i < F->memo.n; ++i) free(F->memo.m[i].D);
  free(F->memo.m);
  free(F->memo.slot);
  for (int e = 0; e < 32; ++e) {
    free(F->dirs[e]);
    free(F->father[e]);
  }
  free(F->m2l); free(F->p2p);
  free(F->m2l_off); free(F->m2l_idx); free(F->p2p_off); free(F->p2p_idx);
  if (!F->same) {
    free(F->My);
    free(F->Ly);
  }
  free(F->Mx); free(F->Lx); free(F->Mt); free(F->Lt);
  free_tree(&F->tx);
  if (!F->same) free_tree(&F->ty_own);
  free(F);
}

/* P2M pass: every expansion of every source leaf. */
static void op_p2m(ofmm* F, const cplx* qs) {
  otree* T = F->ty;
  int L = F->prm.L;
  int L3 = L * L * L;
#pragma omp parallel for schedule(dynamic, 4)
  for (int64_t ci = 0; ci < T->ncells; ++ci) {
    const ocell* c = &T->cells[ci];
    if (!c->is_leaf || c->nmark == 0) continue;
    double alpha[3], h = level_h(F, c->level);
    cell_alpha(F, c, alpha);
    for (int e = 0; e < c->nmark; ++e)
      oracle_p2m(F->kappa, L, alpha, h, dir_vec(F, c->level, c->mark[e]), c->count,
                 T->spts + 3 * c->first, (const double*)(qs + c->first),
                 (double*)(F->My + (c->exp0 + e) * L3));
  }
}

/* M2M pass, sons to fathers: the father's expansion v gathers, from each son,
   the son's expansion Father(v) (high-frequency son) or its single expansion. */
static void op_m2m(ofmm* F) {
  otree* T = F->ty;
  int L = F->prm.L;
  int L3 = L * L * L;
  for (int l = T->nlevels - 2; l >= 0; --l) {
#pragma omp parallel for schedule(dynamic, 2)
    for (int64_t ci = T->lev_start[l]; ci < T->lev_start[l + 1]; ++ci) {
      const ocell* c = &T->cells[ci];
      if (c->is_leaf || c->nmark == 0) continue;
      double alpha[3], h = level_h(F, l);
      cell_alpha(F, c, alpha);
      for (int e = 0; e < c->nmark; ++e) {
        int32_t v = c->mark[e];
        int32_t u = F->hf[l + 1] ? (int32_t)F->father[dir_level(F, l)][v] : -1;
        for (int a = 0; a < c->nchild; ++a) {
          const ocell* ch = &T->cells[c->child[a]];
          int64_t ce = find_exp(ch, u);
          if (ce < 0) {
            fprintf(stderr, "oracle: missing son expansion\n");
            abort();
          }
          double calpha[3];
          cell_alpha(F, ch, calpha);
          oracle_m2m(F->kappa, L, alpha, h, dir_vec(F, l, v), calpha, level_h(F, l + 1),
                     (const double*)(F->My + ce * L3), (double*)(F->My + (c->exp0 + e) * L3));
        }
      }
    }
  }
}

/* M2L in the Fourier domain (Sec. 4.1.1): M2F once per source expansion,
   one Hadamard product per pair, F2L once per target expansion. */
static void op_m2l(ofmm* F) {
  int L = F->prm.L, P = 2 * L - 1;
  int64_t L3 = (int64_t)L * L * L, P3 = (int64_t)P * P * P;
  otree* TX = &F->tx;
  otree* TY = F->ty;
  free(F->Mt);
  free(F->Lt);
  F->Mt = (cplx*)calloc((size_t)(TY->nexp * P3 + 1), sizeof(cplx));
  F->Lt = (cplx*)calloc((size_t)(TX->nexp * P3 + 1), sizeof(cplx));
  /* M2F: fftn of the zero-padded multipole grid. */
#pragma omp parallel
  {
    cplx* pad = (cplx*)malloc(sizeof(cplx) * P3);
#pragma omp for schedule(dynamic, 16)
    for (int64_t e = 0; e < TY->nexp; ++e) {
      memset(pad, 0, sizeof(cplx) * P3);
      const cplx* M = F->My + e * L3;
      for (int k = 0; k < L3; ++k) {
        int kx = k % L, ky = (k / L) % L, kz = k / (L * L);
        pad[kx + P * ky + P * P * kz] = M[k];
      }
      oracle_dft3(P, (const double*)pad, (double*)(F->Mt + e * P3), -1);
    }
    free(pad);
  }
  /* Hadamard products, accumulated per target cell. */
#pragma omp parallel for schedule(dynamic, 4)
  for (int64_t ti = 0; ti < TX->ncells; ++ti) {
    const ocell* t = &TX->cells[ti];
    for (int64_t a = F->m2l_off[ti]; a < F->m2l_off[ti + 1]; ++a) {
      const om2l* m = &F->m2l[F->m2l_idx[a]];
      const omemo* me = &F->memo.m[m->memo];
      int64_t te = find_exp(t, me->dir);
      int64_t se = find_exp(&TY->cells[m->s], me->dir);
      if (te < 0 || se < 0) {
        fprintf(stderr, "oracle: missing M2L expansion\n");
        abort();
      }
      cplx* Lt = F->Lt + te * P3;
      const cplx* Mt = F->Mt + se * P3;
      for (int64_t x = 0; x < P3; ++x) Lt[x] += me->D[x] * Mt[x];
    }
  }
  /* F2L: inverse DFT (with 1/P^3) and restriction to the L^3 grid. */
#pragma omp parallel
  {
    cplx* back = (cplx*)malloc(sizeof(cplx) * P3);
#pragma omp for schedule(dynamic, 16)
    for (int64_t e = 0; e < TX->nexp; ++e) {
      oracle_dft3(P, (const double*)(F->Lt + e * P3), (double*)back, +1);
      cplx* Lc = F->Lx + e * L3;
      for (int k = 0; k < L3; ++k) {
        int kx = k % L, ky = (k / L) % L, kz = k / (L * L);
        Lc[k] += back[kx + P * ky + P * P * kz] / (double)P3;
      }
    }
    free(back);
  }
}

/* L2L pass, fathers to sons: the son's expansion u gathers every expansion v
   of the father with Father(v) = u (all of them for a low-frequency son). */
static void op_l2l(ofmm* F) {
  otree* T = &F->tx;
  int L = F->prm.L;
  int L3 = L * L * L;
  for (int l = 0; l + 1 < T->nlevels; ++l) {
#pragma omp parallel for schedule(dynamic, 2)
    for (int64_t ci = T->lev_start[l + 1]; ci < T->lev_start[l + 2]; ++ci) {
      const ocell* ch = &T->cells[ci];
      if (ch->nmark == 0) continue;
      const ocell* c = &T->cells[ch->parent];
      double alpha[3], calpha[3];
      cell_alpha(F, c, alpha);
      cell_alpha(F, ch, calpha);
      for (int ce = 0; ce < ch->nmark; ++ce) {
        int32_t u = ch->mark[ce];
        for (int e = 0; e < c->nmark; ++e) {
          int32_t v = c->mark[e];
          int32_t fv = F->hf[l + 1] ? (int32_t)F->father[dir_level(F, l)][v] : -1;
          if (fv != u) continue;
          oracle_l2l(F->kappa, L, alpha, level_h(F, l), dir_vec(F, l, v), calpha,
                     level_h(F, l + 1), (const double*)(F->Lx + (c->exp0 + e) * L3),
                     (double*)(F->Lx + (ch->exp0 + ce) * L3));
        }
      }
    }
  }
}

/* L2P pass: every expansion of every target leaf. */
static void op_l2p(ofmm* F, cplx* ps) {
  otree* T = &F->tx;
  int L = F->prm.L;
  int L3 = L * L * L;
#pragma omp parallel for schedule(dynamic, 4)
  for (int64_t ci = 0; ci < T->ncells; ++ci) {
    const ocell* c = &T->cells[ci];
    if (!c->is_leaf || c->nmark == 0) continue;
    double alpha[3], h = level_h(F, c->level);
    cell_alpha(F, c, alpha);
    for (int e = 0; e < c->nmark; ++e)
      oracle_l2p(F->kappa, L, alpha, h, dir_vec(F, c->level, c->mark[e]),
                 (const double*)(F->Lx + (c->exp0 + e) * L3), c->count, T->spts + 3 * c->first,
                 (double*)(ps + c->first));
  }
}

/* P2P (Sec. 2.2, singular pairs as in Sec. 5.3): direct sum over the pairs
   of cells the traversal kept in the near field.  Each target point walks up
   its ancestors, so every P2P pair whose target cell contains it is used. */
static void op_p2p(ofmm* F, const cplx* qs, cplx* ps) {
  otree* TX = &F->tx;
  otree* TY = F->ty;
#pragma omp parallel for schedule(dynamic, 4)
  for (int64_t ci = 0; ci < TX->ncells; ++ci) {
    const ocell* leaf = &TX->cells[ci];
    if (!leaf->is_leaf) continue;
    for (int64_t i = leaf->first; i < leaf->first + leaf->count; ++i) {
      const double* x = TX->spts + 3 * i;
      cplx acc = 0.0;
      for (int64_t c = ci; c >= 0; c = TX->cells[c].parent) {
        for (int64_t a = F->p2p_off[c]; a < F->p2p_off[c + 1]; ++a) {
          const ocell* s = &TY->cells[F->p2p[2 * F->p2p_idx[a] + 1]];
          for (int64_t j = s->first; j < s->first + s->count; ++j) {
            const double* y = TY->spts + 3 * j;
            double dx = x[0] - y[0], dy = x[1] - y[1], dz = x[2] - y[2];
            double r = sqrt(dx * dx + dy * dy + dz * dz);
            if (r > F->tau) acc += kernel_G(r, F->kappa, F->prm.kernel) * qs[j];
          }
        }
      }
      ps[i] += acc;
    }
  }
}

double oracle_fmm_apply(void* h, const double* q_, double* p_) {
  ofmm* F = (ofmm*)h;
  double t0 = wall_seconds();
  const cplx* q = (const cplx*)q_;
  cplx* p = (cplx*)p_;
  otree* TX = &F->tx;
  otree* TY = F->ty;
  int L = F->prm.L;
  int64_t L3 = (int64_t)L * L * L;
  cplx* qs = (cplx*)malloc(sizeof(cplx) * (TY->n + 1));
  cplx* ps = (cplx*)calloc((size_t)(TX->n + 1), sizeof(cplx));
  for (int64_t i = 0; i < TY->n; ++i) qs[i] = q[TY->perm[i]];
  memset(F->My, 0, sizeof(cplx) * (size_t)(TY->nexp * L3));
  memset(F->Lx, 0, sizeof(cplx) * (size_t)(TX->nexp * L3));
  if (!F->same) memset(F->Mx, 0, sizeof(cplx) * (size_t)(TX->nexp * L3));
  op_p2m(F, qs);
  op_m2m(F);
  op_m2l(F);
  op_l2l(F);
  op_l2p(F, ps);
  op_p2p(F, qs, ps);
  for (int64_t i = 0; i < TX->n; ++i) p[TX->perm[i]] = ps[i];
  free(qs);
  free(ps);
  return wall_seconds() - t0;
}

void oracle_fmm_info(void* h, int64_t* info) {
  ofmm* F = (ofmm*)h;
  memset(info, 0, sizeof(int64_t) * 16);
  info[0] = F->tx.nlevels;
  info[1] = F->ty->nlevels;
  info[2] = F->lstar;
  info[3] = F->tx.ncells;
  info[4] = F->ty->ncells;
  info[5] = F->nm2l;
  info[6] = F->np2p;
  int64_t pp = 0;
  for (int64_t i = 0; i < F->np2p; ++i)
    pp += F->tx.cells[F->p2p[2 * i]].count * F->ty->cells[F->p2p[2 * i + 1]].count;
  info[7] = pp;
  info[8] = F->tx.nexp;
  info[9] = F->ty->nexp;
  info[10] = F->memo.n;
  info[11] = F->maxE;
}

double oracle_fmm_geometry(void* h, double* origin3) {
  ofmm* F = (ofmm*)h;
  if (origin3)
    for (int d = 0; d < 3; ++d) origin3[d] = F->origin[d];
  return F->D;
}

static otree* pick(ofmm* F, int32_t tree) { return tree == 0 ? &F->tx : F->ty; }

int64_t oracle_fmm_perm(void* h, int32_t tree, int64_t* perm) {
  otree* T = pick((ofmm*)h, tree);
  if (perm) memcpy(perm, T->perm, sizeof(int64_t) * T->n);
  return T->n;
}

int64_t oracle_fmm_cells(void* h, int32_t tree, int32_t* level, int64_t* ijk,
                         int64_t* first, int64_t* count, int32_t* is_leaf) {
  otree* T = pick((ofmm*)h, tree);
  if (level)
    for (int64_t i = 0; i < T->ncells; ++i) {
      const ocell* c = &T->cells[i];
      level[i] = c->level;
      for (int d = 0; d < 3; ++d) ijk[3 * i + d] = c->ijk[d];
      first[i] = c->first;
      count[i] = c->count;
      is_leaf[i] = c->is_leaf;
    }
  return T->ncells;
}

int64_t oracle_fmm_m2l(void* h, int32_t* level, int64_t* t, int64_t* s, int32_t* delta, int32_t* dir) {
  ofmm* F = (ofmm*)h;
  if (level)
    for (int64_t i = 0; i < F->nm2l; ++i) {
      const om2l* m = &F->m2l[i];
      level[i] = m->level;
      t[i] = m->t;
      s[i] = m->s;
      for (int d = 0; d < 3; ++d) delta[3 * i + d] = m->d[d];
      dir[i] = F->memo.m[m->memo].dir;
    }
  return F->nm2l;
}

int64_t oracle_fmm_p2p(void* h, int64_t* t, int64_t* s) {
  ofmm* F = (ofmm*)h;
  if (t)
    for (int64_t i = 0; i < F->np2p; ++i) {
      t[i] = F->p2p[2 * i];
      s[i] = F->p2p[2 * i + 1];
    }
  return F->np2p;
}

int64_t oracle_fmm_expansions(void* h, int32_t tree, int64_t* cell, int32_t* dir, double* M, double* Lc) {
  ofmm* F = (ofmm*)h;
  otree* T = pick(F, tree);
  if (!cell) return T->nexp;
  int L = F->prm.L;
  int64_t L3 = (int64_t)L * L * L;
  const cplx* Ms = (tree == 0) ? F->Mx : F->My;
  const cplx* Ls = (tree == 0) ? F->Lx : F->Ly;
  for (int64_t ci = 0; ci < T->ncells; ++ci) {
    const ocell* c = &T->cells[ci];
    for (int e = 0; e < c->nmark; ++e) {
      cell[c->exp0 + e] = ci;
      dir[c->exp0 + e] = c->mark[e];
    }
  }
  if (M) memcpy(M, Ms, sizeof(cplx) * (size_t)(T->nexp * L3));
  if (Lc) memcpy(Lc, Ls, sizeof(cplx) * (size_t)(T->nexp * L3));
  return T->nexp;
}
