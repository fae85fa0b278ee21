/*
 * defmm oracle -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, FP64 CPU implementation of the directional equispaced-
 * interpolation FMM (defmm) and of the O(N^2) direct sum it approximates.
 * Only the test-suite, the smoke check and the benchmark's CPU-baseline leg
 * may load it.  It shares no code with the GPU library.
 *
 * Complex arrays are interleaved (re, im) doubles, i.e. C99 `double complex`.
 */
#ifndef DEFMM_ORACLE_H
#define DEFMM_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { ORACLE_HELMHOLTZ = 0, ORACLE_YUKAWA = 1 }; /* G = e^{i kappa r}/(4 pi r) or e^{-kappa r}/(4 pi r) */

typedef struct {
  int32_t L;            /* interpolation nodes per dimension (P = 2L-1)            */
  int32_t ncrit;        /* a cell is a leaf iff it holds <= ncrit points             */
  double eta;           /* MAC constant (eq. macdirref)                              */
  double hf_threshold;  /* level is high-frequency iff kappa * w > hf_threshold      */
  int32_t dir_refine;   /* extra 4-fold refinements of the cube-face direction set   */
  int32_t kernel;       /* ORACLE_HELMHOLTZ or ORACLE_YUKAWA (all levels low-frequency) */
} oracle_params;

/* Ground truth (eq. fmmsum): p(x_i) = sum_y G(x_i,y) q(y), G(x,y)=0 if |x-y|<=tau. */
void oracle_direct_sum(const double* X, int64_t nx, const double* Y, int64_t ny,
                       const double* q, double kappa, double tau,
                       const int64_t* targets, int64_t nt, double* p, int32_t kernel);

/* Building blocks (each pinned on its own by the CPU tests). */
void oracle_lagrange_1d(int32_t L, double t, double* out);           /* l_m(t), m<L   */
int64_t oracle_directions(int32_t E, double* dirs, int64_t* father); /* 6*4^E dirs     */
void oracle_spectrum(double kappa, double h, int32_t L, const int32_t* delta,
                     double* D, int32_t kernel);                        /* fftn(c), P^3 */
void oracle_m2l_fft(double kappa, double h, int32_t L, const int32_t* delta,
                    const double* M, double* Lout, int32_t kernel);     /* circulant M2L */
void oracle_m2l_dense(double kappa, double h, int32_t L, const int32_t* delta,
                      const double* M, double* Lout, int32_t kernel);   /* dense M2L     */
void oracle_dft3(int32_t P, const double* in, double* out, int32_t sign);

/* Single-expansion operators (Sec. 2.2); u/v = unit direction or NULL.
   alpha/h: lower corner and side of the cell; calpha/ch: those of the son.
   m2m/l2l/l2p accumulate into their output. */
void oracle_p2m(double kappa, int32_t L, const double* alpha, double h, const double* u,
                int64_t n, const double* y, const double* q, double* M);
void oracle_m2m(double kappa, int32_t L, const double* alpha, double h, const double* v,
                const double* calpha, double ch, const double* Mc, double* M);
void oracle_l2l(double kappa, int32_t L, const double* alpha, double h, const double* v,
                const double* calpha, double ch, const double* Lp, double* Lc);
void oracle_l2p(double kappa, int32_t L, const double* alpha, double h, const double* u,
                const double* Lc, int64_t n, const double* x, double* p);

/* Full FMM.  same_points != 0 means X == Y (one tree). */
void* oracle_fmm_create(const double* X, int64_t nx, const double* Y, int64_t ny,
                        int32_t same_points, double kappa, const oracle_params* prm);
void oracle_fmm_destroy(void* h);
/* q: ny complex (caller order); p: nx complex (caller order). Returns seconds. */
double oracle_fmm_apply(void* h, const double* q, double* p);
/* info[0..15]: levels_x, levels_y, lstar, cells_x, cells_y, m2l pairs, p2p pairs,
   p2p point pairs, eff. expansions x, eff. expansions y, unique (level,delta),
   max direction level used, D (as bits), 0... */
void oracle_fmm_info(void* h, int64_t* info);
double oracle_fmm_geometry(void* h, double* origin3);  /* returns D */
int64_t oracle_fmm_perm(void* h, int32_t tree, int64_t* perm);
int64_t oracle_fmm_cells(void* h, int32_t tree, int32_t* level, int64_t* ijk,
                         int64_t* first, int64_t* count, int32_t* is_leaf);
int64_t oracle_fmm_m2l(void* h, int32_t* level, int64_t* t, int64_t* s,
                       int32_t* delta, int32_t* dir);
int64_t oracle_fmm_p2p(void* h, int64_t* t, int64_t* s);
/* Expansions of a tree after apply: cell id, direction (-1 = non-directional),
   multipole and local node values (L^3 complex each). */
int64_t oracle_fmm_expansions(void* h, int32_t tree, int64_t* cell, int32_t* dir,
                              double* M, double* Lc);

#ifdef __cplusplus
}
#endif
#endif
