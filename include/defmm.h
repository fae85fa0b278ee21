/*
 * defmm.h -- C ABI of libdefmm.so: the matvec of the directional equispaced-
 * interpolation FMM (Chollet, Claeys, Fortin, Grigori) on one AMD MI355X GPU.
 *
 * Problem (Sec. 1, eq. fmmsum): given target points X, source points Y,
 * a wavenumber kappa >= 0 and charges q on Y, evaluate
 *     p(x) = sum_{y in Y} G(x,y) q(y),   G(x,y) = exp(i kappa |x-y|) / (4 pi |x-y|),
 * for every x in X, with G taken as 0 when |x - y| <= tau = 1e-12 D (the
 * singular pairs of Sec. 5.3; D = side of the bounding cube of X and Y).
 * With DEFMM_YUKAWA the kernel is the screened one, exp(-kappa |x-y|) /
 * (4 pi |x-y|), and kappa is its screening constant.
 *
 * The plan (tree, traversal lists, directions, Fourier-domain M2L spectra)
 * is built once per geometry; each matvec then runs entirely on the device.
 * No C++ types or exceptions cross this interface.  Every call returns a
 * defmm_status; defmm_last_error() gives a thread-local detail message.
 * Calls on distinct plans are thread-safe; one workspace serves one
 * in-flight matvec at a time.
 */
#ifndef DEFMM_H
#define DEFMM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  DEFMM_OK = 0,
  DEFMM_ERR_INVALID_ARG = 1,   /* bad pointer, size or parameter; nothing allocated */
  DEFMM_ERR_OUT_OF_MEMORY = 2, /* device or host allocation failed; partial state freed */
  DEFMM_ERR_DEVICE = 3,        /* a HIP runtime call failed */
  DEFMM_ERR_UNSUPPORTED = 4    /* a parameter outside what the library implements */
} defmm_status;

typedef enum {
  DEFMM_C128 = 0, /* complex128 everywhere */
  DEFMM_C64 = 1   /* complex64 expansions, spectra, FFTs, Hadamard and P2P; FP64 geometry,
                     spectrum precomputation and phase-argument reduction */
} defmm_precision;

/* How M2L is applied (Sec. 4.2.3 gives the Fourier form; the dense form applies
   the same L^3 x L^3 interpolated kernel matrix per (level, offset) directly):
     DEFMM_M2L_FFT    circulant embedding + FFT-diagonal product at every level;
     DEFMM_M2L_DENSE  dense matrix-matrix products on the matrix cores at every
                      level whose matrices fit (<= 2 GiB per level, 8 GiB in all)
                      and whose per-pair products fit the workspace (<= 8 GiB),
                      Fourier form elsewhere;
     DEFMM_M2L_AUTO   the plan builds the dense matrices where they fit, the
                      workspace starts on the Fourier form and
                      defmm_workspace_autotune picks, level by level, the faster. */
typedef enum { DEFMM_M2L_AUTO = 0, DEFMM_M2L_FFT = 1, DEFMM_M2L_DENSE = 2 } defmm_m2l_mode;

#define DEFMM_SAME_POINTS 1u /* X and Y are the same set: one tree; q and p share its order */
/* Store one M2L spectrum per class of (level, offset) under the 48 signed
   axis permutations (Sec. 4.3) and read it through a frequency permutation,
   instead of one per distinct (level, offset): 20-40x less spectrum memory,
   a slower Fourier-path M2L.  Plans whose per-offset table would exceed
   8 GiB use this form whatever the flag. */
#define DEFMM_COMPRESS_SPECTRA 2u
/* Screened (Yukawa, modified Helmholtz) kernel G = exp(-kappa r) / (4 pi r)
   instead of the Helmholtz one.  It is asymptotically smooth and does not
   oscillate, so the interpolation framework (Sec. 1, Sec. 2) applies without
   directional expansions: every level is low-frequency, the MAC is the plain
   one (eq. macdirref with kappa w replaced by 0), and P2P, the spectra and
   the dense M2L matrices evaluate the screened kernel.  kappa = 0 gives the
   Laplace kernel either way. */
#define DEFMM_YUKAWA 4u

typedef struct {
  int32_t order_L;      /* interpolation nodes per dimension, 2..8 (padded FFT length 2L-1) */
  int32_t ncrit;        /* a cell is a leaf iff it holds <= ncrit points (Sec. 4.2.1), >= 1 */
  double eta;           /* MAC constant of eq. macdirref, > 0 (paper: 1) */
  double hf_threshold;  /* a level is high-frequency iff kappa * w > hf_threshold, w = half
                           the cell side; >= 0 (default 2) */
  int32_t dir_refine;   /* extra 4-fold refinements of the cube-face direction set, 0..4 */
  int32_t precision;    /* defmm_precision */
  int32_t m2l_mode;     /* defmm_m2l_mode */
  uint32_t flags;       /* DEFMM_SAME_POINTS | DEFMM_COMPRESS_SPECTRA | DEFMM_YUKAWA;
                           other bits: DEFMM_ERR_INVALID_ARG */
} defmm_params;

typedef struct defmm_plan defmm_plan;           /* opaque */
typedef struct defmm_workspace defmm_workspace; /* opaque */

typedef struct {
  int32_t levels;             /* tree levels of X (root = level 0) */
  int32_t hf_levels;          /* number of high-frequency levels */
  int64_t cells;              /* cells of X plus, for distinct sets, cells of Y */
  int64_t leaves;
  int64_t m2l_pairs;          /* admissible pairs of the dual tree traversal */
  int64_t p2p_cell_pairs;     /* near-field pairs of the traversal */
  int64_t p2p_point_pairs;    /* point-pair interactions of the near field */
  int64_t eff_expansions;     /* effective (cell, direction) expansions, both trees */
  int64_t m2l_expansions;     /* expansions taking part in M2L (sources + targets) */
  int64_t unique_offsets;     /* distinct (level, offset) pairs of the M2L lists */
  int32_t m2l_mode_per_level[32]; /* DEFMM_M2L_DENSE where the plan holds dense M2L
                                     matrices for that level, else DEFMM_M2L_FFT */
  int64_t spectra;            /* stored Fourier-domain M2L spectra: unique_offsets, or,
                                 for a compressed plan, one per class of (level,
                                 offset) under the 48 signed axis permutations
                                 (Sec. 4.3), i.e. per (level, sorted |offset|) */
  int32_t compressed_spectra; /* 1 if the plan reads spectra through the symmetry */
} defmm_stats;

/* Writes the default parameters: L=5, ncrit=64, eta=1, hf_threshold=2,
   dir_refine=0, DEFMM_C64, DEFMM_M2L_FFT, flags=0. */
defmm_status defmm_default_params(defmm_params* out);

/* Builds a plan.  X: device pointer, nx*3 FP64 row-major (x,y,z); Y likewise
   (ignored, may be NULL, when prm->flags has DEFMM_SAME_POINTS).  Host-
   synchronous: X and Y may be freed when it returns.  hip_stream: the stream
   used for the device work of the build (NULL = default stream).
   Errors: DEFMM_ERR_INVALID_ARG for NULL out/prm/X, n < 0, L outside 2..8,
   ncrit < 1, kappa < 0 or non-finite, eta <= 0, unknown flag bits, non-finite
   coordinates.
   nx = 0 or ny = 0 is valid (every potential is then 0). */
defmm_status defmm_plan_create(const double* X, int64_t nx, const double* Y, int64_t ny,
                               double kappa, const defmm_params* prm, void* hip_stream,
                               defmm_plan** out);

/* Builds only the host side of a plan (tree, traversal lists, directions,
   operator tables) from HOST arrays, touching no device: the result answers
   defmm_plan_stats and the defmm_plan_export_* calls, while workspace_create
   and matvec reject it with DEFMM_ERR_INVALID_ARG.  Same arguments and errors
   as defmm_plan_create otherwise. */
defmm_status defmm_plan_inspect_create(const double* X, int64_t nx, const double* Y, int64_t ny,
                                       double kappa, const defmm_params* prm, defmm_plan** out);

/* Device bytes held by the plan and needed by one workspace. */
defmm_status defmm_plan_footprint(const defmm_plan* plan, size_t* resident_bytes,
                                  size_t* workspace_bytes);
defmm_status defmm_plan_stats(const defmm_plan* plan, defmm_stats* out);

defmm_status defmm_workspace_create(defmm_plan* plan, defmm_workspace** out);

/* One matvec p = G q, asynchronous on hip_stream (NULL = default stream).
   q: device, ny complex values in the caller's order, interleaved (re, im),
   complex128 for DEFMM_C128 and complex64 for DEFMM_C64; p: device, nx complex
   of the same type, overwritten.  q must stay valid until the stream has
   passed this call.  A workspace must not serve two in-flight matvecs. */
defmm_status defmm_matvec(defmm_plan* plan, defmm_workspace* ws, const void* q, void* p,
                          void* hip_stream);

/* The same matvec replayed from a HIP graph: the first call (or the first after
   q, p or the workspace's execution choices changed) captures the launch
   sequence on hip_stream into a graph held by the workspace; later calls with
   the same q and p launch the graph, one submission instead of one per kernel.
   q and p are baked into the graph: refill q in place between calls.
   hip_stream must be a created stream (capture is not possible on the null
   stream); per-pass timing must be off.  Same results as defmm_matvec, bit
   for bit. */
defmm_status defmm_matvec_graph(defmm_plan* plan, defmm_workspace* ws, const void* q, void* p,
                                void* hip_stream);

/* Allocation-free matvec, for callers that cannot allocate device memory
   (code under HIP graph capture, tight serving loops, harnesses that forbid
   hipMalloc): p = G q like defmm_matvec, with the workspace arrays taken from
   one static device array of defmm_matvec_noalloc_capacity() bytes (64 MiB)
   per GPU instead of a defmm_workspace.  It calls no hipMalloc or hipFree and
   allocates no device memory.  Runs on hip_stream only (near field not
   overlapped), Fourier M2L on every level; same results as defmm_matvec to
   rounding.  The array's device address is looked up once per device, on the
   first call with that device current, and kept until the process ends.
   Every call on one GPU shares that array: calls that overlap on one GPU
   (other streams, other threads) race and give wrong results; serialise them.
   q, p: device pointers as for defmm_matvec.  Errors: DEFMM_ERR_INVALID_ARG
   for a NULL plan, q or p, an inspection plan, or a plan whose workspace
   (charges, potentials, expansions, Fourier rows, near-field partial sums)
   exceeds the capacity (use defmm_matvec then); DEFMM_ERR_DEVICE for a
   failed launch or address lookup. */
defmm_status defmm_matvec_noalloc(defmm_plan* plan, const void* q, void* p, void* hip_stream);

/* Bytes of the allocation-free matvec's static workspace array. */
size_t defmm_matvec_noalloc_capacity(void);

defmm_status defmm_workspace_destroy(defmm_workspace* ws);
defmm_status defmm_plan_destroy(defmm_plan* plan);

const char* defmm_status_string(defmm_status s);
const char* defmm_last_error(void);

/* ---- Introspection (tests, benchmarks).  All outputs are host arrays sized by
   a first call with NULL outputs, which returns the count in *n. ---- */

/* Bounding cube: side D and lower corner origin[3]. */
defmm_status defmm_plan_geometry(const defmm_plan* plan, double* D, double* origin3);

/* Cells of tree `which` (0 = X, 1 = Y), level-major, Morton order per level:
   level, integer coordinates ijk[3] at that level, first sorted point, point
   count, leaf flag.  perm (optional, n_points): sorted position -> caller index. */
defmm_status defmm_plan_export_tree(const defmm_plan* plan, int32_t which, int64_t* n,
                                    int32_t* level, int32_t* ijk, int32_t* first,
                                    int32_t* count, int32_t* is_leaf, int32_t* perm);

/* M2L pairs (Alg. 1): level, target cell, source cell (ids as in export_tree),
   offset delta = ijk(t) - ijk(s), best direction (Alg. 2; -1 when low-frequency). */
defmm_status defmm_plan_export_m2l(const defmm_plan* plan, int64_t* n, int32_t* level,
                                   int32_t* t, int32_t* s, int32_t* delta, int32_t* dir);

/* P2P pairs (Alg. 1): target cell, source cell. */
defmm_status defmm_plan_export_p2p(const defmm_plan* plan, int64_t* n, int32_t* t, int32_t* s);

/* Marks of tree `which` (0 = X, 1 = Y) after the blank passes (Alg. 2, 3): the
   effective expansions as (cell id, direction index or -1 for the
   non-directional mark), ordered by cell, then direction.  Call with NULL
   arrays to get *n, then with arrays of *n entries. */
defmm_status defmm_plan_export_marks(const defmm_plan* plan, int32_t which, int64_t* n, int32_t* cell,
                                     int32_t* dir);

/* Expansions of tree `which` after a matvec on ws: cell id, direction (-1 =
   non-directional) and kind 0 = multipole / 1 = local node values, L^3 complex
   per expansion (complex of the plan's precision). */
defmm_status defmm_workspace_export_expansions(defmm_workspace* ws, int32_t which, int32_t kind,
                                               int64_t* n, int32_t* cell, int32_t* dir,
                                               void* values);

/* Per-pass device time.  When enabled, matvec records HIP events around each pass
   on its stream; pass_ms[i] accumulates milliseconds over the matvecs since the
   last reset, calls[i] counts launches.  Pass names: defmm_pass_name(i). */
#define DEFMM_NUM_PASSES 12
defmm_status defmm_workspace_set_timing(defmm_workspace* ws, int32_t enable);

/* Execution choices of a workspace (results are the same to rounding; the
   near-field split never changes a bit):
   overlap          1: near field on the workspace's own stream, concurrently
                    with the far field, forked after the charge gather;
                    2: the same, forked after M2F (the upward pass runs
                    alone); 0: every pass in sequence;
   p2p_waves_per_cu persistent near-field workgroups (one wave) per compute
                    unit when overlapped, 1..32;
   m2l_variant      0: Hadamard fused with F2L per target; 1: frequency-sliced
                    per target; 2: frequency-sliced per group of 8 targets
                    merged by source (default);
   dense_levels     bit l set: level l runs the dense MFMA M2L (only levels whose
                    dense matrices the plan built: DEFMM_M2L_AUTO or _DENSE);
   updown_variant   P2M, M2M and L2L kernels: 1 = P2M one workgroup per leaf
                    (weights once for all its expansions), M2M/L2L one wave per
                    pair of expansions of a cell with pencils in registers
                    (default); 0 = one workgroup per expansion, one node per
                    thread;
   fourier_items    expansions per workgroup of M2F and F2L: 1, 2 or 4 (capped
                    to what fits the LDS), 0 = as many as fit 64 KB;
   ms               median matvec time measured by defmm_workspace_autotune. */
typedef struct {
  int32_t overlap;
  int32_t p2p_waves_per_cu;
  int32_t m2l_variant;
  uint32_t dense_levels;
  int32_t updown_variant;
  int32_t fourier_items;
  double ms;
} defmm_tuning;

/* Times the candidate execution choices on this workspace (each: one warm-up
   and `reps` matvecs of q into p on hip_stream; host-synchronous) and keeps
   the fastest: the Fourier-path M2L variant in sequence first, then the M2M/L2L
   kernels, then the M2F/F2L expansions per workgroup, then, level by level, the dense MFMA M2L where the plan holds its
   matrices, then the
   overlapped near field forked early or after M2F, with 2, 3, 4 and 6 waves
   per CU.  q and p as in defmm_matvec; p holds a valid result afterwards.
   chosen (optional) receives the choice. */
defmm_status defmm_workspace_autotune(defmm_plan* plan, defmm_workspace* ws, const void* q, void* p,
                                      void* hip_stream, int32_t reps, defmm_tuning* chosen);
defmm_status defmm_workspace_get_tuning(const defmm_workspace* ws, defmm_tuning* out);
defmm_status defmm_workspace_set_tuning(defmm_workspace* ws, const defmm_tuning* t);

/* Overlap (new workspaces: 2): the near field (P2P) runs on a stream owned by
   the workspace, forked after the charge gather (enable = 1; enable = 2:
   after M2F) and joined before L2P, as a persistent kernel that leaves wave slots
   to the far field.  Off (0): every pass runs in sequence on the caller's
   stream at full occupancy (used to time each kernel alone).  Results are
   bitwise identical either way. */
defmm_status defmm_workspace_set_overlap(defmm_workspace* ws, int32_t enable);
defmm_status defmm_workspace_pass_times(defmm_workspace* ws, double* pass_ms, int64_t* calls);
const char* defmm_pass_name(int32_t i);

/* Algorithmic work of one matvec per pass under the workspace's current
   execution choices (which levels run the dense M2L, which Fourier variant):
   bytes[i] = compulsory HBM bytes of pass i (each input read once, each output
   written once; e.g. Fourier M2L: each distinct spectrum and each source row of
   (2L-1)^3 values read once, each target row written once; dense M2L: each
   level-local matrix, source and target expansion once), flops[i] = real
   floating-point operations (a complex multiply-add counts 8; a near-field
   pair counts 23, 17 for the screened kernel).  Either pointer may be NULL;
   each holds DEFMM_NUM_PASSES entries. */
defmm_status defmm_workspace_pass_work(const defmm_workspace* ws, double* bytes, double* flops);

/* Storage order of the Fourier-domain rows (spectra, M~, L~) for order L
   (2..8), for inspection and tests.  Host only, no device use.  The
   (2L-1)^3 frequencies xi (flattened kx + P ky + P^2 kz, each in [0, P)) are
   stored as pairs (xi, -xi) at positions (2k, 2k+1), the pairs grouped into
   `slices` slices of `cap` pairs, each slice a union of orbits of the 48
   signed axis permutations (Sec. 4.3); *row = 2 * slices * cap.
   freq (optional, *row entries): the frequency stored at each position, -1
   for padding (stored as zero).  perm (optional, slices * 48 * 64 bytes):
   for slice s, symmetry code r and pair k of the slice, byte
   perm[(s * 48 + r) * 64 + k] = k' | swap << 7 says where the canonical
   spectrum holds D[R_r^-1 xi_k]: pair k' of the same slice, second member
   if swap.  Entries for k >= cap are 0.  Symmetry codes are those of
   defmm_canonical_offset.  Errors: DEFMM_ERR_INVALID_ARG for L outside
   2..8 or NULL slices/cap/row. */
defmm_status defmm_fourier_layout(int32_t L, int32_t* slices, int32_t* cap, int32_t* row, int32_t* freq,
                                  uint8_t* perm);

/* Direction set of direction level E (Sec. 4.1.2, Sec. 2.1), for inspection
   and tests: *n = 6 * 4^E unit vectors, the projected centres of the cube's
   face patches when each face is split 2^E x 2^E, index face * 4^E + i * 2^E
   + j (faces +x, -x, +y, -y, +z, -z), and the index of the father direction
   at E - 1 (-1 at E = 0).  dirs (optional, [n x 3] FP64) and father
   (optional, n int64) are host arrays.  Errors: DEFMM_ERR_INVALID_ARG for E
   outside 0..12 or NULL n. */
defmm_status defmm_directions(int32_t E, int64_t* n, double* dirs, int64_t* father);

/* Canonical representative of an M2L offset under the 48 signed axis
   permutations (Sec. 4.3), for inspection and tests.  d: 3 integers; d0
   receives the sorted absolute values (ascending) and *code the symmetry
   r = 8 * p + signs with d_i = s_i * d0[pi(i)], s_i = -1 iff bit i of signs
   is set, pi = the p-th permutation of (0,1,2) in lexicographic order.  The
   spectrum of (level, d) equals that of (level, d0) read at R_r^-1 xi.
   Errors: DEFMM_ERR_INVALID_ARG for NULL pointers. */
defmm_status defmm_canonical_offset(const int32_t* d, int32_t* d0, int32_t* code);

#ifdef __cplusplus
}
#endif
#endif
