/*
 * mlmc.h - C ABI of the MI355X (gfx950) library for the per-sample spectral
 * hot path of multilevel Monte Carlo on honeycomb materials with random
 * vacancies (Plechac & von Schwerin, "Multi-level Monte Carlo acceleration
 * of computations on multi-layer materials with random defects").
 *
 * Per sample and per Brillouin-zone point the library assembles the complex
 * Hermitian Bloch Hamiltonian H(k) of an N x N supercell with vacancies,
 * computes all its eigenvalues and accumulates the smoothed integrated
 * density of states (IDoS) per unit area; on top of that it accumulates the
 * per-level sums of the MC / MLMC estimators.
 *
 * Conventions shared by every entry point
 *   - Every call returns an mlmc_status (0 = success, negative = error).  No
 *     call throws, aborts or prints.  mlmc_status_string() names a status and
 *     mlmc_last_error() gives a detail message for the calling thread.
 *   - Arguments named d_* are device pointers owned by the caller; h_* and
 *     plain pointers to structs are host pointers.  Arguments are validated
 *     before anything is launched; a failed validation launches nothing.
 *   - Work is enqueued on `stream` (a hipStream_t; NULL is the default
 *     stream) and is asynchronous: outputs are valid once the stream has
 *     synchronised.  The only calls that may block are the setup calls
 *     (mlmc_lattice_create / _destroy, mlmc_context_create / _destroy /
 *     _timer) and mlmc_context_timer_read.
 *   - Hot-path calls allocate no device memory.  Scratch memory is a caller
 *     workspace whose size mlmc_workspace_bytes reports.
 *   - The library keeps no mutable state between calls outside the handles
 *     the caller creates and destroys (lattices, pipeline contexts): calls
 *     on different streams with different workspaces and contexts share
 *     nothing and may be made from any thread.  mlmc_last_error() is
 *     per thread.
 *   - Results are deterministic: fixed reduction orders and no floating-point
 *     atomics.  Per-outcome results (masks, H(k), eigenvalues, IDoS) do not
 *     depend on which other outcomes share a call; level sums are
 *     bitwise reproducible for equal inputs and equal workspace size.
 *   - Orbital numbering: orbital m of cell (i, j) (position i*a1 + j*a2 of the
 *     N x N supercell) has index (i*N + j)*n_orb + m.  Present orbitals keep
 *     this order and are renumbered 0..n-1.
 */
#ifndef MLMC_H
#define MLMC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef void *mlmc_stream; /* a hipStream_t */

typedef enum {
    MLMC_OK = 0,
    MLMC_ERR_INVALID_ARG = -1, /* an argument is out of range or inconsistent       */
    MLMC_ERR_UNSUPPORTED = -2, /* valid request the library does not implement      */
    MLMC_ERR_WORKSPACE = -3,   /* workspace pointer NULL or smaller than required    */
    MLMC_ERR_HIP = -4          /* the HIP runtime reported an error (detail string)  */
} mlmc_status;

typedef enum {
    MLMC_C128 = 0, /* complex double, interleaved (re, im) */
    MLMC_C64 = 1   /* complex float, interleaved (re, im)  */
} mlmc_dtype;

typedef enum {
    MLMC_PREC_FP64 = 0, /* every step in double precision                              */
    MLMC_PREC_MIXED = 1 /* tridiagonal reduction in single precision; Sturm bisection,
                           IDoS and level sums in double precision                     */
} mlmc_precision;

typedef enum {
    MLMC_KGRID_MP = 0,     /* K x K Monkhorst-Pack: kappa = (2r - K + 1) / (2K)           */
    MLMC_KGRID_GAMMA = 1,  /* K x K Gamma-centred:  kappa = r / K                         */
    MLMC_KGRID_RHOMBI = 2  /* the three-rhombus lattice of Section 4.2: 3 K^2 points       */
} mlmc_kgrid_kind;

typedef enum {
    MLMC_SMOOTH_GAUSS = 0, /* g(x) = erfc(x / sqrt 2) / 2                               */
    MLMC_SMOOTH_CUBIC = 1  /* g(x) = 1/2 - 9x/8 + 5x^3/8 on [-1, 1], 1 below, 0 above     */
} mlmc_smoother;

/* One row of a tight-binding hopping table (Section 3.1, eq. (tightbinding)).
 * It adds h * exp(i k.(R + r_to - r_from)) to H[from, to] and the complex
 * conjugate to H[to, from] for every cell; R = (R[0], R[1]) is the cell
 * offset of the target orbital in units of a1, a2.  A row with R = 0 and
 * from_orb == to_orb is an on-site energy and is added once (its imaginary
 * part must be 0). */
typedef struct {
    int32_t R[2];
    int32_t from_orb;
    int32_t to_orb;
    double re;
    double im;
} mlmc_hop;

/* Host description of a honeycomb lattice model (Sections 3.1-3.2). */
typedef struct {
    uint32_t lattice_id;            /* selects the vacancy random stream (tag)          */
    int32_t n_orb;                  /* orbitals per primitive cell (1..64)              */
    int32_t n_groups;               /* vacancy groups per cell (1..16)                  */
    int32_t n_hops;                 /* rows of `hops` (1..65536)                        */
    double cell_area;               /* |F| of the primitive cell, Angstrom^2 (> 0)      */
    const double *orb_frac;         /* [n_orb][2] positions in fractions of a1, a2      */
    const int32_t *orb_group;       /* [n_orb] group of each orbital, 0..n_groups-1     */
    const uint8_t *group_removable; /* [n_groups] 1: the group may be vacant            */
    const mlmc_hop *hops;           /* [n_hops]                                         */
    /* Non-orthogonal basis (Section 3.1, generalised problem H c = E S c):
     * n_overlap > 0 rows of an overlap table, S(k) = I + its Bloch sum with
     * the conventions of `hops`; n_overlap = 0 and overlap = NULL for an
     * orthogonal basis (S = I). */
    int32_t n_overlap;              /* 0..65536                                         */
    const mlmc_hop *overlap;        /* [n_overlap]                                      */
} mlmc_lattice_desc;

typedef struct mlmc_lattice_s *mlmc_lattice; /* opaque device-resident lattice */

/* Opaque pipeline context of level estimates (mlmc_context_create). */
typedef struct mlmc_context_s *mlmc_context;

/* The operations that take a caller workspace (mlmc_workspace_bytes). */
typedef enum {
    MLMC_OP_BATCHED_EIGVALSH = 0,             /* mlmc_batched_eigvalsh: dtype, prec, ld, batch          */
    MLMC_OP_BATCHED_EIGVALSH_GENERALIZED = 1, /* mlmc_batched_eigvalsh_generalized: dtype, prec, ld, batch */
    MLMC_OP_LEVEL_ESTIMATE = 2,               /* mlmc_level_estimate and mlmc_level_outcomes: lat, N_fine,
                                                 coupled, K_fine, K_coarse, kgrid, chunk_samples, prec,
                                                 n_eps                                                   */
    MLMC_OP_LEVEL_OUTCOMES_SINGLE_PASS = 3,   /* mlmc_level_outcomes taking chunk_samples outcomes in one
                                                 pass (one buffer set): the fields of MLMC_OP_LEVEL_ESTIMATE */
    MLMC_OP_BATCHED_EIGH = 4,                 /* mlmc_batched_eigh: dtype, prec, ld, batch                */
    MLMC_OP_BATCHED_EIGH_GENERALIZED = 5      /* mlmc_batched_eigh_generalized: dtype, prec, ld, batch    */
} mlmc_op;

/* Arguments of a workspace query; fields an operation does not use are ignored. */
typedef struct {
    mlmc_op op;
    mlmc_dtype dtype;
    mlmc_precision prec;
    int64_t ld;            /* matrix side bound                                  */
    int64_t batch;         /* matrices per call                                  */
    mlmc_lattice lat;
    int32_t N_fine;
    int32_t coupled;       /* 0 or 1                                             */
    int32_t K_fine;
    int32_t K_coarse;
    mlmc_kgrid_kind kgrid;
    int64_t chunk_samples; /* samples per pass of a level call (>= 1)            */
    int32_t n_eps;
} mlmc_workspace_request;

const char *mlmc_status_string(int status);
const char *mlmc_last_error(void);

/* Copy a lattice description to the current HIP device (setup, blocking,
 * allocates device memory).  The handle is bound to that device; the host
 * arrays of `desc` may be freed afterwards.  Validates ranges and that the
 * on-site rows are real. */
mlmc_status mlmc_lattice_create(const mlmc_lattice_desc *desc, mlmc_lattice *out);
/* Release a handle (blocking; waits for the device).  NULL is accepted. */
mlmc_status mlmc_lattice_destroy(mlmc_lattice lat);
/* Orbitals of the pristine N x N supercell (= n_orb * N * N); the matrix
 * side bound `ld` of every per-outcome array. */
mlmc_status mlmc_lattice_max_orbitals(mlmc_lattice lat, int32_t N, int64_t *n_max);

/* Vacancy outcomes (Section 3.2: every removable group of every cell is
 * vacant independently with probability p).
 * Philox4x64-10 (Salmon et al., SC'11) with key (seed, tag) and counter
 * (first_sample + s, floor(g/4), 0, 0); group g = (i*N + j)*n_groups + local
 * of sample s takes word g mod 4 and is vacant iff it is removable and
 * (word >> 11) < floor(p * 2^53).  The MLMC level call uses
 * tag = (lattice_id << 32) | N.
 * d_mask: [n_samples][N][N][n_groups] uint8, 1 = vacant (written).
 * Errors: N < 1, p outside [0, 1], n_samples < 0. */
mlmc_status mlmc_sample_vacancies(mlmc_lattice lat, int32_t N, double p, uint64_t seed, uint64_t tag,
                                  int64_t first_sample, int64_t n_samples, uint8_t *d_mask, mlmc_stream stream);

/* Control-variate partition (Section 3.3, Figure "CV"): each outcome of an N
 * x N supercell (N even) is cut into four quarters that keep their vacancies;
 * quarter q = 2*qi + qj holds cells i in [qi*N/2, (qi+1)*N/2), j in
 * [qj*N/2, (qj+1)*N/2), renumbered as an N/2 supercell that is then
 * re-periodised.
 * d_mask: [n_samples][N][N][G]; d_quarters: [n_samples][4][N/2][N/2][G]. */
mlmc_status mlmc_partition_masks(mlmc_lattice lat, int32_t N, const uint8_t *d_mask, int64_t n_samples,
                                 uint8_t *d_quarters, mlmc_stream stream);

/* Number of points of a Brillouin-zone grid: K^2 (MLMC_KGRID_MP,
 * MLMC_KGRID_GAMMA) or 3 K^2 (MLMC_KGRID_RHOMBI).  Host only.
 * Errors: bad kind, K < 1 or K > 4096, NULL n_k. */
mlmc_status mlmc_kgrid_points(mlmc_kgrid_kind kind, int32_t K, int32_t *n_k);

/* Brillouin-zone grid in reduced coordinates of the supercell reciprocal
 * lattice, with the weights of the nearest-point rule (Section 4.3).
 *   MP, GAMMA: a uniform K x K grid of the supercell zone with equal weights
 *     (the reading used by the main workloads); point r1*K + r2, weight 1/K^2.
 *   RHOMBI: Section 4.2's lattice: the hexagonal zone as three rhombi with
 *     the common corner Gamma, each cut into K x K rhombi whose corners are
 *     the k-points; corners shared by two rhombi or equal modulo a reciprocal
 *     lattice vector count once.  These are the 3 K^2 points
 *     (a, b) / (3K) with a + b divisible by 3, listed in increasing (a, b),
 *     each of weight 1 / (3 K^2).
 * d_kred: [n_k][2], d_kweight: [n_k] with n_k from mlmc_kgrid_points. */
mlmc_status mlmc_kgrid(mlmc_kgrid_kind kind, int32_t K, double *d_kred, double *d_kweight, mlmc_stream stream);

/* Bloch Hamiltonians H(k) (Section 3.1, eq. (tightbinding), orthogonal form;
 * vacant sites' rows and columns removed, Section 3.2).  For outcome s and
 * k-point k, unit u = s*n_k + k receives the n_u x n_u Hermitian matrix in the
 * leading block of d_H + u*ld*ld (column-major, leading dimension ld), with
 * H[a, b] += h * exp(2 pi i (kappa1 d1 + kappa2 d2) / N), d = R + frac(to) -
 * frac(from) the unwrapped atom-to-atom displacement (atom gauge).
 * d_mask: [n_samples][N][N][G]; d_kred: [n_k][2]; d_n: [n_samples*n_k] out.
 * dtype selects complex128 or complex64 storage.  Entries outside the n_u x
 * n_u block are not written.  Errors: ld < n_orb*N*N, n_k < 1. */
mlmc_status mlmc_build_hamiltonians(mlmc_lattice lat, int32_t N, const uint8_t *d_mask, int64_t n_samples,
                                    const double *d_kred, int32_t n_k, mlmc_dtype dtype, void *d_H, int64_t ld,
                                    int32_t *d_n, mlmc_stream stream);

/* Overlap matrices S(k) of a lattice with a non-orthogonal basis (Section
 * 3.1): the unit matrix plus the Bloch sum of the lattice's overlap table,
 * with the layout, phases and removed rows and columns of
 * mlmc_build_hamiltonians for the same outcomes and k-points.
 * Errors: the lattice has no overlap table, ld < n_orb*N*N, n_k < 1. */
mlmc_status mlmc_build_overlaps(mlmc_lattice lat, int32_t N, const uint8_t *d_mask, int64_t n_samples,
                                const double *d_kred, int32_t n_k, mlmc_dtype dtype, void *d_S, int64_t ld,
                                int32_t *d_n, mlmc_stream stream);

/* Bytes of caller workspace an operation needs (host only, no device work).
 *   MLMC_OP_BATCHED_EIGVALSH: `batch` matrices of side bound ld (0 for the
 *     LDS-resident path, ld <= 128 complex128 / 180 complex64).
 *   MLMC_OP_BATCHED_EIGVALSH_GENERALIZED: `batch` pencils of side bound ld.
 *   MLMC_OP_LEVEL_ESTIMATE: a level call that processes chunk_samples samples
 *     per pass (the call uses the largest chunk that fits the workspace it is
 *     given), with three buffer sets that consecutive chunks take in turn.
 *   MLMC_OP_LEVEL_OUTCOMES_SINGLE_PASS: mlmc_level_outcomes on up to
 *     chunk_samples outcomes in a single pass with one buffer set (about a
 *     third of the matrix memory of the pipelined layout).
 *   MLMC_OP_BATCHED_EIGH: `batch` matrices of side bound ld.  LDS-resident
 *     sides: 7*ld*ld doubles each, ld*ld rounded up to even (the tridiagonal
 *     eigenvectors and the inverse iteration's scratch).  Larger sides: a
 *     copy of each matrix, the two-stage buffers, every panel's block
 *     reflector (16*ld + 256 complex per 16 columns), for complex64 the
 *     vectors in complex128, and the band inverse iteration's LU factors and
 *     vector (about 804*ld bytes per wavefront).
 * Errors: NULL arguments, unknown op, the operation's own argument checks
 * (MLMC_ERR_UNSUPPORTED for sizes beyond the library's limits). */
mlmc_status mlmc_workspace_bytes(const mlmc_workspace_request *req, size_t *bytes);

/* All eigenvalues of a batch of Hermitian matrices (the dense full
 * eigensolve of each H(k), Section 4.2; E_n(k) is the n-th smallest
 * eigenvalue, Section 4.3).  Householder reduction to real tridiagonal form
 * (LDS-resident for ld <= 128 complex128 / 180 complex64, else in device
 * memory), then Sturm-count bisection in double precision (Newton points
 * inside the certified brackets; each eigenvalue within 1e-12 eV, or a few
 * ulps of the spectral radius if that is larger).
 * d_H: the matrices, column-major with leading dimension ld; only the lower
 * triangle of the leading n_b x n_b block of matrix b is read, and it is
 * overwritten.  d_offsets == NULL: matrix b starts at element b*ld*ld
 * ([batch][ld][ld]).  Otherwise the layout is ragged: matrix b starts at
 * element d_offsets[b] (device array [batch]) and occupies ld*n_b elements
 * (its columns 0..n_b-1), so a batch of uneven sizes can be packed at
 * offsets sum_{a<b} ld*n_a; the caller keeps the matrices inside its buffer
 * and disjoint.  d_n: [batch] sides, each in [0, ld] (a matrix with n_b
 * outside that range gets NaN eigenvalues).  d_w: [batch][ldw], ascending,
 * entries >= n_b untouched.  dtype/prec: (C128, FP64) or (C64, MIXED). */
mlmc_status mlmc_batched_eigvalsh(mlmc_dtype dtype, mlmc_precision prec, void *d_H, int64_t ld,
                                  const int64_t *d_offsets, const int32_t *d_n, int64_t batch, double *d_w,
                                  int64_t ldw, void *d_work, size_t work_bytes, mlmc_stream stream);

/* mlmc_batched_eigvalsh for callers that cannot allocate device memory or
 * bring a workspace (code under HIP graph capture, tight serving loops,
 * harnesses that forbid allocation).  Same arguments, layout and results as
 * mlmc_batched_eigvalsh (the same kernels), without d_work: the two-stage
 * path's scratch is a static 64 MiB device array of the library, one per
 * device, kept from the library's load until the process ends; batches whose
 * workspace exceeds it run in consecutive chunks on `stream`.  The call
 * allocates nothing.  Every call on one device shares that array and leaves
 * its contents behind (nothing in it has to start at zero), so calls that
 * overlap on one device - on different streams, or from different threads
 * without ordering - race; calls on one stream are ordered.
 * Errors: as mlmc_batched_eigvalsh; MLMC_ERR_UNSUPPORTED when one matrix of
 * side ld needs more than the 64 MiB (not the case for any ld the library
 * supports). */
mlmc_status mlmc_batched_eigvalsh_noalloc(mlmc_dtype dtype, mlmc_precision prec, void *d_H, int64_t ld,
                                          const int32_t *d_n, int64_t batch, double *d_w, int64_t ldw,
                                          mlmc_stream stream);

/* Eigenvalues and eigenvectors of a batch of Hermitian matrices: the
 * eigenstates that the Kubo-Greenwood conductivity needs besides the band
 * energies (Section 1; named as the next quantity of interest in Section 5).
 * LDS-resident matrices (ld <= 128 complex128 / 180 complex64): one
 * workgroup per matrix: Householder reduction H = Q T_c Q^H with the
 * reflectors kept, T_c = D T D^H with a diagonal unitary D that makes the
 * sub-diagonal real and non-negative, eigenvalues of T by the bisection of
 * mlmc_batched_eigvalsh, eigenvectors Z of T by inverse iteration with
 * partial pivoting, then V = Q D Z.
 * Larger matrices (ld <= 4096): a copy of the matrices is reduced to a band
 * of half-width 16 (stage 1 of mlmc_batched_eigvalsh in the compute type,
 * each panel's block reflector I - V_p T_p V_p^H kept), the band is chased to
 * tridiagonal form and bisected for the eigenvalues, eigenvectors of the band
 * matrix B come from inverse iteration with a pivoted band LU of B - lam I
 * (one wavefront per eigenvalue), and the block reflectors take them back,
 * last panel first; the band and the reflectors are widened to double for
 * these steps, and complex64 vectors are rounded at the end.
 * Both paths: eigenvalues closer than 1e-3 of the spectral radius form a
 * cluster whose vectors are orthogonalised against each other (after every
 * solve on the LDS path; once, by Gram-Schmidt applied twice, on the banded
 * path); the eigenvalues are refined to the vectors' Rayleigh quotients
 * (ascending, a cluster's columns sorted with them).
 * d_H, d_offsets, d_n, d_w, ldw: as mlmc_batched_eigvalsh, except that the
 * matrices are left unchanged (only the lower triangles are read).  d_V: the
 * eigenvectors, matrix b at element b*ldv*ldv, column-major with leading
 * dimension ldv, column i (entries 0..n_b-1) the unit eigenvector of
 * d_w[b][i]; entries outside the leading n_b x n_b block are untouched.
 * Each vector is determined up to a phase (within a cluster, the cluster's
 * columns up to a unitary mix).  Accuracy: ||H v - w v|| of a few ulps of
 * ||H|| in the compute type (complex128 or complex64), columns orthonormal
 * to the same order.  d_work: mlmc_workspace_bytes(MLMC_OP_BATCHED_EIGH)
 * (7 ld^2 doubles per LDS-resident matrix; above that about 2 ld^2 complex
 * per matrix, plus ld^2 complex128 for complex64 input, and the inverse
 * iteration's factors and vector, about ld * 804 bytes per wavefront in
 * flight).
 * Errors: ld above 4096, or a batch above 65535 beyond the LDS bound
 * (MLMC_ERR_UNSUPPORTED); ldw or ldv < ld, NULL buffers, workspace too
 * small. */
mlmc_status mlmc_batched_eigh(mlmc_dtype dtype, mlmc_precision prec, void *d_H, int64_t ld, const int64_t *d_offsets,
                              const int32_t *d_n, int64_t batch, double *d_w, int64_t ldw, void *d_V, int64_t ldv,
                              void *d_work, size_t work_bytes, mlmc_stream stream);

/* Eigenvalues and eigenvectors of a batch of Hermitian pencils (H, S), S
 * positive definite: H c = E S c, the non-orthogonal basis of Section 3.1,
 * for the eigenstates of Sections 1 and 5.  S = L L^H and C = L^{-1} H
 * L^{-H} as in mlmc_batched_eigvalsh_generalized, the eigenstates y of C as
 * in mlmc_batched_eigh, then c = L^{-H} y (a blocked back-substitution in
 * double), so that the columns are S-orthonormal: c_i^H S c_j = delta_ij.
 * d_H, d_S: [batch][ld][ld] column-major, lower triangles read, both
 * overwritten (C and L).  d_n, d_w, ldw, d_V, ldv: as mlmc_batched_eigh.
 * d_work: mlmc_workspace_bytes(MLMC_OP_BATCHED_EIGH_GENERALIZED) (the
 * Cholesky reduction's workspace plus mlmc_batched_eigh's).  Accuracy:
 * ||H c - E S c|| of a few ulps of ||H|| + |E| ||S|| in the compute type,
 * times the condition of S.  Errors: ld above 2048 (MLMC_ERR_UNSUPPORTED),
 * otherwise as mlmc_batched_eigh. */
mlmc_status mlmc_batched_eigh_generalized(mlmc_dtype dtype, mlmc_precision prec, void *d_H, void *d_S, int64_t ld,
                                          const int32_t *d_n, int64_t batch, double *d_w, int64_t ldw, void *d_V,
                                          int64_t ldv, void *d_work, size_t work_bytes, mlmc_stream stream);

/* All eigenvalues of a batch of Hermitian-definite pencils (H, S) (the
 * generalised problem H c = E S c of a non-orthogonal basis, Section 3.1):
 * S = L L^H (Cholesky) and C = L^{-1} H L^{-H}, both blocked on the GPU,
 * then the eigenvalues of C as in mlmc_batched_eigvalsh.  d_H, d_S: lower
 * triangles of the leading n_b x n_b blocks are read and both are
 * overwritten (S by L).  S must be positive definite (otherwise the
 * eigenvalues come out NaN).  Other arguments as mlmc_batched_eigvalsh.
 * Errors: ld > 2048 (MLMC_ERR_UNSUPPORTED), workspace too small. */
mlmc_status mlmc_batched_eigvalsh_generalized(mlmc_dtype dtype, mlmc_precision prec, void *d_H, void *d_S,
                                              int64_t ld, const int32_t *d_n, int64_t batch, double *d_w,
                                              int64_t ldw, void *d_work, size_t work_bytes, mlmc_stream stream);

/* Smoothed IDoS per unit area of each outcome (eq. (IDoS) with the
 * nearest-point band approximation and the smoothing of eq.
 * (MLMC_smoothing), Section 4.3):
 *   I_s(eps_j) = 1/area * sum_k w_k sum_{i < n_{s,k}} g((E_{s,k,i} - eps_j)/delta)
 * d_w: [n_samples*n_k][ldw] ascending eigenvalues; d_n: [n_samples*n_k];
 * d_kweight: [n_k]; area = N*N*|F|; d_eps: [n_eps]; d_idos: [n_samples][n_eps].
 * The Gaussian is evaluated for |x| < 10 and taken as exactly 1 / 0 beyond
 * (|error| < 1e-23 per state); the cubic has compact support [-1, 1]. */
mlmc_status mlmc_idos(const double *d_w, int64_t ldw, const int32_t *d_n, int64_t n_samples, int32_t n_k,
                      const double *d_kweight, double area, const double *d_eps, int32_t n_eps, double delta,
                      mlmc_smoother smoother, double *d_idos, mlmc_stream stream);

/* Per-level sums of eq. (MLMC) and of its variance (Section 2.2):
 *   Y_s = Q_s (d_idos_quarters == NULL) or Q_s - (1/4) sum_q Q_{s,q};
 *   d_stats[0][j] += sum_s Y_s(j), [1] += sum Y^2, [2] += sum Q_s(j),
 *   [3] += sum Q_s^2, accumulated in sample order in double precision.
 * d_idos_fine: [n_samples][n_eps]; d_idos_quarters: [n_samples][4][n_eps];
 * d_stats: [4][n_eps] (caller initialises). */
mlmc_status mlmc_level_stats(const double *d_idos_fine, const double *d_idos_quarters, int64_t n_samples,
                             int32_t n_eps, double *d_stats, mlmc_stream stream);

/* Pipeline context of level estimates (setup calls; they create and destroy
 * HIP streams and events and may block).  A context holds, for the current
 * device: two streams besides the caller's (default priority; one runs the
 * band-to-tridiagonal chase, the other the bisection, IDoS and level sums),
 * the events that order them against the caller's stream, the buffer-set
 * rotation of consecutive calls, and an optional launch timer.  Level calls
 * that pass the same context enqueue one at a time (the context's own lock);
 * calls with different contexts share nothing.  A context is bound to the
 * device current at creation.  Streams that share one of the runtime's few
 * hardware queues per process run their work in order; the context's four
 * streams (two caller streams, chase, back) are created one after another so
 * that they get separate queues, which holds in a process whose other streams
 * are idle.  Create a context once per concurrent pipeline and keep it: after
 * other streams have been created and destroyed, a new context's chase
 * stream can share a queue with one of its caller streams, and its chases
 * then no longer overlap the reduction of the next chunk (measured: 23.0k
 * against 25.9k FP64 eigensolves/s on the graphene N = 16 workload). */
mlmc_status mlmc_context_create(mlmc_context *out);
/* One of two caller streams the context owns (index 0 or 1; default
 * priority, non-blocking), created together with its back and chase streams
 * so that the four are spread over the runtime's hardware queues; level calls
 * alternating between them overlap as described at mlmc_level_estimate.
 * The streams are destroyed with the context. */
mlmc_status mlmc_context_stream(mlmc_context ctx, int32_t index, mlmc_stream *out);
/* Launch choices of a context's level calls (the autotuner's knobs):
 *   chase_workgroups: persistent workgroups of a chunk's band-to-tridiagonal
 *     chase on the chase stream, beside the next chunk's dense-to-band stage
 *     (0: 3/4 of the CUs); a call's last chunk is chased on one workgroup per
 *     matrix;
 *   bisect_workgroups: workgroups of a chunk's bisection on the back stream
 *     (0: one per CU);
 *   update_tile_rows: tiles of the dense-to-band stage's rank-2k update,
 *     32 x 64 (32: 16 KiB of LDS, small enough to share a CU with a chase
 *     workgroup) or 64 x 64 (64); 0 means 32.
 * Results do not depend on the workgroup counts; the update tile changes the
 * rounding of the reduction only (both within the accuracy stated for
 * mlmc_batched_eigvalsh). */
typedef struct {
    int64_t chase_workgroups;
    int64_t bisect_workgroups;
    int32_t update_tile_rows;
} mlmc_launch_config;
mlmc_status mlmc_context_configure(mlmc_context ctx, const mlmc_launch_config *cfg);
/* Waits for the context's streams, then destroys its events and streams.
 * NULL is accepted.  The caller must not use the context afterwards. */
mlmc_status mlmc_context_destroy(mlmc_context ctx);
/* Launch timing of the level calls made with `ctx` (diagnostics): capacity
 * > 0 creates that many start/stop HIP event pairs up front (a setup call),
 * and each kernel launch of those calls then records one pair on the stream
 * it is launched on, until all pairs are used (later launches are counted as
 * dropped).  Calling again with the same capacity forgets the records and
 * keeps the events; 0 destroys them.  detail != 0: the kernels of the
 * dense-to-band stage are also timed one by one (a pair each, inside the
 * "band_reduce" pair of their launch). */
mlmc_status mlmc_context_timer(mlmc_context ctx, int64_t capacity, int32_t detail);
/* Total event-measured duration (ms) and count of the recorded launches of
 * kernel `name` since the timer was last (re)set: "sample_vacancies",
 * "partition", "kgrid", "assemble", "small_fused", "band_reduce" (dense to
 * band, several kernels per launch), "chase" (band to tridiagonal, one
 * kernel), "overlap_reduce" (Cholesky and reduction of a generalised
 * problem, several kernels), "bisect", "idos" or "level_stats"; with detail
 * also "s1_panel" (panel QR), "s1_hemm" (Hermitian product), "s1_wfactor"
 * and "s1_update" (rank-2k update), one launch per panel each; `dropped`
 * (may be NULL) receives the launches not timed.  Blocks until the recorded
 * launches have completed. */
mlmc_status mlmc_context_timer_read(mlmc_context ctx, const char *name, double *total_ms, int64_t *launches,
                                    int64_t *dropped);

/* One MLMC level over samples first_sample .. first_sample+M-1 (Sections 2.2
 * and 3.3): sample outcomes on the N_fine supercell (tag (lattice_id << 32) |
 * N_fine), compute Q_f = IDoS on the K_fine grid and, when coupled, the four
 * quarter IDoS Q_q on the K_coarse grid of the N_fine/2 supercell, and add
 * the sums of Y = Q_f [- (1/4) sum_q Q_q], Y^2, Q_f, Q_f^2 into d_stats
 * ([4][n_eps], accumulated; the caller initialises it).
 * Samples are processed in chunks that fit the workspace.
 * ctx == NULL: every step runs on `stream`, and the call keeps nothing.
 * With a context (mlmc_context_create, same device): each chunk's
 * bisection, IDoS and level sums run on the context's back stream while
 * `stream` goes on with the next chunk, and the two-stage path's
 * band-to-tridiagonal chase runs on its chase stream, on the number of CUs
 * mlmc_chase_cus reports, beside the next chunk's dense-to-band stage.  The
 * work is ordered by the context's events, `stream` waits for the context's
 * streams before the call returns, and the sums are added in sample order as
 * on one stream, so the result is the same bit for bit.  The workspace may be
 * handed from one call to the next of the same context on another stream
 * without synchronising: a call starts after the previous call's front part,
 * and reuses a buffer set only after the previous call has released it, so
 * consecutive calls on alternating streams with the same workspace, lattice,
 * sizes, precision and chunk overlap (one call's last chase and bisection
 * beside the next call's first reduction; such a call also leaves its last
 * chunk's chase on the mlmc_chase_cus share instead of the whole device);
 * with any other layout a call waits for all of the context's earlier work.
 * Other work that uses the workspace is the caller's to order; two contexts
 * must not share a workspace while both have work in flight.
 * d_first_sample (may be NULL): a device-resident int64 added to
 * first_sample when the sampling kernels run, and advanced by M at the end
 * of the call (on `stream`); with it, a HIP graph that captures the call
 * (ctx == NULL) draws the next M samples on every replay.  The call records
 * no memset and allocates nothing, so it can be captured.
 * Errors: N_fine < 1, coupled with odd N_fine, K < 1, p outside [0, 1],
 * delta <= 0, workspace too small for one sample. */
mlmc_status mlmc_level_estimate(mlmc_lattice lat, int32_t N_fine, int32_t coupled, double p, int32_t K_fine,
                                int32_t K_coarse, mlmc_kgrid_kind kind, uint64_t seed, int64_t first_sample,
                                int64_t M, const double *d_eps, int32_t n_eps, double delta, mlmc_smoother smoother,
                                mlmc_precision prec, double *d_stats, void *d_work, size_t work_bytes,
                                int64_t *d_first_sample, mlmc_context ctx, mlmc_stream stream);

/* The level of mlmc_level_estimate over M given outcomes instead of drawn
 * ones (d_mask: [M][N_fine][N_fine][n_groups], 1 = vacant, e.g. from
 * mlmc_sample_vacancies with each outcome's own seed and index), with
 * per-outcome outputs: row s of d_Y ([M][n_eps]) receives Y_s = Q_s [- (1/4)
 * sum_q Q_{s,q}] and row s of d_Q ([M][n_eps]) the fine IDoS Q_s; d_stats
 * ([4][n_eps], accumulated) receives the level sums as in
 * mlmc_level_estimate.  Any of the three may be NULL, not all.  Every
 * outcome's rows depend on that outcome alone (not on the others of the
 * call), which is what a server that batches requests relies on.  When the
 * workspace holds all M outcomes in a single pass with one buffer set
 * (MLMC_OP_LEVEL_OUTCOMES_SINGLE_PASS), the call takes that pass; otherwise
 * it works in chunks like mlmc_level_estimate.  Context and streams as
 * mlmc_level_estimate.
 * Errors: as mlmc_level_estimate, NULL mask, no output. */
mlmc_status mlmc_level_outcomes(mlmc_lattice lat, int32_t N_fine, int32_t coupled, int32_t K_fine, int32_t K_coarse,
                                mlmc_kgrid_kind kind, const uint8_t *d_mask, int64_t M, const double *d_eps,
                                int32_t n_eps, double delta, mlmc_smoother smoother, mlmc_precision prec,
                                double *d_stats, double *d_Y, double *d_Q, void *d_work, size_t work_bytes,
                                mlmc_context ctx, mlmc_stream stream);

/* Workgroups (one per CU) that the chase of a level call with a context
 * occupies on the current device with precision prec: 3/4 of the CUs (the chase runs beside
 * the next chunk's dense-to-band stage; the last chunk of a call is chased on
 * the whole device).  Errors: no device, bad prec. */
mlmc_status mlmc_chase_cus(mlmc_precision prec, int64_t *cus);

/* Sample allocation of eq. (opt_samples) (host, no device work):
 *   M_l = (C_alpha / (theta tol))^2 sqrt(V_l / W_l) sum_k sqrt(W_k V_k)
 * V, W, M_out: host arrays [L] (real-valued; the caller rounds up).
 * Errors: L < 1, any V < 0 or W <= 0, theta or tol <= 0. */
mlmc_status mlmc_optimal_samples(int32_t L, const double *V, const double *W, double C_alpha, double theta,
                                 double tol, double *M_out);

/* Density of states from the integrated density of states by numerical
 * differentiation (Section 4.3): on the increasing energy grid eps[0..n_eps)
 * dos[j] approximates dI/deps at eps[j] with the second-order three-point
 * formula, centred at interior points (unequal spacings allowed) and
 * one-sided at the two ends.  Host arrays; no device work.
 * Errors: n_eps < 3, NULL pointer, eps not strictly increasing. */
mlmc_status mlmc_dos(int32_t n_eps, const double *eps, const double *idos, double *dos);

#ifdef __cplusplus
}
#endif

#endif /* MLMC_H */
