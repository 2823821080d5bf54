/*
 * FP64 CPU oracle for the per-sample spectral hot path of the multilevel
 * Monte Carlo method for honeycomb materials with random vacancies
 * (Plechac & von Schwerin, "Multi-level Monte Carlo acceleration of
 * computations on multi-layer materials with random defects").
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, plain reference that the
 * GPU library is checked against.  Only the test suite, the smoke check and
 * the CPU-baseline leg of the benchmark may load it.  It shares no code,
 * header, table or helper with the HIP library.
 *
 * Every routine is the plain definition or a textbook algorithm written out
 * in double precision:
 *   - Philox4x64-10 counter-based generator (Salmon, Moraes, Dror, Shaw,
 *     "Parallel random numbers: as easy as 1, 2, 3", SC'11) drives the iid
 *     vacancy outcomes of Section 3.2;
 *   - the Bloch Hamiltonian of the supercell follows the tight-binding model
 *     of Section 3.1, eq. (tightbinding), with vacant sites' rows and columns
 *     removed (Section 3.2);
 *   - the control-variate partition into four re-periodised quarters follows
 *     Section 3.3 (Figure "CV");
 *   - for a non-orthogonal basis (overlap matrix S, Section 3.1) the
 *     generalised problem H c = E S c is reduced to C = L^{-1} H L^{-H} with
 *     the Cholesky factor S = L L^H (Golub & Van Loan, Alg. 4.2.1 and
 *     Sec. 8.7.2) before the Hermitian eigensolver;
 *   - eigenvalues: unblocked Householder reduction of the Hermitian matrix to
 *     real symmetric tridiagonal form (Golub & Van Loan, Matrix Computations,
 *     Sec. 8.3.1, Hermitian form) followed by the implicit symmetric QR
 *     iteration with Wilkinson shift (Golub & Van Loan, Alg. 8.3.2/8.3.3);
 *   - the smoothed integrated density of states is eq. (IDoS) with the
 *     nearest-point band approximation and the smoothing of
 *     eq. (MLMC_smoothing) (Section 4.3), summed with Neumaier compensation;
 *   - the per-level sums are the ingredients of eq. (MLMC) and of the
 *     estimator variance of Section 2.2.
 * Parity pins for each routine live in the test suite.
 */
#include <complex.h>
#include <float.h>
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef double complex cplx;

#define ORA_OK 0
#define ORA_ERR_ARG (-1)
#define ORA_ERR_NOT_CONVERGED (-5)
#define ORA_ERR_NOMEM (-6)

/* Lattice description as the oracle receives it (host arrays). */
typedef struct {
    int32_t lattice_id;
    int32_t n_orb;
    int32_t n_groups;
    int32_t n_hops;
    double cell_area;          /* |F|, Angstrom^2 */
    const double *orb_frac;    /* [n_orb][2] fractional positions          */
    const int32_t *orb_group;  /* [n_orb] vacancy group of each orbital    */
    const uint8_t *removable;  /* [n_groups] 1 if the group can be vacant  */
    const int32_t *hop_R;      /* [n_hops][2] cell offset of the target    */
    const int32_t *hop_from;   /* [n_hops]                                 */
    const int32_t *hop_to;     /* [n_hops]                                 */
    const double *hop_re;      /* [n_hops]                                 */
    const double *hop_im;      /* [n_hops]                                 */
    /* Non-orthogonal basis (Section 3.1, generalised problem H c = E S c):  */
    /* has_overlap = 1 adds an overlap table; S = I + its Bloch sum.         */
    int32_t has_overlap;
    int32_t n_ovl;
    const int32_t *ovl_R;      /* [n_ovl][2] */
    const int32_t *ovl_from;   /* [n_ovl]    */
    const int32_t *ovl_to;     /* [n_ovl]    */
    const double *ovl_re;      /* [n_ovl]    */
    const double *ovl_im;      /* [n_ovl]    */
} ora_lattice;

/* ------------------------------------------------------------------------ */
/* Philox4x64-10                                                             */
/* ------------------------------------------------------------------------ */

void ora_philox4x64_10(const uint64_t ctr_in[4], const uint64_t key_in[2], uint64_t out[4])
{
    const uint64_t mul0 = 0xD2E7470EE14C6C93ULL, mul1 = 0xCA5A826395121157ULL;
    const uint64_t weyl0 = 0x9E3779B97F4A7C15ULL, weyl1 = 0xBB67AE8584CAA73BULL;
    uint64_t x0 = ctr_in[0], x1 = ctr_in[1], x2 = ctr_in[2], x3 = ctr_in[3];
    uint64_t k0 = key_in[0], k1 = key_in[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += weyl0;
            k1 += weyl1;
        }
        unsigned __int128 prod0 = (unsigned __int128)mul0 * x0;
        unsigned __int128 prod1 = (unsigned __int128)mul1 * x2;
        uint64_t hi0 = (uint64_t)(prod0 >> 64), lo0 = (uint64_t)prod0;
        uint64_t hi1 = (uint64_t)(prod1 >> 64), lo1 = (uint64_t)prod1;
        uint64_t y0 = hi1 ^ x1 ^ k0;
        uint64_t y1 = lo1;
        uint64_t y2 = hi0 ^ x3 ^ k1;
        uint64_t y3 = lo0;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* ------------------------------------------------------------------------ */
/* Vacancy outcomes (Section 3.2): every removable group of every cell is     */
/* vacant independently with probability p.                                  */
/*                                                                           */
/* Group g = (i*N + j)*G + local_group of sample s uses word g mod 4 of the  */
/* Philox block with counter (s, floor(g/4), 0, 0) and key (seed, tag); the  */
/* group is vacant iff it is removable and (word >> 11) < floor(p * 2^53).   */
/* ------------------------------------------------------------------------ */

int ora_sample_vacancies(const ora_lattice *L, int32_t N, double p, uint64_t seed, uint64_t tag,
                         int64_t first_sample, int64_t n_samples, uint8_t *mask)
{
    if (N < 1 || !(p >= 0.0 && p <= 1.0) || n_samples < 0) return ORA_ERR_ARG;
    const uint64_t threshold = (uint64_t)floor(p * 9007199254740992.0); /* p * 2^53 */
    const int64_t groups = (int64_t)N * N * L->n_groups;
    const uint64_t key[2] = {seed, tag};
    for (int64_t s = 0; s < n_samples; ++s) {
        for (int64_t g = 0; g < groups; ++g) {
            uint64_t ctr[4] = {(uint64_t)(first_sample + s), (uint64_t)(g / 4), 0, 0};
            uint64_t words[4];
            ora_philox4x64_10(ctr, key, words);
            uint64_t u53 = words[g % 4] >> 11;
            int local = (int)(g % L->n_groups);
            mask[s * groups + g] = (uint8_t)(L->removable[local] && u53 < threshold);
        }
    }
    return ORA_OK;
}

/* Control-variate partition (Section 3.3): quarter q = 2*qi + qj keeps the   */
/* cells with i in [qi*N/2, (qi+1)*N/2) and j in [qj*N/2, (qj+1)*N/2) and    */
/* their outcomes; the quarter is then treated as an N/2 supercell.          */
int ora_partition_masks(int32_t N, int32_t G, const uint8_t *mask, uint8_t *quarters)
{
    if (N < 2 || N % 2 != 0) return ORA_ERR_ARG;
    const int h = N / 2;
    for (int q = 0; q < 4; ++q) {
        const int qi = q / 2, qj = q % 2;
        for (int i = 0; i < h; ++i)
            for (int j = 0; j < h; ++j)
                for (int g = 0; g < G; ++g) {
                    int src_cell = (qi * h + i) * N + (qj * h + j);
                    quarters[((int64_t)q * h * h + (int64_t)i * h + j) * G + g] = mask[(int64_t)src_cell * G + g];
                }
    }
    return ORA_OK;
}

/* Number of k-points of a grid: K x K for the Monkhorst-Pack (0) and
 * Gamma-centred (1) grids, 3 K^2 for the three-rhombus lattice (2). */
int ora_kgrid_points(int32_t kind, int32_t K)
{
    if (K < 1) return -1;
    if (kind == 0 || kind == 1) return K * K;
    if (kind == 2) return 3 * K * K;
    return -1;
}

static int imod(int a, int m)
{
    int r = a % m;
    return r < 0 ? r + m : r;
}

/* Brillouin-zone grids in reduced coordinates of the supercell reciprocal
 * lattice, with weights.
 *   kind 0, 1: a uniform K x K grid (Monkhorst-Pack or Gamma-centred), equal
 *              weights (the reading of Sections 4.2-4.3 used by the main
 *              workloads).
 *   kind 2:    the three-rhombus lattice of Section 4.2.  The hexagonal zone
 *              is the union of three rhombi with the common corner Gamma,
 *              each spanned by two zone corners 120 degrees apart; in reduced
 *              coordinates the corners used are c1 = (2/3, 1/3),
 *              c3 = (-1/3, 1/3) and c5 = (-1/3, -2/3), and the rhombi are
 *              (c1, c3), (c3, c5), (c5, c1).  Each rhombus is cut into K x K
 *              equal rhombi and the k-points are their corners,
 *              (m/K) u + (n/K) v for 0 <= m, n <= K.  Corners shared by two
 *              rhombi, and corners that differ by a reciprocal lattice vector
 *              (the same point of the periodic band structure), are kept once.
 *              The kept points form a uniform lattice, so every one has the
 *              same nearest-point cell (Section 4.3): weight 1 / (number of
 *              points).  Points are listed in increasing (3K kappa1, 3K kappa2).
 */
int ora_kgrid(int32_t kind, int32_t K, double *kred, double *kweight)
{
    const int nk = ora_kgrid_points(kind, K);
    if (nk < 0) return ORA_ERR_ARG;
    if (kind == 0 || kind == 1) {
        for (int r1 = 0; r1 < K; ++r1)
            for (int r2 = 0; r2 < K; ++r2) {
                int idx = r1 * K + r2;
                if (kind == 0) {
                    kred[2 * idx + 0] = (2.0 * r1 - K + 1.0) / (2.0 * K);
                    kred[2 * idx + 1] = (2.0 * r2 - K + 1.0) / (2.0 * K);
                } else {
                    kred[2 * idx + 0] = (double)r1 / K;
                    kred[2 * idx + 1] = (double)r2 / K;
                }
                kweight[idx] = 1.0 / ((double)K * K);
            }
        return ORA_OK;
    }
    /* zone corners times 3 (integer numerators over 3) */
    const int corner[3][2] = {{2, 1}, {-1, 1}, {-1, -2}};
    const int M3 = 3 * K;
    unsigned char *seen = (unsigned char *)calloc((size_t)M3 * M3, 1);
    if (!seen) return ORA_ERR_NOMEM;
    for (int r = 0; r < 3; ++r) {
        const int *u = corner[r], *v = corner[(r + 1) % 3];
        for (int m = 0; m <= K; ++m)
            for (int n = 0; n <= K; ++n) {
                /* (m/K) u/3 + (n/K) v/3 = (m u + n v) / (3K) */
                const int a = imod(m * u[0] + n * v[0], M3), b = imod(m * u[1] + n * v[1], M3);
                seen[(size_t)a * M3 + b] = 1;
            }
    }
    int count = 0;
    for (int a = 0; a < M3; ++a)
        for (int b = 0; b < M3; ++b)
            if (seen[(size_t)a * M3 + b]) {
                if (count < nk) {
                    kred[2 * count + 0] = (double)a / (double)M3;
                    kred[2 * count + 1] = (double)b / (double)M3;
                }
                ++count;
            }
    free(seen);
    if (count != nk) return ORA_ERR_ARG;
    for (int i = 0; i < nk; ++i) kweight[i] = 1.0 / (double)nk;
    return ORA_OK;
}

static int wrap(int a, int N)
{
    int r = a % N;
    return r < 0 ? r + N : r;
}

/* Bloch Hamiltonian H(k) of one N x N supercell outcome (Section 3.1,        */
/* eq. (tightbinding), orthogonal form; vacancies of Section 3.2).            */
/*                                                                           */
/* Orbital (cell (i,j), m) has index (i*N + j)*n_orb + m; present orbitals   */
/* keep that order and are renumbered 0..n-1.  A hopping row (R, from, to,   */
/* h) adds h*exp(2*pi*i*(k1*d1 + k2*d2)/N) to H[a, b] and its conjugate to    */
/* H[b, a] for every present pair a = (c, from), b = (c + R mod N, to), where */
/* d = R + frac(to) - frac(from) is the unwrapped displacement in units of    */
/* a1, a2 (the atom-to-atom vector of eq. (tightbinding)).  On-site rows     */
/* (R = 0, from == to) are added once.  H is written column-major with       */
/* leading dimension ld; *n_out receives n.                                   */
/* Bloch sum of one hopping table over the present orbitals of an outcome   */
/* (Section 3.1, eq. (tightbinding); vacant rows and columns removed,         */
/* Section 3.2), with the unit matrix added first when unit_diag is set.      */
static int assemble_table(const ora_lattice *L, int32_t N, const uint8_t *mask, double k1, double k2, int n_tab,
                          const int32_t *tR, const int32_t *tfrom, const int32_t *tto, const double *tre,
                          const double *tim, int unit_diag, cplx *H, int64_t ld, int32_t *n_out)
{
    const int n_orb = L->n_orb, G = L->n_groups;
    const int total = N * N * n_orb;
    int *index = (int *)malloc(sizeof(int) * (size_t)total);
    if (!index) return ORA_ERR_NOMEM;
    int n = 0;
    for (int c = 0; c < N * N; ++c)
        for (int m = 0; m < n_orb; ++m)
            index[c * n_orb + m] = mask[c * G + L->orb_group[m]] ? -1 : n++;
    if (ld < n) {
        free(index);
        return ORA_ERR_ARG;
    }
    for (int64_t col = 0; col < n; ++col)
        for (int64_t row = 0; row < n; ++row) H[row + col * ld] = (unit_diag && row == col) ? 1.0 : 0.0;
    for (int h = 0; h < n_tab; ++h) {
        const int R1 = tR[2 * h], R2 = tR[2 * h + 1];
        const int from = tfrom[h], to = tto[h];
        const cplx amp = tre[h] + I * tim[h];
        const double d1 = R1 + L->orb_frac[2 * to] - L->orb_frac[2 * from];
        const double d2 = R2 + L->orb_frac[2 * to + 1] - L->orb_frac[2 * from + 1];
        double x = (k1 * d1 + k2 * d2) / N;
        x -= floor(x);
        const cplx z = amp * (cos(2.0 * M_PI * x) + I * sin(2.0 * M_PI * x));
        const int onsite = (R1 == 0 && R2 == 0 && from == to);
        for (int i = 0; i < N; ++i)
            for (int j = 0; j < N; ++j) {
                const int a = index[(i * N + j) * n_orb + from];
                const int b = index[(wrap(i + R1, N) * N + wrap(j + R2, N)) * n_orb + to];
                if (a < 0 || b < 0) continue;
                if (onsite) {
                    H[a + (int64_t)a * ld] += amp;
                } else {
                    H[a + (int64_t)b * ld] += z;
                    H[b + (int64_t)a * ld] += conj(z);
                }
            }
    }
    free(index);
    *n_out = n;
    return ORA_OK;
}

int ora_build_hamiltonian(const ora_lattice *L, int32_t N, const uint8_t *mask, double k1, double k2,
                          cplx *H, int64_t ld, int32_t *n_out)
{
    return assemble_table(L, N, mask, k1, k2, L->n_hops, L->hop_R, L->hop_from, L->hop_to, L->hop_re, L->hop_im, 0,
                          H, ld, n_out);
}

/* Overlap matrix S(k) of a non-orthogonal basis: the unit matrix plus the  */
/* Bloch sum of the overlap table (same phase convention as H(k)).          */
int ora_build_overlap(const ora_lattice *L, int32_t N, const uint8_t *mask, double k1, double k2,
                      cplx *S, int64_t ld, int32_t *n_out)
{
    if (!L->has_overlap) return ORA_ERR_ARG;
    return assemble_table(L, N, mask, k1, k2, L->n_ovl, L->ovl_R, L->ovl_from, L->ovl_to, L->ovl_re, L->ovl_im, 1,
                          S, ld, n_out);
}

/* Cholesky factorisation S = L L^H of a Hermitian positive definite matrix  */
/* (Golub & Van Loan, Alg. 4.2.1, column by column); L overwrites the lower  */
/* triangle.  Returns ORA_ERR_ARG when a pivot is not positive.              */
int ora_cholesky(int32_t n, cplx *S, int64_t ld)
{
    for (int j = 0; j < n; ++j) {
        double djj = creal(S[j + (int64_t)j * ld]);
        for (int k = 0; k < j; ++k) djj -= creal(S[j + (int64_t)k * ld] * conj(S[j + (int64_t)k * ld]));
        if (!(djj > 0.0)) return ORA_ERR_ARG;
        const double ljj = sqrt(djj);
        S[j + (int64_t)j * ld] = ljj;
        for (int i = j + 1; i < n; ++i) {
            cplx sij = S[i + (int64_t)j * ld];
            for (int k = 0; k < j; ++k) sij -= S[i + (int64_t)k * ld] * conj(S[j + (int64_t)k * ld]);
            S[i + (int64_t)j * ld] = sij / ljj;
        }
    }
    return ORA_OK;
}

int ora_eigvalsh(int32_t n, cplx *A, int64_t ld, double *w);

/* Eigenvalues of the Hermitian-definite pencil (H, S): with S = L L^H the  */
/* pencil has the eigenvalues of the Hermitian C = L^{-1} H L^{-H}.  Y =     */
/* L^{-1} H by forward substitution, then C = L^{-1} Y^H (= Y L^{-H}, as C   */
/* is Hermitian), then the Hermitian eigensolver.  H and S are overwritten.  */
int ora_eigvalsh_generalized(int32_t n, cplx *H, cplx *S, int64_t ld, double *w)
{
    if (n < 0) return ORA_ERR_ARG;
    if (n == 0) return ORA_OK;
    int st = ora_cholesky(n, S, ld);
    if (st != ORA_OK) return st;
    cplx *Y = (cplx *)malloc(sizeof(cplx) * (size_t)n * (size_t)n);
    if (!Y) return ORA_ERR_NOMEM;
    for (int c = 0; c < n; ++c)            /* Y[:, c] = L^{-1} H[:, c] */
        for (int i = 0; i < n; ++i) {
            cplx v = H[i + (int64_t)c * ld];
            for (int k = 0; k < i; ++k) v -= S[i + (int64_t)k * ld] * Y[k + (size_t)c * n];
            Y[i + (size_t)c * n] = v / creal(S[i + (int64_t)i * ld]);
        }
    for (int c = 0; c < n; ++c)            /* C[:, c] = L^{-1} (Y^H)[:, c] */
        for (int i = 0; i < n; ++i) {
            cplx v = conj(Y[c + (size_t)i * n]);
            for (int k = 0; k < i; ++k) v -= S[i + (int64_t)k * ld] * H[k + (int64_t)c * ld];
            H[i + (int64_t)c * ld] = v / creal(S[i + (int64_t)i * ld]);
        }
    free(Y);
    for (int c = 0; c < n; ++c)            /* the Hermitian part of the computed C */
        for (int i = c; i < n; ++i) {
            const cplx m = 0.5 * (H[i + (int64_t)c * ld] + conj(H[c + (int64_t)i * ld]));
            H[i + (int64_t)c * ld] = m;
            H[c + (int64_t)i * ld] = conj(m);
        }
    return ora_eigvalsh(n, H, ld, w);
}

/* Householder reduction of a Hermitian matrix (full storage, column-major)  */
/* to real symmetric tridiagonal form T = Q^H A Q with diagonal d[n] and     */
/* non-negative sub-diagonal e[n-1] (the moduli of the reduced complex       */
/* sub-diagonal, which a diagonal unitary scaling makes real).  A is          */
/* overwritten.                                                               */
int ora_tridiagonalize(int32_t n, cplx *A, int64_t ld, double *d, double *e)
{
    if (n < 0) return ORA_ERR_ARG;
    if (n == 0) return ORA_OK;
    cplx *v = (cplx *)malloc(sizeof(cplx) * (size_t)n);
    cplx *p = (cplx *)malloc(sizeof(cplx) * (size_t)n);
    cplx *w = (cplx *)malloc(sizeof(cplx) * (size_t)n);
    if (!v || !p || !w) {
        free(v); free(p); free(w);
        return ORA_ERR_NOMEM;
    }
    for (int j = 0; j + 2 < n; ++j) {
        const int m = n - j - 1;             /* length of the column below the diagonal */
        cplx *x = &A[(j + 1) + (int64_t)j * ld];
        double nrm2 = 0.0;
        for (int i = 0; i < m; ++i) nrm2 += creal(x[i]) * creal(x[i]) + cimag(x[i]) * cimag(x[i]);
        const double xnorm = sqrt(nrm2);
        e[j] = xnorm;
        if (xnorm == 0.0) continue;          /* column already reduced */
        const double ax0 = cabs(x[0]);
        const cplx phase = ax0 > 0.0 ? x[0] / ax0 : 1.0;
        const cplx alpha = -phase * xnorm;   /* reflected column is alpha * e_1 */
        for (int i = 0; i < m; ++i) v[i] = x[i];
        v[0] -= alpha;
        double vnorm2 = 0.0;
        for (int i = 0; i < m; ++i) vnorm2 += creal(v[i]) * creal(v[i]) + cimag(v[i]) * cimag(v[i]);
        const double tau = 2.0 / vnorm2;     /* reflector I - tau v v^H */
        cplx *A22 = &A[(j + 1) + (int64_t)(j + 1) * ld];
        for (int r = 0; r < m; ++r) {
            cplx s = 0.0;
            for (int c = 0; c < m; ++c) s += A22[r + (int64_t)c * ld] * v[c];
            p[r] = tau * s;
        }
        cplx vhp = 0.0;
        for (int i = 0; i < m; ++i) vhp += conj(v[i]) * p[i];
        const double K = 0.5 * tau * creal(vhp);
        for (int i = 0; i < m; ++i) w[i] = p[i] - K * v[i];
        for (int c = 0; c < m; ++c)
            for (int r = 0; r < m; ++r)
                A22[r + (int64_t)c * ld] -= v[r] * conj(w[c]) + w[r] * conj(v[c]);
        x[0] = alpha;
        for (int i = 1; i < m; ++i) x[i] = 0.0;
        for (int i = 0; i < m; ++i) A[j + (int64_t)(j + 1 + i) * ld] = conj(x[i]);
    }
    for (int j = 0; j < n; ++j) d[j] = creal(A[j + (int64_t)j * ld]);
    if (n >= 2) e[n - 2] = cabs(A[(n - 1) + (int64_t)(n - 2) * ld]);
    free(v); free(p); free(w);
    return ORA_OK;
}

/* One implicit symmetric QR step with Wilkinson shift on the unreduced       */
/* block a[lo..hi], b[lo..hi-1] (Golub & Van Loan, Alg. 8.3.2).  Rotation     */
/* k acts on indices (k, k+1) as (u, v) -> (c u + s v, -s u + c v).          */
static void qr_step(double *a, double *b, int lo, int hi)
{
    const double half_gap = 0.5 * (a[hi - 1] - a[hi]);
    const double bt = b[hi - 1];
    const double denom = half_gap + copysign(hypot(half_gap, bt), half_gap);
    const double mu = a[hi] - bt * bt / denom;
    double x = a[lo] - mu, z = b[lo];
    for (int k = lo; k < hi; ++k) {
        const double r = hypot(x, z);
        double c = 1.0, s = 0.0;
        if (r > 0.0) {
            c = x / r;
            s = z / r;
        }
        if (k > lo) b[k - 1] = r;
        const double ak = a[k], ak1 = a[k + 1], bk = b[k];
        a[k] = c * c * ak + 2.0 * c * s * bk + s * s * ak1;
        a[k + 1] = s * s * ak - 2.0 * c * s * bk + c * c * ak1;
        b[k] = c * s * (ak1 - ak) + (c * c - s * s) * bk;
        if (k + 1 < hi) {
            const double bk1 = b[k + 1];
            z = s * bk1;           /* bulge at (k+2, k) */
            b[k + 1] = c * bk1;
            x = b[k];
        }
    }
}

static int cmp_double(const void *pa, const void *pb)
{
    const double a = *(const double *)pa, b = *(const double *)pb;
    return (a > b) - (a < b);
}

static int negligible(double b, double a0, double a1)
{
    return fabs(b) <= DBL_EPSILON * (fabs(a0) + fabs(a1)) || fabs(b) < DBL_MIN;
}

/* Eigenvalues of the symmetric tridiagonal (d, e) by the symmetric QR        */
/* algorithm with deflation (Golub & Van Loan, Alg. 8.3.3); ascending.        */
int ora_tridiag_eigvals(int32_t n, const double *d, const double *e, double *w)
{
    if (n < 0) return ORA_ERR_ARG;
    if (n == 0) return ORA_OK;
    double *a = (double *)malloc(sizeof(double) * (size_t)n);
    double *b = (double *)malloc(sizeof(double) * (size_t)(n > 1 ? n - 1 : 1));
    if (!a || !b) {
        free(a); free(b);
        return ORA_ERR_NOMEM;
    }
    memcpy(a, d, sizeof(double) * (size_t)n);
    if (n > 1) memcpy(b, e, sizeof(double) * (size_t)(n - 1));
    int hi = n - 1;
    long iterations = 0;
    const long max_iterations = 30L * n;
    int status = ORA_OK;
    while (hi > 0) {
        if (negligible(b[hi - 1], a[hi - 1], a[hi])) {
            b[hi - 1] = 0.0;
            --hi;
            continue;
        }
        int lo = hi - 1;
        while (lo > 0 && !negligible(b[lo - 1], a[lo - 1], a[lo])) --lo;
        if (lo > 0) b[lo - 1] = 0.0;
        if (++iterations > max_iterations) {
            status = ORA_ERR_NOT_CONVERGED;
            break;
        }
        qr_step(a, b, lo, hi);
    }
    qsort(a, (size_t)n, sizeof(double), cmp_double);
    memcpy(w, a, sizeof(double) * (size_t)n);
    free(a); free(b);
    return status;
}

/* All eigenvalues (ascending) of a Hermitian matrix; A is overwritten.      */
int ora_eigvalsh(int32_t n, cplx *A, int64_t ld, double *w)
{
    if (n == 0) return ORA_OK;
    double *d = (double *)malloc(sizeof(double) * (size_t)n);
    double *e = (double *)malloc(sizeof(double) * (size_t)n);
    if (!d || !e) {
        free(d); free(e);
        return ORA_ERR_NOMEM;
    }
    int st = ora_tridiagonalize(n, A, ld, d, e);
    if (st == ORA_OK) st = ora_tridiag_eigvals(n, d, e, w);
    free(d); free(e);
    return st;
}

/* Eigenvalues and eigenvectors of a Hermitian matrix (eigenstates of H(k),  */
/* the input of the conductivity the paper names as the next quantity of     */
/* interest).  Textbook path (Golub & Van Loan Sections 8.3.1 and 8.3.5):    */
/* Householder reduction A = Q T_c Q^H keeping the reflectors; the complex   */
/* sub-diagonal alpha_j of T_c made real by D = diag(delta), delta_0 = 1,    */
/* delta_{j+1} = delta_j alpha_j / |alpha_j|, so T_c = D T D^H with T real;  */
/* the symmetric QR algorithm on T accumulating its rotations in Z (T = Z    */
/* diag(w) Z^T); then V = Q D Z.  w ascending, V[:, i] (column-major, ldv)   */
/* the unit eigenvector of w[i].  A is overwritten.                          */
int ora_eigh(int32_t n, cplx *A, int64_t ld, double *w, cplx *V, int64_t ldv)
{
    if (n < 0 || ld < n || ldv < n) return ORA_ERR_ARG;
    if (n == 0) return ORA_OK;
    cplx *R = (cplx *)calloc((size_t)n * (size_t)n, sizeof(cplx));   /* reflector j in column j */
    double *tau = (double *)calloc((size_t)n, sizeof(double));
    cplx *delta = (cplx *)malloc(sizeof(cplx) * (size_t)n);
    cplx *p = (cplx *)malloc(sizeof(cplx) * (size_t)n);
    cplx *q = (cplx *)malloc(sizeof(cplx) * (size_t)n);
    double *a = (double *)malloc(sizeof(double) * (size_t)n);
    double *b = (double *)calloc((size_t)n, sizeof(double));
    double *Z = (double *)calloc((size_t)n * (size_t)n, sizeof(double));
    int *order = (int *)malloc(sizeof(int) * (size_t)n);
    int status = ORA_OK;
    if (!R || !tau || !delta || !p || !q || !a || !b || !Z || !order) {
        status = ORA_ERR_NOMEM;
        goto done;
    }
    /* Householder reduction, the reflectors kept (as in ora_tridiagonalize) */
    for (int j = 0; j + 2 < n; ++j) {
        const int m = n - j - 1;
        cplx *x = &A[(j + 1) + (int64_t)j * ld];
        double nrm2 = 0.0;
        for (int i = 0; i < m; ++i) nrm2 += creal(x[i]) * creal(x[i]) + cimag(x[i]) * cimag(x[i]);
        const double xnorm = sqrt(nrm2);
        if (xnorm == 0.0) continue;
        const double ax0 = cabs(x[0]);
        const cplx phase = ax0 > 0.0 ? x[0] / ax0 : 1.0;
        const cplx alpha = -phase * xnorm;
        cplx *v = &R[(int64_t)j * n];
        for (int i = 0; i < m; ++i) v[i] = x[i];
        v[0] -= alpha;
        double vnorm2 = 0.0;
        for (int i = 0; i < m; ++i) vnorm2 += creal(v[i]) * creal(v[i]) + cimag(v[i]) * cimag(v[i]);
        tau[j] = 2.0 / vnorm2;
        cplx *A22 = &A[(j + 1) + (int64_t)(j + 1) * ld];
        for (int r = 0; r < m; ++r) {
            cplx s = 0.0;
            for (int c = 0; c < m; ++c) s += A22[r + (int64_t)c * ld] * v[c];
            p[r] = tau[j] * s;
        }
        cplx vhp = 0.0;
        for (int i = 0; i < m; ++i) vhp += conj(v[i]) * p[i];
        const double K = 0.5 * tau[j] * creal(vhp);
        for (int i = 0; i < m; ++i) q[i] = p[i] - K * v[i];
        for (int c = 0; c < m; ++c)
            for (int r = 0; r < m; ++r)
                A22[r + (int64_t)c * ld] -= v[r] * conj(q[c]) + q[r] * conj(v[c]);
        x[0] = alpha;
        for (int i = 1; i < m; ++i) x[i] = 0.0;
    }
    /* real tridiagonal T = D^H T_c D */
    delta[0] = 1.0;
    for (int j = 0; j < n; ++j) a[j] = creal(A[j + (int64_t)j * ld]);
    for (int j = 0; j + 1 < n; ++j) {
        const cplx al = A[(j + 1) + (int64_t)j * ld];
        const double m = cabs(al);
        b[j] = m;
        delta[j + 1] = m > 0.0 ? delta[j] * (al / m) : delta[j];
    }
    /* symmetric QR on (a, b) with the rotations accumulated in Z */
    for (int i = 0; i < n; ++i) Z[i + (int64_t)i * n] = 1.0;
    {
        int hi = n - 1;
        long iterations = 0;
        const long max_iterations = 30L * n;
        while (hi > 0) {
            if (negligible(b[hi - 1], a[hi - 1], a[hi])) {
                b[hi - 1] = 0.0;
                --hi;
                continue;
            }
            int lo = hi - 1;
            while (lo > 0 && !negligible(b[lo - 1], a[lo - 1], a[lo])) --lo;
            if (lo > 0) b[lo - 1] = 0.0;
            if (++iterations > max_iterations) {
                status = ORA_ERR_NOT_CONVERGED;
                goto done;
            }
            /* the step of qr_step, each rotation also applied to Z's columns k, k+1 */
            const double half_gap = 0.5 * (a[hi - 1] - a[hi]);
            const double bt = b[hi - 1];
            const double denom = half_gap + copysign(hypot(half_gap, bt), half_gap);
            const double mu = a[hi] - bt * bt / denom;
            double xx = a[lo] - mu, zz = b[lo];
            for (int k = lo; k < hi; ++k) {
                const double r = hypot(xx, zz);
                double c = 1.0, s = 0.0;
                if (r > 0.0) {
                    c = xx / r;
                    s = zz / r;
                }
                if (k > lo) b[k - 1] = r;
                const double ak = a[k], ak1 = a[k + 1], bk = b[k];
                a[k] = c * c * ak + 2.0 * c * s * bk + s * s * ak1;
                a[k + 1] = s * s * ak - 2.0 * c * s * bk + c * c * ak1;
                b[k] = c * s * (ak1 - ak) + (c * c - s * s) * bk;
                if (k + 1 < hi) {
                    const double bk1 = b[k + 1];
                    zz = s * bk1;
                    b[k + 1] = c * bk1;
                    xx = b[k];
                }
                for (int i = 0; i < n; ++i) {
                    const double zk = Z[i + (int64_t)k * n], zk1 = Z[i + (int64_t)(k + 1) * n];
                    Z[i + (int64_t)k * n] = c * zk + s * zk1;
                    Z[i + (int64_t)(k + 1) * n] = -s * zk + c * zk1;
                }
            }
        }
    }
    /* ascending order */
    for (int i = 0; i < n; ++i) order[i] = i;
    for (int i = 1; i < n; ++i) {  /* insertion sort by eigenvalue (stable) */
        const int o = order[i];
        int k = i - 1;
        while (k >= 0 && a[order[k]] > a[o]) {
            order[k + 1] = order[k];
            --k;
        }
        order[k + 1] = o;
    }
    /* V = Q D Z: column i starts as D z, then the reflectors in reverse order */
    for (int i = 0; i < n; ++i) {
        const int o = order[i];
        w[i] = a[o];
        cplx *vi = &V[(int64_t)i * ldv];
        for (int r = 0; r < n; ++r) vi[r] = delta[r] * Z[r + (int64_t)o * n];
        for (int j = n - 3; j >= 0; --j) {
            if (tau[j] == 0.0) continue;
            const int m = n - j - 1;
            const cplx *v = &R[(int64_t)j * n];
            cplx s = 0.0;
            for (int r = 0; r < m; ++r) s += conj(v[r]) * vi[j + 1 + r];
            s *= tau[j];
            for (int r = 0; r < m; ++r) vi[j + 1 + r] -= v[r] * s;
        }
    }
done:
    free(R); free(tau); free(delta); free(p); free(q); free(a); free(b); free(Z); free(order);
    return status;
}

/* Smoothed step of eq. (MLMC_smoothing).  smoother 0: Gaussian CDF           */
/* erfc(x/sqrt 2)/2; smoother 1: the cubic 1/2 - 9x/8 + 5x^3/8 on [-1, 1]     */
/* (1 below, 0 above), the polynomial of least degree meeting the endpoint   */
/* and q = 0, 1 moment conditions.                                            */
double ora_smooth_step(int32_t smoother, double x)
{
    if (smoother == 0) return 0.5 * erfc(x / M_SQRT2);
    if (x <= -1.0) return 1.0;
    if (x >= 1.0) return 0.0;
    return 0.5 - 1.125 * x + 0.625 * x * x * x;
}

/* Smoothed IDoS of one outcome (eq. (IDoS) with the nearest-point band      */
/* approximation and eq. (MLMC_smoothing)):                                   */
/*   I(eps_j) = 1/area * sum_k kweight[k] * sum_{i < n[k]} g((w[k][i] - eps_j)/delta)  */
/* with area = N^2 |F|.  The double sum is Neumaier-compensated.              */
int ora_idos(const double *w, int64_t ldw, const int32_t *n, int32_t n_k, const double *kweight,
             double area, const double *eps, int32_t n_eps, double delta, int32_t smoother, double *out)
{
    if (!(delta > 0.0) || !(area > 0.0) || n_eps < 0 || n_k < 0) return ORA_ERR_ARG;
    for (int j = 0; j < n_eps; ++j) {
        double sum = 0.0, comp = 0.0;
        for (int k = 0; k < n_k; ++k)
            for (int i = 0; i < n[k]; ++i) {
                const double term = kweight[k] * ora_smooth_step(smoother, (w[k * ldw + i] - eps[j]) / delta);
                const double t = sum + term;
                if (fabs(sum) >= fabs(term))
                    comp += (sum - t) + term;
                else
                    comp += (term - t) + sum;
                sum = t;
            }
        out[j] = (sum + comp) / area;
    }
    return ORA_OK;
}

/* ------------------------------------------------------------------------ */
/* One sample of a level (Sections 2.2 and 3.3).                              */
/*   Q_f  : IDoS of the N x N outcome on the K_f x K_f grid;                  */
/*   Q_q  : IDoS of quarter q (an N/2 supercell) on the K_c x K_c grid.       */
/* ------------------------------------------------------------------------ */

static int outcome_idos(const ora_lattice *L, int32_t N, const uint8_t *mask, int32_t kind, int32_t K,
                        const double *eps, int32_t n_eps, double delta, int32_t smoother, double *out)
{
    const int nk = ora_kgrid_points(kind, K);
    if (nk < 0) return ORA_ERR_ARG;
    const int nmax = N * N * L->n_orb;
    double *kred = (double *)malloc(sizeof(double) * 2 * (size_t)nk);
    double *kw = (double *)malloc(sizeof(double) * (size_t)nk);
    double *w = (double *)malloc(sizeof(double) * (size_t)nk * (size_t)(nmax > 0 ? nmax : 1));
    int32_t *nn = (int32_t *)malloc(sizeof(int32_t) * (size_t)nk);
    cplx *H = (cplx *)malloc(sizeof(cplx) * (size_t)(nmax > 0 ? nmax : 1) * (size_t)(nmax > 0 ? nmax : 1));
    cplx *S = L->has_overlap
                  ? (cplx *)malloc(sizeof(cplx) * (size_t)(nmax > 0 ? nmax : 1) * (size_t)(nmax > 0 ? nmax : 1))
                  : NULL;
    int st = ORA_OK;
    if (!kred || !kw || !w || !nn || !H || (L->has_overlap && !S)) st = ORA_ERR_NOMEM;
    if (st == ORA_OK) st = ora_kgrid(kind, K, kred, kw);
    for (int k = 0; st == ORA_OK && k < nk; ++k) {
        st = ora_build_hamiltonian(L, N, mask, kred[2 * k], kred[2 * k + 1], H, nmax, &nn[k]);
        if (st == ORA_OK && L->has_overlap) {
            int32_t ns = 0;
            st = ora_build_overlap(L, N, mask, kred[2 * k], kred[2 * k + 1], S, nmax, &ns);
            if (st == ORA_OK) st = ora_eigvalsh_generalized(nn[k], H, S, nmax, &w[(size_t)k * nmax]);
        } else if (st == ORA_OK) {
            st = ora_eigvalsh(nn[k], H, nmax, &w[(size_t)k * nmax]);
        }
    }
    if (st == ORA_OK)
        st = ora_idos(w, nmax, nn, nk, kw, (double)N * N * L->cell_area, eps, n_eps, delta, smoother, out);
    free(kred); free(kw); free(w); free(nn); free(H); free(S);
    return st;
}

int ora_sample_qoi(const ora_lattice *L, int32_t N, const uint8_t *mask, int32_t coupled, int32_t K_fine,
                   int32_t K_coarse, int32_t kind, const double *eps, int32_t n_eps, double delta,
                   int32_t smoother, double *Q_fine, double *Q_quarters)
{
    int st = outcome_idos(L, N, mask, kind, K_fine, eps, n_eps, delta, smoother, Q_fine);
    if (st != ORA_OK || !coupled) return st;
    const int h = N / 2, G = L->n_groups;
    uint8_t *quarters = (uint8_t *)malloc((size_t)4 * h * h * G);
    if (!quarters) return ORA_ERR_NOMEM;
    st = ora_partition_masks(N, G, mask, quarters);
    for (int q = 0; st == ORA_OK && q < 4; ++q)
        st = outcome_idos(L, h, quarters + (size_t)q * h * h * G, kind, K_coarse, eps, n_eps, delta, smoother,
                          Q_quarters + (size_t)q * n_eps);
    free(quarters);
    return st;
}

typedef struct {
    const ora_lattice *L;
    int32_t N, coupled, K_fine, K_coarse, kind, n_eps, smoother;
    double delta;
    const double *eps;
    const uint8_t *masks;
    int64_t M, groups;
    int tid, n_threads;
    double *Q_fine;      /* [M][n_eps] */
    double *Q_quarters;  /* [M][4][n_eps] or NULL */
    int status;
} level_job;

static void *level_worker(void *arg)
{
    level_job *job = (level_job *)arg;
    for (int64_t s = job->tid; s < job->M; s += job->n_threads) {
        int st = ora_sample_qoi(job->L, job->N, job->masks + s * job->groups, job->coupled, job->K_fine,
                                job->K_coarse, job->kind, job->eps, job->n_eps, job->delta, job->smoother,
                                job->Q_fine + s * job->n_eps,
                                job->coupled ? job->Q_quarters + s * 4 * job->n_eps : NULL);
        if (st != ORA_OK) {
            job->status = st;
            break;
        }
    }
    return NULL;
}

/* Per-level sums over M samples with global indices first..first+M-1:       */
/*   Y = Q_f (uncoupled) or Y = Q_f - (1/4) sum_q Q_q (coupled, eq. (MLMC));  */
/*   stats[0] += sum Y, stats[1] += sum Y^2, stats[2] += sum Q_f,             */
/*   stats[3] += sum Q_f^2, each of length n_eps, accumulated in sample order.*/
/* The vacancy stream tag is (lattice_id << 32) | N.  Samples are spread over */
/* n_threads POSIX threads (one sample per thread at a time).  Optional       */
/* Y_out / Qf_out ([M][n_eps]) receive the per-sample values.                 */
int ora_level_estimate(const ora_lattice *L, int32_t N, int32_t coupled, double p, int32_t K_fine, int32_t K_coarse,
                       int32_t kind, uint64_t seed, int64_t first_sample, int64_t M, const double *eps,
                       int32_t n_eps, double delta, int32_t smoother, int32_t n_threads, double *stats,
                       double *Y_out, double *Qf_out)
{
    if (N < 1 || M < 0 || n_eps < 1 || !(delta > 0.0) || K_fine < 1) return ORA_ERR_ARG;
    if (coupled && (N % 2 != 0 || K_coarse < 1)) return ORA_ERR_ARG;
    if (n_threads < 1) n_threads = 1;
    const int64_t groups = (int64_t)N * N * L->n_groups;
    const uint64_t tag = ((uint64_t)(uint32_t)L->lattice_id << 32) | (uint64_t)(uint32_t)N;
    uint8_t *masks = (uint8_t *)malloc((size_t)(M > 0 ? M : 1) * (size_t)groups);
    double *Qf = (double *)malloc(sizeof(double) * (size_t)(M > 0 ? M : 1) * n_eps);
    double *Qq = coupled ? (double *)malloc(sizeof(double) * (size_t)(M > 0 ? M : 1) * 4 * n_eps) : NULL;
    int st = ORA_OK;
    if (!masks || !Qf || (coupled && !Qq)) st = ORA_ERR_NOMEM;
    if (st == ORA_OK) st = ora_sample_vacancies(L, N, p, seed, tag, first_sample, M, masks);
    if (st == ORA_OK) {
        level_job *jobs = (level_job *)calloc((size_t)n_threads, sizeof(level_job));
        pthread_t *th = (pthread_t *)calloc((size_t)n_threads, sizeof(pthread_t));
        if (!jobs || !th) st = ORA_ERR_NOMEM;
        /* Thread t takes samples t, t + n_threads, ... */
        int started = 0;
        for (int t = 0; st == ORA_OK && t < n_threads; ++t) {
            level_job j = {L, N, coupled, K_fine, K_coarse, kind, n_eps, smoother, delta, eps, masks,
                           M, groups, t, n_threads, Qf, Qq, ORA_OK};
            jobs[t] = j;
        }
        for (int t = 0; st == ORA_OK && t < n_threads; ++t) {
            if (pthread_create(&th[t], NULL, level_worker, &jobs[t]) != 0) break;
            ++started;
        }
        if (st == ORA_OK && started < n_threads) {
            /* Not every thread started: join those that did, then run every
             * sample again on this thread alone (the results do not depend
             * on the split). */
            for (int t = 0; t < started; ++t) pthread_join(th[t], NULL);
            started = 0;
            level_job j = {L, N, coupled, K_fine, K_coarse, kind, n_eps, smoother, delta, eps, masks,
                           M, groups, 0, 1, Qf, Qq, ORA_OK};
            jobs[0] = j;
            level_worker(&jobs[0]);
            st = jobs[0].status;
        } else {
            /* Join every started thread before reading any status or freeing
             * the buffers they use. */
            for (int t = 0; t < started; ++t) pthread_join(th[t], NULL);
            for (int t = 0; st == ORA_OK && t < started; ++t)
                if (jobs[t].status != ORA_OK) st = jobs[t].status;
        }
        free(jobs); free(th);
    }
    if (st == ORA_OK) {
        for (int64_t s = 0; s < M; ++s)
            for (int j = 0; j < n_eps; ++j) {
                const double qf = Qf[s * n_eps + j];
                double y = qf;
                if (coupled) {
                    const double *q = Qq + s * 4 * n_eps;
                    y = qf - 0.25 * (q[j] + q[n_eps + j] + q[2 * n_eps + j] + q[3 * n_eps + j]);
                }
                stats[j] += y;
                stats[n_eps + j] += y * y;
                stats[2 * n_eps + j] += qf;
                stats[3 * n_eps + j] += qf * qf;
                if (Y_out) Y_out[s * n_eps + j] = y;
                if (Qf_out) Qf_out[s * n_eps + j] = qf;
            }
    }
    free(masks); free(Qf); free(Qq);
    return st;
}
