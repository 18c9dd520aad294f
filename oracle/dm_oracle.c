/*
 * Plain FP64 density-matrix oracle -- TEST INFRASTRUCTURE ONLY.
 *
 * Only the tests, the smoke check and the CPU-baseline leg of the benchmark
 * use this file.  It shares no code with the GPU library.
 *
 * Storage: rho is a row-major 2^n x 2^n complex matrix, R[r * D + c] with
 * D = 2^n, interleaved (re, im) doubles.  Qubit q is bit q of the row (and of
 * the column) index.  A k-qubit operator M on targets t[0..k-1] has matrix
 * index sum_j b(t[j]) 2^j (t[0] is the least significant bit).
 *
 * What is computed is the plain definition of the paper's density-matrix
 * emulation (Sec. 2, density-matrix representation with general Kraus
 * operators; Sec. 3.1 channel definitions):
 *   unitary / general matrix:  rho <- M rho M^dagger
 *   Kraus map {K_j}:           rho <- sum_j K_j rho K_j^dagger
 * each operator embedded as identity on the other qubits.  Ops are applied in
 * order, one at a time, with no fusion.  OpenMP may split the outer loops;
 * every output element is written by exactly one thread, so results do not
 * depend on the thread count.
 *
 * Read-outs (Sec. 2: expectation values of Pauli strings; density-matrix
 * elements): trace, diagonal probabilities, <Z_i>, <Z_i Z_j>, purity Tr rho^2
 * and Tr(P rho) for a Pauli string P.  Sums use Neumaier compensation in a
 * fixed sequential order.
 */
#include <complex.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef double complex cplx;

/* Row/column index with bit t[j] set to bit j of `sub`, on top of `base`. */
static inline uint64_t deposit(uint64_t base, int k, const int *t, unsigned sub)
{
    uint64_t r = base;
    for (int j = 0; j < k; ++j)
        if (sub >> j & 1u) r |= (uint64_t)1 << t[j];
    return r;
}

/* For each row a of the d x d matrices M[0..nm-1], the columns b whose entry
 * M[a][b] is not an exact zero: cols[(j*d + a)*d + 0 .. cnt[j*d + a] - 1].
 * A product with an exact zero entry adds an exact zero to a sum, so the sums
 * below leave those terms out and are unchanged (at most the sign of a zero
 * result differs).  Pauli-product Kraus operators and diagonal gates have one
 * nonzero per row, which is where this saves time. */
static void nonzero_cols(const cplx *M, int nm, unsigned d, unsigned char *cols, unsigned char *cnt)
{
    for (int j = 0; j < nm; ++j)
        for (unsigned a = 0; a < d; ++a) {
            unsigned c = 0;
            for (unsigned b = 0; b < d; ++b)
                if (M[((size_t)j * d + a) * d + b] != 0) cols[((size_t)j * d + a) * d + c++] = (unsigned char)b;
            cnt[(size_t)j * d + a] = (unsigned char)c;
        }
}

/* True if none of the target bits is set in x. */
static inline int targets_clear(uint64_t x, int k, const int *t)
{
    for (int j = 0; j < k; ++j)
        if (x >> t[j] & 1u) return 0;
    return 1;
}

void orc_init_zero(double *R, int n)
{
    uint64_t D = (uint64_t)1 << n;
    memset(R, 0, sizeof(double) * 2 * D * D);
    R[0] = 1.0;
}

void orc_init_basis(double *R, int n, uint64_t b)
{
    uint64_t D = (uint64_t)1 << n;
    memset(R, 0, sizeof(double) * 2 * D * D);
    R[2 * (b * D + b)] = 1.0;
}

/* Product of single-qubit diagonal states p0[j]|0><0| + (1-p0[j])|1><1|
 * (thermal initial state, Sec. 8 superconducting error model). */
void orc_init_product_diag(double *R, int n, const double *p0)
{
    uint64_t D = (uint64_t)1 << n;
    memset(R, 0, sizeof(double) * 2 * D * D);
    for (uint64_t r = 0; r < D; ++r) {
        double v = 1.0;
        for (int j = 0; j < n; ++j)
            v *= (r >> j & 1u) ? (1.0 - p0[j]) : p0[j];
        R[2 * (r * D + r)] = v;
    }
}

/* rho <- M rho M^dagger for a k-qubit matrix M (row-major, interleaved). */
void orc_apply_matrix(double *Rd, int n, int k, const int *t, const double *Md)
{
    cplx *R = (cplx *)Rd;
    const cplx *M = (const cplx *)Md;
    const int64_t D = (int64_t)1 << n;
    const unsigned d = 1u << k;
    unsigned char *nzc = malloc((size_t)d * d), *nzn = malloc(d);
    if (!nzc || !nzn) { free(nzc); free(nzn); return; }
    nonzero_cols(M, 1, d, nzc, nzn);

    /* left multiplication: rho <- M rho; each group of d rows that differ
     * only in the target bits is combined column by column */
#pragma omp parallel for schedule(static)
    for (int64_t r0 = 0; r0 < D; ++r0) {
        if (!targets_clear((uint64_t)r0, k, t)) continue;
        cplx v[64], w[64];
        uint64_t rows[64];
        for (unsigned a = 0; a < d; ++a) rows[a] = deposit(r0, k, t, a);
        for (int64_t c = 0; c < D; ++c) {
            for (unsigned a = 0; a < d; ++a) v[a] = R[rows[a] * D + c];
            for (unsigned a = 0; a < d; ++a) {
                cplx s = 0;
                for (unsigned i = 0; i < nzn[a]; ++i) {
                    unsigned b = nzc[a * d + i];
                    s += M[a * d + b] * v[b];
                }
                w[a] = s;
            }
            for (unsigned a = 0; a < d; ++a) R[rows[a] * D + c] = w[a];
        }
    }
    /* right multiplication: rho <- rho M^dagger, row by row;
     * (rho M^dagger)_{r,c} = sum_c' rho_{r,c'} conj(M_{c,c'}) */
#pragma omp parallel for schedule(static)
    for (int64_t r = 0; r < D; ++r) {
        cplx v[64], w[64];
        for (int64_t c0 = 0; c0 < D; ++c0) {
            if (!targets_clear((uint64_t)c0, k, t)) continue;
            for (unsigned b = 0; b < d; ++b)
                v[b] = R[r * D + deposit(c0, k, t, b)];
            for (unsigned a = 0; a < d; ++a) {
                cplx s = 0;
                for (unsigned i = 0; i < nzn[a]; ++i) {
                    unsigned b = nzc[a * d + i];
                    s += v[b] * conj(M[a * d + b]);
                }
                w[a] = s;
            }
            for (unsigned a = 0; a < d; ++a)
                R[r * D + deposit(c0, k, t, a)] = w[a];
        }
    }
    free(nzc);
    free(nzn);
}

/* rho <- sum_j K_j rho K_j^dagger.  K holds nk matrices of size 2^k x 2^k,
 * one after another.  Each d x d block of rho whose rows and columns differ
 * only in the target bits is replaced in place by sum_j K_j B K_j^dagger. */
void orc_apply_kraus(double *Rd, int n, int k, const int *t, int nk, const double *Kd)
{
    cplx *R = (cplx *)Rd;
    const cplx *K = (const cplx *)Kd;
    const int64_t D = (int64_t)1 << n;
    const unsigned d = 1u << k;
    unsigned char *nzc = malloc((size_t)nk * d * d), *nzn = malloc((size_t)nk * d);
    if (!nzc || !nzn) { free(nzc); free(nzn); return; }
    nonzero_cols(K, nk, d, nzc, nzn);

#pragma omp parallel for schedule(static)
    for (int64_t r0 = 0; r0 < D; ++r0) {
        if (!targets_clear((uint64_t)r0, k, t)) continue;
        cplx B[16 * 16], KB[16 * 16], out[16 * 16];
        for (int64_t c0 = 0; c0 < D; ++c0) {
            if (!targets_clear((uint64_t)c0, k, t)) continue;
            for (unsigned a = 0; a < d; ++a)
                for (unsigned b = 0; b < d; ++b)
                    B[a * d + b] = R[deposit(r0, k, t, a) * D + deposit(c0, k, t, b)];
            for (unsigned i = 0; i < d * d; ++i) out[i] = 0;
            for (int j = 0; j < nk; ++j) {
                const cplx *Kj = K + (size_t)j * d * d;
                const unsigned char *cj = nzc + (size_t)j * d * d, *nj = nzn + (size_t)j * d;
                /* KB = K_j B */
                for (unsigned a = 0; a < d; ++a)
                    for (unsigned b = 0; b < d; ++b) {
                        cplx s = 0;
                        for (unsigned i = 0; i < nj[a]; ++i) {
                            unsigned m = cj[a * d + i];
                            s += Kj[a * d + m] * B[m * d + b];
                        }
                        KB[a * d + b] = s;
                    }
                /* out += KB K_j^dagger */
                for (unsigned a = 0; a < d; ++a)
                    for (unsigned b = 0; b < d; ++b) {
                        cplx s = 0;
                        for (unsigned i = 0; i < nj[b]; ++i) {
                            unsigned m = cj[b * d + i];
                            s += KB[a * d + m] * conj(Kj[b * d + m]);
                        }
                        out[a * d + b] += s;
                    }
            }
            for (unsigned a = 0; a < d; ++a)
                for (unsigned b = 0; b < d; ++b)
                    R[deposit(r0, k, t, a) * D + deposit(c0, k, t, b)] = out[a * d + b];
        }
    }
    free(nzc);
    free(nzn);
}

/* ---- compensated summation (Neumaier) -------------------------------- */
typedef struct { double s, c; } nsum;
static inline void nadd(nsum *a, double x)
{
    double t = a->s + x;
    if ((t < 0 ? -t : t) >= (a->s < 0 ? -a->s : a->s))
        a->c += (a->s - t) + x;
    else
        a->c += (x - t) + a->s;
    a->s = t;
}
static inline double nval(const nsum *a) { return a->s + a->c; }

void orc_trace(const double *R, int n, double *re, double *im)
{
    uint64_t D = (uint64_t)1 << n;
    nsum a = {0, 0}, b = {0, 0};
    for (uint64_t r = 0; r < D; ++r) {
        nadd(&a, R[2 * (r * D + r)]);
        nadd(&b, R[2 * (r * D + r) + 1]);
    }
    *re = nval(&a);
    *im = nval(&b);
}

/* p_r = Re rho_{rr}; not clamped, not renormalised. */
void orc_probs(const double *R, int n, double *out)
{
    uint64_t D = (uint64_t)1 << n;
    for (uint64_t r = 0; r < D; ++r) out[r] = R[2 * (r * D + r)];
}

/* <Z_i> = sum_r (-1)^{r_i} rho_{rr}, i = 0..n-1 */
void orc_expec_z(const double *R, int n, double *out)
{
    uint64_t D = (uint64_t)1 << n;
    for (int i = 0; i < n; ++i) {
        nsum a = {0, 0};
        for (uint64_t r = 0; r < D; ++r) {
            double p = R[2 * (r * D + r)];
            nadd(&a, (r >> i & 1u) ? -p : p);
        }
        out[i] = nval(&a);
    }
}

/* <Z_i Z_j> for the listed pairs. */
void orc_expec_zz(const double *R, int n, const int *pairs, int npairs, double *out)
{
    uint64_t D = (uint64_t)1 << n;
    for (int k = 0; k < npairs; ++k) {
        int i = pairs[2 * k], j = pairs[2 * k + 1];
        nsum a = {0, 0};
        for (uint64_t r = 0; r < D; ++r) {
            double p = R[2 * (r * D + r)];
            int s = (int)((r >> i) ^ (r >> j)) & 1;
            nadd(&a, s ? -p : p);
        }
        out[k] = nval(&a);
    }
}

/* Tr rho^2 = sum_{r,c} |rho_{rc}|^2 for Hermitian rho; here computed as the
 * plain sum of squared magnitudes over all entries. */
double orc_purity(const double *R, int n)
{
    uint64_t D = (uint64_t)1 << n;
    nsum a = {0, 0};
    for (uint64_t i = 0; i < 2 * D * D; ++i) nadd(&a, R[i] * R[i]);
    return nval(&a);
}

/* Tr(P rho) = sum_{r,c} P_{rc} rho_{cr} for P = (x) sigma_{codes[q]} on qubit q
 * (0=I, 1=X, 2=Y, 3=Z).  Each column c of P has exactly one nonzero row r. */
void orc_expec_pauli(const double *Rd, int n, const int *codes, double *re, double *im)
{
    const cplx *R = (const cplx *)Rd;
    static const cplx I2[2][2] = {{1, 0}, {0, 1}};
    const cplx X2[2][2] = {{0, 1}, {1, 0}};
    const cplx Y2[2][2] = {{0, -I}, {I, 0}};
    const cplx Z2[2][2] = {{1, 0}, {0, -1}};
    uint64_t D = (uint64_t)1 << n;
    uint64_t xmask = 0;
    for (int q = 0; q < n; ++q)
        if (codes[q] == 1 || codes[q] == 2) xmask |= (uint64_t)1 << q;
    nsum a = {0, 0}, b = {0, 0};
    for (uint64_t c = 0; c < D; ++c) {
        uint64_t r = c ^ xmask;
        cplx p = 1;
        for (int q = 0; q < n; ++q) {
            int rb = (int)(r >> q & 1u), cb = (int)(c >> q & 1u);
            const cplx (*S)[2] = codes[q] == 0 ? I2 : codes[q] == 1 ? X2 : codes[q] == 2 ? Y2 : Z2;
            p *= S[rb][cb];
        }
        cplx v = p * R[c * D + r];
        nadd(&a, creal(v));
        nadd(&b, cimag(v));
    }
    *re = nval(&a);
    *im = nval(&b);
}
