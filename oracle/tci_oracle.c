/*
 * CPU FP64 oracle for the two-site MPS update.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file: only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark use it.  It shares no code, header, table or helper
 * with the GPU library.
 *
 * Everything here is plain, slow and written to be checked by eye against
 * the definitions in arXiv:2512.23917 (Tensor Computing Interface, TCI).
 * "Spec" below means the paper's appendix that specifies the TCI API.
 *   - row-major tensors (memory order kept by Spec, manipulation, reshape),
 *   - transpose: Sec. II.B, transpose equation,
 *   - label-based contraction: Sec. II.B contraction equations and Spec,
 *     linear algebra, contract,
 *   - SVD after matricisation: Sec. II.B decomposition equations and Spec,
 *     linear algebra, svd,
 *   - truncation: Spec, linear algebra, trunc_svd (rules a-c and the
 *     relative truncation-error equation),
 *   - thin QR: Spec, linear algebra, qr,
 *   - Hermitian eigensolve: Spec, linear algebra, eigh (ascending).
 * All arithmetic is complex128 (real inputs are embedded with zero
 * imaginary part) and accumulates in double precision.
 *
 * Status codes: 0 ok, 1 invalid argument, 2 shape, 3 label, 7 not converged.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef double complex cplx;

#define ORC_OK 0
#define ORC_INVALID 1
#define ORC_SHAPE 2
#define ORC_LABEL 3
#define ORC_NOT_CONVERGED 7
#define ORC_MAX_ORDER 16

/* ------------------------------------------------------------------ */
/* Transpose (Section II.B): out.shape[b] = in.shape[perm[b]] and       */
/* out[c] = in[c'] with c'[perm[b]] = c[b].                              */
/* ------------------------------------------------------------------ */
int orc_permute(const cplx *in, int order, const int64_t *shape,
                const int32_t *perm, cplx *out)
{
    if (order < 0 || order > ORC_MAX_ORDER) return ORC_INVALID;
    int seen[ORC_MAX_ORDER] = {0};
    for (int b = 0; b < order; ++b) {
        if (perm[b] < 0 || perm[b] >= order || seen[perm[b]]) return ORC_INVALID;
        seen[perm[b]] = 1;
    }
    int64_t in_stride[ORC_MAX_ORDER], out_shape[ORC_MAX_ORDER];
    int64_t total = 1;
    for (int b = order - 1; b >= 0; --b) {
        in_stride[b] = total;
        total *= shape[b];
    }
    for (int b = 0; b < order; ++b) out_shape[b] = shape[perm[b]];
#pragma omp parallel for schedule(static)
    for (int64_t lin = 0; lin < total; ++lin) {
        int64_t rem = lin, src = 0;
        for (int b = order - 1; b >= 0; --b) {
            int64_t cb = rem % out_shape[b];
            rem /= out_shape[b];
            src += cb * in_stride[perm[b]];
        }
        out[lin] = in[src];
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------ */
/* Label-based contraction (Spec, linear algebra, "contract").                 */
/* Labels appearing in both a and b but not in c are summed over; the   */
/* labels of c give the free bonds and their order.  A label repeated   */
/* inside one operand is rejected, as is a label of c found in neither  */
/* or in both operands, and a label found in one operand only that is   */
/* missing from c (no implicit sums, no batch labels).                  */
/* out_shape receives the shape of c.                                    */
/* ------------------------------------------------------------------ */
static int find_label(const int32_t *labels, int n, int32_t lab)
{
    for (int i = 0; i < n; ++i)
        if (labels[i] == lab) return i;
    return -1;
}

int orc_contract_check(int ra, const int64_t *sa, const int32_t *la,
                       int rb, const int64_t *sb, const int32_t *lb,
                       int rc, const int32_t *lc, int64_t *out_shape)
{
    if (ra < 0 || rb < 0 || rc < 0 || ra > ORC_MAX_ORDER || rb > ORC_MAX_ORDER ||
        rc > ORC_MAX_ORDER)
        return ORC_INVALID;
    for (int i = 0; i < ra; ++i)
        if (find_label(la, i, la[i]) >= 0) return ORC_LABEL;
    for (int i = 0; i < rb; ++i)
        if (find_label(lb, i, lb[i]) >= 0) return ORC_LABEL;
    for (int i = 0; i < rc; ++i)
        if (find_label(lc, i, lc[i]) >= 0) return ORC_LABEL;
    for (int i = 0; i < rc; ++i) {
        int ia = find_label(la, ra, lc[i]);
        int ib = find_label(lb, rb, lc[i]);
        if ((ia >= 0) == (ib >= 0)) return ORC_LABEL;
        out_shape[i] = ia >= 0 ? sa[ia] : sb[ib];
    }
    for (int i = 0; i < ra; ++i) {
        int ib = find_label(lb, rb, la[i]);
        int ic = find_label(lc, rc, la[i]);
        if (ib < 0 && ic < 0) return ORC_LABEL;
        if (ib >= 0 && sb[ib] != sa[i]) return ORC_SHAPE;
    }
    for (int i = 0; i < rb; ++i) {
        int ia = find_label(la, ra, lb[i]);
        int ic = find_label(lc, rc, lb[i]);
        if (ia < 0 && ic < 0) return ORC_LABEL;
    }
    return ORC_OK;
}

int orc_contract(const cplx *a, int ra, const int64_t *sa, const int32_t *la,
                 const cplx *b, int rb, const int64_t *sb, const int32_t *lb,
                 cplx *c, int rc, const int32_t *lc)
{
    int64_t sc[ORC_MAX_ORDER];
    int st = orc_contract_check(ra, sa, la, rb, sb, lb, rc, lc, sc);
    if (st != ORC_OK) return st;

    int64_t stride_a[ORC_MAX_ORDER], stride_b[ORC_MAX_ORDER];
    int64_t acc = 1;
    for (int i = ra - 1; i >= 0; --i) { stride_a[i] = acc; acc *= sa[i]; }
    acc = 1;
    for (int i = rb - 1; i >= 0; --i) { stride_b[i] = acc; acc *= sb[i]; }

    /* For each free bond of c: its stride inside a (or 0) and inside b (or 0). */
    int64_t c_in_a[ORC_MAX_ORDER], c_in_b[ORC_MAX_ORDER];
    for (int i = 0; i < rc; ++i) {
        int ia = find_label(la, ra, lc[i]);
        int ib = find_label(lb, rb, lc[i]);
        c_in_a[i] = ia >= 0 ? stride_a[ia] : 0;
        c_in_b[i] = ib >= 0 ? stride_b[ib] : 0;
    }
    /* Summed bonds: labels of a that also appear in b and not in c. */
    int ns = 0;
    int64_t s_dim[ORC_MAX_ORDER], s_in_a[ORC_MAX_ORDER], s_in_b[ORC_MAX_ORDER];
    int64_t n_sum = 1;
    for (int i = 0; i < ra; ++i) {
        int ib = find_label(lb, rb, la[i]);
        if (ib >= 0 && find_label(lc, rc, la[i]) < 0) {
            s_dim[ns] = sa[i];
            s_in_a[ns] = stride_a[i];
            s_in_b[ns] = stride_b[ib];
            n_sum *= sa[i];
            ++ns;
        }
    }
    int64_t n_out = 1;
    for (int i = 0; i < rc; ++i) n_out *= sc[i];

#pragma omp parallel for schedule(static)
    for (int64_t lin = 0; lin < n_out; ++lin) {
        int64_t rem = lin, off_a = 0, off_b = 0;
        for (int i = rc - 1; i >= 0; --i) {
            int64_t ci = rem % sc[i];
            rem /= sc[i];
            off_a += ci * c_in_a[i];
            off_b += ci * c_in_b[i];
        }
        cplx sum = 0.0;
        for (int64_t s = 0; s < n_sum; ++s) {
            int64_t r2 = s, oa = off_a, ob = off_b;
            for (int k = ns - 1; k >= 0; --k) {
                int64_t ck = r2 % s_dim[k];
                r2 /= s_dim[k];
                oa += ck * s_in_a[k];
                ob += ck * s_in_b[k];
            }
            sum += a[oa] * b[ob];
        }
        c[lin] = sum;
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------ */
/* Thin SVD by one-sided Jacobi (Hestenes) on the columns of an m x n   */
/* matrix with m >= n; the m < n case works on the conjugate transpose. */
/* Spec, linear algebra, "svd": A' = U S V^dagger, s non-increasing, kappa =   */
/* min(m, n), u is m x kappa, vh is kappa x n, both row-major.           */
/* Column pairs are visited in round-robin order: every round holds     */
/* n/2 disjoint pairs which are independent and run in parallel.        */
/* A pair (i, j) is rotated unless |<x_i, x_j>| <= tol ||x_i|| ||x_j||   */
/* with tol = rows * 2^-53.  After convergence s_j = ||x_j||,           */
/* u_j = x_j / s_j, V is the product of the rotations.                  */
/* The returned factors are put in a fixed gauge: u_j is multiplied by  */
/* the phase that makes its largest-modulus entry (first on ties) real  */
/* and positive, and row j of vh by the inverse phase.                  */
/* ------------------------------------------------------------------ */
static void rotate_pair(cplx *xi, cplx *xj, int64_t len, double c, double s, cplx eph)
{
    /* [x_i', x_j'] = [x_i, x_j] diag(1, eph) [[c, s], [-s, c]], eph = e^{-i phi} */
    for (int64_t r = 0; r < len; ++r) {
        cplx a = xi[r], b = eph * xj[r];
        xi[r] = c * a - s * b;
        xj[r] = s * a + c * b;
    }
}

static int jacobi_columns(cplx *x, int64_t m, int64_t n, cplx *v, int *sweeps_out)
{
    /* x: n columns of length m, column-major.  v: n x n column-major. */
    const double tol = (double)m * ldexp(1.0, -53);
    int64_t np = n + (n & 1); /* round-robin needs an even count; index n is a dummy */
    int64_t *slot = (int64_t *)malloc(sizeof(int64_t) * (size_t)np);
    for (int64_t i = 0; i < np; ++i) slot[i] = i;
    int converged = 0, sweep = 0;
    const int max_sweeps = 80;
    for (sweep = 0; sweep < max_sweeps && !converged; ++sweep) {
        int64_t rotations = 0;
        for (int64_t round = 0; round < np - 1; ++round) {
#pragma omp parallel for schedule(dynamic, 4) reduction(+ : rotations)
            for (int64_t p = 0; p < np / 2; ++p) {
                int64_t i = slot[p], j = slot[np - 1 - p];
                if (i >= n || j >= n) continue;
                if (i > j) { int64_t t = i; i = j; j = t; }
                cplx *xi = x + i * m, *xj = x + j * m;
                double alpha = 0.0, beta = 0.0;
                cplx gamma = 0.0;
                for (int64_t r = 0; r < m; ++r) {
                    alpha += creal(xi[r]) * creal(xi[r]) + cimag(xi[r]) * cimag(xi[r]);
                    beta += creal(xj[r]) * creal(xj[r]) + cimag(xj[r]) * cimag(xj[r]);
                    gamma += conj(xi[r]) * xj[r];
                }
                double g = cabs(gamma);
                if (g == 0.0 || g <= tol * sqrt(alpha) * sqrt(beta)) continue;
                cplx eph = conj(gamma) / g; /* e^{-i phi}, gamma = |gamma| e^{i phi} */
                double zeta = (beta - alpha) / (2.0 * g);
                double t = (zeta >= 0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
                double c = 1.0 / sqrt(1.0 + t * t), s = c * t;
                rotate_pair(xi, xj, m, c, s, eph);
                rotate_pair(v + i * n, v + j * n, n, c, s, eph);
                ++rotations;
            }
            /* round-robin: keep slot[0], rotate the others by one place */
            int64_t last = slot[np - 1];
            for (int64_t q = np - 1; q > 1; --q) slot[q] = slot[q - 1];
            slot[1] = last;
        }
        if (rotations == 0) converged = 1;
    }
    free(slot);
    if (sweeps_out) *sweeps_out = sweep;
    return converged ? ORC_OK : ORC_NOT_CONVERGED;
}

/* Complete column j of the m x k column-major u (zero column) to a unit  */
/* vector orthogonal to the other non-zero columns, by Gram-Schmidt on   */
/* the standard basis vectors.                                            */
static void complete_column(cplx *u, int64_t m, int64_t k, int64_t j, const int *filled)
{
    for (int64_t e = 0; e < m; ++e) {
        cplx *col = u + j * m;
        for (int64_t r = 0; r < m; ++r) col[r] = (r == e) ? 1.0 : 0.0;
        for (int pass = 0; pass < 2; ++pass)
            for (int64_t q = 0; q < k; ++q) {
                if (q == j || !filled[q]) continue;
                cplx *o = u + q * m, d = 0.0;
                for (int64_t r = 0; r < m; ++r) d += conj(o[r]) * col[r];
                for (int64_t r = 0; r < m; ++r) col[r] -= d * o[r];
            }
        double nn = 0.0;
        for (int64_t r = 0; r < m; ++r) nn += creal(col[r] * conj(col[r]));
        nn = sqrt(nn);
        if (nn > 0.5) {
            for (int64_t r = 0; r < m; ++r) col[r] /= nn;
            return;
        }
    }
}

typedef struct { double s; int64_t idx; } sval_t;
static int cmp_sval(const void *pa, const void *pb)
{
    const sval_t *a = (const sval_t *)pa, *b = (const sval_t *)pb;
    if (a->s > b->s) return -1;
    if (a->s < b->s) return 1;
    return (a->idx < b->idx) ? -1 : (a->idx > b->idx);
}

/* tall case, m >= n: u m x n, s n, vh n x n (row-major outputs) */
static int svd_tall(const cplx *a, int64_t m, int64_t n, cplx *u, double *s, cplx *vh,
                    int *sweeps)
{
    cplx *x = (cplx *)malloc(sizeof(cplx) * (size_t)(m * n));
    cplx *v = (cplx *)calloc((size_t)(n * n), sizeof(cplx));
    for (int64_t i = 0; i < m; ++i)
        for (int64_t j = 0; j < n; ++j) x[j * m + i] = a[i * n + j];
    for (int64_t j = 0; j < n; ++j) v[j * n + j] = 1.0;
    int st = jacobi_columns(x, m, n, v, sweeps);

    sval_t *order = (sval_t *)malloc(sizeof(sval_t) * (size_t)n);
    for (int64_t j = 0; j < n; ++j) {
        double nn = 0.0;
        for (int64_t r = 0; r < m; ++r) nn += creal(x[j * m + r] * conj(x[j * m + r]));
        order[j].s = sqrt(nn);
        order[j].idx = j;
    }
    qsort(order, (size_t)n, sizeof(sval_t), cmp_sval);

    /* column-major u so columns are contiguous during completion */
    cplx *ucm = (cplx *)calloc((size_t)(m * n), sizeof(cplx));
    int *filled = (int *)calloc((size_t)n, sizeof(int));
    for (int64_t k = 0; k < n; ++k) {
        int64_t j = order[k].idx;
        s[k] = order[k].s;
        if (order[k].s > 0.0) {
            for (int64_t r = 0; r < m; ++r) ucm[k * m + r] = x[j * m + r] / order[k].s;
            filled[k] = 1;
        }
    }
    for (int64_t k = 0; k < n; ++k)
        if (!filled[k]) { complete_column(ucm, m, n, k, filled); filled[k] = 1; }

    for (int64_t k = 0; k < n; ++k) {
        int64_t j = order[k].idx;
        /* gauge: largest-modulus entry of u_k real positive */
        int64_t best = 0;
        double bm = -1.0;
        for (int64_t r = 0; r < m; ++r) {
            double mod = cabs(ucm[k * m + r]);
            if (mod > bm) { bm = mod; best = r; }
        }
        cplx ph = bm > 0 ? conj(ucm[k * m + best]) / bm : 1.0;
        for (int64_t r = 0; r < m; ++r) u[r * n + k] = ucm[k * m + r] * ph;
        /* vh row k = conj(V column j) * conj(ph) */
        for (int64_t q = 0; q < n; ++q) vh[k * n + q] = conj(v[j * n + q]) * conj(ph);
    }
    free(x); free(v); free(order); free(ucm); free(filled);
    return st;
}

int orc_svd(const cplx *a, int64_t m, int64_t n, cplx *u, double *s, cplx *vh, int *sweeps)
{
    if (m < 1 || n < 1) return ORC_INVALID;
    if (m >= n) return svd_tall(a, m, n, u, s, vh, sweeps);
    /* A^dagger = U' S V'^dagger  =>  A = V' S U'^dagger */
    int64_t k = m;
    cplx *ah = (cplx *)malloc(sizeof(cplx) * (size_t)(m * n));
    for (int64_t i = 0; i < m; ++i)
        for (int64_t j = 0; j < n; ++j) ah[j * m + i] = conj(a[i * n + j]);
    cplx *u2 = (cplx *)malloc(sizeof(cplx) * (size_t)(n * k));
    cplx *vh2 = (cplx *)malloc(sizeof(cplx) * (size_t)(k * k));
    int st = svd_tall(ah, n, m, u2, s, vh2, sweeps);
    /* u = V' = vh2^dagger (m x k); vh = U'^dagger (k x n) */
    for (int64_t i = 0; i < m; ++i)
        for (int64_t q = 0; q < k; ++q) u[i * k + q] = conj(vh2[q * k + i]);
    for (int64_t q = 0; q < k; ++q)
        for (int64_t j = 0; j < n; ++j) vh[q * n + j] = conj(u2[j * k + q]);
    /* re-apply the gauge on u (the transposed problem fixed it on V') */
    for (int64_t q = 0; q < k; ++q) {
        int64_t best = 0;
        double bm = -1.0;
        for (int64_t i = 0; i < m; ++i) {
            double mod = cabs(u[i * k + q]);
            if (mod > bm) { bm = mod; best = i; }
        }
        cplx ph = bm > 0 ? conj(u[best * k + q]) / bm : 1.0;
        for (int64_t i = 0; i < m; ++i) u[i * k + q] *= ph;
        for (int64_t j = 0; j < n; ++j) vh[q * n + j] *= conj(ph);
    }
    free(ah); free(u2); free(vh2);
    return st;
}

/* ------------------------------------------------------------------ */
/* Truncation strategy, Spec, linear algebra, "trunc_svd" form (2).            */
/*  a) discard every s_i < s_min (absolute threshold);                  */
/*  b) if at most chi_min values remain, keep exactly those;            */
/*  c) otherwise start at chi = chi_min and add values in descending    */
/*     order until eps(chi) <= target or chi = chi_max (never beyond    */
/*     the values left by a).                                           */
/* eps(chi) = sum_{i>=chi} s_i^2 / sum_i s_i^2 over ALL kappa values,  */
/* taken as 0 when the total is 0.  chi is clamped to at least 1 so a   */
/* bond never has zero width.  s must be sorted non-increasingly.        */
/* ------------------------------------------------------------------ */
int orc_trunc_rule(const double *s, int64_t kappa, int64_t chi_min, int64_t chi_max,
                   double target, double s_min, int64_t *chi_out, double *err_out)
{
    if (kappa < 1 || chi_max < 1 || chi_min < 1 || chi_min > chi_max) return ORC_INVALID;
    /* tail[i] = sum_{j >= i} s_j^2, summed from the smallest value up */
    double *tail = (double *)malloc(sizeof(double) * (size_t)(kappa + 1));
    tail[kappa] = 0.0;
    for (int64_t i = kappa - 1; i >= 0; --i) tail[i] = tail[i + 1] + s[i] * s[i];
    double total = tail[0];
    int64_t n_a = 0;
    while (n_a < kappa && s[n_a] >= s_min) ++n_a;
    int64_t chi;
    if (n_a <= chi_min) {
        chi = n_a;
    } else {
        int64_t limit = chi_max < n_a ? chi_max : n_a;
        chi = chi_min;
        while (chi < limit && total > 0.0 && tail[chi] / total > target) ++chi;
    }
    if (chi < 1) chi = 1;
    *chi_out = chi;
    *err_out = total > 0.0 ? tail[chi] / total : 0.0;
    free(tail);
    return ORC_OK;
}

/* ------------------------------------------------------------------ */
/* Thin QR by Householder reflections, Spec, linear algebra, "qr":             */
/* A' (m x n) = Q R, rho = min(m, n), Q m x rho with orthonormal        */
/* columns, R rho x n upper trapezoidal.  The gauge is fixed by making   */
/* every diagonal entry of R real and non-negative.                     */
/* ------------------------------------------------------------------ */
int orc_qr(const cplx *a, int64_t m, int64_t n, cplx *q, cplx *r)
{
    if (m < 1 || n < 1) return ORC_INVALID;
    int64_t rho = m < n ? m : n;
    cplx *w = (cplx *)malloc(sizeof(cplx) * (size_t)(m * n));
    memcpy(w, a, sizeof(cplx) * (size_t)(m * n));
    cplx *vs = (cplx *)calloc((size_t)(m * rho), sizeof(cplx)); /* reflector k in column k */
    double *taus = (double *)calloc((size_t)rho, sizeof(double));
    for (int64_t k = 0; k < rho; ++k) {
        /* x = w[k:m, k]; H = I - tau v v^dagger with v = x - beta e1, beta real */
        double xn2 = 0.0;
        for (int64_t i = k; i < m; ++i) xn2 += creal(w[i * n + k] * conj(w[i * n + k]));
        double xn = sqrt(xn2);
        cplx x0 = w[k * n + k];
        double ax0 = cabs(x0);
        cplx ph = ax0 > 0 ? x0 / ax0 : 1.0;
        cplx beta = -ph * xn; /* v = x - beta e1 avoids cancellation */
        cplx *v = vs + k * m;
        for (int64_t i = 0; i < m; ++i) v[i] = 0.0;
        v[k] = x0 - beta;
        for (int64_t i = k + 1; i < m; ++i) v[i] = w[i * n + k];
        double vn2 = 0.0;
        for (int64_t i = k; i < m; ++i) vn2 += creal(v[i] * conj(v[i]));
        taus[k] = vn2 > 0 ? 2.0 / vn2 : 0.0;
        /* apply H to columns k..n-1 of w */
        for (int64_t j = k; j < n; ++j) {
            cplx d = 0.0;
            for (int64_t i = k; i < m; ++i) d += conj(v[i]) * w[i * n + j];
            d *= taus[k];
            for (int64_t i = k; i < m; ++i) w[i * n + j] -= d * v[i];
        }
    }
    /* R = top rho rows of w (upper part); Q = H_0 ... H_{rho-1} applied to I[:, :rho] */
    for (int64_t i = 0; i < rho; ++i)
        for (int64_t j = 0; j < n; ++j) r[i * n + j] = (j >= i) ? w[i * n + j] : 0.0;
    for (int64_t i = 0; i < m; ++i)
        for (int64_t j = 0; j < rho; ++j) q[i * rho + j] = (i == j) ? 1.0 : 0.0;
    for (int64_t k = rho - 1; k >= 0; --k) {
        cplx *v = vs + k * m;
        for (int64_t j = 0; j < rho; ++j) {
            cplx d = 0.0;
            for (int64_t i = k; i < m; ++i) d += conj(v[i]) * q[i * rho + j];
            d *= taus[k];
            for (int64_t i = k; i < m; ++i) q[i * rho + j] -= d * v[i];
        }
    }
    /* gauge: diag(R) real >= 0 */
    for (int64_t i = 0; i < rho; ++i) {
        cplx d = r[i * n + i];
        double ad = cabs(d);
        cplx ph = ad > 0 ? conj(d) / ad : 1.0;
        for (int64_t j = 0; j < n; ++j) r[i * n + j] *= ph;
        for (int64_t k = 0; k < m; ++k) q[k * rho + i] *= conj(ph);
    }
    free(w); free(vs); free(taus);
    return ORC_OK;
}

/* ------------------------------------------------------------------ */
/* Hermitian eigensolve by the cyclic two-sided Jacobi method,          */
/* Spec, linear algebra, "eigh": H = V diag(w) V^dagger with w ascending.       */
/* Each rotation J = diag(1, e^{-i phi}) [[c, s], [-s, c]] annihilates   */
/* H[p][q] = |H[p][q]| e^{i phi}.  Sweeps stop when every off-diagonal  */
/* entry satisfies |H[p][q]| <= 2^-53 * sqrt(|H[p][p] H[q][q]|) or is   */
/* below 2^-53 * 1e-3 * ||H||_F.  Eigenvector gauge: largest-modulus    */
/* entry (first on ties) real and positive.                             */
/* ------------------------------------------------------------------ */
typedef struct { double w; int64_t idx; } eval_t;
static int cmp_eval(const void *pa, const void *pb)
{
    const eval_t *a = (const eval_t *)pa, *b = (const eval_t *)pb;
    if (a->w < b->w) return -1;
    if (a->w > b->w) return 1;
    return (a->idx < b->idx) ? -1 : (a->idx > b->idx);
}

int orc_eigh(const cplx *h, int64_t n, double *w, cplx *v, int *sweeps_out)
{
    if (n < 1) return ORC_INVALID;
    cplx *a = (cplx *)malloc(sizeof(cplx) * (size_t)(n * n));
    cplx *z = (cplx *)calloc((size_t)(n * n), sizeof(cplx));
    double fro = 0.0;
    for (int64_t i = 0; i < n; ++i)
        for (int64_t j = 0; j < n; ++j) {
            /* use the Hermitian part so round-off asymmetry cannot leak in */
            a[i * n + j] = 0.5 * (h[i * n + j] + conj(h[j * n + i]));
            fro += creal(a[i * n + j] * conj(a[i * n + j]));
        }
    fro = sqrt(fro);
    for (int64_t i = 0; i < n; ++i) z[i * n + i] = 1.0;
    const double eps = ldexp(1.0, -53);
    int converged = (n == 1), sweep = 0;
    for (sweep = 0; sweep < 100 && !converged; ++sweep) {
        int64_t rotations = 0;
        for (int64_t p = 0; p < n - 1; ++p)
            for (int64_t q = p + 1; q < n; ++q) {
                cplx hpq = a[p * n + q];
                double g = cabs(hpq);
                double app = creal(a[p * n + p]), aqq = creal(a[q * n + q]);
                if (g == 0.0 || g <= eps * sqrt(fabs(app * aqq)) || g <= eps * 1e-3 * fro)
                    continue;
                cplx eph = conj(hpq) / g;
                double zeta = (aqq - app) / (2.0 * g);
                double t = (zeta >= 0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
                double c = 1.0 / sqrt(1.0 + t * t), s = c * t;
                /* columns: A <- A J */
                for (int64_t k = 0; k < n; ++k) {
                    cplx x = a[k * n + p], y = eph * a[k * n + q];
                    a[k * n + p] = c * x - s * y;
                    a[k * n + q] = s * x + c * y;
                }
                /* rows: A <- J^dagger A */
                for (int64_t k = 0; k < n; ++k) {
                    cplx x = a[p * n + k], y = conj(eph) * a[q * n + k];
                    a[p * n + k] = c * x - s * y;
                    a[q * n + k] = s * x + c * y;
                }
                a[p * n + q] = 0.0;
                a[q * n + p] = 0.0;
                a[p * n + p] = creal(a[p * n + p]);
                a[q * n + q] = creal(a[q * n + q]);
                for (int64_t k = 0; k < n; ++k) {
                    cplx x = z[k * n + p], y = eph * z[k * n + q];
                    z[k * n + p] = c * x - s * y;
                    z[k * n + q] = s * x + c * y;
                }
                ++rotations;
            }
        if (rotations == 0) converged = 1;
    }
    eval_t *ord = (eval_t *)malloc(sizeof(eval_t) * (size_t)n);
    for (int64_t i = 0; i < n; ++i) { ord[i].w = creal(a[i * n + i]); ord[i].idx = i; }
    qsort(ord, (size_t)n, sizeof(eval_t), cmp_eval);
    for (int64_t k = 0; k < n; ++k) {
        int64_t j = ord[k].idx;
        w[k] = ord[k].w;
        int64_t best = 0;
        double bm = -1.0;
        for (int64_t r = 0; r < n; ++r) {
            double mod = cabs(z[r * n + j]);
            if (mod > bm) { bm = mod; best = r; }
        }
        cplx ph = bm > 0 ? conj(z[best * n + j]) / bm : 1.0;
        for (int64_t r = 0; r < n; ++r) v[r * n + k] = z[r * n + j] * ph;
    }
    if (sweeps_out) *sweeps_out = sweep;
    free(a); free(z); free(ord);
    return converged ? ORC_OK : ORC_NOT_CONVERGED;
}

/* ------------------------------------------------------------------ */
/* Philox4x32-10 counter-based generator (Salmon, Moraes, Dror, Shaw,   */
/* "Parallel random numbers: as easy as 1, 2, 3", SC'11).  Used by the  */
/* randomized SVD sketch: block i of four 32-bit outputs is             */
/* philox(counter = (i_lo, i_hi, stream, 0), key = (seed_lo, seed_hi)). */
/* ------------------------------------------------------------------ */
static void philox_round(uint32_t ctr[4], const uint32_t key[2])
{
    const uint64_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
    uint64_t p0 = M0 * (uint64_t)ctr[0], p1 = M1 * (uint64_t)ctr[2];
    uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    uint32_t n0 = hi1 ^ ctr[1] ^ key[0];
    uint32_t n1 = lo1;
    uint32_t n2 = hi0 ^ ctr[3] ^ key[1];
    uint32_t n3 = lo0;
    ctr[0] = n0; ctr[1] = n1; ctr[2] = n2; ctr[3] = n3;
}

void orc_philox4x32_10_raw(const uint32_t *ctr_in, const uint32_t *key_in, uint32_t *out)
{
    uint32_t ctr[4] = {ctr_in[0], ctr_in[1], ctr_in[2], ctr_in[3]};
    uint32_t key[2] = {key_in[0], key_in[1]};
    for (int r = 0; r < 10; ++r) {
        philox_round(ctr, key);
        if (r < 9) { key[0] += 0x9E3779B9u; key[1] += 0xBB67AE85u; }
    }
    memcpy(out, ctr, sizeof(ctr));
}

void orc_philox4x32_10(uint64_t seed, uint32_t stream, uint64_t first_block, int64_t n_blocks,
                       uint32_t *out)
{
    const uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    for (int64_t b = 0; b < n_blocks; ++b) {
        uint64_t idx = first_block + (uint64_t)b;
        const uint32_t ctr[4] = {(uint32_t)idx, (uint32_t)(idx >> 32), stream, 0u};
        orc_philox4x32_10_raw(ctr, key, out + 4 * b);
    }
}
