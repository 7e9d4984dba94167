/*
 * Plain CPU oracle for the FEM SpMV / CG hot path.  TEST INFRASTRUCTURE ONLY:
 * nothing in the product library calls, links or includes this file; only the
 * test suite, the smoke check and the CPU-baseline leg of the benchmark do.
 *
 * Everything here is the slow, obviously-correct definition of what the GPU
 * path computes, in IEEE double precision (single precision where the
 * mixed-precision variant fixes it), single-threaded, compiled with
 * -ffp-contract=off so that no multiply-add is fused behind our back.
 *
 * Status codes returned by the solvers (defined here, independently of the
 * library):  0 converged, 1 not converged within maxit, 2 breakdown
 * (p^T A p <= 0 or a non-finite scalar), 3 bad argument (e.g. a zero
 * diagonal entry with the Jacobi preconditioner).
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_OK 0
#define OR_NOT_CONVERGED 1
#define OR_BREAKDOWN 2
#define OR_ARG 3

/* ------------------------------------------------------------------------
 * Sparse matrix-vector product, statement of the problem (section "Description
 * of Current GPU Methods": y = A x for given x).  Row i of a CSR matrix is
 * summed in increasing storage order k = rowptr[i] .. rowptr[i+1]-1.
 * ---------------------------------------------------------------------- */
void or_spmv(int32_t n_rows, const int32_t *rowptr, const int32_t *col,
             const double *val, const double *x, double *y)
{
    for (int32_t i = 0; i < n_rows; ++i) {
        double s = 0.0;
        for (int32_t k = rowptr[i]; k < rowptr[i + 1]; ++k)
            s += val[k] * x[col[k]];
        y[i] = s;
    }
}

/* The same row sums with the rows split over OpenMP threads (each row is
 * still summed by one thread in storage order, so the result is bitwise
 * that of or_spmv).  Used only to time the oracle on all host cores.
 * Returns the number of threads used. */
int or_spmv_par(int32_t n_rows, const int32_t *rowptr, const int32_t *col,
                const double *val, const double *x, double *y)
{
    int used = 1;
#pragma omp parallel
    {
#pragma omp single
        used = omp_get_num_threads();
#pragma omp for schedule(static)
        for (int32_t i = 0; i < n_rows; ++i) {
            double s = 0.0;
            for (int32_t k = rowptr[i]; k < rowptr[i + 1]; ++k)
                s += val[k] * x[col[k]];
            y[i] = s;
        }
    }
    return used;
}

/* Componentwise magnitude bound (|A| |x|)_i, the scale of the rounding error
 * of row i; used to state the FP64 SpMV tolerance componentwise. */
void or_spmv_abs(int32_t n_rows, const int32_t *rowptr, const int32_t *col,
                 const double *val, const double *x, double *y)
{
    for (int32_t i = 0; i < n_rows; ++i) {
        double s = 0.0;
        for (int32_t k = rowptr[i]; k < rowptr[i + 1]; ++k)
            s += fabs(val[k]) * fabs(x[col[k]]);
        y[i] = s;
    }
}

/* Multi-right-hand-side product Y = A X; X is n_cols x k and Y is n_rows x k,
 * both row-major with row strides ldx, ldy.  Column c of Y is exactly the
 * single-vector product with column c of X. */
void or_spmm(int32_t n_rows, const int32_t *rowptr, const int32_t *col,
             const double *val, int32_t k, const double *X, int64_t ldx,
             double *Y, int64_t ldy)
{
    for (int32_t i = 0; i < n_rows; ++i)
        for (int32_t c = 0; c < k; ++c) {
            double s = 0.0;
            for (int32_t e = rowptr[i]; e < rowptr[i + 1]; ++e)
                s += val[e] * X[(int64_t)col[e] * ldx + c];
            Y[(int64_t)i * ldy + c] = s;
        }
}

/* ------------------------------------------------------------------------
 * Renumbering (sections "ELL-WARP with row reordering (K1r)" and "K1r with
 * sorted column index numbering (K1rs)").  With a permutation P (new index i
 * holds old index P[i]) the relabelled vector is x'(i) = x(P(i)) and a column
 * index c becomes c' = P^{-1}(c); K1rs additionally sorts each row's
 * relabelled columns ascending, moving the values with them.
 * ---------------------------------------------------------------------- */
void or_gather(int32_t n, const int32_t *perm, const double *x, double *xp)
{
    for (int32_t i = 0; i < n; ++i)
        xp[i] = x[perm[i]];
}

void or_scatter(int32_t n, const int32_t *perm, const double *xp, double *x)
{
    for (int32_t i = 0; i < n; ++i)
        x[perm[i]] = xp[i];
}

void or_inverse_perm(int32_t n, const int32_t *perm, int32_t *iperm)
{
    for (int32_t i = 0; i < n; ++i)
        iperm[perm[i]] = i;
}

/* Row i of the output is row rperm[i] of the input (rperm NULL: identity);
 * every column index c becomes ciperm[c] (ciperm NULL: unchanged); with
 * sort_cols the entries of each output row are ordered by column (a stable
 * insertion sort, values follow their columns).  Output arrays have room for
 * n_rows+1 and nnz entries. */
void or_permute(int32_t n_rows, const int32_t *rowptr, const int32_t *col,
                const double *val, const int32_t *rperm,
                const int32_t *ciperm, int32_t sort_cols,
                int32_t *orowptr, int32_t *ocol, double *oval)
{
    orowptr[0] = 0;
    for (int32_t i = 0; i < n_rows; ++i) {
        int32_t src = rperm ? rperm[i] : i;
        int32_t len = rowptr[src + 1] - rowptr[src];
        int32_t o = orowptr[i];
        for (int32_t e = 0; e < len; ++e) {
            int32_t c = col[rowptr[src] + e];
            ocol[o + e] = ciperm ? ciperm[c] : c;
            oval[o + e] = val[rowptr[src] + e];
        }
        if (sort_cols) {
            for (int32_t a = 1; a < len; ++a) {
                int32_t c = ocol[o + a];
                double v = oval[o + a];
                int32_t b = a - 1;
                while (b >= 0 && ocol[o + b] > c) {
                    ocol[o + b + 1] = ocol[o + b];
                    oval[o + b + 1] = oval[o + b];
                    --b;
                }
                ocol[o + b + 1] = c;
                oval[o + b + 1] = v;
            }
        }
        orowptr[i + 1] = o + len;
    }
}

/* ------------------------------------------------------------------------
 * Low-precision storage.  FP32: round-to-nearest (ties to even) of the double
 * value, which is what the C conversion does under the default rounding mode.
 * BF16: the upper 16 bits of the FP32 value rounded to nearest, ties to even,
 * taken on the FP32 bit pattern (so FP64 -> BF16 is a two-step rounding,
 * FP64 -> FP32 -> BF16); NaN stays a quiet NaN of the same sign.
 * ---------------------------------------------------------------------- */
float or_round_f32(double v) { return (float)v; }

uint16_t or_f32_to_bf16(float f)
{
    uint32_t u;
    memcpy(&u, &f, 4);
    if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x007fffffu))
        return (uint16_t)((u >> 16) | 0x0040u);          /* quiet NaN */
    uint32_t lsb = (u >> 16) & 1u;
    uint32_t r = u + 0x7fffu + lsb;                       /* nearest, ties even */
    return (uint16_t)(r >> 16);
}

float or_bf16_to_f32(uint16_t h)
{
    uint32_t u = (uint32_t)h << 16;
    float f;
    memcpy(&f, &u, 4);
    return f;
}

void or_round_array_f32(int64_t n, const double *v, float *out)
{
    for (int64_t i = 0; i < n; ++i)
        out[i] = or_round_f32(v[i]);
}

void or_round_array_bf16(int64_t n, const double *v, uint16_t *out)
{
    for (int64_t i = 0; i < n; ++i)
        out[i] = or_f32_to_bf16(or_round_f32(v[i]));
}

/* Single-precision product with single-precision values (BF16 values are
 * passed widened to float, which is exact): y_i = sum_k a_k x_{c_k}, summed
 * in float in storage order. */
void or_spmv_f32(int32_t n_rows, const int32_t *rowptr, const int32_t *col,
                 const float *val, const float *x, float *y)
{
    for (int32_t i = 0; i < n_rows; ++i) {
        float s = 0.0f;
        for (int32_t k = rowptr[i]; k < rowptr[i + 1]; ++k)
            s += val[k] * x[col[k]];
        y[i] = s;
    }
}

/* ------------------------------------------------------------------------
 * Conjugate gradients.  The paper solves K dx = R with a standard
 * Jacobi-preconditioned conjugate-gradient method, at least one SpMV per
 * iteration (sections "Computational Cost of the Finite Element Method" and
 * "Description of Current GPU Methods"), without printing the iteration.
 * This is the textbook preconditioned CG (Hestenes and Stiefel; Saad,
 * Iterative Methods for Sparse Linear Systems, Algorithm 9.1) with
 * M = diag(A) (precond = 1) or M = I (precond = 0):
 *
 *   r = b - A x, z = M^-1 r, p = z, rho = r.z
 *   repeat: q = A p; gamma = p.q  (gamma <= 0 or non-finite: breakdown)
 *           alpha = rho / gamma; x += alpha p; r -= alpha q
 *           if |r| <= rtol |b|: recompute r_t = b - A x; stop if
 *               |r_t| <= rtol |b|, else replace r by r_t
 *           z = M^-1 r; rho' = r.z; beta = rho' / rho; rho = rho'
 *           p = z + beta p
 *
 * b = 0 returns x = 0 after 0 iterations.  x holds the initial guess on
 * entry.  *iters counts executed iterations; *relres is the true relative
 * residual |b - A x| / |b| of the returned x.
 * ---------------------------------------------------------------------- */
static double dot(int32_t n, const double *a, const double *b)
{
    double s = 0.0;
    for (int32_t i = 0; i < n; ++i)
        s += a[i] * b[i];
    return s;
}

static int diag_inverse(int32_t n, const int32_t *rowptr, const int32_t *col,
                        const double *val, double *dinv)
{
    for (int32_t i = 0; i < n; ++i) {
        double d = 0.0;
        for (int32_t k = rowptr[i]; k < rowptr[i + 1]; ++k)
            if (col[k] == i)
                d += val[k];
        if (d == 0.0 || !isfinite(d))
            return OR_ARG;
        dinv[i] = 1.0 / d;
    }
    return OR_OK;
}

static void true_residual(int32_t n, const int32_t *rowptr,
                          const int32_t *col, const double *val,
                          const double *b, const double *x, double *r)
{
    or_spmv(n, rowptr, col, val, x, r);
    for (int32_t i = 0; i < n; ++i)
        r[i] = b[i] - r[i];
}

int or_pcg(int32_t n, const int32_t *rowptr, const int32_t *col,
           const double *val, const double *b, double *x, int32_t precond,
           double rtol, int32_t maxit, int32_t *iters, double *relres)
{
    *iters = 0;
    *relres = 0.0;
    double bnorm = sqrt(dot(n, b, b));
    if (bnorm == 0.0) {
        for (int32_t i = 0; i < n; ++i)
            x[i] = 0.0;
        return OR_OK;
    }
    double *r = malloc(sizeof(double) * n), *z = malloc(sizeof(double) * n);
    double *p = malloc(sizeof(double) * n), *q = malloc(sizeof(double) * n);
    double *dinv = malloc(sizeof(double) * n);
    int status = OR_NOT_CONVERGED;
    if (precond) {
        if (diag_inverse(n, rowptr, col, val, dinv) != OR_OK) {
            status = OR_ARG;
            goto done;
        }
    } else {
        for (int32_t i = 0; i < n; ++i)
            dinv[i] = 1.0;
    }
    double tol = rtol * bnorm;
    true_residual(n, rowptr, col, val, b, x, r);
    if (sqrt(dot(n, r, r)) <= tol) {
        status = OR_OK;
        goto done;
    }
    for (int32_t i = 0; i < n; ++i) {
        z[i] = dinv[i] * r[i];
        p[i] = z[i];
    }
    double rho = dot(n, r, z);
    for (int32_t it = 1; it <= maxit; ++it) {
        or_spmv(n, rowptr, col, val, p, q);
        double gamma = dot(n, p, q);
        *iters = it;
        if (!(gamma > 0.0) || !isfinite(gamma)) {
            status = OR_BREAKDOWN;
            goto done;
        }
        double alpha = rho / gamma;
        for (int32_t i = 0; i < n; ++i) {
            x[i] += alpha * p[i];
            r[i] -= alpha * q[i];
        }
        if (sqrt(dot(n, r, r)) <= tol) {
            true_residual(n, rowptr, col, val, b, x, r);
            if (sqrt(dot(n, r, r)) <= tol) {
                status = OR_OK;
                goto done;
            }
        }
        for (int32_t i = 0; i < n; ++i)
            z[i] = dinv[i] * r[i];
        double rho_new = dot(n, r, z);
        double beta = rho_new / rho;
        if (!isfinite(beta)) {
            status = OR_BREAKDOWN;
            goto done;
        }
        rho = rho_new;
        for (int32_t i = 0; i < n; ++i)
            p[i] = z[i] + beta * p[i];
    }
done:
    true_residual(n, rowptr, col, val, b, x, r);
    *relres = sqrt(dot(n, r, r)) / bnorm;
    free(r); free(z); free(p); free(q); free(dinv);
    return status;
}

/* ------------------------------------------------------------------------
 * Mixed-precision iterative refinement.  Outer loop in double precision:
 *   r = b - A x  (FP64 matrix);  stop when |r| <= rtol |b|
 *   solve A_lo d = r approximately by the same preconditioned CG run in
 *   single precision (values a_lo, vectors and every sum in float), from
 *   d = 0, until |r_inner| <= inner_rtol |r| or max_inner iterations
 *   x += d  (FP64)
 * a_lo holds the stored low-precision values (FP32, or BF16 widened to
 * float).  *outer counts refinement steps, *inner the inner iterations over
 * all steps.  The Jacobi scaling of the inner solve uses diag(A_lo).
 * With scale = s != NULL the inner system is the Jacobi-scaled one,
 * S A S d' = S r with S = diag(s), s_i = diag(A)_i^-1/2 (a_lo then holds
 * round(S A S), and the caller passes precond = 0 since that diagonal is
 * 1): the inner right-hand side is float(s_i r_i) and the FP64 update
 * x_i += s_i d'_i -- exactly A d = r for d = S d'.
 * ---------------------------------------------------------------------- */
static float dotf(int32_t n, const float *a, const float *b)
{
    float s = 0.0f;
    for (int32_t i = 0; i < n; ++i)
        s += a[i] * b[i];
    return s;
}

static int32_t inner_cg_f32(int32_t n, const int32_t *rowptr,
                            const int32_t *col, const float *a,
                            const float *dinv, const float *rhs, float *d,
                            float tol, int32_t maxit, float *r, float *z,
                            float *p, float *q, int *bad)
{
    *bad = 0;
    for (int32_t i = 0; i < n; ++i) {
        d[i] = 0.0f;
        r[i] = rhs[i];
        z[i] = dinv[i] * r[i];
        p[i] = z[i];
    }
    float rho = dotf(n, r, z);
    int32_t it;
    for (it = 1; it <= maxit; ++it) {
        or_spmv_f32(n, rowptr, col, a, p, q);
        float gamma = dotf(n, p, q);
        if (!(gamma > 0.0f) || !isfinite(gamma)) {
            *bad = 1;
            return it;
        }
        float alpha = rho / gamma;
        for (int32_t i = 0; i < n; ++i) {
            d[i] += alpha * p[i];
            r[i] -= alpha * q[i];
        }
        if (sqrtf(dotf(n, r, r)) <= tol)
            return it;
        for (int32_t i = 0; i < n; ++i)
            z[i] = dinv[i] * r[i];
        float rho_new = dotf(n, r, z);
        float beta = rho_new / rho;
        rho = rho_new;
        for (int32_t i = 0; i < n; ++i)
            p[i] = z[i] + beta * p[i];
    }
    return maxit;
}

int or_ir_cg(int32_t n, const int32_t *rowptr, const int32_t *col,
             const double *val, const float *a_lo, const double *b,
             double *x, int32_t precond, double rtol, double inner_rtol,
             int32_t max_outer, int32_t max_inner, int32_t *outer,
             int32_t *inner, double *relres, const double *scale)
{
    *outer = 0;
    *inner = 0;
    *relres = 0.0;
    double bnorm = sqrt(dot(n, b, b));
    if (bnorm == 0.0) {
        for (int32_t i = 0; i < n; ++i)
            x[i] = 0.0;
        return OR_OK;
    }
    double *r = malloc(sizeof(double) * n);
    float *rf = malloc(sizeof(float) * n), *df = malloc(sizeof(float) * n);
    float *w1 = malloc(sizeof(float) * n), *w2 = malloc(sizeof(float) * n);
    float *w3 = malloc(sizeof(float) * n), *w4 = malloc(sizeof(float) * n);
    float *dinv = malloc(sizeof(float) * n);
    int status = OR_NOT_CONVERGED;
    for (int32_t i = 0; i < n; ++i) {
        float dd = 0.0f;
        for (int32_t k = rowptr[i]; k < rowptr[i + 1]; ++k)
            if (col[k] == i)
                dd += a_lo[k];
        if (precond && (dd == 0.0f || !isfinite(dd))) {
            status = OR_ARG;
            goto done;
        }
        dinv[i] = precond ? 1.0f / dd : 1.0f;
    }
    for (;;) {
        true_residual(n, rowptr, col, val, b, x, r);
        double rn = sqrt(dot(n, r, r));
        if (rn <= rtol * bnorm) {
            status = OR_OK;
            break;
        }
        if (*outer >= max_outer)
            break;
        for (int32_t i = 0; i < n; ++i)
            rf[i] = (float)(scale ? scale[i] * r[i] : r[i]);
        float rfn = sqrtf(dotf(n, rf, rf));
        int bad = 0;
        *inner += inner_cg_f32(n, rowptr, col, a_lo, dinv, rf, df,
                               (float)inner_rtol * rfn, max_inner, w1, w2,
                               w3, w4, &bad);
        *outer += 1;
        if (bad) {
            status = OR_BREAKDOWN;
            break;
        }
        for (int32_t i = 0; i < n; ++i)
            x[i] += scale ? scale[i] * (double)df[i] : (double)df[i];
    }
done:
    true_residual(n, rowptr, col, val, b, x, r);
    *relres = sqrt(dot(n, r, r)) / bnorm;
    free(r); free(rf); free(df); free(w1); free(w2); free(w3); free(w4);
    free(dinv);
    return status;
}

/* Refinement with a kept inner search direction: one FP32 CG runs across
 * the refinement steps.  When its residual has fallen by inner_rtol, the
 * correction d is added to x in FP64, the FP64 residual r = b - A x is
 * taken, and the inner CG continues from d = 0 with its residual replaced
 * by float(r): rho and beta are recomputed from the new residual and the
 * search direction p = z + beta p is kept. */
int or_ir_cg_keep(int32_t n, const int32_t *rowptr, const int32_t *col,
                  const double *val, const float *a_lo, const double *b,
                  double *x, int32_t precond, double rtol, double inner_rtol,
                  int32_t max_outer, int32_t max_inner, int32_t *outer,
                  int32_t *inner, double *relres, const double *scale)
{
    *outer = 0;
    *inner = 0;
    *relres = 0.0;
    double bnorm = sqrt(dot(n, b, b));
    if (bnorm == 0.0) {
        for (int32_t i = 0; i < n; ++i)
            x[i] = 0.0;
        return OR_OK;
    }
    double *r64 = malloc(sizeof(double) * n);
    float *d = malloc(sizeof(float) * n), *r = malloc(sizeof(float) * n);
    float *z = malloc(sizeof(float) * n), *p = malloc(sizeof(float) * n);
    float *q = malloc(sizeof(float) * n), *dinv = malloc(sizeof(float) * n);
    int status = OR_NOT_CONVERGED;
    for (int32_t i = 0; i < n; ++i) {
        float dd = 0.0f;
        for (int32_t k = rowptr[i]; k < rowptr[i + 1]; ++k)
            if (col[k] == i)
                dd += a_lo[k];
        if (precond && (dd == 0.0f || !isfinite(dd))) {
            status = OR_ARG;
            goto done;
        }
        dinv[i] = precond ? 1.0f / dd : 1.0f;
    }
    true_residual(n, rowptr, col, val, b, x, r64);
    if (sqrt(dot(n, r64, r64)) <= rtol * bnorm) {
        status = OR_OK;
        goto done;
    }
    for (int32_t i = 0; i < n; ++i) {
        d[i] = 0.0f;
        r[i] = (float)(scale ? scale[i] * r64[i] : r64[i]);
        z[i] = dinv[i] * r[i];
        p[i] = z[i];
    }
    float rho = dotf(n, r, z);
    float tol = (float)inner_rtol * sqrtf(dotf(n, r, r));
    while (*inner < max_inner) {
        or_spmv_f32(n, rowptr, col, a_lo, p, q);
        *inner += 1;
        float gamma = dotf(n, p, q);
        if (!(gamma > 0.0f) || !isfinite(gamma)) {
            status = OR_BREAKDOWN;
            break;
        }
        float alpha = rho / gamma;
        for (int32_t i = 0; i < n; ++i) {
            d[i] += alpha * p[i];
            r[i] -= alpha * q[i];
        }
        if (sqrtf(dotf(n, r, r)) <= tol) {
            /* FP64 steps: update and residual; then rebase the inner CG */
            for (int32_t i = 0; i < n; ++i)
                x[i] += scale ? scale[i] * (double)d[i] : (double)d[i];
            *outer += 1;
            true_residual(n, rowptr, col, val, b, x, r64);
            if (sqrt(dot(n, r64, r64)) <= rtol * bnorm) {
                status = OR_OK;
                break;
            }
            if (*outer >= max_outer)
                break;
            for (int32_t i = 0; i < n; ++i) {
                d[i] = 0.0f;
                r[i] = (float)(scale ? scale[i] * r64[i] : r64[i]);
            }
            tol = (float)inner_rtol * sqrtf(dotf(n, r, r));
        }
        for (int32_t i = 0; i < n; ++i)
            z[i] = dinv[i] * r[i];
        float rho_new = dotf(n, r, z);
        float beta = rho_new / rho;
        rho = rho_new;
        for (int32_t i = 0; i < n; ++i)
            p[i] = z[i] + beta * p[i];
    }
done:
    true_residual(n, rowptr, col, val, b, x, r64);
    *relres = sqrt(dot(n, r64, r64)) / bnorm;
    free(r64); free(d); free(r); free(z); free(p); free(q); free(dinv);
    return status;
}

/* ------------------------------------------------------------------------
 * Finite-element assembly (section "Description of Current GPU Methods":
 * every global non-zero K_IJ is the sum of the element contributions
 * Ke_ab with I, J the global DOFs of local DOFs a, b; the residual R_I the
 * sum of the element entries Re_a).  Written as the classic sequential
 * element loop: entries start at 0.0 and every contribution is added when
 * its element is visited, elements in increasing order, local (a, b) in
 * row-major order.  edof[e*nde + a] < 0 marks a DOF that is not assembled.
 * The CSR position of (I, J) is found by scanning row I.
 * Returns 0, or 1 + e for the first element e that couples two DOFs whose
 * entry is missing from the pattern.
 * ---------------------------------------------------------------------- */
int64_t or_assemble_matrix(int32_t n_rows, const int32_t *rowptr,
                           const int32_t *col, int32_t n_elem, int32_t nde,
                           const int32_t *edof, const double *ke,
                           double *val)
{
    for (int32_t k = 0; k < rowptr[n_rows]; ++k)
        val[k] = 0.0;
    for (int32_t e = 0; e < n_elem; ++e) {
        const int32_t *ed = edof + (int64_t)e * nde;
        const double *K = ke + (int64_t)e * nde * nde;
        for (int32_t a = 0; a < nde; ++a) {
            const int32_t I = ed[a];
            if (I < 0)
                continue;
            for (int32_t b = 0; b < nde; ++b) {
                const int32_t J = ed[b];
                if (J < 0)
                    continue;
                int32_t k = rowptr[I];
                while (k < rowptr[I + 1] && col[k] != J)
                    ++k;
                if (k == rowptr[I + 1])
                    return 1 + (int64_t)e;
                val[k] += K[a * nde + b];
            }
        }
    }
    return 0;
}

void or_assemble_vector(int32_t n_rows, int32_t n_elem, int32_t nde,
                        const int32_t *edof, const double *re, double *r)
{
    for (int32_t i = 0; i < n_rows; ++i)
        r[i] = 0.0;
    for (int32_t e = 0; e < n_elem; ++e)
        for (int32_t a = 0; a < nde; ++a) {
            const int32_t I = edof[(int64_t)e * nde + a];
            if (I >= 0)
                r[I] += re[(int64_t)e * nde + a];
        }
}
