/*
 * Oracle for the PSD-cone projection: TEST INFRASTRUCTURE ONLY.
 *
 * Only tests/, __graft_entry__.smoke() and bench.py's cpu_baseline leg may
 * load this library.  It shares no code, header, table or helper with the GPU
 * library; the product path never calls it.
 *
 * What it computes is the plain definition of the projection (paper §1,
 * definition of the projection and eq. `projection`):
 *
 *     Pi(X) = argmin_{Y psd} ||X - Y||_F = Q diag(max(lambda, 0)) Q^T
 *
 * where X = Q diag(lambda) Q^T is the full eigendecomposition of X.  The
 * eigendecomposition is the textbook two-sided cyclic Jacobi method
 * (Golub & Van Loan, Matrix Computations, §8.5, which the paper cites for the
 * cost of eigendecomposition in §1), in FP64, with the rotation formulas of
 * the symmetric 2x2 Schur decomposition (same section).  Pairs are visited
 * in round-robin ("tournament") order so that the n/2 rotations of one round
 * touch disjoint index pairs and can run in parallel under OpenMP; this is
 * the parallel-ordering variant that the same section describes, and it does
 * not change what is computed.
 *
 * Input convention: the LOWER triangle of X (column-major, leading dimension
 * ldx) is read, like LAPACK uplo='L'.  All outputs are column-major.
 *
 * Return codes: 0 ok, 1 no convergence within ORACLE_MAX_SWEEPS sweeps,
 * 2 invalid argument, 3 out of memory, 4 non-finite input.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORACLE_MAX_SWEEPS 60

/* Rotation (c, s) that annihilates a_pq of the symmetric 2x2 block
 * [[app, apq], [apq, aqq]] under J^T A J with J = [[c, s], [-s, c]]
 * on rows/columns (p, q).  Golub & Van Loan, symmetric 2x2 Schur. */
static void sym_schur2(double app, double apq, double aqq, double *c, double *s)
{
    if (apq == 0.0) { *c = 1.0; *s = 0.0; return; }
    double tau = (aqq - app) / (2.0 * apq);
    double t;
    if (fabs(tau) > 1e150) {
        /* 1/(|tau| + sqrt(1 + tau^2)) ~ 1/(2|tau|) without overflow */
        t = 1.0 / (2.0 * tau);
    } else if (tau >= 0.0) {
        t = 1.0 / (tau + sqrt(1.0 + tau * tau));
    } else {
        t = -1.0 / (-tau + sqrt(1.0 + tau * tau));
    }
    *c = 1.0 / sqrt(1.0 + t * t);
    *s = t * (*c);
}

/* Round-robin schedule: N players (N even), round r in [0, N-2], slot k in
 * [0, N/2-1].  Slot 0 pairs the fixed player N-1 with r; slot k>0 pairs
 * (r+k) mod (N-1) with (r-k) mod (N-1).  Every pair meets once per sweep. */
static void rr_pair(int N, int r, int k, int *p, int *q)
{
    int a, b;
    if (k == 0) { a = r; b = N - 1; }
    else {
        a = (r + k) % (N - 1);
        b = ((r - k) % (N - 1) + (N - 1)) % (N - 1);
    }
    if (a < b) { *p = a; *q = b; } else { *p = b; *q = a; }
}

static double off_norm2(int n, const double *A, int lda)
{
    double s = 0.0;
    for (int j = 0; j < n; ++j)
        for (int i = 0; i < n; ++i)
            if (i != j) s += A[i + (size_t)j * lda] * A[i + (size_t)j * lda];
    return s;
}

/*
 * Full eigendecomposition of the symmetric matrix whose lower triangle is X.
 * lam[n]: eigenvalues, ascending.  V (n x n, ldv): orthonormal eigenvectors,
 * column i belongs to lam[i].  sweeps_out (may be NULL): sweeps used.
 */
int oracle_eigh(int n, const double *X, int ldx, double *lam, double *V, int ldv,
                int *sweeps_out)
{
    if (n < 0 || ldx < (n > 0 ? n : 1) || ldv < (n > 0 ? n : 1)) return 2;
    if (n == 0) { if (sweeps_out) *sweeps_out = 0; return 0; }
    if (!X || !lam || !V) return 2;

    int lda = n;
    double *A = (double *)malloc(sizeof(double) * (size_t)n * n);
    double *cs = NULL;
    int *pq = NULL;
    int N = (n % 2 == 0) ? n : n + 1;
    int npairs = N / 2;
    if (!A) return 3;
    cs = (double *)malloc(sizeof(double) * 2 * (size_t)npairs);
    pq = (int *)malloc(sizeof(int) * 2 * (size_t)npairs);
    if (!cs || !pq) { free(A); free(cs); free(pq); return 3; }

    /* symmetric copy from the lower triangle; V = I */
    for (int j = 0; j < n; ++j)
        for (int i = j; i < n; ++i) {
            double x = X[i + (size_t)j * ldx];
            if (!isfinite(x)) { free(A); free(cs); free(pq); return 4; }
            A[i + (size_t)j * lda] = x;
            A[j + (size_t)i * lda] = x;
        }
    for (int j = 0; j < n; ++j)
        for (int i = 0; i < n; ++i) V[i + (size_t)j * ldv] = (i == j) ? 1.0 : 0.0;

    double fro2 = 0.0;
    for (int j = 0; j < n; ++j)
        for (int i = 0; i < n; ++i) fro2 += A[i + (size_t)j * lda] * A[i + (size_t)j * lda];
    double fro = sqrt(fro2);
    /* stop once the off-diagonal mass is below 1e-15 of ||A||_F */
    double stop2 = (1e-15 * fro) * (1e-15 * fro);
    /* entries below this are left alone (they are under the rounding level
       of the largest entries and rotating them changes nothing measurable) */
    double skip = 1e-18 * fro;

    int sweep = 0, rc = 1;
    int par = (n >= 96);
    if (n == 1 || off_norm2(n, A, lda) <= stop2) rc = 0;
    for (sweep = 0; rc != 0 && sweep < ORACLE_MAX_SWEEPS; ++sweep) {
        for (int r = 0; r < N - 1; ++r) {
            /* 1. rotation parameters for the n/2 disjoint pairs of this round */
            for (int k = 0; k < npairs; ++k) {
                int p, q;
                rr_pair(N, r, k, &p, &q);
                pq[2 * k] = p; pq[2 * k + 1] = q;
                if (q >= n) { cs[2 * k] = 1.0; cs[2 * k + 1] = 0.0; continue; }
                double apq = A[p + (size_t)q * lda];
                if (fabs(apq) <= skip) { cs[2 * k] = 1.0; cs[2 * k + 1] = 0.0; continue; }
                sym_schur2(A[p + (size_t)p * lda], apq, A[q + (size_t)q * lda],
                           &cs[2 * k], &cs[2 * k + 1]);
            }
            /* 2. columns: A <- A J and V <- V J (pairs are disjoint) */
#pragma omp parallel for schedule(static) if (par)
            for (int k = 0; k < npairs; ++k) {
                int p = pq[2 * k], q = pq[2 * k + 1];
                double c = cs[2 * k], s = cs[2 * k + 1];
                if (q >= n || s == 0.0) continue;
                double *ap = A + (size_t)p * lda, *aq = A + (size_t)q * lda;
                double *vp = V + (size_t)p * ldv, *vq = V + (size_t)q * ldv;
                for (int i = 0; i < n; ++i) {
                    double x = ap[i], y = aq[i];
                    ap[i] = c * x - s * y;
                    aq[i] = s * x + c * y;
                    double u = vp[i], w = vq[i];
                    vp[i] = c * u - s * w;
                    vq[i] = s * u + c * w;
                }
            }
            /* 3. rows: A <- J^T A, one column at a time */
#pragma omp parallel for schedule(static) if (par)
            for (int j = 0; j < n; ++j) {
                double *aj = A + (size_t)j * lda;
                for (int k = 0; k < npairs; ++k) {
                    int p = pq[2 * k], q = pq[2 * k + 1];
                    double c = cs[2 * k], s = cs[2 * k + 1];
                    if (q >= n || s == 0.0) continue;
                    double x = aj[p], y = aj[q];
                    aj[p] = c * x - s * y;
                    aj[q] = s * x + c * y;
                }
            }
            /* 4. the annihilated entries are zero by construction */
            for (int k = 0; k < npairs; ++k) {
                int p = pq[2 * k], q = pq[2 * k + 1];
                if (q >= n || cs[2 * k + 1] == 0.0) continue;
                A[p + (size_t)q * lda] = 0.0;
                A[q + (size_t)p * lda] = 0.0;
            }
        }
        if (off_norm2(n, A, lda) <= stop2) { rc = 0; ++sweep; break; }
    }
    if (sweeps_out) *sweeps_out = sweep;

    /* eigenvalues = diag(A); sort ascending, permuting the columns of V */
    int *idx = (int *)malloc(sizeof(int) * (size_t)n);
    double *d = (double *)malloc(sizeof(double) * (size_t)n);
    double *Vt = (double *)malloc(sizeof(double) * (size_t)n * n);
    if (!idx || !d || !Vt) { free(A); free(cs); free(pq); free(idx); free(d); free(Vt); return 3; }
    for (int i = 0; i < n; ++i) { d[i] = A[i + (size_t)i * lda]; idx[i] = i; }
    /* insertion sort on (value, original index): stable and O(n^2) worst case */
    for (int i = 1; i < n; ++i) {
        int t = idx[i], j = i - 1;
        while (j >= 0 && d[idx[j]] > d[t]) { idx[j + 1] = idx[j]; --j; }
        idx[j + 1] = t;
    }
    for (int j = 0; j < n; ++j) {
        lam[j] = d[idx[j]];
        memcpy(Vt + (size_t)j * n, V + (size_t)idx[j] * ldv, sizeof(double) * (size_t)n);
    }
    for (int j = 0; j < n; ++j)
        memcpy(V + (size_t)j * ldv, Vt + (size_t)j * n, sizeof(double) * (size_t)n);
    free(idx); free(d); free(Vt);
    free(A); free(cs); free(pq);
    return rc;
}

/*
 * Exact projection Pi = V diag(max(lam, 0)) V^T, both triangles written and
 * symmetrized, plus all eigenvalues (ascending) in lam (may be NULL).
 */
int oracle_project(int n, const double *X, int ldx, double *Pi, int ldpi, double *lam)
{
    if (n < 0 || ldpi < (n > 0 ? n : 1) || ldx < (n > 0 ? n : 1)) return 2;
    if (n == 0) return 0;
    if (!Pi) return 2;
    double *w = (double *)malloc(sizeof(double) * (size_t)n);
    double *V = (double *)malloc(sizeof(double) * (size_t)n * n);
    if (!w || !V) { free(w); free(V); return 3; }
    int rc = oracle_eigh(n, X, ldx, w, V, n, NULL);
    if (rc == 0 || rc == 1) {
        /* Pi_ij = sum_k max(lam_k, 0) v_ik v_jk */
#pragma omp parallel for schedule(dynamic, 8) if (n >= 96)
        for (int j = 0; j < n; ++j) {
            double *pj = Pi + (size_t)j * ldpi;
            for (int i = 0; i < n; ++i) pj[i] = 0.0;
            for (int k = 0; k < n; ++k) {
                if (!(w[k] > 0.0)) continue;
                const double *vk = V + (size_t)k * n;
                double a = w[k] * vk[j];
                for (int i = 0; i < n; ++i) pj[i] += a * vk[i];
            }
        }
        for (int j = 0; j < n; ++j)
            for (int i = j + 1; i < n; ++i) {
                double a = 0.5 * (Pi[i + (size_t)j * ldpi] + Pi[j + (size_t)i * ldpi]);
                Pi[i + (size_t)j * ldpi] = a;
                Pi[j + (size_t)i * ldpi] = a;
            }
        if (lam) memcpy(lam, w, sizeof(double) * (size_t)n);
    }
    free(w); free(V);
    return rc;
}

/* Threads OpenMP will use for the parallel regions above. */
int oracle_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
