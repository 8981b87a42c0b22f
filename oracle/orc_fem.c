/* Oracle (test infrastructure): the Eulerian solves on the grid (Sec. I,
 * role (ii)): Galerkin P1 elliptic relaxation (R-19) and the pressure
 * projection (R-27), each solved by a plain Jacobi-preconditioned conjugate
 * gradient method to a tight tolerance (R-28).
 *
 * Element matrices (linear triangle, area A, shape gradients (b_k, c_k)):
 *   mass      M_e[a][b] = A/12 (1 + delta_ab)
 *   stiffness K_e[a][b] = A (b_a b_b + c_a c_b)
 */
#include "orc_internal.h"
#include <math.h>
#include <stdlib.h>
#include <string.h>

typedef struct { int n; int* ptr; int* col; double* val; } csr;

static void csr_pattern(const omesh* m, csr* A)
{
    int n = m->nsn;
    A->n = n;
    A->ptr = orc_alloc(sizeof(int) * (n + 1));
    int* tmp = orc_alloc(sizeof(int) * 64);
    int cap = 64;
    /* count */
    int total = 0;
    int** rows = orc_alloc(sizeof(int*) * n);
    int* rlen = orc_alloc(sizeof(int) * n);
    for (int s = 0; s < n; ++s) {
        int len = 0;
        for (int j = m->inc_ptr[s]; j < m->inc_ptr[s + 1]; ++j) {
            int e = m->inc[j] / 3;
            for (int k = 0; k < 3; ++k) {
                int t = m->tri_s[3 * e + k], dup = 0;
                for (int q = 0; q < len; ++q) if (tmp[q] == t) { dup = 1; break; }
                if (!dup) {
                    if (len == cap) { cap *= 2; tmp = realloc(tmp, sizeof(int) * cap); }
                    tmp[len++] = t;
                }
            }
        }
        /* sort the row */
        for (int a = 1; a < len; ++a) {
            int v = tmp[a], b = a - 1;
            while (b >= 0 && tmp[b] > v) { tmp[b + 1] = tmp[b]; --b; }
            tmp[b + 1] = v;
        }
        rows[s] = orc_alloc(sizeof(int) * len);
        memcpy(rows[s], tmp, sizeof(int) * len);
        rlen[s] = len;
        total += len;
    }
    A->col = orc_alloc(sizeof(int) * total);
    A->val = orc_alloc(sizeof(double) * total);
    for (int s = 0; s < n; ++s) {
        A->ptr[s + 1] = A->ptr[s] + rlen[s];
        memcpy(A->col + A->ptr[s], rows[s], sizeof(int) * rlen[s]);
        free(rows[s]);
    }
    free(rows); free(rlen); free(tmp);
}

static void csr_add(csr* A, int r, int cidx, double v)
{
    for (int j = A->ptr[r]; j < A->ptr[r + 1]; ++j)
        if (A->col[j] == cidx) { A->val[j] += v; return; }
}

static void csr_free(csr* A) { free(A->ptr); free(A->col); free(A->val); }

static void matvec(const csr* A, const double* x, double* y)
{
    for (int i = 0; i < A->n; ++i) {
        double s = 0.0;
        for (int j = A->ptr[i]; j < A->ptr[i + 1]; ++j) s += A->val[j] * x[A->col[j]];
        y[i] = s;
    }
}

static double dot(int n, const double* a, const double* b)
{
    double s = 0.0;
    for (int i = 0; i < n; ++i) s += a[i] * b[i];
    return s;
}

/* Jacobi-preconditioned CG from x = 0; stops at ||r|| <= tol ||b||.
 * If mean_free, the iterate and residual are kept orthogonal to constants
 * (singular Neumann/periodic operator). Returns 0 on convergence. */
static int pcg(const csr* A, const double* b, double tol, int maxit, int mean_free, double* x, int* iters)
{
    int n = A->n;
    double* r = orc_alloc(sizeof(double) * n);
    double* z = orc_alloc(sizeof(double) * n);
    double* p = orc_alloc(sizeof(double) * n);
    double* q = orc_alloc(sizeof(double) * n);
    double* dinv = orc_alloc(sizeof(double) * n);
    for (int i = 0; i < n; ++i) {
        double d = 0.0;
        for (int j = A->ptr[i]; j < A->ptr[i + 1]; ++j) if (A->col[j] == i) d = A->val[j];
        dinv[i] = 1.0 / d;
        x[i] = 0.0;
        r[i] = b[i];
    }
    double bn = sqrt(dot(n, b, b));
    int it = 0, ok = 0;
    if (bn == 0.0) ok = 1;
    for (int i = 0; i < n; ++i) z[i] = dinv[i] * r[i];
    memcpy(p, z, sizeof(double) * n);
    double rz = dot(n, r, z);
    while (!ok && it < maxit) {
        if (sqrt(dot(n, r, r)) <= tol * bn) { ok = 1; break; }
        matvec(A, p, q);
        double alpha = rz / dot(n, p, q);
        for (int i = 0; i < n; ++i) { x[i] += alpha * p[i]; r[i] -= alpha * q[i]; }
        if (mean_free) {
            double mr = 0.0;
            for (int i = 0; i < n; ++i) mr += r[i];
            mr /= n;
            for (int i = 0; i < n; ++i) r[i] -= mr;
        }
        for (int i = 0; i < n; ++i) z[i] = dinv[i] * r[i];
        double rz2 = dot(n, r, z);
        double beta = rz2 / rz;
        rz = rz2;
        for (int i = 0; i < n; ++i) p[i] = z[i] + beta * p[i];
        ++it;
    }
    if (!ok && sqrt(dot(n, r, r)) <= tol * bn) ok = 1;
    if (mean_free) {
        double mx = 0.0;
        for (int i = 0; i < n; ++i) mx += x[i];
        mx /= n;
        for (int i = 0; i < n; ++i) x[i] -= mx;
    }
    *iters = it;
    free(r); free(z); free(p); free(q); free(dinv);
    return ok ? 0 : 1;
}

int orc_helmholtz(const omesh* m, const double* L2, const double* rn, const int* dmask,
                  const double* dval, double tol, int maxit, double* s, int* iters)
{
    int n = m->nsn;
    csr A;
    csr_pattern(m, &A);
    double* b = orc_alloc(sizeof(double) * n);
    for (int e = 0; e < m->ne; ++e) {
        const int* t = m->tri_s + 3 * e;
        const double* rc = m->rec + 8 * (size_t)e;
        double Ae = m->area[e];
        double L2e = ((L2[t[0]] + L2[t[1]]) + L2[t[2]]) / 3.0;
        for (int a = 0; a < 3; ++a)
            for (int c = 0; c < 3; ++c) {
                double Mab = Ae / 12.0 * (a == c ? 2.0 : 1.0);
                double Kab = Ae * (rc[2 + a] * rc[2 + c] + rc[5 + a] * rc[5 + c]);
                csr_add(&A, t[a], t[c], Mab + L2e * Kab);
                b[t[a]] += Mab * rn[t[c]];
            }
    }
    /* Dirichlet rows: identity; known values moved to the right-hand side */
    for (int i = 0; i < n; ++i) {
        if (dmask[i]) continue;
        for (int j = A.ptr[i]; j < A.ptr[i + 1]; ++j)
            if (dmask[A.col[j]]) { b[i] -= A.val[j] * dval[A.col[j]]; A.val[j] = 0.0; }
    }
    for (int i = 0; i < n; ++i) {
        if (!dmask[i]) continue;
        for (int j = A.ptr[i]; j < A.ptr[i + 1]; ++j) A.val[j] = (A.col[j] == i) ? 1.0 : 0.0;
        b[i] = dval[i];
    }
    int rc = pcg(&A, b, tol, maxit, 0, s, iters);
    free(b);
    csr_free(&A);
    return rc;
}

int orc_projection(const omesh* m, const double* U1, const double* U2, double dt,
                   double tol, int maxit, double* phi, int* iters)
{
    int n = m->nsn;
    csr A;
    csr_pattern(m, &A);
    double* b = orc_alloc(sizeof(double) * n);
    for (int e = 0; e < m->ne; ++e) {
        const int* t = m->tri_s + 3 * e;
        const double* rc = m->rec + 8 * (size_t)e;
        double Ae = m->area[e];
        double ue = ((U1[t[0]] + U1[t[1]]) + U1[t[2]]) / 3.0;
        double ve = ((U2[t[0]] + U2[t[1]]) + U2[t[2]]) / 3.0;
        for (int a = 0; a < 3; ++a) {
            for (int c = 0; c < 3; ++c)
                csr_add(&A, t[a], t[c], Ae * (rc[2 + a] * rc[2 + c] + rc[5 + a] * rc[5 + c]));
            b[t[a]] += Ae * (rc[2 + a] * ue + rc[5 + a] * ve) / dt;
        }
    }
    double mb = 0.0;
    for (int i = 0; i < n; ++i) mb += b[i];
    mb /= n;
    for (int i = 0; i < n; ++i) b[i] -= mb;
    int rc = pcg(&A, b, tol, maxit, 1, phi, iters);
    free(b);
    csr_free(&A);
    return rc;
}
