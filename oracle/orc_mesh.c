/* Oracle (test infrastructure): derivation of the unstructured-mesh tables.
 *
 * The grid serves three roles in the method (Sec. I): statistics at
 * gridpoints, Eulerian solves and particle tracking. This file derives what
 * those roles need from a plain triangle list, written for clarity:
 *  - element records of the barycentric formula (R-05),
 *  - neighbours across each edge, edge k being opposite vertex k (R-04),
 *  - partner elements across periodic edges, matched by exactly equal
 *    coordinates after the shift (R-15),
 *  - statistics nodes with periodic images merged (R-33),
 *  - lumped node areas, node->element incidence, wall normals (R-19).
 */
#include "orc_internal.h"
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

int orc_err(orc_ctx* c, int code, const char* fmt, ...)
{
    if (c) {
        va_list ap; va_start(ap, fmt);
        vsnprintf(c->err, sizeof c->err, fmt, ap);
        va_end(ap);
    }
    return code;
}

void* orc_alloc(size_t n)
{
    void* p = calloc(n ? n : 1, 1);
    if (!p) { fprintf(stderr, "oracle: out of memory (%zu bytes)\n", n); abort(); }
    return p;
}

/* R-05: D = (x2-x1)(y3-y1) - (x3-x1)(y2-y1) as two products and one
 * subtraction; b_k = (y_{k+1}-y_{k+2})/D, c_k = (x_{k+2}-x_{k+1})/D. */
static double elem_record(const double* X, const double* Y, const int* v, double* rec)
{
    double x1 = X[v[0]], y1 = Y[v[0]], x2 = X[v[1]], y2 = Y[v[1]], x3 = X[v[2]], y3 = Y[v[2]];
    double p = (x2 - x1) * (y3 - y1);
    double q = (x3 - x1) * (y2 - y1);
    double D = p - q;
    double xs[3] = {x1, x2, x3}, ys[3] = {y1, y2, y3};
    rec[0] = x1; rec[1] = y1;
    for (int k = 0; k < 3; ++k) {
        int k1 = (k + 1) % 3, k2 = (k + 2) % 3;
        rec[2 + k] = (ys[k1] - ys[k2]) / D;
        rec[5 + k] = (xs[k2] - xs[k1]) / D;
    }
    return D;
}

/* R-05: lambda_k = fma(c_k, dy, fma(b_k, dx, delta_k1)), dx = x - x1, dy = y - y1 */
void omesh_bary(const omesh* m, int e, double x, double y, double lam[3])
{
    const double* r = m->rec + 8 * (size_t)e;
    double dx = x - r[0], dy = y - r[1];
    for (int k = 0; k < 3; ++k)
        lam[k] = fma(r[5 + k], dy, fma(r[2 + k], dx, k == 0 ? 1.0 : 0.0));
}

typedef struct { int a, b, e, k; } edge_t;

static int edge_cmp(const void* pa, const void* pb)
{
    const edge_t* A = pa; const edge_t* B = pb;
    int a0 = A->a < A->b ? A->a : A->b, a1 = A->a < A->b ? A->b : A->a;
    int b0 = B->a < B->b ? B->a : B->b, b1 = B->a < B->b ? B->b : B->a;
    if (a0 != b0) return a0 < b0 ? -1 : 1;
    if (a1 != b1) return a1 < b1 ? -1 : 1;
    if (A->e != B->e) return A->e < B->e ? -1 : 1;
    return A->k - B->k;
}

static int same_edge(const edge_t* A, const edge_t* B)
{
    int a0 = A->a < A->b ? A->a : A->b, a1 = A->a < A->b ? A->b : A->a;
    int b0 = B->a < B->b ? B->a : B->b, b1 = B->a < B->b ? B->b : B->a;
    return a0 == b0 && a1 == b1;
}

static int uf_find(int* par, int i)
{
    while (par[i] != i) i = par[i];
    return i;
}

static void uf_union(int* par, int i, int j)
{
    int a = uf_find(par, i), b = uf_find(par, j);
    if (a == b) return;
    if (a < b) par[b] = a; else par[a] = b;   /* lowest raw id represents the class */
}

int omesh_build(orc_ctx* c, omesh* m, const orc_mesh_desc* d)
{
    memset(m, 0, sizeof *m);
    if (!d || d->n_nodes < 3 || d->n_elems < 1 || !d->xy || !d->tri || !d->edge_tag)
        return orc_err(c, ORC_E_INVALID, "mesh: missing arrays or empty mesh");
    if (d->n_bc < 0 || (d->n_bc > 0 && !d->bc))
        return orc_err(c, ORC_E_INVALID, "mesh: bad boundary table");
    int nn = d->n_nodes, ne = d->n_elems;
    m->nn = nn; m->ne = ne; m->nbc = d->n_bc;
    m->x = orc_alloc(sizeof(double) * nn); m->y = orc_alloc(sizeof(double) * nn);
    for (int i = 0; i < nn; ++i) { m->x[i] = d->xy[2 * i]; m->y[i] = d->xy[2 * i + 1]; }
    m->tri = orc_alloc(sizeof(int) * 3 * ne); m->tag = orc_alloc(sizeof(int) * 3 * ne);
    m->bc = orc_alloc(sizeof(orc_bc) * (d->n_bc + 1));
    memcpy(m->bc, d->bc, sizeof(orc_bc) * d->n_bc);
    for (int i = 0; i < 3 * ne; ++i) {
        m->tri[i] = d->tri[i]; m->tag[i] = d->edge_tag[i];
        if (m->tri[i] < 0 || m->tri[i] >= nn)
            return orc_err(c, ORC_E_MESH, "mesh: element %d references node %d", i / 3, m->tri[i]);
        if (m->tag[i] < -1 || m->tag[i] >= d->n_bc)
            return orc_err(c, ORC_E_MESH, "mesh: element %d edge %d has tag %d", i / 3, i % 3, m->tag[i]);
    }
    for (int b = 0; b < d->n_bc; ++b)
        if (m->bc[b].type != ORC_BC_WALL && m->bc[b].type != ORC_BC_PERIODIC)
            return orc_err(c, ORC_E_MESH, "mesh: boundary %d has unknown type", b);

    /* element records and positivity */
    m->rec = orc_alloc(sizeof(double) * 8 * ne);
    m->area = orc_alloc(sizeof(double) * ne);
    for (int e = 0; e < ne; ++e) {
        double D = elem_record(m->x, m->y, m->tri + 3 * e, m->rec + 8 * e);
        if (!(D > 0.0))
            return orc_err(c, ORC_E_MESH, "mesh: element %d is not counter-clockwise (D=%g)", e, D);
        m->area[e] = 0.5 * D;
    }

    /* neighbours: pair up the edges sharing the same two vertices */
    edge_t* E = orc_alloc(sizeof(edge_t) * 3 * ne);
    for (int e = 0; e < ne; ++e)
        for (int k = 0; k < 3; ++k) {
            edge_t* t = E + 3 * e + k;
            t->a = m->tri[3 * e + (k + 1) % 3]; t->b = m->tri[3 * e + (k + 2) % 3];
            t->e = e; t->k = k;
        }
    qsort(E, 3 * (size_t)ne, sizeof(edge_t), edge_cmp);
    m->nbr = orc_alloc(sizeof(int) * 3 * ne);
    m->partner = orc_alloc(sizeof(int) * 3 * ne);
    for (int i = 0; i < 3 * ne; ++i) { m->nbr[i] = -1; m->partner[i] = -1; }
    int rc = ORC_OK;
    for (int i = 0; i < 3 * ne && rc == ORC_OK;) {
        int j = i + 1;
        while (j < 3 * ne && same_edge(&E[i], &E[j])) ++j;
        int cnt = j - i;
        if (cnt == 1) {
            if (m->tag[3 * E[i].e + E[i].k] < 0)
                rc = orc_err(c, ORC_E_MESH, "mesh: boundary edge of element %d has no tag", E[i].e);
        } else if (cnt == 2) {
            const edge_t *P = &E[i], *Q = &E[i + 1];
            if (P->a != Q->b || P->b != Q->a)
                rc = orc_err(c, ORC_E_MESH, "mesh: inconsistent orientation at elements %d,%d", P->e, Q->e);
            else if (m->tag[3 * P->e + P->k] >= 0 || m->tag[3 * Q->e + Q->k] >= 0)
                rc = orc_err(c, ORC_E_MESH, "mesh: interior edge of element %d carries a boundary tag", P->e);
            m->nbr[3 * P->e + P->k] = Q->e;
            m->nbr[3 * Q->e + Q->k] = P->e;
        } else {
            rc = orc_err(c, ORC_E_MESH, "mesh: non-manifold edge (%d elements)", cnt);
        }
        i = j;
    }
    free(E);
    if (rc) return rc;

    /* periodic partners, by exact coordinate match after the shift (R-15) */
    int* par = orc_alloc(sizeof(int) * nn);
    for (int i = 0; i < nn; ++i) par[i] = i;
    for (int e = 0; e < ne; ++e)
        for (int k = 0; k < 3; ++k) {
            int t = m->tag[3 * e + k];
            if (t < 0 || m->bc[t].type != ORC_BC_PERIODIC) continue;
            int a = m->tri[3 * e + (k + 1) % 3], b = m->tri[3 * e + (k + 2) % 3];
            double sx = m->bc[t].shift[0], sy = m->bc[t].shift[1];
            double ax = m->x[a] + sx, ay = m->y[a] + sy, bx = m->x[b] + sx, by = m->y[b] + sy;
            int found = -1, fk = -1;
            for (int e2 = 0; e2 < ne && found < 0; ++e2)
                for (int k2 = 0; k2 < 3; ++k2) {
                    int t2 = m->tag[3 * e2 + k2];
                    if (t2 < 0 || m->bc[t2].type != ORC_BC_PERIODIC) continue;
                    int a2 = m->tri[3 * e2 + (k2 + 1) % 3], b2 = m->tri[3 * e2 + (k2 + 2) % 3];
                    if (m->x[a2] == bx && m->y[a2] == by && m->x[b2] == ax && m->y[b2] == ay) {
                        if (m->bc[t2].shift[0] != -sx || m->bc[t2].shift[1] != -sy) {
                            free(par);
                            return orc_err(c, ORC_E_MESH, "mesh: periodic shifts of boundaries %d and %d are not opposite", t, t2);
                        }
                        found = e2; fk = k2; break;
                    }
                }
            if (found < 0) {
                free(par);
                return orc_err(c, ORC_E_MESH, "mesh: periodic edge of element %d has no partner", e);
            }
            m->partner[3 * e + k] = found;
            uf_union(par, a, m->tri[3 * found + (fk + 2) % 3]);
            uf_union(par, b, m->tri[3 * found + (fk + 1) % 3]);
        }

    /* statistics nodes: one per class of periodic images (R-33) */
    m->snode = orc_alloc(sizeof(int) * nn);
    m->rep = orc_alloc(sizeof(int) * nn);
    m->nsn = 0;
    for (int i = 0; i < nn; ++i) {
        int r = uf_find(par, i);
        if (r == i) { m->snode[i] = m->nsn; m->rep[m->nsn] = i; m->nsn++; }
    }
    for (int i = 0; i < nn; ++i) m->snode[i] = m->snode[uf_find(par, i)];
    free(par);
    int nsn = m->nsn;
    m->tri_s = orc_alloc(sizeof(int) * 3 * ne);
    m->vol = orc_alloc(sizeof(double) * nsn);
    for (int e = 0; e < ne; ++e)
        for (int k = 0; k < 3; ++k) {
            int s = m->snode[m->tri[3 * e + k]];
            m->tri_s[3 * e + k] = s;
            m->vol[s] += m->area[e] / 3.0;
        }
    /* incidence lists, in increasing (element, vertex) order */
    m->inc_ptr = orc_alloc(sizeof(int) * (nsn + 1));
    for (int i = 0; i < 3 * ne; ++i) m->inc_ptr[m->tri_s[i] + 1]++;
    for (int s = 0; s < nsn; ++s) m->inc_ptr[s + 1] += m->inc_ptr[s];
    m->inc = orc_alloc(sizeof(int) * 3 * ne);
    int* fill = orc_alloc(sizeof(int) * nsn);
    for (int i = 0; i < 3 * ne; ++i) {
        int s = m->tri_s[i];
        m->inc[m->inc_ptr[s] + fill[s]++] = i;
    }
    free(fill);

    /* wall nodes and their normals: normalised sum of the outward unit
     * normals of the adjacent wall edges (R-19) */
    m->is_wall = orc_alloc(sizeof(int) * nsn);
    m->wnx = orc_alloc(sizeof(double) * nsn);
    m->wny = orc_alloc(sizeof(double) * nsn);
    for (int e = 0; e < ne; ++e)
        for (int k = 0; k < 3; ++k) {
            int t = m->tag[3 * e + k];
            if (t < 0 || m->bc[t].type != ORC_BC_WALL) continue;
            int a = m->tri[3 * e + (k + 1) % 3], b = m->tri[3 * e + (k + 2) % 3];
            double dx = m->x[b] - m->x[a], dy = m->y[b] - m->y[a];
            double L = sqrt(dx * dx + dy * dy);
            int ends[2] = {m->snode[a], m->snode[b]};
            for (int q = 0; q < 2; ++q) {
                m->is_wall[ends[q]] = 1;
                m->wnx[ends[q]] += dy / L;
                m->wny[ends[q]] += -dx / L;
            }
        }
    for (int s = 0; s < nsn; ++s)
        if (m->is_wall[s]) {
            double L = sqrt(m->wnx[s] * m->wnx[s] + m->wny[s] * m->wny[s]);
            m->wnx[s] /= L; m->wny[s] /= L;
        }
    return ORC_OK;
}

void omesh_free(omesh* m)
{
    free(m->x); free(m->y); free(m->tri); free(m->tag); free(m->bc); free(m->nbr);
    free(m->partner); free(m->snode); free(m->rep); free(m->tri_s); free(m->rec);
    free(m->area); free(m->vol); free(m->inc_ptr); free(m->inc); free(m->is_wall);
    free(m->wnx); free(m->wny);
    memset(m, 0, sizeof *m);
}
