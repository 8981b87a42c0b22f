/* Oracle (test infrastructure): context, cases, uploads and readbacks. */
#include "orc_internal.h"
#include <math.h>
#include <stdlib.h>
#include <string.h>

orc_ctx* orc_create(void)
{
    orc_ctx* c = orc_alloc(sizeof(orc_ctx));
    return c;
}

static void case_free(ocase* cs)
{
    omesh_free(&cs->m);
    free(cs->x); free(cs->y); free(cs->u); free(cs->v); free(cs->w); free(cs->om); free(cs->wt);
    free(cs->psi); free(cs->elem); free(cs->id); free(cs->bin);
    free(cs->F); free(cs->Ffrz); free(cs->stats); free(cs->sums); free(cs->cmean); free(cs->ccount); free(cs->P); free(cs->gphi);
    free(cs);
}

void orc_destroy(orc_ctx* c)
{
    if (!c) return;
    for (int i = 0; i < c->ncase; ++i) case_free(c->cases[i]);
    free(c->cases);
    free(c);
}

const char* orc_last_error(const orc_ctx* c) { return c ? c->err : "null context"; }

static ocase* get_case(orc_ctx* c, int32_t cs)
{
    if (!c || cs < 0 || cs >= c->ncase) return NULL;
    return c->cases[cs];
}

int orc_add_case(orc_ctx* c, const orc_mesh_desc* m, const orc_params* p, int32_t* case_id)
{
    if (!c || !m || !p || !case_id) return orc_err(c, ORC_E_INVALID, "add_case: null argument");
    if (p->n_scalars < 0 || p->n_scalars > ORC_MAXS)
        return orc_err(c, ORC_E_INVALID, "add_case: n_scalars must be 0..%d", ORC_MAXS);
    if (p->n_bins != 1 && p->n_bins != 8) return orc_err(c, ORC_E_INVALID, "add_case: n_bins must be 1 or 8");
    if (p->mode < 0 || p->mode > 2) return orc_err(c, ORC_E_INVALID, "add_case: bad mode");
    if (!(p->dt > 0.0) || !(p->nu >= 0.0)) return orc_err(c, ORC_E_INVALID, "add_case: dt must be > 0, nu >= 0");
    if (!(p->n_eff_min >= 0.0)) return orc_err(c, ORC_E_INVALID, "add_case: n_eff_min must be >= 0");
    if (p->reaction < 0 || p->reaction > 2) return orc_err(c, ORC_E_INVALID, "add_case: reaction must be 0, 1 or 2");
    if (p->rebin < 0 || p->rebin > 1) return orc_err(c, ORC_E_INVALID, "add_case: rebin must be 0 or 1");
    if (p->reaction == 2 && p->n_scalars < 3)
        return orc_err(c, ORC_E_INVALID, "add_case: reaction 2 (A + B -> P) needs at least 3 scalars");
    for (int a = 0; a < ORC_MAXS; ++a)
        if (!(p->k_react[a] >= 0.0 && p->k_react[a] < 1e300))
            return orc_err(c, ORC_E_INVALID, "add_case: k_react must be finite and >= 0");
    ocase* cs = orc_alloc(sizeof(ocase));
    cs->p = *p;
    int rc = omesh_build(c, &cs->m, m);
    if (rc) { case_free(cs); return rc; }
    int nsn = cs->m.nsn, ne = cs->m.ne, ns = p->n_scalars;
    cs->F = orc_alloc(sizeof(double) * (size_t)nsn * ORC_NF);
    cs->Ffrz = orc_alloc(sizeof(double) * (size_t)nsn * ORC_NF);
    cs->stats = orc_alloc(sizeof(double) * (size_t)nsn * (12 + 2 * ns));
    cs->sums = orc_alloc(sizeof(double) * (size_t)nsn * (12 + 2 * ns));
    cs->cmean = orc_alloc(sizeof(double) * (size_t)ne * 8 * (ns > 0 ? ns : 1));
    cs->ccount = orc_alloc(sizeof(int32_t) * (size_t)ne * 8);
    cs->P = orc_alloc(sizeof(double) * nsn);
    cs->gphi = orc_alloc(sizeof(double) * (size_t)nsn * 2);
    c->cases = realloc(c->cases, sizeof(ocase*) * (c->ncase + 1));
    c->cases[c->ncase] = cs;
    *case_id = c->ncase++;
    return ORC_OK;
}

int orc_mesh_info(orc_ctx* c, int32_t ci, int32_t* n_stat_nodes, int32_t* stat_node, int32_t* nbr,
                  double* rec, double* vol)
{
    ocase* cs = get_case(c, ci);
    if (!cs) return orc_err(c, ORC_E_INVALID, "mesh_info: bad case");
    const omesh* m = &cs->m;
    if (n_stat_nodes) *n_stat_nodes = m->nsn;
    if (stat_node) for (int i = 0; i < m->nn; ++i) stat_node[i] = m->snode[i];
    if (nbr) for (int i = 0; i < 3 * m->ne; ++i) nbr[i] = m->nbr[i];
    if (rec) memcpy(rec, m->rec, sizeof(double) * 8 * (size_t)m->ne);
    if (vol) for (int i = 0; i < m->nn; ++i) vol[i] = m->vol[m->snode[i]];
    return ORC_OK;
}

int orc_particles_upload(orc_ctx* c, int32_t ci, const orc_particles* p)
{
    ocase* cs = get_case(c, ci);
    if (!cs || !p || p->n < 0) return orc_err(c, ORC_E_INVALID, "particles_upload: bad argument");
    int64_t n = p->n;
    int ns = cs->p.n_scalars;
    for (int64_t i = 0; i < n; ++i)
        if (p->elem[i] < 0 || p->elem[i] >= cs->m.ne)
            return orc_err(c, ORC_E_INVALID, "particles_upload: particle %lld has element %d", (long long)i, p->elem[i]);
    free(cs->x); free(cs->y); free(cs->u); free(cs->v); free(cs->w); free(cs->om); free(cs->wt);
    free(cs->psi); free(cs->elem); free(cs->id); free(cs->bin);
    size_t d = sizeof(double) * (size_t)n;
    cs->np = n;
    cs->x = orc_alloc(d); cs->y = orc_alloc(d); cs->u = orc_alloc(d); cs->v = orc_alloc(d);
    cs->w = orc_alloc(d); cs->om = orc_alloc(d); cs->wt = orc_alloc(d);
    cs->psi = orc_alloc(d * (ns > 0 ? ns : 1));
    cs->elem = orc_alloc(sizeof(int32_t) * (size_t)n);
    cs->id = orc_alloc(sizeof(uint32_t) * (size_t)n);
    cs->bin = orc_alloc((size_t)n);
    memcpy(cs->x, p->x, d); memcpy(cs->y, p->y, d); memcpy(cs->u, p->u, d); memcpy(cs->v, p->v, d);
    memcpy(cs->w, p->w, d); memcpy(cs->om, p->omega, d); memcpy(cs->wt, p->weight, d);
    if (ns > 0) memcpy(cs->psi, p->psi, d * ns);
    memcpy(cs->elem, p->elem, sizeof(int32_t) * (size_t)n);
    memcpy(cs->id, p->id, sizeof(uint32_t) * (size_t)n);
    if (p->bin) memcpy(cs->bin, p->bin, (size_t)n);
    return ORC_OK;
}

int orc_particles_download(orc_ctx* c, int32_t ci, orc_particles* p)
{
    ocase* cs = get_case(c, ci);
    if (!cs || !p || p->n != cs->np) return orc_err(c, ORC_E_INVALID, "particles_download: bad argument");
    size_t d = sizeof(double) * (size_t)cs->np;
    int ns = cs->p.n_scalars;
    memcpy(p->x, cs->x, d); memcpy(p->y, cs->y, d); memcpy(p->u, cs->u, d); memcpy(p->v, cs->v, d);
    memcpy(p->w, cs->w, d); memcpy(p->omega, cs->om, d); memcpy(p->weight, cs->wt, d);
    if (ns > 0 && p->psi) memcpy(p->psi, cs->psi, d * ns);
    memcpy(p->elem, cs->elem, sizeof(int32_t) * (size_t)cs->np);
    memcpy(p->id, cs->id, sizeof(uint32_t) * (size_t)cs->np);
    if (p->bin) memcpy(p->bin, cs->bin, (size_t)cs->np);
    return ORC_OK;
}

int orc_fields_upload(orc_ctx* c, int32_t ci, const double* F, uint32_t freeze_mask)
{
    ocase* cs = get_case(c, ci);
    if (!cs || !F || (freeze_mask >> ORC_NF)) return orc_err(c, ORC_E_INVALID, "fields_upload: bad argument");
    for (int s = 0; s < cs->m.nsn; ++s)
        memcpy(cs->F + (size_t)s * ORC_NF, F + (size_t)cs->m.rep[s] * ORC_NF, sizeof(double) * ORC_NF);
    memcpy(cs->Ffrz, cs->F, sizeof(double) * (size_t)cs->m.nsn * ORC_NF);
    cs->freeze = freeze_mask;
    return ORC_OK;
}

int orc_pressure_upload(orc_ctx* c, int32_t ci, const double* P)
{
    ocase* cs = get_case(c, ci);
    if (!cs || !P) return orc_err(c, ORC_E_INVALID, "pressure_upload: bad argument");
    const int nsn = cs->m.nsn;
    for (int s = 0; s < nsn; ++s) cs->P[s] = P[cs->m.rep[s]];
    double* gx = orc_alloc(sizeof(double) * nsn);
    double* gy = orc_alloc(sizeof(double) * nsn);
    orc_recover_grad(&cs->m, cs->P, gx, gy);
    for (int s = 0; s < nsn; ++s) { cs->gphi[2 * (size_t)s] = gx[s]; cs->gphi[2 * (size_t)s + 1] = gy[s]; }
    free(gx); free(gy);
    return ORC_OK;
}

int orc_fields_download(orc_ctx* c, int32_t ci, double* F)
{
    ocase* cs = get_case(c, ci);
    if (!cs || !F) return orc_err(c, ORC_E_INVALID, "fields_download: bad argument");
    for (int i = 0; i < cs->m.nn; ++i)
        memcpy(F + (size_t)i * ORC_NF, cs->F + (size_t)cs->m.snode[i] * ORC_NF, sizeof(double) * ORC_NF);
    return ORC_OK;
}

int orc_pressure_download(orc_ctx* c, int32_t ci, double* P)
{
    ocase* cs = get_case(c, ci);
    if (!cs || !P) return orc_err(c, ORC_E_INVALID, "pressure_download: bad argument");
    for (int i = 0; i < cs->m.nn; ++i) P[i] = cs->P[cs->m.snode[i]];
    return ORC_OK;
}

int orc_init(orc_ctx* c)
{
    if (!c) return ORC_E_INVALID;
    for (int i = 0; i < c->ncase; ++i) {
        int rc = orc_case_init(c, c->cases[i]);
        if (rc) return rc;
    }
    c->initialised = 1;
    return ORC_OK;
}

int orc_rebin(orc_ctx* c)
{
    if (!c) return ORC_E_INVALID;
    for (int i = 0; i < c->ncase; ++i) orc_case_rebin(c->cases[i]);
    return ORC_OK;
}

int orc_step(orc_ctx* c, int32_t n_steps)
{
    if (!c) return ORC_E_INVALID;
    if (!c->initialised) return orc_err(c, ORC_E_STATE, "step: call orc_init (or orc_rebin) first");
    for (int s = 0; s < n_steps; ++s) {
        for (int i = 0; i < c->ncase; ++i) {
            int rc = orc_case_step(c, c->cases[i], c->step);
            if (rc) return rc;
        }
        c->step++;
    }
    return ORC_OK;
}

int orc_set_step_index(orc_ctx* c, uint32_t n)
{
    if (!c) return ORC_E_INVALID;
    c->step = n;
    c->initialised = 1;
    return ORC_OK;
}

int orc_stats(orc_ctx* c, int32_t ci, double* out)
{
    ocase* cs = get_case(c, ci);
    if (!cs || !out) return orc_err(c, ORC_E_INVALID, "stats: bad argument");
    int nst = 12 + 2 * cs->p.n_scalars;
    for (int i = 0; i < cs->m.nn; ++i)
        memcpy(out + (size_t)i * nst, cs->stats + (size_t)cs->m.snode[i] * nst, sizeof(double) * nst);
    return ORC_OK;
}

int orc_node_sums(orc_ctx* c, int32_t ci, double* out)
{
    ocase* cs = get_case(c, ci);
    if (!cs || !out) return orc_err(c, ORC_E_INVALID, "node_sums: bad argument");
    int nsu = 12 + 2 * cs->p.n_scalars;
    for (int i = 0; i < cs->m.nn; ++i)
        memcpy(out + (size_t)i * nsu, cs->sums + (size_t)cs->m.snode[i] * nsu, sizeof(double) * nsu);
    return ORC_OK;
}

int orc_cell_means(orc_ctx* c, int32_t ci, double* mean, int32_t* count)
{
    ocase* cs = get_case(c, ci);
    if (!cs) return orc_err(c, ORC_E_INVALID, "cell_means: bad case");
    int ns = cs->p.n_scalars;
    if (mean && ns > 0) memcpy(mean, cs->cmean, sizeof(double) * (size_t)cs->m.ne * 8 * ns);
    if (count) memcpy(count, cs->ccount, sizeof(int32_t) * (size_t)cs->m.ne * 8);
    return ORC_OK;
}

int orc_counters(orc_ctx* c, int32_t ci, int64_t* out)
{
    ocase* cs = get_case(c, ci);
    if (!cs || !out) return orc_err(c, ORC_E_INVALID, "counters: bad argument");
    memcpy(out, cs->cnt, sizeof cs->cnt);
    return ORC_OK;
}

int orc_bary(orc_ctx* c, int32_t ci, int32_t e, double x, double y, double lam[3])
{
    ocase* cs = get_case(c, ci);
    if (!cs || e < 0 || e >= cs->m.ne) return orc_err(c, ORC_E_INVALID, "bary: bad argument");
    omesh_bary(&cs->m, e, x, y, lam);
    return ORC_OK;
}

int32_t orc_locate_brute(orc_ctx* c, int32_t ci, double x, double y)
{
    ocase* cs = get_case(c, ci);
    if (!cs) return -1;
    const omesh* m = &cs->m;
    for (int e = 0; e < m->ne; ++e) {
        double l[3];
        omesh_bary(m, e, x, y, l);
        if (l[0] >= 0.0 && l[1] >= 0.0 && l[2] >= 0.0) return e;
    }
    return -1;
}

int32_t orc_walk(orc_ctx* c, int32_t ci, int32_t e0, double* x, double* y, double* u3)
{
    ocase* cs = get_case(c, ci);
    if (!cs || e0 < 0 || e0 >= cs->m.ne) return -1;
    return orc_walk_case(cs, e0, x, y, u3);
}

static void to_stat(const omesh* m, const double* raw, double* st)
{
    for (int s = 0; s < m->nsn; ++s) st[s] = raw[m->rep[s]];
}

static void to_raw(const omesh* m, const double* st, double* raw)
{
    for (int i = 0; i < m->nn; ++i) raw[i] = st[m->snode[i]];
}

int orc_recover(orc_ctx* c, int32_t ci, const double* f, double* gx, double* gy, double* lap)
{
    ocase* cs = get_case(c, ci);
    if (!cs) return orc_err(c, ORC_E_INVALID, "recover: bad case");
    const omesh* m = &cs->m;
    int n = m->nsn;
    double* t = orc_alloc(sizeof(double) * 4 * (size_t)n);
    to_stat(m, f, t);
    orc_recover_grad(m, t, t + n, t + 2 * n);
    orc_recover_lap(m, t + n, t + 2 * n, t + 3 * n);
    if (gx) to_raw(m, t + n, gx);
    if (gy) to_raw(m, t + 2 * n, gy);
    if (lap) to_raw(m, t + 3 * n, lap);
    free(t);
    return ORC_OK;
}

int orc_fem_helmholtz(orc_ctx* c, int32_t ci, const double* L2, const double* r,
                      const int32_t* dmask, const double* dval, double tol, double* s)
{
    ocase* cs = get_case(c, ci);
    if (!cs) return orc_err(c, ORC_E_INVALID, "helmholtz: bad case");
    const omesh* m = &cs->m;
    int n = m->nsn;
    double* t = orc_alloc(sizeof(double) * 4 * (size_t)n);
    int* dm = orc_alloc(sizeof(int) * n);
    to_stat(m, L2, t); to_stat(m, r, t + n); to_stat(m, dval, t + 2 * n);
    for (int q = 0; q < n; ++q) dm[q] = dmask[m->rep[q]];
    int it = 0;
    int rc = orc_helmholtz(m, t, t + n, dm, t + 2 * n, tol, 100000, t + 3 * n, &it);
    to_raw(m, t + 3 * n, s);
    free(t); free(dm);
    return rc ? orc_err(c, 3, "helmholtz: no convergence") : ORC_OK;
}

int orc_fem_projection(orc_ctx* c, int32_t ci, const double* U1, const double* U2,
                       double dt, double tol, double* phi)
{
    ocase* cs = get_case(c, ci);
    if (!cs) return orc_err(c, ORC_E_INVALID, "projection: bad case");
    const omesh* m = &cs->m;
    int n = m->nsn;
    double* t = orc_alloc(sizeof(double) * 3 * (size_t)n);
    to_stat(m, U1, t); to_stat(m, U2, t + n);
    int it = 0;
    int rc = orc_projection(m, t, t + n, dt, tol, 100000, t + 2 * n, &it);
    to_raw(m, t + 2 * n, phi);
    free(t);
    return rc ? orc_err(c, 3, "projection: no convergence") : ORC_OK;
}

int orc_set_stats(orc_ctx* c, int32_t ci, const double* stats)
{
    ocase* cs = get_case(c, ci);
    if (!cs || !stats) return orc_err(c, ORC_E_INVALID, "set_stats: bad argument");
    int nst = 12 + 2 * cs->p.n_scalars;
    for (int s = 0; s < cs->m.nsn; ++s)
        memcpy(cs->stats + (size_t)s * nst, stats + (size_t)cs->m.rep[s] * nst, sizeof(double) * nst);
    cs->have_stats = 1;
    return ORC_OK;
}

int orc_derive(orc_ctx* c, int32_t ci, int32_t project)
{
    ocase* cs = get_case(c, ci);
    if (!cs) return orc_err(c, ORC_E_INVALID, "derive: bad case");
    return orc_derive_fields(c, cs, project != 0);
}

int orc_relax_source(const orc_params* p, const double stress[6], const double grad[6], double k, double eps,
                     const double n[2], double r[5], double dval[5], double* L2, double* Av)
{
    if (!p || !stress || !grad || !n || !r || !dval || !L2) return ORC_E_INVALID;
    double R[3][3] = {{stress[0], stress[3], stress[4]}, {stress[3], stress[1], stress[5]},
                      {stress[4], stress[5], stress[2]}};
    double dU[3][3] = {{grad[0], grad[1], 0.0}, {grad[2], grad[3], 0.0}, {grad[4], grad[5], 0.0}};
    orc_relax_node(p, R, dU, k, eps, n[0], n[1], r, dval, L2, Av);
    return ORC_OK;
}

int orc_particles_init(orc_ctx* c, int32_t ci, int32_t ppe, const orc_init_params* ip)
{
    ocase* cs = get_case(c, ci);
    if (!cs || !ip || ppe < 1) return orc_err(c, ORC_E_INVALID, "particles_init: bad argument");
    const omesh* m = &cs->m;
    const int ns = cs->p.n_scalars;
    const int64_t n = (int64_t)m->ne * ppe;
    free(cs->x); free(cs->y); free(cs->u); free(cs->v); free(cs->w); free(cs->om); free(cs->wt);
    free(cs->psi); free(cs->elem); free(cs->id); free(cs->bin);
    size_t d = sizeof(double) * (size_t)n;
    cs->np = n;
    cs->x = orc_alloc(d); cs->y = orc_alloc(d); cs->u = orc_alloc(d); cs->v = orc_alloc(d);
    cs->w = orc_alloc(d); cs->om = orc_alloc(d); cs->wt = orc_alloc(d);
    cs->psi = orc_alloc(d * (ns > 0 ? ns : 1));
    cs->elem = orc_alloc(sizeof(int32_t) * (size_t)n);
    cs->id = orc_alloc(sizeof(uint32_t) * (size_t)n);
    cs->bin = orc_alloc((size_t)n);
    for (int64_t i = 0; i < n; ++i) {
        const int e = (int)(i / ppe);
        double u[10];
        orc_init_uniforms(cs->p.seed, (uint32_t)i, cs->p.stream, u);
        /* R-29: uniform in the element */
        const int* t = m->tri + 3 * e;
        double s = sqrt(u[0]);
        double l0 = 1.0 - s, l1 = s * (1.0 - u[1]), l2 = s * u[1];
        double x = (l0 * m->x[t[0]] + l1 * m->x[t[1]]) + l2 * m->x[t[2]];
        double y = (l0 * m->y[t[0]] + l1 * m->y[t[1]]) + l2 * m->y[t[2]];
        /* R-30: Gaussian velocity components, Gamma(4, scale) frequency */
        double r0 = sqrt(-2.0 * orc_ln(u[2])), s0, c0;
        orc_sincos2pi(u[3], &s0, &c0);
        double r1 = sqrt(-2.0 * orc_ln(u[4])), s1, c1;
        orc_sincos2pi(u[5], &s1, &c1);
        cs->x[i] = x; cs->y[i] = y;
        cs->u[i] = ip->u_std * (r0 * c0);
        cs->v[i] = ip->u_std * (r0 * s0);
        cs->w[i] = ip->u_std * (r1 * c1);
        cs->om[i] = -ip->omega_scale * (((orc_ln(u[6]) + orc_ln(u[7])) + orc_ln(u[8])) + orc_ln(u[9]));
        /* R-31 mass weight, R-32 identity */
        cs->wt[i] = m->area[e] / (double)ppe;
        cs->elem[i] = e;
        cs->id[i] = (uint32_t)i;
        cs->bin[i] = 0;
        for (int a = 0; a < ns; ++a) {
            double val = 0.0;
            if (ip->disk[a][2] > 0.0) {
                double dx = x - ip->disk[a][0], dy = y - ip->disk[a][1];
                if (dx * dx + dy * dy < ip->disk[a][2] * ip->disk[a][2]) val = ip->disk[a][3];
            }
            cs->psi[(size_t)a * n + i] = val;
        }
    }
    memset(cs->cnt, 0, sizeof cs->cnt);
    return ORC_OK;
}
