/* Oracle (test infrastructure): one forward-Euler time step of the particle
 * system, written as the plain definition, one particle at a time in index
 * order, followed by the grid statistics and the Eulerian fields.
 *
 * Order within a step (R-08): interpolate F^n at X^n -> IECM mixing with the
 * cell means of state n -> velocity, position and frequency increments ->
 * walk with boundary conditions -> concentrated sources -> node statistics of
 * state n+1 -> velocity bins against F^n -> cell means -> derived fields,
 * elliptic relaxation and projection -> F^{n+1}.
 */
#include "orc_internal.h"
#include <math.h>
#include <stdlib.h>
#include <string.h>

static int nstat_of(const ocase* cs) { return 12 + 2 * cs->p.n_scalars; }
static int nsum_of(const ocase* cs) { return 12 + 2 * cs->p.n_scalars; }

/* R-06: f = fma(l3, f3, fma(l2, f2, l1*f1)) for every field slot */
static void interpolate(const ocase* cs, int e, const double lam[3], double f[ORC_NF])
{
    const int* s = cs->m.tri_s + 3 * e;
    const double *F0 = cs->F + (size_t)s[0] * ORC_NF, *F1 = cs->F + (size_t)s[1] * ORC_NF,
                 *F2 = cs->F + (size_t)s[2] * ORC_NF;
    for (int q = 0; q < ORC_NF; ++q) f[q] = fma(lam[2], F2[q], fma(lam[1], F1[q], lam[0] * F0[q]));
}

/* One particle, Eq.(2), (4), (5) and (9) by forward Euler (R-03). */
/* Closed reaction source S_alpha(psi) of the scalar equation, Eq.(8)-(9),
 * for particle p (R-35): first-order decay, or A + B -> P with the rate
 * k_0 psi_A psi_B consuming A and B and producing P. */
static void reaction_source(const orc_params* P, const double* psi, int64_t np, int64_t p, double S[ORC_MAXS])
{
    const int ns = P->n_scalars;
    if (P->reaction == 1) {
        for (int a = 0; a < ns; ++a) S[a] = -P->k_react[a] * psi[(size_t)a * np + p];
    } else if (P->reaction == 2) {
        double r = P->k_react[0] * psi[p] * psi[(size_t)np + p];
        S[0] = -r;
        S[1] = -r;
        S[2] = r;
    }
}

static void advance_particle(ocase* cs, int64_t p, uint32_t n)
{
    const orc_params* P = &cs->p;
    const omesh* m = &cs->m;
    const int ns = P->n_scalars;
    const double dt = P->dt;
    int e = cs->elem[p];
    double lam[3], f[ORC_NF], xi[6];
    omesh_bary(m, e, cs->x[p], cs->y[p], lam);
    interpolate(cs, e, lam, f);
    orc_gauss6(P->seed, cs->id[p], n, P->stream, xi);

    /* Eq.(9), IECM plus the closed reaction source, forward Euler:
     * psi <- psi - (dt/t_m)(psi - <phi|V>) + dt S(psi), with the cell
     * estimate of the conditional mean (R-23), 1/t_m = Cphi/2 <omega>_e
     * (R-24), and S evaluated on the composition before the step (R-35) */
    if (ns > 0) {
        double S[ORC_MAXS] = {0.0, 0.0, 0.0, 0.0};
        reaction_source(P, cs->psi, cs->np, p, S);
        const int* s = m->tri_s + 3 * e;
        double om_e = ((cs->F[(size_t)s[0] * ORC_NF + F_OMEGA] + cs->F[(size_t)s[1] * ORC_NF + F_OMEGA])
                       + cs->F[(size_t)s[2] * ORC_NF + F_OMEGA]) / 3.0;
        double fm = dt * ((0.5 * P->Cphi) * om_e);
        if (fm > 1.0) fm = 1.0;
        int b = cs->bin[p];
        for (int a = 0; a < ns; ++a) {
            double mean = cs->cmean[((size_t)e * 8 + b) * ns + a];
            double* ps = cs->psi + (size_t)a * cs->np + p;
            *ps = (*ps - fm * (*ps - mean)) + dt * S[a];
        }
    }

    /* R-27: the projection of the last step corrects the velocity,
     * U <- U - dt grad <P>(X), before the step uses it */
    double u = cs->u[p], v = cs->v[p], w = cs->w[p];
    {
        /* zero unless a projection ran (mode 2) or a pressure was uploaded */
        const int* sg = m->tri_s + 3 * e;
        const double* g0 = cs->gphi + 2 * (size_t)sg[0];
        const double* g1 = cs->gphi + 2 * (size_t)sg[1];
        const double* g2 = cs->gphi + 2 * (size_t)sg[2];
        double gx = fma(lam[2], g2[0], fma(lam[1], g1[0], lam[0] * g0[0]));
        double gy = fma(lam[2], g2[1], fma(lam[1], g1[1], lam[0] * g0[1]));
        u = u - dt * gx;
        v = v - dt * gy;
    }

    /* Eq.(4) with the generalized Langevin model; the dW_j of the viscous
     * term is the same increment as in Eq.(2) (R-01) */
    double d1 = u - f[F_U1], d2 = v - f[F_U2], d3 = w - f[F_U3];
    double tnu = 2.0 * P->nu;
    double sq_nu = sqrt(tnu * dt);
    double c0e = f[F_C0EPS] > 0.0 ? f[F_C0EPS] : 0.0;
    double sq_c0 = sqrt(c0e * dt);
    double du = dt * ((-f[F_DPX] + tnu * f[F_LAP1]) + (f[F_G11] * d1 + f[F_G12] * d2))
              + sq_nu * (f[F_DU1X] * xi[0] + f[F_DU1Y] * xi[1]) + sq_c0 * xi[2];
    double dv = dt * ((-f[F_DPY] + tnu * f[F_LAP2]) + (f[F_G21] * d1 + f[F_G22] * d2))
              + sq_nu * (f[F_DU2X] * xi[0] + f[F_DU2Y] * xi[1]) + sq_c0 * xi[3];
    double dw = dt * (tnu * f[F_LAP3] + f[F_G33] * d3)
              + sq_nu * (f[F_DU3X] * xi[0] + f[F_DU3Y] * xi[1]) + sq_c0 * xi[4];

    /* Eq.(2): X^{n+1} = X^n + U^n dt + (2 nu)^{1/2} dW */
    double x = (cs->x[p] + u * dt) + sq_nu * xi[0];
    double y = (cs->y[p] + v * dt) + sq_nu * xi[1];
    double U3[3] = {u + du, v + dv, w + dw};

    /* Eq.(5) with S_omega of Eq.(6) interpolated from the nodes (R-17) */
    double om = cs->om[p], W = f[F_OMEGA], S = f[F_SOMEGA];
    double drift = ((-P->C3 * W) * (om - W)) - ((S * W) * om);
    double omp = om > 0.0 ? om : 0.0;
    double diff = sqrt((((2.0 * P->C3 * P->C4) * (W * W)) * omp) * dt);
    double omn = (om + dt * drift) + diff * xi[5];
    if (omn < 0.0) { omn = -omn; cs->cnt[CNT_OMEGA_FLIP]++; }   /* R-21 */

    /* tracking with wall and periodic conditions (R-12..R-15) */
    int en = orc_walk_case(cs, e, &x, &y, U3);

    /* concentrated sources (R-26) */
    for (int a = 0; a < ns; ++a) {
        double r = P->src[a][2];
        if (r > 0.0) {
            double dx = x - P->src[a][0], dy = y - P->src[a][1];
            if (dx * dx + dy * dy < r * r) cs->psi[(size_t)a * cs->np + p] = P->src[a][3];
        }
    }
    cs->x[p] = x; cs->y[p] = y;
    cs->u[p] = U3[0]; cs->v[p] = U3[1]; cs->w[p] = U3[2];
    cs->om[p] = omn; cs->elem[p] = en;
}

/* R-11: mass-weighted P1 kernel estimator at the statistics nodes, two
 * passes (means, then central moments about the nodal means). */
int orc_node_moments(ocase* cs)
{
    const omesh* m = &cs->m;
    const int ns = cs->p.n_scalars, nst = nstat_of(cs), nsu = nsum_of(cs), nsn = m->nsn;
    double* S = cs->sums;
    memset(S, 0, sizeof(double) * (size_t)nsn * nsu);
    for (int64_t p = 0; p < cs->np; ++p) {
        int e = cs->elem[p];
        double lam[3];
        omesh_bary(m, e, cs->x[p], cs->y[p], lam);
        double Q[3] = {cs->u[p], cs->v[p], cs->w[p]};
        for (int k = 0; k < 3; ++k) {
            double* r = S + (size_t)m->tri_s[3 * e + k] * nsu;
            double wn = cs->wt[p] * lam[k];
            r[0] += wn;
            for (int i = 0; i < 3; ++i) r[1 + i] += wn * Q[i];
            r[4] += wn * Q[0] * Q[0]; r[5] += wn * Q[1] * Q[1]; r[6] += wn * Q[2] * Q[2];
            r[7] += wn * Q[0] * Q[1]; r[8] += wn * Q[0] * Q[2]; r[9] += wn * Q[1] * Q[2];
            r[10] += wn * cs->om[p];
            r[11 + 2 * ns] += wn * wn;
            for (int a = 0; a < ns; ++a) {
                double ps = cs->psi[(size_t)a * cs->np + p];
                r[11 + a] += wn * ps;
                r[11 + ns + a] += wn * ps * ps;
            }
        }
    }
    /* means; an empty node, or (once there are previous statistics) one whose
     * effective sample size W^2 / sum (w N)^2 is below n_eff_min, keeps its
     * previous statistics (R-34) */
    char* live = orc_alloc((size_t)nsn);
    for (int s = 0; s < nsn; ++s) {
        double* st = cs->stats + (size_t)s * nst;
        const double* r = S + (size_t)s * nsu;
        if (r[0] > 0.0 && (!cs->have_stats || r[0] * r[0] >= cs->p.n_eff_min * r[11 + 2 * ns])) {
            live[s] = 1;
            st[0] = r[0];
            st[1] = r[0] / m->vol[s];
            for (int i = 0; i < 3; ++i) st[2 + i] = r[1 + i] / r[0];
            st[11] = r[10] / r[0];
            for (int a = 0; a < ns; ++a) st[12 + a] = r[11 + a] / r[0];
            for (int q = 5; q <= 10; ++q) st[q] = 0.0;
            for (int a = 0; a < ns; ++a) st[12 + ns + a] = 0.0;
        } else {
            live[s] = 0;
            st[0] = r[0];
            st[1] = r[0] / m->vol[s];
            cs->cnt[CNT_EMPTY_NODE]++;
        }
    }
    /* central moments */
    for (int64_t p = 0; p < cs->np; ++p) {
        int e = cs->elem[p];
        double lam[3];
        omesh_bary(m, e, cs->x[p], cs->y[p], lam);
        double Q[3] = {cs->u[p], cs->v[p], cs->w[p]};
        for (int k = 0; k < 3; ++k) {
            int s = m->tri_s[3 * e + k];
            if (!live[s]) continue;
            double* st = cs->stats + (size_t)s * nst;
            double wn = cs->wt[p] * lam[k];
            double d[3];
            for (int i = 0; i < 3; ++i) d[i] = Q[i] - st[2 + i];
            st[5] += wn * d[0] * d[0]; st[6] += wn * d[1] * d[1]; st[7] += wn * d[2] * d[2];
            st[8] += wn * d[0] * d[1]; st[9] += wn * d[0] * d[2]; st[10] += wn * d[1] * d[2];
            for (int a = 0; a < ns; ++a) {
                double dp = cs->psi[(size_t)a * cs->np + p] - st[12 + a];
                st[12 + ns + a] += wn * dp * dp;
            }
        }
    }
    for (int s = 0; s < nsn; ++s) {
        if (!live[s]) continue;
        double* st = cs->stats + (size_t)s * nst;
        for (int q = 5; q <= 10; ++q) st[q] /= st[0];
        for (int a = 0; a < ns; ++a) st[12 + ns + a] /= st[0];
    }
    free(live);
    cs->have_stats = 1;
    return ORC_OK;
}

/* R-23: octant of U - <U>(X) with <U> interpolated from the fields in force;
 * cell means over (element, bin); bins with fewer than n_min particles of an
 * element are pooled into one residual cell. */
int orc_case_rebin(ocase* cs)
{
    const omesh* m = &cs->m;
    const int ns = cs->p.n_scalars, ne = m->ne, nb = cs->p.n_bins;
    double* sw = orc_alloc(sizeof(double) * (size_t)ne * 8);
    double* swp = orc_alloc(sizeof(double) * (size_t)ne * 8 * (ns > 0 ? ns : 1));
    memset(cs->ccount, 0, sizeof(int32_t) * (size_t)ne * 8);
    for (int64_t p = 0; p < cs->np; ++p) {
        int e = cs->elem[p];
        int b = 0;
        if (nb == 8) {
            double lam[3], f[ORC_NF];
            omesh_bary(m, e, cs->x[p], cs->y[p], lam);
            interpolate(cs, e, lam, f);
            if (cs->u[p] - f[F_U1] >= 0.0) b += 1;
            if (cs->v[p] - f[F_U2] >= 0.0) b += 2;
            if (cs->w[p] - f[F_U3] >= 0.0) b += 4;
        }
        cs->bin[p] = (uint8_t)b;
        size_t c = (size_t)e * 8 + b;
        cs->ccount[c]++;
        sw[c] += cs->wt[p];
        for (int a = 0; a < ns; ++a) swp[c * ns + a] += cs->wt[p] * cs->psi[(size_t)a * cs->np + p];
    }
    for (int e = 0; e < ne; ++e) {
        double rw = 0.0, rp[ORC_MAXS] = {0, 0, 0, 0};
        for (int b = 0; b < 8; ++b) {
            size_t c = (size_t)e * 8 + b;
            if (cs->ccount[c] > 0 && cs->ccount[c] < cs->p.n_min) {
                rw += sw[c];
                for (int a = 0; a < ns; ++a) rp[a] += swp[c * ns + a];
            }
        }
        for (int b = 0; b < 8; ++b) {
            size_t c = (size_t)e * 8 + b;
            for (int a = 0; a < ns; ++a) {
                double mval = 0.0;
                if (cs->ccount[c] >= cs->p.n_min) mval = swp[c * ns + a] / sw[c];
                else if (rw > 0.0) mval = rp[a] / rw;
                cs->cmean[c * ns + a] = mval;
            }
        }
    }
    free(sw); free(swp);
    return ORC_OK;
}

/* R-16: area-weighted average of the element gradients of the P1 field */
void orc_recover_grad(const omesh* m, const double* f, double* gx, double* gy)
{
    for (int s = 0; s < m->nsn; ++s) {
        double A = 0.0, sx = 0.0, sy = 0.0;
        for (int j = m->inc_ptr[s]; j < m->inc_ptr[s + 1]; ++j) {
            int e = m->inc[j] / 3;
            const double* r = m->rec + 8 * (size_t)e;
            const int* t = m->tri_s + 3 * e;
            double ex = (f[t[0]] * r[2] + f[t[1]] * r[3]) + f[t[2]] * r[4];
            double ey = (f[t[0]] * r[5] + f[t[1]] * r[6]) + f[t[2]] * r[7];
            sx += m->area[e] * ex; sy += m->area[e] * ey; A += m->area[e];
        }
        gx[s] = sx / A; gy[s] = sy / A;
    }
}

/* R-16: nodal Laplacian = area-weighted average of the element divergence of
 * the P1 interpolant of the recovered gradient */
void orc_recover_lap(const omesh* m, const double* gx, const double* gy, double* lap)
{
    for (int s = 0; s < m->nsn; ++s) {
        double A = 0.0, sd = 0.0;
        for (int j = m->inc_ptr[s]; j < m->inc_ptr[s + 1]; ++j) {
            int e = m->inc[j] / 3;
            const double* r = m->rec + 8 * (size_t)e;
            const int* t = m->tri_s + 3 * e;
            double div = 0.0;
            for (int k = 0; k < 3; ++k) div += r[2 + k] * gx[t[k]] + r[5 + k] * gy[t[k]];
            sd += m->area[e] * div; A += m->area[e];
        }
        lap[s] = sd / A;
    }
}

static double det3(const double R[3][3])
{
    return R[0][0] * (R[1][1] * R[2][2] - R[1][2] * R[2][1])
         - R[0][1] * (R[1][0] * R[2][2] - R[1][2] * R[2][0])
         + R[0][2] * (R[1][0] * R[2][1] - R[1][1] * R[2][0]);
}

/* R-19 at one node (the elliptic relaxation of Dreeben & Pope, cited after
 * Eq.(4)): for the five components (11, 12, 21, 22, 33) of the relaxed
 * tensor, the right-hand side
 *   r_ij = 1/2 (1 - C1) eps delta_ij + k H_ijkl d<U_k>/dx_l,
 *   H_ijkl d_l U_k = (C2 A_v + g5/3) d_j U_i - (g5/3) d_i U_j
 *                    + g5 b_ik d_j U_k - g5 b_il d_l U_j,
 * b_ij = <u_i u_j>/(2k) - delta_ij/3, A_v = min(1, Cv det<uu> / (2k/3)^3),
 * the wall value -4.5 eps n_i n_j (used where the node is on a wall), and the
 * squared length scale L^2, L = CL max(k^3/2 / eps, Ceta nu^3/4 / eps^1/4).
 * R is <u_i u_j>, dU[i][j] = d<U_i>/dx_j (j = 3 is zero, R-01); K and E are
 * the floored k and eps (R-18). */
void orc_relax_node(const orc_params* P, const double R[3][3], const double dU[3][3], double K, double E,
                    double nx, double ny, double r[5], double dval[5], double* L2, double* Av_out)
{
    static const int ci[5] = {0, 0, 1, 1, 2}, cj[5] = {0, 1, 0, 1, 2};
    double b[3][3];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) b[i][j] = R[i][j] / (2.0 * K) - (i == j ? 1.0 / 3.0 : 0.0);
    double k23 = (2.0 / 3.0) * K;
    double Av = P->Cv * det3(R) / (k23 * k23 * k23);
    if (Av > 1.0) Av = 1.0;
    double cA = P->C2 * Av + P->gamma5 / 3.0;
    for (int q = 0; q < 5; ++q) {
        int i = ci[q], j = cj[q];
        double h = cA * dU[i][j] - (P->gamma5 / 3.0) * dU[j][i];
        for (int kk = 0; kk < 3; ++kk) h += P->gamma5 * b[i][kk] * dU[kk][j];
        for (int l = 0; l < 3; ++l) h -= P->gamma5 * b[i][l] * dU[j][l];
        double val = K * h;
        if (i == j) val += 0.5 * (1.0 - P->C1) * E;
        r[q] = val;
        double nvec[3] = {nx, ny, 0.0};
        dval[q] = -4.5 * E * nvec[i] * nvec[j];
    }
    double nu34 = sqrt(P->nu * sqrt(P->nu));
    double lt = K * sqrt(K) / E;
    double lk = P->Ceta * nu34 / sqrt(sqrt(E));
    double L = P->CL * (lt > lk ? lt : lk);
    *L2 = L * L;
    if (Av_out) *Av_out = Av;
}

/* Eulerian fields from the node statistics (R-16..R-20, R-27). */
int orc_derive_fields(orc_ctx* c, ocase* cs, int project)
{
    const orc_params* P = &cs->p;
    const omesh* m = &cs->m;
    const int nsn = m->nsn, nst = nstat_of(cs);
    if (P->mode == ORC_MODE_FROZEN) return ORC_OK;
    double* tmp = orc_alloc(sizeof(double) * (size_t)nsn * 6);
    double *f = tmp, *gx = tmp + nsn, *gy = tmp + 2 * nsn, *lap = tmp + 3 * nsn;
    for (int i = 0; i < 3; ++i) {
        for (int s = 0; s < nsn; ++s) {
            f[s] = cs->stats[(size_t)s * nst + 2 + i];
            cs->F[(size_t)s * ORC_NF + F_U1 + i] = f[s];
        }
        orc_recover_grad(m, f, gx, gy);
        orc_recover_lap(m, gx, gy, lap);
        for (int s = 0; s < nsn; ++s) {
            cs->F[(size_t)s * ORC_NF + F_DU1X + 2 * i] = gx[s];
            cs->F[(size_t)s * ORC_NF + F_DU1X + 2 * i + 1] = gy[s];
            cs->F[(size_t)s * ORC_NF + F_LAP1 + i] = lap[s];
        }
    }
    double* kf = orc_alloc(sizeof(double) * nsn);
    double* ef = orc_alloc(sizeof(double) * nsn);
    for (int s = 0; s < nsn; ++s) {
        const double* st = cs->stats + (size_t)s * nst;
        double* F = cs->F + (size_t)s * ORC_NF;
        double k = 0.5 * ((st[5] + st[6]) + st[7]);
        double om = st[11];
        double eps = k * om;
        kf[s] = k; ef[s] = eps;
        if (kf[s] < P->k_floor) { kf[s] = P->k_floor; cs->cnt[CNT_K_FLOOR]++; }
        if (ef[s] < P->eps_floor) { ef[s] = P->eps_floor; cs->cnt[CNT_EPS_FLOOR]++; }
        /* production P = -<u_i u_j> d<U_i>/dx_j, i = 1..3, j = 1..2 (Eq.(6)) */
        double u11 = st[5], u22 = st[6], u12 = st[8], u13 = st[9], u23 = st[10];
        double prod = -(((u11 * F[F_DU1X] + u12 * F[F_DU1Y]) + (u12 * F[F_DU2X] + u22 * F[F_DU2Y]))
                        + (u13 * F[F_DU3X] + u23 * F[F_DU3Y]));
        F[F_OMEGA] = om;
        F[F_SOMEGA] = P->Cw2 - P->Cw1 * prod / ef[s];
        if (P->mode == ORC_MODE_SLM) {
            /* R-20: G_ij = -(1/2 + 3/4 C0) <omega> delta_ij, C0 eps = C0 k <omega> */
            double g = -(0.5 + 0.75 * P->C0) * om;
            F[F_G11] = g; F[F_G22] = g; F[F_G33] = g; F[F_G12] = 0.0; F[F_G21] = 0.0;
            F[F_C0EPS] = P->C0 * eps;
            F[F_DPX] = P->dpdx[0]; F[F_DPY] = P->dpdx[1];
        }
    }
    int rc = ORC_OK;
    if (P->mode == ORC_MODE_ER) {
        /* R-19: elliptic relaxation, wp_ij - div(L^2 grad wp_ij) = r_ij with
         * the nodal sources, wall values and length scale of orc_relax_node;
         * G_ij = (wp_ij - eps/2 delta_ij)/k */
        double* L2 = orc_alloc(sizeof(double) * nsn);
        double* r = orc_alloc(sizeof(double) * (size_t)nsn * 5);
        double* dv = orc_alloc(sizeof(double) * (size_t)nsn * 5);
        int* dm = orc_alloc(sizeof(int) * nsn);
        for (int s = 0; s < nsn; ++s) {
            const double* st = cs->stats + (size_t)s * nst;
            const double* F = cs->F + (size_t)s * ORC_NF;
            double R[3][3] = {{st[5], st[8], st[9]}, {st[8], st[6], st[10]}, {st[9], st[10], st[7]}};
            double dU[3][3] = {{F[F_DU1X], F[F_DU1Y], 0.0}, {F[F_DU2X], F[F_DU2Y], 0.0},
                               {F[F_DU3X], F[F_DU3Y], 0.0}};   /* dU[i][j] = d<U_i>/dx_j */
            double rq[5], dq[5], av;
            orc_relax_node(P, R, dU, kf[s], ef[s], m->wnx[s], m->wny[s], rq, dq, &L2[s], &av);
            for (int q = 0; q < 5; ++q) {
                r[(size_t)q * nsn + s] = rq[q];
                dv[(size_t)q * nsn + s] = dq[q];
            }
            dm[s] = m->is_wall[s];
        }
        double* wp = orc_alloc(sizeof(double) * (size_t)nsn * 5);
        for (int q = 0; q < 5 && rc == ORC_OK; ++q) {
            int it = 0;
            rc = orc_helmholtz(m, L2, r + (size_t)q * nsn, dm, dv + (size_t)q * nsn, 1e-13, 100000,
                               wp + (size_t)q * nsn, &it);
            cs->cnt[CNT_CG_ER] += it;
            if (rc) orc_err(c, rc, "elliptic relaxation solve did not converge");
        }
        for (int s = 0; s < nsn; ++s) {
            const double* st = cs->stats + (size_t)s * nst;
            double* F = cs->F + (size_t)s * ORC_NF;
            double K = kf[s], E = ef[s];
            double w11 = wp[s], w12 = wp[nsn + s], w21 = wp[2 * (size_t)nsn + s],
                   w22 = wp[3 * (size_t)nsn + s], w33 = wp[4 * (size_t)nsn + s];
            F[F_G11] = (w11 - 0.5 * E) / K;
            F[F_G12] = w12 / K;
            F[F_G21] = w21 / K;
            F[F_G22] = (w22 - 0.5 * E) / K;
            F[F_G33] = (w33 - 0.5 * E) / K;
            double tr = (st[5] * w11 + st[8] * w12) + (st[8] * w21 + st[6] * w22) + st[7] * w33;
            double c0e = -(2.0 / 3.0) * tr / K;
            F[F_C0EPS] = c0e > 0.0 ? c0e : 0.0;
        }
        free(wp); free(L2); free(r); free(dv); free(dm);

        /* R-27: pressure projection on the grid (Chorin's, not incremental):
         * <P> = phi with grad^2 phi = div <U> / dt; the particles take the
         * correction -dt grad <P> at the start of the next step */
        if (rc == ORC_OK && project) {
            double* U1 = orc_alloc(sizeof(double) * nsn);
            double* U2 = orc_alloc(sizeof(double) * nsn);
            double* phi = orc_alloc(sizeof(double) * nsn);
            for (int s = 0; s < nsn; ++s) { U1[s] = cs->stats[(size_t)s * nst + 2]; U2[s] = cs->stats[(size_t)s * nst + 3]; }
            int it = 0;
            rc = orc_projection(m, U1, U2, P->dt, 1e-13, 100000, phi, &it);
            cs->cnt[CNT_CG_P] += it;
            if (rc) orc_err(c, rc, "pressure projection solve did not converge");
            for (int s = 0; s < nsn; ++s) cs->P[s] = phi[s];
            free(U1); free(U2); free(phi);
        }
        /* the predictor sees the driving gradient alone; the projection's
         * gradient acts through the correction */
        orc_recover_grad(m, cs->P, gx, gy);
        for (int s = 0; s < nsn; ++s) {
            cs->F[(size_t)s * ORC_NF + F_DPX] = P->dpdx[0];
            cs->F[(size_t)s * ORC_NF + F_DPY] = P->dpdx[1];
            cs->gphi[2 * (size_t)s] = gx[s];
            cs->gphi[2 * (size_t)s + 1] = gy[s];
        }
    }
    free(kf); free(ef); free(tmp);
    /* slots the caller froze keep their uploaded values */
    for (int s = 0; s < nsn; ++s)
        for (int q = 0; q < ORC_NF; ++q)
            if ((cs->freeze >> q) & 1u) cs->F[(size_t)s * ORC_NF + q] = cs->Ffrz[(size_t)s * ORC_NF + q];
    return rc;
}

int orc_case_init(orc_ctx* c, ocase* cs)
{
    orc_node_moments(cs);
    int rc = orc_derive_fields(c, cs, 0);
    if (rc) return rc;
    return orc_case_rebin(cs);
}

int orc_case_step(orc_ctx* c, ocase* cs, uint32_t n)
{
    for (int64_t p = 0; p < cs->np; ++p) advance_particle(cs, p, n);
    orc_node_moments(cs);
    orc_case_rebin(cs);              /* bins against F^n, the fields of this step */
    int rc = orc_derive_fields(c, cs, 1);
    /* R-36: bins and cell means against F^{n+1}, the fields the next step uses */
    if (rc == ORC_OK && cs->p.rebin) orc_case_rebin(cs);
    return rc;
}
