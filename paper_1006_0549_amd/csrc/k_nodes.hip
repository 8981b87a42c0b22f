// Node- and element-level kernels of a time step, all in FP64 (the Eulerian
// side of the method: Sec. I grid roles (i) statistics and (ii) Eulerian
// solves). Each kernel covers every case of the context in one launch:
// threads map to global statistics nodes or elements and look up their case.
// The node kernels take their blocks in XCD order (xcd_block): neighbouring
// nodes, which read each other's values, then share an L2.
//
//   (node statistics and cell means come from the scatter passes, k_scatter.hip)
//   k_fields_grad  <U>, <omega>, recovered gradients of <U> (R-16)
//   k_fields_derived  Laplacians (R-16), k, eps, production, S_omega
//                  (Eq.(6), R-17, R-18), simplified Langevin G_ij (R-20) or
//                  the elliptic-relaxation sources, length scale and wall values (R-19)
//   k_er_assemble  Galerkin (M + K_L) matrix, M r right-hand sides, Dirichlet rows
//   k_galerkin     coarse-level values of the relaxation hierarchies; the
//                  solves themselves are in k_mg.hip (R-28)
//   k_er_finish    G_ij and C0 eps from the relaxed tensor (R-19)
//   k_proj_rhs / k_proj_finish  pressure projection (R-27)
//   k_fields_elem  element-major copy of the fields in the particle precision
#include "pdfmc_dev.h"
#include "pdfmc_nodes.h"

namespace pdfmc {

__global__ void k_fill_f64(double* __restrict__ a, int64_t n, double v)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) a[i] = v;
}

__global__ void k_fill_i32(int32_t* __restrict__ a, int64_t n, int32_t v)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) a[i] = v;
}

__global__ void k_step_increment(uint32_t* step) { if (threadIdx.x == 0 && blockIdx.x == 0) step[0] += 1u; }

// R-16: area-weighted average of the element gradients of a P1 field
__device__ inline void recover_grad(const NodeArgs& A, const double* f, int fstride, int s, double& gx, double& gy)
{
    double Asum = 0.0, sx = 0.0, sy = 0.0;
    for (int j = A.inc_ptr[s]; j < A.inc_ptr[s + 1]; ++j) {
        const int e = A.inc[j] / 3;
        const double* r = A.rec + 8 * (int64_t)e;
        const int4 t = A.tri_s[e];
        const double f0 = f[(int64_t)t.x * fstride], f1 = f[(int64_t)t.y * fstride], f2 = f[(int64_t)t.z * fstride];
        const double ex = (f0 * r[2] + f1 * r[3]) + f2 * r[4];
        const double ey = (f0 * r[5] + f1 * r[6]) + f2 * r[7];
        const double ae = A.area[e];
        sx += ae * ex; sy += ae * ey; Asum += ae;
    }
    gx = sx / Asum; gy = sy / Asum;
}

// the same for three consecutive fields f[0], f[1], f[2] in one pass over
// the incident elements (each component's sums in the same order)
__device__ inline void recover_grad3(const NodeArgs& A, const double* f, int fstride, int s, double (&gx)[3],
                                     double (&gy)[3])
{
    double Asum = 0.0, sx[3] = {0.0, 0.0, 0.0}, sy[3] = {0.0, 0.0, 0.0};
    for (int j = A.inc_ptr[s]; j < A.inc_ptr[s + 1]; ++j) {
        const int e = A.inc[j] / 3;
        const double* r = A.rec + 8 * (int64_t)e;
        const int4 t = A.tri_s[e];
        const double ae = A.area[e];
        const double* p0 = f + (int64_t)t.x * fstride;
        const double* p1 = f + (int64_t)t.y * fstride;
        const double* p2 = f + (int64_t)t.z * fstride;
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            const double f0 = p0[i], f1 = p1[i], f2 = p2[i];
            const double ex = (f0 * r[2] + f1 * r[3]) + f2 * r[4];
            const double ey = (f0 * r[5] + f1 * r[6]) + f2 * r[7];
            sx[i] += ae * ex; sy[i] += ae * ey;
        }
        Asum += ae;
    }
#pragma unroll
    for (int i = 0; i < 3; ++i) { gx[i] = sx[i] / Asum; gy[i] = sy[i] / Asum; }
}

__global__ void k_fields_grad(NodeArgs A)
{
    const int s = xcd_block((int)blockIdx.x, (int)gridDim.x) * blockDim.x + threadIdx.x;
    if (s >= A.nn) return;
    const CaseDev& C = A.cases[A.node_case[s]];
    if (C.mode == 0) return;
    double* F = A.F + (int64_t)s * NF;
    const double* st = A.stats + (int64_t)s * NST;
    F[F_U1] = st[2]; F[F_U2] = st[3]; F[F_U3] = st[4];
    F[F_OMEGA] = st[11];
    double gx[3], gy[3];
    recover_grad3(A, A.stats + 2, NST, s, gx, gy);
    for (int i = 0; i < 3; ++i) {
        F[F_DU1X + 2 * i] = gx[i];
        F[F_DU1X + 2 * i + 1] = gy[i];
    }
}

__device__ inline double det3(const double R[3][3])
{
    return R[0][0] * (R[1][1] * R[2][2] - R[1][2] * R[2][1])
         - R[0][1] * (R[1][0] * R[2][2] - R[1][2] * R[2][0])
         + R[0][2] * (R[1][0] * R[2][1] - R[1][1] * R[2][0]);
}

__global__ void k_fields_derived(NodeArgs A)
{
    const int s = xcd_block((int)blockIdx.x, (int)gridDim.x) * blockDim.x + threadIdx.x;
    if (s >= A.nn) return;
    const int c = A.node_case[s];
    const CaseDev& C = A.cases[c];
    if (C.mode == 0) return;
    double* F = A.F + (int64_t)s * NF;
    const double* st = A.stats + (int64_t)s * NST;
    // Laplacian: area-weighted element divergence of the recovered gradient
    // (R-16), the three components in one pass over the incident elements
    {
        double Asum = 0.0, sd[3] = {0.0, 0.0, 0.0};
        for (int j = A.inc_ptr[s]; j < A.inc_ptr[s + 1]; ++j) {
            const int e = A.inc[j] / 3;
            const double* r = A.rec + 8 * (int64_t)e;
            const int4 t = A.tri_s[e];
            const int tt[3] = {t.x, t.y, t.z};
            const double ae = A.area[e];
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                double div = 0.0;
                for (int k = 0; k < 3; ++k) {
                    const double* Fk = A.F + (int64_t)tt[k] * NF;
                    div += r[2 + k] * Fk[F_DU1X + 2 * i] + r[5 + k] * Fk[F_DU1X + 2 * i + 1];
                }
                sd[i] += ae * div;
            }
            Asum += ae;
        }
        for (int i = 0; i < 3; ++i) F[F_LAP1 + i] = sd[i] / Asum;
    }
    const double k = 0.5 * ((st[5] + st[6]) + st[7]);
    const double om = st[11];
    const double eps = k * om;
    double kf = k, ef = eps;
    unsigned long long* cnt = A.counters + (int64_t)c * NCNT;
    if (kf < C.k_floor) { kf = C.k_floor; atomicAdd(cnt + C_K_FLOOR, 1ull); }
    if (ef < C.eps_floor) { ef = C.eps_floor; atomicAdd(cnt + C_EPS_FLOOR, 1ull); }
    A.kf[s] = kf; A.ef[s] = ef;
    const double u11 = st[5], u22 = st[6], u33 = st[7], u12 = st[8], u13 = st[9], u23 = st[10];
    const double prod = -(((u11 * F[F_DU1X] + u12 * F[F_DU1Y]) + (u12 * F[F_DU2X] + u22 * F[F_DU2Y]))
                          + (u13 * F[F_DU3X] + u23 * F[F_DU3Y]));
    F[F_SOMEGA] = C.Cw2 - C.Cw1 * prod / ef;
    if (C.mode == 1) {
        const double g = -(0.5 + 0.75 * C.C0) * om;
        F[F_G11] = g; F[F_G22] = g; F[F_G33] = g; F[F_G12] = 0.0; F[F_G21] = 0.0;
        F[F_C0EPS] = C.C0 * eps;
        F[F_DPX] = C.dpdx[0]; F[F_DPY] = C.dpdx[1];
        return;
    }
    // mode 2: sources of the elliptic-relaxation equation (R-19)
    const double Rm[3][3] = {{u11, u12, u13}, {u12, u22, u23}, {u13, u23, u33}};
    const double dU[3][3] = {{F[F_DU1X], F[F_DU1Y], 0.0}, {F[F_DU2X], F[F_DU2Y], 0.0}, {F[F_DU3X], F[F_DU3Y], 0.0}};
    double b[3][3];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) b[i][j] = Rm[i][j] / (2.0 * kf) - (i == j ? 1.0 / 3.0 : 0.0);
    const double k23 = (2.0 / 3.0) * kf;
    double Av = C.Cv * det3(Rm) / (k23 * k23 * k23);
    if (Av > 1.0) Av = 1.0;
    const double cA = C.C2 * Av + C.gamma5 / 3.0;
    const int ci[NER] = {0, 0, 1, 1, 2}, cj[NER] = {0, 1, 0, 1, 2};
    const double nvec[3] = {A.wnx[s], A.wny[s], 0.0};
    for (int q = 0; q < NER; ++q) {
        const int i = ci[q], j = cj[q];
        double h = cA * dU[i][j] - (C.gamma5 / 3.0) * dU[j][i];
        for (int kk = 0; kk < 3; ++kk) h += C.gamma5 * b[i][kk] * dU[kk][j];
        for (int l = 0; l < 3; ++l) h -= C.gamma5 * b[i][l] * dU[j][l];
        double val = kf * h;
        if (i == j) val += 0.5 * (1.0 - C.C1) * ef;
        A.er_r[(int64_t)s * NER + q] = val;
        A.er_dval[(int64_t)q * A.nn + s] = -4.5 * ef * nvec[i] * nvec[j];
    }
    const double lt = kf * __builtin_sqrt(kf) / ef;
    const double lk = C.Ceta * C.nu34 / __builtin_sqrt(__builtin_sqrt(ef));
    const double L = C.CL * (lt > lk ? lt : lk);
    A.L2[s] = L * L;
}

// Galerkin matrix (M + K_L) with L^2 per element = mean of the nodal values,
// right-hand sides M r for the five components, Dirichlet rows at walls.
// One thread per row; the row's entries are accumulated in incidence order.
// The matrix is stored per case in ELL form (column-major, local columns).
__global__ void k_er_assemble(NodeArgs A)
{
    const int s = xcd_block((int)blockIdx.x, (int)gridDim.x) * blockDim.x + threadIdx.x;
    if (s >= A.nn) return;
    const CaseDev& C = A.cases[A.node_case[s]];
    if (C.mode != 2) return;
    const int n = C.nsn, i = s - C.noff, len = A.ell_len[s];
    double* val = A.er_val + C.ell_off;
    const int32_t* col = A.ell_col + C.ell_off;
    for (int k = 0; k < C.ell_w; ++k) val[(int64_t)k * n + i] = 0.0;
    double rhs[NER] = {0, 0, 0, 0, 0};
    for (int j = A.inc_ptr[s]; j < A.inc_ptr[s + 1]; ++j) {
        const int ent = A.inc[j];
        const int e = ent / 3, a = ent % 3;
        const double* rc = A.rec + 8 * (int64_t)e;
        const int4 t4 = A.tri_s[e];
        const int t[3] = {t4.x, t4.y, t4.z};
        const double Ae = A.area[e];
        const double L2e = ((A.L2[t[0]] + A.L2[t[1]]) + A.L2[t[2]]) / 3.0;
        for (int cc = 0; cc < 3; ++cc) {
            const double Mab = Ae / 12.0 * (a == cc ? 2.0 : 1.0);
            const double Kab = Ae * (rc[2 + a] * rc[2 + cc] + rc[5 + a] * rc[5 + cc]);
            A.er_val[A.incpos[3 * (int64_t)j + cc]] += Mab + L2e * Kab;
            for (int q = 0; q < NER; ++q) rhs[q] += Mab * A.er_r[(int64_t)t[cc] * NER + q];
        }
    }
    if (A.is_wall[s]) {
        for (int k = 0; k < len; ++k) val[(int64_t)k * n + i] = (col[(int64_t)k * n + i] == i) ? 1.0 : 0.0;
        for (int q = 0; q < NER; ++q) A.er_b[(int64_t)s * NER + q] = A.er_dval[(int64_t)q * A.nn + s];
        return;
    }
    for (int k = 0; k < len; ++k) {
        const int64_t at = (int64_t)k * n + i;
        const int g = C.noff + col[at];
        if (A.is_wall[g]) {
            for (int q = 0; q < NER; ++q) rhs[q] -= val[at] * A.er_dval[(int64_t)q * A.nn + g];
            val[at] = 0.0;
        }
    }
    for (int q = 0; q < NER; ++q) A.er_b[(int64_t)s * NER + q] = rhs[q];
}

// Stiffness matrix of the projection (constant; assembled once).
__global__ void k_stiffness_assemble(NodeArgs A)
{
    const int s = xcd_block((int)blockIdx.x, (int)gridDim.x) * blockDim.x + threadIdx.x;
    if (s >= A.nn) return;
    const CaseDev& C = A.cases[A.node_case[s]];
    if (C.mode != 2) return;
    const int n = C.nsn, i = s - C.noff;
    for (int k = 0; k < C.ell_w; ++k) A.pk_val[C.ell_off + (int64_t)k * n + i] = 0.0;
    for (int j = A.inc_ptr[s]; j < A.inc_ptr[s + 1]; ++j) {
        const int ent = A.inc[j];
        const int e = ent / 3, a = ent % 3;
        const double* rc = A.rec + 8 * (int64_t)e;
        const double Ae = A.area[e];
        for (int cc = 0; cc < 3; ++cc)
            A.pk_val[A.incpos[3 * (int64_t)j + cc]] += Ae * (rc[2 + a] * rc[2 + cc] + rc[5 + a] * rc[5 + cc]);
    }
}

__global__ void k_er_finish(NodeArgs A)
{
    const int s = xcd_block((int)blockIdx.x, (int)gridDim.x) * blockDim.x + threadIdx.x;
    if (s >= A.nn) return;
    const CaseDev& C = A.cases[A.node_case[s]];
    if (C.mode != 2) return;
    double* F = A.F + (int64_t)s * NF;
    const double* st = A.stats + (int64_t)s * NST;
    const double K = A.kf[s], E = A.ef[s];
    const double* wx = A.er_x + (int64_t)s * NER;
    const double w11 = wx[0], w12 = wx[1], w21 = wx[2], w22 = wx[3], w33 = wx[4];
    F[F_G11] = (w11 - 0.5 * E) / K;
    F[F_G12] = w12 / K;
    F[F_G21] = w21 / K;
    F[F_G22] = (w22 - 0.5 * E) / K;
    F[F_G33] = (w33 - 0.5 * E) / K;
    const double tr = (st[5] * w11 + st[8] * w12) + (st[8] * w21 + st[6] * w22) + st[7] * w33;
    const double c0e = -(2.0 / 3.0) * tr / K;
    F[F_C0EPS] = c0e > 0.0 ? c0e : 0.0;
}

// right-hand side of the projection: (1/dt) sum_e A_e grad N_a . <U>_e
__global__ void k_proj_rhs(NodeArgs A)
{
    const int s = xcd_block((int)blockIdx.x, (int)gridDim.x) * blockDim.x + threadIdx.x;
    if (s >= A.nn) return;
    const CaseDev& C = A.cases[A.node_case[s]];
    if (C.mode != 2) return;
    double b = 0.0;
    for (int j = A.inc_ptr[s]; j < A.inc_ptr[s + 1]; ++j) {
        const int ent = A.inc[j];
        const int e = ent / 3, a = ent % 3;
        const double* rc = A.rec + 8 * (int64_t)e;
        const int4 t = A.tri_s[e];
        const double* S0 = A.stats + (int64_t)t.x * NST;
        const double* S1 = A.stats + (int64_t)t.y * NST;
        const double* S2 = A.stats + (int64_t)t.z * NST;
        const double ue = ((S0[2] + S1[2]) + S2[2]) / 3.0;
        const double ve = ((S0[3] + S1[3]) + S2[3]) / 3.0;
        b += A.area[e] * (rc[2 + a] * ue + rc[5 + a] * ve) / C.dt;
    }
    A.pb[s] = b;
}

// <P> += phi, then d<P>/dx_j = driving gradient + recovered gradient of <P>
__global__ void k_proj_update(NodeArgs A)
{
    const int s = xcd_block((int)blockIdx.x, (int)gridDim.x) * blockDim.x + threadIdx.x;
    if (s >= A.nn) return;
    const CaseDev& C = A.cases[A.node_case[s]];
    if (C.mode != 2) return;
    A.P[s] = A.phi[s];     // R-27: the projection is not incremental
}

__global__ void k_proj_grad(NodeArgs A)
{
    const int s = xcd_block((int)blockIdx.x, (int)gridDim.x) * blockDim.x + threadIdx.x;
    if (s >= A.nn) return;
    const CaseDev& C = A.cases[A.node_case[s]];
    if (C.mode != 2) return;
    // the predictor sees the driving gradient alone; the gradient of <P>
    // corrects the particle velocities at the start of the next step
    double gx, gy;
    recover_grad(A, A.P, 1, s, gx, gy);
    A.F[(int64_t)s * NF + F_DPX] = C.dpdx[0];
    A.F[(int64_t)s * NF + F_DPY] = C.dpdx[1];
    A.gphi[2 * (int64_t)s] = gx;
    A.gphi[2 * (int64_t)s + 1] = gy;
}

// Field slots a case keeps frozen go back to their uploaded values after the
// fields have been derived from the statistics (the particles then see the
// uploaded values; fields derived within the step used the computed ones).
__global__ void k_fields_freeze(const CaseDev* __restrict__ cases, const int32_t* __restrict__ node_case,
                                const double* __restrict__ Ffrz, double* __restrict__ F, int nn)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)nn * NF) return;
    const int64_t s = i / NF;
    const int q = (int)(i - s * NF);
    if ((cases[node_case[s]].freeze >> q) & 1u) F[i] = Ffrz[i];
}

// Element-major copy of the nodal fields in the particle precision: row k of
// element e holds the fields of its vertex k, so that a particle reads its
// element's three rows from one place right after its element id.
template <typename R>
__global__ void k_fields_elem(const double* __restrict__ F, const double* __restrict__ gphi, const int4* __restrict__ tri_s,
                              R* __restrict__ Fel, int ne)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)ne * 3 * NFE) return;
    const int64_t r = i / NFE;
    const int q = (int)(i - r * NFE);
    const int64_t e = r / 3;
    const int k = (int)(r - e * 3);
    const int4 t = tri_s[e];
    const int s = k == 0 ? t.x : (k == 1 ? t.y : t.z);
    Fel[i] = q < NF ? (R)F[(int64_t)s * NF + q] : (R)gphi[2 * (int64_t)s + (q - FE_GPX)];
}
template __global__ void k_fields_elem<double>(const double*, const double*, const int4*, double*, int);
template __global__ void k_fields_elem<float>(const double*, const double*, const int4*, float*, int);

// ---------------------------------------------------------------- multigrid

// LPE lanes per coarse entry (more where the entries gather longer
// contribution lists); the group's partial sums meet by shuffles
template <int LPE>
__device__ inline void galerkin_body(const GalJob& J)
{
    const int sub = threadIdx.x % LPE;
    const int g0 = (blockIdx.x * blockDim.x + threadIdx.x) / LPE, gs = gridDim.x * blockDim.x / LPE;
    for (int k = g0; k < J.nnz; k += gs) {
        double s = 0.0;
        for (int j = J.gptr[k] + sub; j < J.gptr[k + 1]; j += LPE) s += J.gcoef[j] * J.src[J.gidx[j]];
        for (int d = LPE / 2; d >= 1; d >>= 1) s += __shfl_xor(s, d);
        if (sub == 0) J.dst[J.gdst[k]] = s;
    }
}

// one job (hierarchy) per blockIdx.y, each with its own lanes per entry, so
// that a coarse value's summation order does not depend on the other jobs
__global__ void k_galerkin(const GalJob* __restrict__ jobs)
{
    const GalJob J = jobs[blockIdx.y];
    if (J.lpe >= 16) galerkin_body<16>(J);
    else if (J.lpe >= 4) galerkin_body<4>(J);
    else galerkin_body<1>(J);
}

}  // namespace pdfmc
