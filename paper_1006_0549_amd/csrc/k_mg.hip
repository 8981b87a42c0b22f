// FP64 multigrid-preconditioned conjugate gradients for the Eulerian systems
// of every case (elliptic relaxation, reading R-19; projection, R-27; stopping
// rule, R-28), split into phases so that one system spreads over many
// workgroups.
//
// One PCG iteration k, each phase a kernel over all systems at once:
//   PA(k)  convergence test on ||r_k||; p_k = z_k + beta p_{k-1} (computed on
//          the fly at the neighbours); q = A p_k; accumulate p.q
//   PB(k)  alpha; x += alpha p_k; r_{k+1} = r_k - alpha q; first two smoothing
//          steps of the fine level (from zero, fused: the first step is local)
//   V-cycle on r_{k+1}: residual -> restriction -> [pre-smoothing, residual,
//          restriction on further large levels] -> one workgroup per system
//          for the small levels and the dense coarsest solve -> prolongation
//          -> two post-smoothing steps, the second of which gives z_{k+1} on
//          level 0 and accumulates r.z and sum z.
// Scalars are accumulated with FP64 atomics into rotating per-iteration slots
// (slot k mod 4); a slot is cleared two phases after its last reader. The
// first lanes of each workgroup gather the slot words in one round trip and
// share them through LDS. Level sizes are fixed per system, so a fixed number
// of iterations can be replayed from a graph; systems that have converged leave every later phase at once,
// and k_mg_finish completes any system that needs more iterations in one
// workgroup, with the same phase bodies.
#include "pdfmc_kernels.h"

namespace pdfmc {

namespace {

constexpr int MGB = 256;   // rows per workgroup in the row-parallel phases

// loads that bypass the non-coherent L1 (values written by atomics of the
// same kernel)
__device__ inline double aload(const double* p)
{
    return __longlong_as_double(
        __hip_atomic_load((const long long*)p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
}
__device__ inline int aloadi(const int* p) { return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT); }

__device__ inline double* slot(const MgJob& J, int k) { return J.acc + ((k + 4) & 3) * MG_SLOT; }
__device__ inline double* setup_slot(const MgJob& J) { return J.acc + 4 * MG_SLOT; }
// slot layout: [0] p.q  [1] r.r  [2] sum r  [3] r.z  [4] sum z

// The accumulator words a phase needs, gathered by the first lanes in one
// round trip and shared through LDS:
//   w[0..4]   slot k      w[5..9]  slot k-1     w[10..14] slot k-2
//   w[15..17] set-up slot
// COHERENT: the words were written by atomics of this same kernel (one
// workgroup completing a system), so the loads must bypass the L1.
constexpr int NW = 18;
template <bool COHERENT>
__device__ inline void gather_words(const MgJob& J, int k, double* w)
{
    __syncthreads();
    const int t = threadIdx.x;
    if (t < NW) {
        const double* src = t < 5 ? slot(J, k) + t : t < 10 ? slot(J, k - 1) + (t - 5)
                          : t < 15 ? slot(J, k - 2) + (t - 10) : setup_slot(J) + (t - 15);
        w[t] = COHERENT ? aload(src) : *src;
    }
    __syncthreads();
}

// r.z of a slot (words s[0..4]), with z made mean-free for singular systems
__device__ inline double rz_w(const MgJob& J, const double* s)
{
    return J.mean_free ? s[3] - (s[4] / J.n) * s[2] : s[3];
}

// Sum NV per-thread values over the workgroup and add them to dst[k].
template <int NV>
__device__ inline void block_accumulate(const double (&v)[NV], double* const (&dst)[NV])
{
    __shared__ double sh[16 * 4];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
#pragma unroll
    for (int k = 0; k < NV; ++k) {
        double x = v[k];
        for (int d = 32; d >= 1; d >>= 1) x += __shfl_xor(x, d);
        if (lane == 0) sh[wid * 4 + k] = x;
    }
    __syncthreads();
    if (threadIdx.x < NV) {
        double s = 0.0;
        for (int w = 0; w < nw; ++w) s += sh[w * 4 + threadIdx.x];
        unsafeAtomicAdd(dst[threadIdx.x], s);
    }
    // workgroup-scope release: the atomics above have completed before any
    // thread of this workgroup reads the accumulators again (k_mg_finish);
    // other workgroups read them only in later kernels. An agent-scope fence
    // here would write back the whole L2 of the XCD from every workgroup.
    __threadfence_block();
    __syncthreads();
}

// Scalars of a phase.
struct Scal {
    double a, b;
    int flag;
};

// PA: flag = converged (||r_k||^2 <= tol^2 ||b||^2); a = beta, b = mean of z
template <bool COHERENT>
__device__ inline Scal pa_scalars(const MgJob& J, int k)
{
    __shared__ double w[NW];
    gather_words<COHERENT>(J, k, w);
    Scal s{0.0, 0.0, 0};
    s.flag = w[5 + 1] <= J.tol * J.tol * w[15 + 2] ? 1 : 0;
    if (!s.flag) {
        s.a = k == 0 ? 0.0 : rz_w(J, w + 5) / rz_w(J, w + 10);
        s.b = J.mean_free ? w[5 + 4] / J.n : 0.0;
    }
    return s;
}

// PB: a = alpha; flag = zero right-hand side (first pass only)
template <bool COHERENT>
__device__ inline Scal pb_scalars(const MgJob& J, int k, bool first)
{
    __shared__ double w[NW];
    gather_words<COHERENT>(J, k, w);
    Scal s{0.0, 0.0, 0};
    s.flag = first && (w[15 + 2] <= 1e-28 * w[15 + 1]) ? 1 : 0;
    s.a = first ? 0.0 : rz_w(J, w + 5) / w[0];
    return s;
}

// y_i = sum_k A(k, i) x(col(k, i)); the width is a multiple of 4 and the
// four loads of a group are issued together
__device__ inline double ell_row(const EllDev& A, const double* __restrict__ x, int i)
{
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
    const int64_t n = A.n;
    for (int k = 0; k < A.w; k += 4) {
        const int64_t a = (int64_t)k * n + i;
        const int c0 = A.col[a], c1 = A.col[a + n], c2 = A.col[a + 2 * n], c3 = A.col[a + 3 * n];
        const double v0 = A.val[a], v1 = A.val[a + n], v2 = A.val[a + 2 * n], v3 = A.val[a + 3 * n];
        const double x0 = x[c0], x1 = x[c1], x2 = x[c2], x3 = x[c3];
        s0 += v0 * x0;
        s1 += v1 * x1;
        s2 += v2 * x2;
        s3 += v3 * x3;
    }
    return (s0 + s1) + (s2 + s3);
}

template <typename F>
__device__ inline double ell_row_f(const EllDev& A, F get, int i)
{
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
    const int64_t n = A.n;
    for (int k = 0; k < A.w; k += 4) {
        const int64_t a = (int64_t)k * n + i;
        const int c0 = A.col[a], c1 = A.col[a + n], c2 = A.col[a + 2 * n], c3 = A.col[a + 3 * n];
        const double v0 = A.val[a], v1 = A.val[a + n], v2 = A.val[a + 2 * n], v3 = A.val[a + 3 * n];
        const double x0 = get(c0), x1 = get(c1), x2 = get(c2), x3 = get(c3);
        s0 += v0 * x0;
        s1 += v1 * x1;
        s2 += v2 * x2;
        s3 += v3 * x3;
    }
    return (s0 + s1) + (s2 + s3);
}

// two smoothing steps from zero for row i; b(j) gives the right-hand side
template <typename F>
__device__ inline double pre_row(const AmgDev& H, int l, F b, int i)
{
    const double* dinv = H.dinv[l];
    const double sa = H.sa[l];
    const double s = ell_row_f(H.A[l], [&](int j) { return sa * dinv[j] * b(j); }, i);
    const double bi = b(i);
    return H.se[l] * (sa * dinv[i] * bi) + H.sc[l] * dinv[i] * (bi - s);
}

__device__ inline const double* level_rhs(const MgJob& J, int l, int k)
{
    return l == 0 ? J.r[(k + 1) & 1] : J.lb[l];
}

// ---------------------------------------------------------------- phase bodies
// Each body handles rows i0, i0 + st, ... < i1 of one system. All threads of
// the workgroup call the accumulating bodies (they synchronise).

__device__ void pa_body(const MgJob& J, const AmgDev& H, int k, Scal sc, int i0, int i1, int st)
{
    const double beta = sc.a, mz = sc.b;
    const double* z = J.ly[0];
    const double* pold = J.p[(k - 1) & 1];
    double* pnew = J.p[k & 1];
    auto pv = [&](int j) { return k == 0 ? z[j] - mz : (z[j] - mz) + beta * pold[j]; };
    double pq = 0.0;
    for (int i = i0; i < i1; i += st) {
        const double s = ell_row_f(H.A[0], pv, i);
        const double pi = pv(i);
        pnew[i] = pi;
        J.q[i] = s;
        pq += pi * s;
    }
    block_accumulate<1>({pq}, {slot(J, k)});
}

__device__ void pb_body(const MgJob& J, const AmgDev& H, int k, bool first, Scal sc, bool leader, int i0, int i1,
                        int st)
{
    const bool zero_rhs = sc.flag != 0;
    const double alpha = sc.a;
    if (leader) {
        double* sn = slot(J, k + 1);
        for (int t = 0; t < MG_SLOT; ++t) sn[t] = 0.0;
    }
    const double* rold = J.r[k & 1];
    double* rnew = J.r[(k + 1) & 1];
    const double* pk = J.p[k & 1];
    const double* q = J.q;
    auto bget = [&](int j) -> double { return zero_rhs ? 0.0 : (first ? rold[j] : rold[j] - alpha * q[j]); };
    const bool smooth = H.nbig >= 1;
    double rr = 0.0, sr = 0.0;
    for (int i = i0; i < i1; i += st) {
        if (zero_rhs) J.x[i] = 0.0;
        else if (!first) J.x[i] += alpha * pk[i];
        const double rn = bget(i);
        rnew[i] = rn;
        rr += rn * rn;
        sr += rn;
        if (smooth) J.ly[0][i] = pre_row(H, 0, bget, i);
    }
    block_accumulate<2>({rr, sr}, {slot(J, k) + 1, slot(J, k) + 2});
}

__device__ inline void res_rows(const MgJob& J, const AmgDev& H, int l, int k, int i0, int i1, int st)
{
    const double* b = level_rhs(J, l, k);
    for (int i = i0; i < i1; i += st) J.lt[l][i] = b[i] - ell_row(H.A[l], J.ly[l], i);
}

__device__ inline void restrict_rows(const MgJob& J, const AmgDev& H, int l, int i0, int i1, int st)
{
    for (int i = i0; i < i1; i += st) J.lb[l][i] = ell_row(H.R[l - 1], J.lt[l - 1], i);
}

__device__ inline void pre_rows(const MgJob& J, const AmgDev& H, int l, int k, int i0, int i1, int st)
{
    const double* b = level_rhs(J, l, k);
    for (int i = i0; i < i1; i += st) J.ly[l][i] = pre_row(H, l, [&](int j) { return b[j]; }, i);
}

// prolongation: lt = y + P y_c
__device__ inline void prolong_rows(const MgJob& J, const AmgDev& H, int l, int i0, int i1, int st)
{
    for (int i = i0; i < i1; i += st) J.lt[l][i] = J.ly[l][i] + ell_row(H.P[l], J.ly[l + 1], i);
}

// first post-smoothing step: la = lt + sa D^-1 (b - A lt)
__device__ inline void post1_rows(const MgJob& J, const AmgDev& H, int l, int k, int i0, int i1, int st)
{
    const double* b = level_rhs(J, l, k);
    const double* dinv = H.dinv[l];
    for (int i = i0; i < i1; i += st)
        J.la[l][i] = J.lt[l][i] + H.sa[l] * dinv[i] * (b[i] - ell_row(H.A[l], J.lt[l], i));
}

// second post-smoothing step: y = la + (se - 1)(la - lt) + sc D^-1 (b - A la)
__device__ inline void post2_rows(const MgJob& J, const AmgDev& H, int l, int k, int i0, int i1, int st,
                                  double& rz, double& sz)
{
    const double* b = level_rhs(J, l, k);
    const double* dinv = H.dinv[l];
    const double em1 = H.se[l] - 1.0, sc = H.sc[l];
    for (int i = i0; i < i1; i += st) {
        const double a = J.la[l][i];
        const double y = a + em1 * (a - J.lt[l][i]) + sc * dinv[i] * (b[i] - ell_row(H.A[l], J.la[l], i));
        J.ly[l][i] = y;
        rz += b[i] * y;
        sz += y;
    }
}

// The small levels (nbig and below) of one system's V-cycle, in one workgroup.
__device__ void tail_body(const MgJob& J, const AmgDev& H, int k)
{
    const int tid = threadIdx.x, nt = blockDim.x;
    const int l0 = H.nbig, nl = H.nlev;
    if (l0 >= 1) {
        restrict_rows(J, H, l0, tid, H.n[l0], nt);
        __syncthreads();
    }
    for (int l = l0; l < nl - 1; ++l) {
        pre_rows(J, H, l, k, tid, H.n[l], nt);
        __syncthreads();
        res_rows(J, H, l, k, tid, H.n[l], nt);
        __syncthreads();
        restrict_rows(J, H, l + 1, tid, H.n[l + 1], nt);
        __syncthreads();
    }
    {
        // dense coarse solve, 16 lanes per row (nc <= 64 rows)
        const int l = nl - 1, nc = H.n[l];
        const double* b = level_rhs(J, l, k);
        for (int t = tid; t < 16 * AMG_MAXC; t += nt) {
            const int i = t >> 4, part = t & 15;
            double s = 0.0;
            if (i < nc)
                for (int j = part; j < nc; j += 16) s += H.ainv[i * AMG_MAXC + j] * b[j];
            s += __shfl_xor(s, 8);
            s += __shfl_xor(s, 4);
            s += __shfl_xor(s, 2);
            s += __shfl_xor(s, 1);
            if (i < nc && part == 0) J.ly[l][i] = s;
        }
        __syncthreads();
    }
    for (int l = nl - 2; l >= l0; --l) {
        prolong_rows(J, H, l, tid, H.n[l], nt);
        __syncthreads();
        post1_rows(J, H, l, k, tid, H.n[l], nt);
        __syncthreads();
        double rz = 0.0, sz = 0.0;
        post2_rows(J, H, l, k, tid, H.n[l], nt, rz, sz);
        __syncthreads();
    }
    if (l0 == 0) {
        // z = ly[0] is complete: accumulate r.z and sum z
        const double* r = J.r[(k + 1) & 1];
        double rz = 0.0, sz = 0.0;
        for (int i = tid; i < J.n; i += nt) {
            rz += r[i] * J.ly[0][i];
            sz += J.ly[0][i];
        }
        block_accumulate<2>({rz, sz}, {slot(J, k) + 3, slot(J, k) + 4});
    }
}


}  // namespace

// ---------------------------------------------------------------- kernels

// Inverse diagonals of every level; tab entries: (hierarchy, level, first row)
__global__ void k_mg_dinv(const AmgDev* __restrict__ hs, const int4* __restrict__ tab)
{
    const int4 e = tab[blockIdx.x];
    const AmgDev& H = hs[e.x];
    const EllDev& A = H.A[e.y];
    const int i = e.z + threadIdx.x;
    if (i >= A.n) return;
    double d = 1.0;
    for (int k = 0; k < A.w; ++k) {
        const int64_t a = (int64_t)k * A.n + i;
        if (A.col[a] == i) { d = A.val[a]; break; }
    }
    H.dinv[e.y][i] = 1.0 / d;
}

// Inverse of the (slightly shifted) coarsest matrix by Gauss-Jordan
// elimination in LDS, one workgroup per hierarchy.
__global__ void __launch_bounds__(1024) k_mg_coarse(const AmgDev* __restrict__ hs)
{
    const AmgDev& H = hs[blockIdx.x];
    const EllDev& Ac = H.A[H.nlev - 1];
    const int nc = Ac.n;
    __shared__ double a[AMG_MAXC * AMG_MAXC];
    __shared__ double prow[AMG_MAXC], pcol[AMG_MAXC];
    for (int q = threadIdx.x; q < AMG_MAXC * AMG_MAXC; q += blockDim.x) a[q] = 0.0;
    __syncthreads();
    for (int i = threadIdx.x; i < nc; i += blockDim.x)
        for (int k = 0; k < Ac.w; ++k) {
            const int64_t at = (int64_t)k * nc + i;
            a[i * AMG_MAXC + Ac.col[at]] += Ac.val[at];
        }
    __syncthreads();
    for (int i = threadIdx.x; i < nc; i += blockDim.x) a[i * AMG_MAXC + i] *= (1.0 + H.coarse_shift);
    __syncthreads();
    for (int k = 0; k < nc; ++k) {
        for (int j = threadIdx.x; j < nc; j += blockDim.x) {
            prow[j] = a[k * AMG_MAXC + j];
            pcol[j] = a[j * AMG_MAXC + k];
        }
        __syncthreads();
        const double ip = 1.0 / prow[k];
        for (int q = threadIdx.x; q < nc * nc; q += blockDim.x) {
            const int i = q / nc, j = q % nc;
            double v;
            if (i == k && j == k) v = ip;
            else if (i == k) v = prow[j] * ip;
            else if (j == k) v = -pcol[i] * ip;
            else v = a[i * AMG_MAXC + j] - pcol[i] * prow[j] * ip;
            a[i * AMG_MAXC + j] = v;
        }
        __syncthreads();
    }
    for (int q = threadIdx.x; q < nc * AMG_MAXC; q += blockDim.x) H.ainv[q] = a[q];
}

// Set-up 1: sum b and sum b^2 (tab entries: (job, first row) over level 0)
__global__ void __launch_bounds__(MGB) k_mg_setup1(const MgJob* __restrict__ jobs, const int4* __restrict__ tab, const int32_t* __restrict__ st)
{
    const int4 e = tab[blockIdx.x];
    const MgJob& J = jobs[e.x];
    if (blockIdx.x == 0 && threadIdx.x == 0) *J.need = 0u;
    const int i = e.y + threadIdx.x;
    const double b = i < J.n ? J.b[i] : 0.0;
    double* su = setup_slot(J);
    block_accumulate<2>({b, b * b}, {su, su + 1});
}

// Set-up 2: mean-free right-hand side, r = b - A x (warm start) or r = b
// with x = 0, ||b||^2
__global__ void __launch_bounds__(MGB) k_mg_setup2(const MgJob* __restrict__ jobs, const AmgDev* __restrict__ hs,
                                                   const int4* __restrict__ tab, const int32_t* __restrict__ st)
{
    const int4 e = tab[blockIdx.x];
    const MgJob& J = jobs[e.x];
    const AmgDev& H = hs[e.z];
    double* su = setup_slot(J);
    const double mb = J.mean_free ? su[0] / J.n : 0.0;
    const int i = e.y + threadIdx.x;
    double bb = 0.0;
    if (i < J.n) {
        const double b = J.b[i] - mb;
        J.b[i] = b;
        if (J.warm) {
            J.r[1][i] = b - ell_row(H.A[0], J.x, i);
        } else {
            J.x[i] = 0.0;
            J.r[1][i] = b;
        }
        bb = b * b;
    }
    block_accumulate<1>({bb}, {su + 2});
}

__global__ void __launch_bounds__(MGB) k_mg_pa(const MgJob* __restrict__ jobs, const AmgDev* __restrict__ hs,
                                               const int4* __restrict__ tab, const int32_t* __restrict__ st, int k)
{
    const int4 e = tab[blockIdx.x];
    const MgJob& J = jobs[e.x];
    if (st[2 * e.x] != 0 || k >= J.maxit) return;
    const Scal sc = pa_scalars<false>(J, k);
    if (sc.flag) {
        if (e.y == 0 && threadIdx.x == 0) { J.state[0] = 1; J.state[1] = k; }
        return;
    }
    pa_body(J, hs[e.z], k, sc, e.y + threadIdx.x, min(e.y + MGB, J.n), MGB);
}

__global__ void __launch_bounds__(MGB) k_mg_pb(const MgJob* __restrict__ jobs, const AmgDev* __restrict__ hs,
                                               const int4* __restrict__ tab, const int32_t* __restrict__ st, int k, int first)
{
    const int4 e = tab[blockIdx.x];
    const MgJob& J = jobs[e.x];
    if (st[2 * e.x] != 0 || k >= J.maxit) return;
    const Scal sc = pb_scalars<false>(J, k, first != 0);
    pb_body(J, hs[e.z], k, first != 0, sc, e.y == 0 && threadIdx.x == 0, e.y + threadIdx.x, min(e.y + MGB, J.n),
            MGB);
}

// residual of level l (tab: rows of level l of the systems with nbig > l)
__global__ void __launch_bounds__(MGB) k_mg_res(const MgJob* __restrict__ jobs, const AmgDev* __restrict__ hs,
                                                const int4* __restrict__ tab, const int32_t* __restrict__ st, int l, int k)
{
    const int4 e = tab[blockIdx.x];
    const MgJob& J = jobs[e.x];
    if (st[2 * e.x] != 0 || k >= J.maxit) return;
    const AmgDev& H = hs[e.z];
    const int i = e.y + threadIdx.x;
    if (i < H.n[l]) res_rows(J, H, l, k, i, i + 1, 1);
}

// restriction to level l >= 1 (the pre-smoothing of level l needs every row
// of the restricted right-hand side, so it is a phase of its own)
__global__ void __launch_bounds__(MGB) k_mg_restrict(const MgJob* __restrict__ jobs, const AmgDev* __restrict__ hs,
                                                     const int4* __restrict__ tab, const int32_t* __restrict__ st, int l, int k)
{
    const int4 e = tab[blockIdx.x];
    const MgJob& J = jobs[e.x];
    if (st[2 * e.x] != 0 || k >= J.maxit) return;
    const AmgDev& H = hs[e.z];
    const int i = e.y + threadIdx.x;
    if (i < H.n[l]) restrict_rows(J, H, l, i, i + 1, 1);
}

__global__ void __launch_bounds__(MGB) k_mg_pre(const MgJob* __restrict__ jobs, const AmgDev* __restrict__ hs,
                                                const int4* __restrict__ tab, const int32_t* __restrict__ st, int l, int k)
{
    const int4 e = tab[blockIdx.x];
    const MgJob& J = jobs[e.x];
    if (st[2 * e.x] != 0 || k >= J.maxit) return;
    const AmgDev& H = hs[e.z];
    const int i = e.y + threadIdx.x;
    if (i < H.n[l]) pre_rows(J, H, l, k, i, i + 1, 1);
}

__global__ void __launch_bounds__(1024) k_mg_tail(const MgJob* __restrict__ jobs, const AmgDev* __restrict__ hs,
                                                 const int32_t* __restrict__ st, int k)
{
    const MgJob& J = jobs[blockIdx.x];
    if (st[2 * blockIdx.x] != 0 || J.n <= 0 || k >= J.maxit) return;
    tail_body(J, hs[J.hier], k);
}

__global__ void __launch_bounds__(MGB) k_mg_prolong(const MgJob* __restrict__ jobs, const AmgDev* __restrict__ hs,
                                                    const int4* __restrict__ tab, const int32_t* __restrict__ st, int l, int k)
{
    const int4 e = tab[blockIdx.x];
    const MgJob& J = jobs[e.x];
    if (st[2 * e.x] != 0 || k >= J.maxit) return;
    const AmgDev& H = hs[e.z];
    const int i = e.y + threadIdx.x;
    if (i < H.n[l]) prolong_rows(J, H, l, i, i + 1, 1);
}

__global__ void __launch_bounds__(MGB) k_mg_post1(const MgJob* __restrict__ jobs, const AmgDev* __restrict__ hs,
                                                  const int4* __restrict__ tab, const int32_t* __restrict__ st, int l, int k)
{
    const int4 e = tab[blockIdx.x];
    const MgJob& J = jobs[e.x];
    if (st[2 * e.x] != 0 || k >= J.maxit) return;
    const AmgDev& H = hs[e.z];
    const int i = e.y + threadIdx.x;
    if (i < H.n[l]) post1_rows(J, H, l, k, i, i + 1, 1);
}

__global__ void __launch_bounds__(MGB) k_mg_post2(const MgJob* __restrict__ jobs, const AmgDev* __restrict__ hs,
                                                  const int4* __restrict__ tab, const int32_t* __restrict__ st, int l, int k)
{
    const int4 e = tab[blockIdx.x];
    const MgJob& J = jobs[e.x];
    if (st[2 * e.x] != 0 || k >= J.maxit) return;
    const AmgDev& H = hs[e.z];
    const int i = e.y + threadIdx.x;
    double rz = 0.0, sz = 0.0;
    if (i < H.n[l]) post2_rows(J, H, l, k, i, i + 1, 1, rz, sz);
    if (l == 0) block_accumulate<2>({rz, sz}, {slot(J, k) + 3, slot(J, k) + 4});
}

// Completes, in one workgroup per system, every system that has not
// converged within the first k0 iterations; then makes singular solutions
// mean-free, counts iterations and failures, and clears the per-system state
// for the next solve.
__global__ void __launch_bounds__(1024) k_mg_finish(const MgJob* __restrict__ jobs, const AmgDev* __restrict__ hs, int k0)
{
    const MgJob& J = jobs[blockIdx.x];
    const int n = J.n;
    if (n <= 0) return;
    const AmgDev& H = hs[J.hier];
    const int tid = threadIdx.x, nt = blockDim.x;
    __shared__ int st[2];
    if (tid == 0) { st[0] = aloadi(J.state); st[1] = aloadi(J.state + 1); }
    __syncthreads();
    bool done = st[0] != 0;
    int it = done ? st[1] : 0;
    for (int k = min(k0, J.maxit); !done; ++k) {
        const Scal sa = pa_scalars<true>(J, k);
        if (sa.flag) { done = true; it = k; break; }
        if (k >= J.maxit) { it = k; break; }
        pa_body(J, H, k, sa, tid, n, nt);
        const Scal sb = pb_scalars<true>(J, k, false);
        pb_body(J, H, k, false, sb, tid == 0, tid, n, nt);
        if (H.nbig >= 1) {
            res_rows(J, H, 0, k, tid, n, nt);
            __syncthreads();
            for (int l = 1; l < H.nbig; ++l) {
                restrict_rows(J, H, l, tid, H.n[l], nt);
                __syncthreads();
                pre_rows(J, H, l, k, tid, H.n[l], nt);
                __syncthreads();
                res_rows(J, H, l, k, tid, H.n[l], nt);
                __syncthreads();
            }
        }
        tail_body(J, H, k);
        __syncthreads();
        for (int l = H.nbig - 1; l >= 0; --l) {
            prolong_rows(J, H, l, tid, H.n[l], nt);
            __syncthreads();
            post1_rows(J, H, l, k, tid, H.n[l], nt);
            __syncthreads();
            double rz = 0.0, sz = 0.0;
            post2_rows(J, H, l, k, tid, H.n[l], nt, rz, sz);
            if (l == 0) block_accumulate<2>({rz, sz}, {slot(J, k) + 3, slot(J, k) + 4});
            else __syncthreads();
        }
    }
    if (J.mean_free) {
        double s = 0.0;
        for (int i = tid; i < n; i += nt) s += J.x[i];
        __shared__ double sh[16];
        for (int d = 32; d >= 1; d >>= 1) s += __shfl_xor(s, d);
        if ((tid & 63) == 0) sh[tid >> 6] = s;
        __syncthreads();
        double m = 0.0;
        for (int w = 0; w < (nt + 63) / 64; ++w) m += sh[w];
        m /= n;
        for (int i = tid; i < n; i += nt) J.x[i] -= m;
    }
    __syncthreads();
    if (tid == 0) {
        atomicAdd(J.iters, (unsigned long long)it);
        if (!done) atomicAdd(J.fails, 1ull);
        atomicMax(J.need, (unsigned int)it);
        J.state[0] = 0;
        J.state[1] = 0;
    }
    for (int t = tid; t < MG_NSLOT * MG_SLOT; t += nt) J.acc[t] = 0.0;
}

}  // namespace pdfmc
