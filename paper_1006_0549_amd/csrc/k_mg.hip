// FP64 multigrid-preconditioned conjugate gradients for the Eulerian systems
// of every case (elliptic relaxation, reading R-19; projection, R-27; stopping
// rule, R-28), split into phases so that one system spreads over many
// workgroups.
//
// A system carries NV right-hand sides that share its matrix: the five
// components of the relaxed tensor (NV = 5, one Krylov sequence per column)
// or the pressure increment (NV = 1). Vectors are interleaved, entry v of row
// i at i * NV + v, and one lane handles one (row, column) pair: the NV lanes of
// a row read each matrix entry at the same address and the NV values of a
// neighbour as one contiguous access.
//
// One PCG iteration k, each phase a kernel over all systems at once:
//   PA(k)  convergence test on ||r_k|| per column; p_k = z_k + beta p_{k-1}
//          (computed on the fly at the neighbours); q = A p_k; accumulate p.q
//   PB(k)  alpha; x += alpha p_k; r_{k+1} = r_k - alpha q; first two smoothing
//          steps of the fine level (from zero, fused: the first step is local)
//   V-cycle on r_{k+1}: residual -> restriction -> [pre-smoothing, residual,
//          restriction on further large levels] -> one workgroup per system
//          for the small levels and the dense coarsest solve -> prolongation
//          -> two post-smoothing steps, the second of which gives z_{k+1} on
//          level 0 and accumulates r.z and sum z.
// A converged column keeps its x and r (p = 0, alpha = 0); a system is done
// when all its columns are. Scalars go into rotating per-iteration slots
// (slot k mod 4, one per column): each row-parallel workgroup stores its
// share, and k_mg_reduce adds a system's shares in block order into the slot;
// the one workgroup of a system in the tail and the completion adds its sum
// onto the cleared word. So every scalar is summed in a fixed order. A slot
// is cleared two phases after its last reader. The first lanes of each workgroup
// gather the slot words in one round trip and share them through LDS. Level
// sizes are fixed per system, so a fixed number of iterations can be replayed
// from a graph; systems that have converged leave every later phase at once,
// and k_mg_finish completes any system that needs more iterations in one
// workgroup, with the same phase bodies.
#include "pdfmc_kernels.h"

namespace pdfmc {

namespace {

constexpr int MGB = 256;   // threads of the row-parallel phases
constexpr int MGT = 1024;  // threads of the one-workgroup-per-system tail
constexpr int MGW = 512;   // threads of the one-workgroup-per-system completion
constexpr int NVMAX = NER;

// loads that bypass the non-coherent L1 (values written by atomics of the
// same kernel)
__device__ inline double aload(const double* p)
{
    return __longlong_as_double(
        __hip_atomic_load((const long long*)p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
}
__device__ inline int aloadi(const int* p) { return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT); }

// slot of iteration k for column v: [0] p.q  [1] r.r  [2] sum r  [3] r.z  [4] sum z
__device__ inline double* slot(const MgJob& J, int k, int v) { return J.acc + ((((k + 4) & 3) * J.nv) + v) * MG_SLOT; }
// set-up slot of column v: [0] sum b  [1] sum b^2 (raw)  [2] ||b||^2 (mean-free)
__device__ inline double* setup_slot(const MgJob& J, int v) { return J.acc + (4 * J.nv + v) * MG_SLOT; }

// The accumulator words a phase needs, gathered by the first lanes in one
// round trip and shared through LDS; for column v, w[NW v + ...]:
//   [0..4] slot k   [5..9] slot k-1   [10..14] slot k-2   [15..17] set-up slot
// COHERENT: the words were written by atomics of this same kernel (one
// workgroup completing a system), so the loads must bypass the L1.
constexpr int NW = 18;
template <int NV, bool COHERENT>
__device__ inline void gather_words(const MgJob& J, int k, double* w)
{
    __syncthreads();
    const int t = threadIdx.x;
    if (t < NW * NV) {
        const int v = t / NW, u = t - v * NW;
        const double* src = u < 5 ? slot(J, k, v) + u : u < 10 ? slot(J, k - 1, v) + (u - 5)
                          : u < 15 ? slot(J, k - 2, v) + (u - 10) : setup_slot(J, v) + (u - 15);
        w[t] = COHERENT ? aload(src) : *src;
    }
    __syncthreads();
}

// r.z of a slot (words s[0..4]), with z made mean-free for singular systems
__device__ inline double rz_w(const MgJob& J, const double* s)
{
    return J.mean_free ? s[3] - (s[4] / J.n) * s[2] : s[3];
}

// Sum M per-lane values over the workgroup, separately for each column
// (lane t holds column t % NV), in a fixed order. With part, the workgroup's
// sums go to part[v M + m] with plain stores (a row-parallel phase: one of
// many workgroups of the system; k_mg_reduce adds them in block order);
// without, they are added to dst(v, m) (the one workgroup of a system in
// k_mg_tail and k_mg_finish: a single addition onto a cleared word).
template <int NV, int M, typename D>
__device__ inline void block_accumulate(const double (&val)[M], D dst, double* part)
{
    const int t = threadIdx.x, nt = blockDim.x;
    if constexpr (NV == 1) {
        __shared__ double sh[16 * M];
        const int lane = t & 63, wid = t >> 6, nw = (nt + 63) >> 6;
#pragma unroll
        for (int m = 0; m < M; ++m) {
            double x = val[m];
            for (int d = 32; d >= 1; d >>= 1) x += __shfl_xor(x, d);
            if (lane == 0) sh[wid * M + m] = x;
        }
        __syncthreads();
        if (t < M) {
            double s = 0.0;
            for (int w = 0; w < nw; ++w) s += sh[w * M + t];
            if (part) part[t] = s;
            else unsafeAtomicAdd(dst(0, t), s);
        }
    } else {
        // lanes t and t + 64 NV hold the same column: fold each wave group of
        // 64 NV lanes... simply stage everything in LDS and let NV * M lanes sum
        __shared__ double sh[MGT * M];
#pragma unroll
        for (int m = 0; m < M; ++m) sh[m * nt + t] = val[m];
        __syncthreads();
        if (t < NV * M) {
            const int v = t % NV, m = t / NV;
            double s = 0.0;
            for (int u = v; u < nt; u += NV) s += sh[m * nt + u];
            if (part) part[v * M + m] = s;
            else unsafeAtomicAdd(dst(v, m), s);
        }
    }
    // workgroup-scope release: the atomics above have completed before any
    // thread of this workgroup reads the accumulators again (k_mg_finish);
    // other workgroups read them only in later kernels. An agent-scope fence
    // here would write back the whole L2 of the XCD from every workgroup.
    __threadfence_block();
    __syncthreads();
}

// Scalars of one column for a phase.
struct Scal {
    double a;     // PA: beta; PB: alpha (0 for converged columns)
    double b;     // PA: mean of z (singular systems)
    bool conv;    // column converged: ||r_k||^2 <= tol^2 ||b||^2
    bool zr;      // PB, first pass: zero right-hand side
    bool all;     // PA: every column of the system converged
};

template <int NV, bool COHERENT>
__device__ inline Scal pa_scalars(const MgJob& J, int k, int v)
{
    __shared__ double w[NW * NVMAX];
    gather_words<NV, COHERENT>(J, k, w);
    Scal s;
    s.all = true;
#pragma unroll
    for (int u = 0; u < NV; ++u) s.all = s.all && (w[NW * u + 6] <= J.tol * J.tol * w[NW * u + 17]);
    const double* x = w + NW * v;
    s.conv = x[5 + 1] <= J.tol * J.tol * x[15 + 2];
    s.zr = false;
    s.a = (k == 0 || s.conv) ? 0.0 : rz_w(J, x + 5) / rz_w(J, x + 10);
    s.b = J.mean_free ? x[5 + 4] / J.n : 0.0;
    return s;
}

template <int NV, bool COHERENT>
__device__ inline Scal pb_scalars(const MgJob& J, int k, bool first, int v)
{
    __shared__ double w[NW * NVMAX];
    gather_words<NV, COHERENT>(J, k, w);
    Scal s;
    const double* x = w + NW * v;
    s.all = false;
    s.conv = !first && x[5 + 1] <= J.tol * J.tol * x[15 + 2];
    s.zr = first && x[15 + 2] <= 1e-28 * x[15 + 1];
    s.a = (first || s.conv) ? 0.0 : rz_w(J, x + 5) / x[0];
    s.b = 0.0;
    return s;
}

// sum_k A(k, i) get(col(k, i)) over the row's entries rounded up to a
// multiple of 4 (padding entries are zero); the loads of a group of four
// entries are issued together
template <typename F>
__device__ inline double ell_row_f(const EllDev& A, F get, int i)
{
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
    const int64_t n = A.n;
    const int w = A.len ? min((A.len[i] + 3) & ~3, A.w) : A.w;
    for (int k = 0; k < w; k += 4) {
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

// column v of the product with an interleaved vector of NV columns
template <int NV>
__device__ inline double ell_row(const EllDev& A, const double* __restrict__ x, int i, int v)
{
    return ell_row_f(A, [&](int j) { return x[(int64_t)j * NV + v]; }, i);
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
// A body handles the (row, column) pairs t = t0, t0 + st, ... < t1 of one
// system, row t / NV and column t % NV. All threads of the workgroup call the
// accumulating bodies (they synchronise); their v is the column of the lane.

template <int NV>
__device__ __forceinline__ void pa_body(const MgJob& J, const AmgDev& H, int k, const Scal& sc, int v, int t0,
                                        int t1, int st, double* part)
{
    const double* z = J.ly[0];
    const double* pold = J.p[(k - 1) & 1];
    double* pnew = J.p[k & 1];
    auto pv = [&](int j) -> double {
        const int64_t a = (int64_t)j * NV + v;
        const double zz = z[a] - sc.b;
        return k == 0 ? zz : zz + sc.a * pold[a];
    };
    double pq = 0.0;
    if (!sc.conv)
        for (int t = t0; t < t1; t += st) {
            const int i = t / NV;
            const double s = ell_row_f(H.A[0], pv, i);
            const double pi = pv(i);
            pnew[t] = pi;
            J.q[t] = s;
            pq += pi * s;
        }
    else
        for (int t = t0; t < t1; t += st) {
            pnew[t] = 0.0;
            J.q[t] = 0.0;
        }
    block_accumulate<NV, 1>({pq}, [&](int u, int) { return slot(J, k, u); }, part);
}

template <int NV>
__device__ __forceinline__ void pb_body(const MgJob& J, const AmgDev& H, int k, bool first, const Scal& sc,
                                        bool leader, int v, int t0, int t1, int st, double* part)
{
    if (leader)
        for (int u = 0; u < NV * MG_SLOT; ++u) slot(J, k + 1, 0)[u] = 0.0;
    const double* rold = J.r[k & 1];
    double* rnew = J.r[(k + 1) & 1];
    const double* pk = J.p[k & 1];
    const double* q = J.q;
    auto bget = [&](int j) -> double {
        const int64_t a = (int64_t)j * NV + v;
        return sc.zr ? 0.0 : (first ? rold[a] : rold[a] - sc.a * q[a]);
    };
    const bool smooth = H.nbig >= 1;
    double rr = 0.0, sr = 0.0;
    for (int t = t0; t < t1; t += st) {
        const int i = t / NV;
        if (sc.zr) J.x[t] = 0.0;
        else if (!first) J.x[t] += sc.a * pk[t];
        const double rn = bget(i);
        rnew[t] = rn;
        rr += rn * rn;
        sr += rn;
        if (smooth) J.ly[0][t] = pre_row(H, 0, bget, i);
    }
    block_accumulate<NV, 2>({rr, sr}, [&](int u, int m) { return slot(J, k, u) + 1 + m; }, part);
}

template <int NV>
__device__ inline void res_pairs(const MgJob& J, const AmgDev& H, int l, int k, int t0, int t1, int st)
{
    const double* b = level_rhs(J, l, k);
    for (int t = t0; t < t1; t += st) J.lt[l][t] = b[t] - ell_row<NV>(H.A[l], J.ly[l], t / NV, t % NV);
}

template <int NV>
__device__ inline void restrict_pairs(const MgJob& J, const AmgDev& H, int l, int t0, int t1, int st)
{
    for (int t = t0; t < t1; t += st) J.lb[l][t] = ell_row<NV>(H.R[l - 1], J.lt[l - 1], t / NV, t % NV);
}

template <int NV>
__device__ inline void pre_pairs(const MgJob& J, const AmgDev& H, int l, int k, int t0, int t1, int st)
{
    const double* b = level_rhs(J, l, k);
    for (int t = t0; t < t1; t += st) {
        const int v = t % NV;
        J.ly[l][t] = pre_row(H, l, [&](int j) { return b[(int64_t)j * NV + v]; }, t / NV);
    }
}

// prolongation: lt = y + P y_c
template <int NV>
__device__ inline void prolong_pairs(const MgJob& J, const AmgDev& H, int l, int t0, int t1, int st)
{
    for (int t = t0; t < t1; t += st) J.lt[l][t] = J.ly[l][t] + ell_row<NV>(H.P[l], J.ly[l + 1], t / NV, t % NV);
}

// first post-smoothing step: la = lt + sa D^-1 (b - A lt)
template <int NV>
__device__ inline void post1_pairs(const MgJob& J, const AmgDev& H, int l, int k, int t0, int t1, int st)
{
    const double* b = level_rhs(J, l, k);
    const double* dinv = H.dinv[l];
    for (int t = t0; t < t1; t += st) {
        const int i = t / NV;
        J.la[l][t] = J.lt[l][t] + H.sa[l] * dinv[i] * (b[t] - ell_row<NV>(H.A[l], J.lt[l], i, t % NV));
    }
}

// second post-smoothing step: y = la + (se - 1)(la - lt) + sc D^-1 (b - A la);
// rz and sz accumulate r.z and sum z (used on level 0)
template <int NV>
__device__ inline void post2_pairs(const MgJob& J, const AmgDev& H, int l, int k, int t0, int t1, int st, double& rz,
                                   double& sz)
{
    const double* b = level_rhs(J, l, k);
    const double* dinv = H.dinv[l];
    const double em1 = H.se[l] - 1.0, sc = H.sc[l];
    for (int t = t0; t < t1; t += st) {
        const int i = t / NV;
        const double a = J.la[l][t];
        const double y = a + em1 * (a - J.lt[l][t]) + sc * dinv[i] * (b[t] - ell_row<NV>(H.A[l], J.la[l], i, t % NV));
        J.ly[l][t] = y;
        rz += b[t] * y;
        sz += y;
    }
}

template <int NV>
__device__ inline void accumulate_rz(const MgJob& J, int k, double rz, double sz, double* part)
{
    block_accumulate<NV, 2>({rz, sz}, [&](int u, int m) { return slot(J, k, u) + 3 + m; }, part);
}

// No pair: the start of the pair loops for lanes beyond the multiple of NV.
constexpr int NO_PAIR = 0x3fffffff;

// The small levels (nbig and below) of one system's V-cycle, in one
// workgroup; the pair loops use the first nt lanes (a multiple of NV), the
// others only join the barriers and reductions.
template <int NV>
__device__ __forceinline__ void tail_body(const MgJob& J, const AmgDev& H, int k, int nt)
{
    const int tid = (int)threadIdx.x < nt ? (int)threadIdx.x : NO_PAIR;
    const int l0 = H.nbig, nl = H.nlev;
    if (l0 >= 1) {
        restrict_pairs<NV>(J, H, l0, tid, NV * H.n[l0], nt);
        __syncthreads();
    }
    for (int l = l0; l < nl - 1; ++l) {
        pre_pairs<NV>(J, H, l, k, tid, NV * H.n[l], nt);
        __syncthreads();
        res_pairs<NV>(J, H, l, k, tid, NV * H.n[l], nt);
        __syncthreads();
        restrict_pairs<NV>(J, H, l + 1, tid, NV * H.n[l + 1], nt);
        __syncthreads();
    }
    {
        // dense coarse solve, 16 lanes per (row, column) pair (nc <= 64 rows)
        const int l = nl - 1, nc = H.n[l];
        const double* b = level_rhs(J, l, k);
        for (int t = threadIdx.x; t < 16 * AMG_MAXC * NV; t += blockDim.x) {
            const int pr = t >> 4, part = t & 15;
            const int i = pr / NV, v = pr % NV;
            double s = 0.0;
            if (i < nc)
                for (int j = part; j < nc; j += 16) s += H.ainv[i * AMG_MAXC + j] * b[(int64_t)j * NV + v];
            s += __shfl_xor(s, 8);
            s += __shfl_xor(s, 4);
            s += __shfl_xor(s, 2);
            s += __shfl_xor(s, 1);
            if (i < nc && part == 0) J.ly[l][pr] = s;
        }
        __syncthreads();
    }
    for (int l = nl - 2; l >= l0; --l) {
        prolong_pairs<NV>(J, H, l, tid, NV * H.n[l], nt);
        __syncthreads();
        post1_pairs<NV>(J, H, l, k, tid, NV * H.n[l], nt);
        __syncthreads();
        double rz = 0.0, sz = 0.0;
        post2_pairs<NV>(J, H, l, k, tid, NV * H.n[l], nt, rz, sz);
        __syncthreads();
    }
    if (l0 == 0) {
        // z = ly[0] is complete: accumulate r.z and sum z
        const double* r = J.r[(k + 1) & 1];
        double rz = 0.0, sz = 0.0;
        for (int t = tid; t < NV * J.n; t += nt) {
            rz += r[t] * J.ly[0][t];
            sz += J.ly[0][t];
        }
        accumulate_rz<NV>(J, k, rz, sz, nullptr);
    }
}

// (row, column) pairs of a row-parallel workgroup: rows e.y .. e.y + MGB/NV
template <int NV>
struct Pairs {
    int t0, t1, v;
    bool live;     // the lane holds a pair of the block
};
template <int NV>
__device__ inline Pairs<NV> block_pairs(int row0, int rows)
{
    constexpr int RPB = MGB / NV;
    Pairs<NV> p;
    const int t = threadIdx.x;
    p.v = t % NV;
    p.live = t < RPB * NV && row0 + t / NV < rows;
    p.t0 = NV * row0 + t;
    p.t1 = p.live ? p.t0 + 1 : p.t0;
    return p;
}

// the partial sums of the row-parallel workgroup whose first row is row0
template <int NV>
__device__ inline double* block_part(const MgJob& J, int row0)
{
    return J.part + (int64_t)(row0 / (MGB / NV)) * MG_PART;
}

// ---------------------------------------------------------------- kernel bodies

template <int NV>
__device__ void setup1_body(const MgJob& J, int row0)
{
    const Pairs<NV> q = block_pairs<NV>(row0, J.n);
    const double x = q.live ? J.b[q.t0] : 0.0;
    block_accumulate<NV, 2>({x, x * x}, [&](int u, int m) { return setup_slot(J, u) + m; }, block_part<NV>(J, row0));
}

template <int NV>
__device__ void setup2_body(const MgJob& J, const AmgDev& H, int row0)
{
    const Pairs<NV> q = block_pairs<NV>(row0, J.n);
    double bb = 0.0;
    if (q.live) {
        const int t = q.t0;
        const double mb = J.mean_free ? setup_slot(J, q.v)[0] / J.n : 0.0;
        const double b = J.b[t] - mb;
        J.b[t] = b;
        if (J.warm) {
            J.r[1][t] = b - ell_row<NV>(H.A[0], J.x, t / NV, q.v);
        } else {
            J.x[t] = 0.0;
            J.r[1][t] = b;
        }
        bb = b * b;
    }
    block_accumulate<NV, 1>({bb}, [&](int u, int) { return setup_slot(J, u) + 2; }, block_part<NV>(J, row0));
}

template <int NV>
__device__ void pa_kernel_body(const MgJob& J, const AmgDev& H, int row0, int k)
{
    const Pairs<NV> q = block_pairs<NV>(row0, J.n);
    const Scal sc = pa_scalars<NV, false>(J, k, q.v);
    if (sc.all) {
        if (row0 == 0 && threadIdx.x == 0) { J.state[0] = 1; J.state[1] = k; }
        return;
    }
    pa_body<NV>(J, H, k, sc, q.v, q.t0, q.t1, 1, block_part<NV>(J, row0));
}

template <int NV>
__device__ void pb_kernel_body(const MgJob& J, const AmgDev& H, int row0, int k, bool first)
{
    const Pairs<NV> q = block_pairs<NV>(row0, J.n);
    const Scal sc = pb_scalars<NV, false>(J, k, first, q.v);
    pb_body<NV>(J, H, k, first, sc, row0 == 0 && threadIdx.x == 0, q.v, q.t0, q.t1, 1, block_part<NV>(J, row0));
}

template <int NV>
__device__ void finish_body(const MgJob& J, const AmgDev& H, int k0)
{
    const int n = J.n;
    const int tid = threadIdx.x;
    // lanes beyond a multiple of NV idle in the pair loops but join every
    // barrier and reduction
    const int nt = (blockDim.x / NV) * NV;
    const int v = tid % NV;
    const int t0 = tid < nt ? tid : NO_PAIR;
    __shared__ int st[2];
    if (tid == 0) { st[0] = aloadi(J.state); st[1] = aloadi(J.state + 1); }
    __syncthreads();
    bool done = st[0] != 0;
    int it = done ? st[1] : 0;
    // from the first iteration the phases did not run for this system
    for (int k = min(min(k0, J.ksw), J.maxit); !done; ++k) {
        const Scal sa = pa_scalars<NV, true>(J, k, v);
        if (sa.all) { done = true; it = k; break; }
        if (k >= J.maxit) { it = k; break; }
        pa_body<NV>(J, H, k, sa, v, t0, NV * n, nt, nullptr);
        const Scal sb = pb_scalars<NV, true>(J, k, false, v);
        pb_body<NV>(J, H, k, false, sb, tid == 0, v, t0, NV * n, nt, nullptr);
        if (H.nbig >= 1) {
            res_pairs<NV>(J, H, 0, k, t0, NV * n, nt);
            __syncthreads();
            for (int l = 1; l < H.nbig; ++l) {
                restrict_pairs<NV>(J, H, l, t0, NV * H.n[l], nt);
                __syncthreads();
                pre_pairs<NV>(J, H, l, k, t0, NV * H.n[l], nt);
                __syncthreads();
                res_pairs<NV>(J, H, l, k, t0, NV * H.n[l], nt);
                __syncthreads();
            }
        }
        tail_body<NV>(J, H, k, nt);
        __syncthreads();
        for (int l = H.nbig - 1; l >= 0; --l) {
            prolong_pairs<NV>(J, H, l, t0, NV * H.n[l], nt);
            __syncthreads();
            post1_pairs<NV>(J, H, l, k, t0, NV * H.n[l], nt);
            __syncthreads();
            double rz = 0.0, sz = 0.0;
            post2_pairs<NV>(J, H, l, k, t0, NV * H.n[l], nt, rz, sz);
            if (l == 0) accumulate_rz<NV>(J, k, rz, sz, nullptr);
            else __syncthreads();
        }
    }
    if (NV == 1 && J.mean_free) {
        // singular system: remove the mean of x
        double s = 0.0;
        for (int i = tid; i < n; i += blockDim.x) s += J.x[i];
        __shared__ double sh[16];
        for (int d = 32; d >= 1; d >>= 1) s += __shfl_xor(s, d);
        if ((tid & 63) == 0) sh[tid >> 6] = s;
        __syncthreads();
        double m = 0.0;
        for (int w = 0; w < (blockDim.x + 63) / 64; ++w) m += sh[w];
        m /= n;
        for (int i = tid; i < n; i += blockDim.x) J.x[i] -= m;
    }
    __syncthreads();
    if (tid == 0) {
        // iterations are counted per column
        atomicAdd(J.iters, (unsigned long long)it * NV);
        if (!done) atomicAdd(J.fails, 1ull);
        atomicMax(J.need, (unsigned int)it);
        J.state[0] = 0;
        J.state[1] = 0;
    }
    for (int u = tid; u < MG_NSLOT * NV * MG_SLOT; u += blockDim.x) J.acc[u] = 0.0;
}

}  // namespace

// ---------------------------------------------------------------- kernels

// instantiate CALL for the column count of system J
#define MG_DISPATCH(J, CALL)  \
    do {                      \
        if ((J).nv == NER) {  \
            CALL(NER);        \
        } else {              \
            CALL(1);          \
        }                     \
    } while (0)

// Inverse diagonals of every level; tab entries: (hierarchy, level, first row)
__global__ void k_mg_dinv(const AmgDev* __restrict__ hs, const int4* __restrict__ tab)
{
    const int4 e = tab[xcd_block((int)blockIdx.x, (int)gridDim.x)];
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
// elimination in LDS, one workgroup per hierarchy: hierarchies first,
// first + stride, ... (the relaxation hierarchies every solve, the constant
// projection hierarchies once).
__global__ void __launch_bounds__(1024) k_mg_coarse(const AmgDev* __restrict__ hs, int first, int stride)
{
    const AmgDev& H = hs[first + stride * (int)blockIdx.x];
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

// Row-parallel phases: tab entries (system, first row, hierarchy, 0); a
// workgroup covers MGB / nv rows of its system.

// Set-up 1: sum b and sum b^2 per column
__global__ void __launch_bounds__(MGB) k_mg_setup1(const MgJob* __restrict__ jobs, const int4* __restrict__ tab,
                                                   const int32_t* __restrict__ st)
{
    const int4 e = tab[xcd_block((int)blockIdx.x, (int)gridDim.x)];
    const MgJob& J = jobs[e.x];
#define SETUP1(NV) setup1_body<NV>(J, e.y)
    MG_DISPATCH(J, SETUP1);
#undef SETUP1
}

// Set-up 2: mean-free right-hand side, r = b - A x (warm start) or r = b
// with x = 0, ||b||^2 per column
__global__ void __launch_bounds__(MGB) k_mg_setup2(const MgJob* __restrict__ jobs, const AmgDev* __restrict__ hs,
                                                   const int4* __restrict__ tab, const int32_t* __restrict__ st)
{
    const int4 e = tab[xcd_block((int)blockIdx.x, (int)gridDim.x)];
    const MgJob& J = jobs[e.x];
#define SETUP2(NV) setup2_body<NV>(J, hs[e.z], e.y)
    MG_DISPATCH(J, SETUP2);
#undef SETUP2
}

__global__ void __launch_bounds__(MGB) k_mg_pa(const MgJob* __restrict__ jobs, const AmgDev* __restrict__ hs,
                                               const int4* __restrict__ tab, const int32_t* __restrict__ st, int k)
{
    const int4 e = tab[xcd_block((int)blockIdx.x, (int)gridDim.x)];
    const MgJob& J = jobs[e.x];
    if (st[2 * e.x] != 0 || k >= J.ksw) return;
#define PA(NV) pa_kernel_body<NV>(J, hs[e.z], e.y, k)
    MG_DISPATCH(J, PA);
#undef PA
}

__global__ void __launch_bounds__(MGB) k_mg_pb(const MgJob* __restrict__ jobs, const AmgDev* __restrict__ hs,
                                               const int4* __restrict__ tab, const int32_t* __restrict__ st, int k,
                                               int first)
{
    const int4 e = tab[xcd_block((int)blockIdx.x, (int)gridDim.x)];
    const MgJob& J = jobs[e.x];
    if (st[2 * e.x] != 0 || k >= J.ksw) return;
#define PB(NV) pb_kernel_body<NV>(J, hs[e.z], e.y, k, first != 0)
    MG_DISPATCH(J, PB);
#undef PB
}

// residual of level l (tab: rows of level l of the systems with nbig > l)
__global__ void __launch_bounds__(MGB) k_mg_res(const MgJob* __restrict__ jobs, const AmgDev* __restrict__ hs,
                                                const int4* __restrict__ tab, const int32_t* __restrict__ st, int l,
                                                int k)
{
    const int4 e = tab[xcd_block((int)blockIdx.x, (int)gridDim.x)];
    const MgJob& J = jobs[e.x];
    if (st[2 * e.x] != 0 || k >= J.ksw) return;
    const AmgDev& H = hs[e.z];
#define RES(NV)                                                  \
    {                                                            \
        const Pairs<NV> q = block_pairs<NV>(e.y, H.n[l]);        \
        res_pairs<NV>(J, H, l, k, q.t0, q.t1, 1);                \
    }
    MG_DISPATCH(J, RES);
#undef RES
}

// restriction to level l >= 1 (the pre-smoothing of level l needs every row
// of the restricted right-hand side, so it is a phase of its own)
__global__ void __launch_bounds__(MGB) k_mg_restrict(const MgJob* __restrict__ jobs, const AmgDev* __restrict__ hs,
                                                     const int4* __restrict__ tab, const int32_t* __restrict__ st,
                                                     int l, int k)
{
    const int4 e = tab[xcd_block((int)blockIdx.x, (int)gridDim.x)];
    const MgJob& J = jobs[e.x];
    if (st[2 * e.x] != 0 || k >= J.ksw) return;
    const AmgDev& H = hs[e.z];
#define RST(NV)                                                  \
    {                                                            \
        const Pairs<NV> q = block_pairs<NV>(e.y, H.n[l]);        \
        restrict_pairs<NV>(J, H, l, q.t0, q.t1, 1);              \
    }
    MG_DISPATCH(J, RST);
#undef RST
}

__global__ void __launch_bounds__(MGB) k_mg_pre(const MgJob* __restrict__ jobs, const AmgDev* __restrict__ hs,
                                                const int4* __restrict__ tab, const int32_t* __restrict__ st, int l,
                                                int k)
{
    const int4 e = tab[xcd_block((int)blockIdx.x, (int)gridDim.x)];
    const MgJob& J = jobs[e.x];
    if (st[2 * e.x] != 0 || k >= J.ksw) return;
    const AmgDev& H = hs[e.z];
#define PRE(NV)                                                  \
    {                                                            \
        const Pairs<NV> q = block_pairs<NV>(e.y, H.n[l]);        \
        pre_pairs<NV>(J, H, l, k, q.t0, q.t1, 1);                \
    }
    MG_DISPATCH(J, PRE);
#undef PRE
}

__global__ void __launch_bounds__(MGT) k_mg_tail(const MgJob* __restrict__ jobs, const AmgDev* __restrict__ hs,
                                                 const int32_t* __restrict__ st, int k)
{
    const MgJob& J = jobs[blockIdx.x];
    if (st[2 * blockIdx.x] != 0 || J.n <= 0 || k >= J.ksw) return;
    // the pair loops use a multiple of NV lanes; the others only join the
    // barriers and reductions
#define TAIL(NV) tail_body<NV>(J, hs[J.hier], k, (MGT / NV) * NV)
    MG_DISPATCH(J, TAIL);
#undef TAIL
}

__global__ void __launch_bounds__(MGB) k_mg_prolong(const MgJob* __restrict__ jobs, const AmgDev* __restrict__ hs,
                                                    const int4* __restrict__ tab, const int32_t* __restrict__ st,
                                                    int l, int k)
{
    const int4 e = tab[xcd_block((int)blockIdx.x, (int)gridDim.x)];
    const MgJob& J = jobs[e.x];
    if (st[2 * e.x] != 0 || k >= J.ksw) return;
    const AmgDev& H = hs[e.z];
#define PRL(NV)                                                  \
    {                                                            \
        const Pairs<NV> q = block_pairs<NV>(e.y, H.n[l]);        \
        prolong_pairs<NV>(J, H, l, q.t0, q.t1, 1);               \
    }
    MG_DISPATCH(J, PRL);
#undef PRL
}

__global__ void __launch_bounds__(MGB) k_mg_post1(const MgJob* __restrict__ jobs, const AmgDev* __restrict__ hs,
                                                  const int4* __restrict__ tab, const int32_t* __restrict__ st, int l,
                                                  int k)
{
    const int4 e = tab[xcd_block((int)blockIdx.x, (int)gridDim.x)];
    const MgJob& J = jobs[e.x];
    if (st[2 * e.x] != 0 || k >= J.ksw) return;
    const AmgDev& H = hs[e.z];
#define PS1(NV)                                                  \
    {                                                            \
        const Pairs<NV> q = block_pairs<NV>(e.y, H.n[l]);        \
        post1_pairs<NV>(J, H, l, k, q.t0, q.t1, 1);              \
    }
    MG_DISPATCH(J, PS1);
#undef PS1
}

__global__ void __launch_bounds__(MGB) k_mg_post2(const MgJob* __restrict__ jobs, const AmgDev* __restrict__ hs,
                                                  const int4* __restrict__ tab, const int32_t* __restrict__ st, int l,
                                                  int k)
{
    const int4 e = tab[xcd_block((int)blockIdx.x, (int)gridDim.x)];
    const MgJob& J = jobs[e.x];
    if (st[2 * e.x] != 0 || k >= J.ksw) return;
    const AmgDev& H = hs[e.z];
#define PS2(NV)                                                  \
    {                                                            \
        const Pairs<NV> q = block_pairs<NV>(e.y, H.n[l]);        \
        double rz = 0.0, sz = 0.0;                               \
        post2_pairs<NV>(J, H, l, k, q.t0, q.t1, 1, rz, sz);      \
        if (l == 0) accumulate_rz<NV>(J, k, rz, sz, block_part<NV>(J, e.y)); \
    }
    MG_DISPATCH(J, PS2);
#undef PS2
}

// The sums of a row-parallel phase: for each system that ran the phase, the
// partials of its workgroups (row-block order) are added in a fixed order
// (16 lanes per word, each over every 16th block in turn, then the 16 lanes
// in order) and stored into the phase's accumulator words, slot k words
// word0 .. word0 + M - 1 (setup: the set-up slot). The same skips as the
// phase: a converged system or one past its cap (not for the set-up); with
// big_only, a system whose level 0 the tail handles (its k_mg_tail adds its
// own sums). So a system's sums depend on its rows alone, in any batch.
__global__ void __launch_bounds__(256) k_mg_reduce(const MgJob* __restrict__ jobs, const AmgDev* __restrict__ hs,
                                                   const int32_t* __restrict__ st, int k, int word0, int M, int setup,
                                                   int big_only)
{
    const MgJob& J = jobs[blockIdx.x];
    if (J.n <= 0) return;
    if (!setup && (st[2 * blockIdx.x] != 0 || k >= J.ksw)) return;
    if (big_only && hs[J.hier].nbig < 1) return;
    __shared__ double sh[MG_PART * 16];
    const int nw = J.nv * M, nb = J.nblk0;
    const int t = threadIdx.x, w = t >> 4, j = t & 15;
    if (w < nw) {
        double s = 0.0;
        for (int b = j; b < nb; b += 16) s += J.part[(int64_t)b * MG_PART + w];
        sh[t] = s;
    }
    __syncthreads();
    if (t < nw) {
        double s = 0.0;
        for (int q = 0; q < 16; ++q) s += sh[t * 16 + q];
        const int v = t / M, m = t - v * M;
        (setup ? setup_slot(J, v) : slot(J, k, v))[word0 + m] = s;
    }
}

// Completes, in one workgroup per system, every system that has not
// converged within the first k0 iterations; then makes singular solutions
// mean-free, counts iterations and failures, and clears the per-system state
// for the next solve.
__global__ void __launch_bounds__(MGW) k_mg_finish(const MgJob* __restrict__ jobs, const AmgDev* __restrict__ hs,
                                                   int k0)
{
    const MgJob& J = jobs[blockIdx.x];
    if (J.n <= 0) return;
#define FIN(NV) finish_body<NV>(J, hs[J.hier], k0)
    MG_DISPATCH(J, FIN);
#undef FIN
}

}  // namespace pdfmc
