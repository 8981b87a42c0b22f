// Projection solve (reading R-27) by the nested-dissection Cholesky factor of
// the constant projection matrix: the right-hand side is made mean-free (the
// Neumann problem's compatibility condition) and the decoupled unknown set to
// zero; a forward sweep over the supernodes from the leaves up (all cases and
// all supernodes of one height in one launch) and a backward sweep from the
// root down give the solution, which is finally made mean-free.
//
// Forward, supernode S: y_S = L11^-1 b_S; b_R -= L21 y_S for the later
// unknowns R it reaches. Siblings reach common ancestors, so S stores its
// updates L21 y_S in a slot of its own, and an ancestor subtracts the updates
// of its unknowns, in supernode order, when it loads b: the same bits on
// every run and in any batch.
// Backward: x_S = L11^-T (y_S - L21^T x_R), the x_R final from higher sweeps.
#include "pdfmc_kernels.h"

namespace pdfmc {

namespace {


__device__ inline double wave_sum(double a)
{
    for (int d = 32; d >= 1; d >>= 1) a += __shfl_xor(a, d);
    return a;
}

// sum over the workgroup (all threads call)
__device__ inline double block_sum(double a)
{
    __shared__ double sh[16];
    a = wave_sum(a);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) sh[wid] = a;
    __syncthreads();
    double s = 0.0;
    for (int w = 0; w < (int)(blockDim.x + 63) / 64; ++w) s += sh[w];
    return s;
}

}  // namespace

// x = b - mean(b) over each case, x[pin] = 0; one workgroup per case
__global__ void __launch_bounds__(1024) k_ds_prep(const DsCase* __restrict__ cs, const double* __restrict__ b,
                                                  double* __restrict__ x)
{
    const DsCase C = cs[blockIdx.x];
    double s = 0.0;
    for (int i = threadIdx.x; i < C.n; i += blockDim.x) s += b[C.noff + i];
    const double mean = block_sum(s) / C.n;
    for (int i = threadIdx.x; i < C.n; i += blockDim.x) x[C.noff + i] = i == C.pin ? 0.0 : b[C.noff + i] - mean;
}

// x -= mean(x) over each case; one workgroup per case
__global__ void __launch_bounds__(1024) k_ds_post(const DsCase* __restrict__ cs, double* __restrict__ x)
{
    const DsCase C = cs[blockIdx.x];
    double s = 0.0;
    for (int i = threadIdx.x; i < C.n; i += blockDim.x) s += x[C.noff + i];
    const double mean = block_sum(s) / C.n;
    for (int i = threadIdx.x; i < C.n; i += blockDim.x) x[C.noff + i] -= mean;
}

// forward sweep over the supernodes list[0 .. gridDim.x) (one height);
// DSB threads per supernode (more for the few large separators near the
// root), LDS for CAP unknowns (small for the many leaves, so that more of
// them share a CU)
template <int DSB, int CAP>
__global__ void __launch_bounds__(DSB) k_ds_forward(const DsNode* __restrict__ nodes, const int32_t* __restrict__ list,
                                                    const int32_t* __restrict__ idx, const double* __restrict__ val,
                                                    double* __restrict__ x, DsUpd U)
{
    const DsNode N = nodes[list[blockIdx.x]];
    const int s = N.s, m = N.m;
    const int32_t* vi = idx + N.idx;
    const double* Li = val + N.val;
    const double* L21 = Li + (int64_t)s * s;
    __shared__ double bs[CAP], ys[CAP];
    for (int t = threadIdx.x; t < s; t += DSB) {
        const int u = vi[t];
        double b = x[u];
        for (int q = U.cptr[u]; q < U.cptr[u + 1]; ++q) b -= U.contrib[U.clist[q]];
        bs[t] = b;
    }
    __syncthreads();
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    constexpr int NWV = DSB / 64;
    for (int i = wv; i < s; i += NWV) {
        const double* row = Li + (int64_t)i * s;
        double a = 0.0;
        for (int j = lane; j <= i; j += 64) a += row[j] * bs[j];
        a = wave_sum(a);
        if (lane == 0) {
            ys[i] = a;
            x[vi[i]] = a;
        }
    }
    __syncthreads();
    for (int r = wv; r < m; r += NWV) {
        const double* row = L21 + (int64_t)r * s;
        double a = 0.0;
        for (int j = lane; j < s; j += 64) a += row[j] * ys[j];
        a = wave_sum(a);
        if (lane == 0) U.contrib[N.cof + r] = a;
    }
}

// backward sweep over the supernodes list[0 .. gridDim.x) (one height)
template <int DSB, int CAP>
__global__ void __launch_bounds__(DSB) k_ds_backward(const DsNode* __restrict__ nodes, const int32_t* __restrict__ list,
                                                     const int32_t* __restrict__ idx, const double* __restrict__ val,
                                                     double* __restrict__ x)
{
    const DsNode N = nodes[list[blockIdx.x]];
    const int s = N.s, m = N.m;
    const int32_t* vi = idx + N.idx;
    const double* Li = val + N.val;
    const double* L21 = Li + (int64_t)s * s;
    __shared__ double xr[CAP], ts[CAP], part[DSB];
    for (int r = threadIdx.x; r < m; r += DSB) xr[r] = x[vi[s + r]];
    __syncthreads();
    // t_j = y_j - sum_r L21[r][j] x_r: for a supernode of at most half the
    // lanes of the split, the rows r are split over G groups of lanes whose
    // partial sums are added through LDS. The split is the supernode's own:
    // 256 lanes for one that the narrow sweep takes (s + m <= 128), all DSB
    // for the others, which always run wide. So its bits do not depend on
    // the variant that the other supernodes of its height need.
    const int sp = (s + 63) & ~63;
    const int gl = s + m <= 128 ? 256 : DSB;
    const int G = sp > 0 && sp <= gl / 2 ? gl / sp : 1;
    if (G > 1) {
        const int g = threadIdx.x / sp, j = threadIdx.x - g * sp;
        double a = 0.0;
        if (j < s && g < G)
            for (int r = g; r < m; r += G) a += L21[(int64_t)r * s + j] * xr[r];
        part[threadIdx.x] = a;
        __syncthreads();
        if (threadIdx.x < s) {
            double t = x[vi[threadIdx.x]];
            for (int q = 0; q < G; ++q) t -= part[q * sp + threadIdx.x];
            ts[threadIdx.x] = t;
        }
    } else {
        for (int j = threadIdx.x; j < s; j += DSB) {
            double a = x[vi[j]];
            for (int r = 0; r < m; ++r) a -= L21[(int64_t)r * s + j] * xr[r];
            ts[j] = a;
        }
    }
    __syncthreads();
    for (int j = threadIdx.x; j < s; j += DSB) {
        double a = 0.0;
        for (int i = j; i < s; ++i) a += Li[(int64_t)i * s + j] * ts[i];
        x[vi[j]] = a;
    }
}

#define DS_INST(B, C)                                                                                           \
    template __global__ void k_ds_forward<B, C>(const DsNode*, const int32_t*, const int32_t*, const double*, double*, \
                                                DsUpd);                                                                 \
    template __global__ void k_ds_backward<B, C>(const DsNode*, const int32_t*, const int32_t*, const double*, double*);
DS_INST(256, DS_SMALL)
DS_INST(1024, DS_SMALL)
DS_INST(1024, DS_MAXS)
#undef DS_INST

}  // namespace pdfmc
