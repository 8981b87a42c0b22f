// Counting sort of the particle arrays by element (periodic re-sort).
//
// Keeping each case's particles grouped by element keeps the gathers of
// element records and nodal fields cache-resident and the runs of equal
// element long, which is what the particle kernel's segmented scatter
// relies on. Order inside an element is not kept (the run heads claim their
// slots with atomics); results do not depend on it beyond the summation
// order of the FP64 node sums.
//   k_sort_hist     per-element counts (one atomic per run of equal element)
//   k_sort_scan     exclusive scan of the counts, one workgroup
//   k_sort_scatter  move every particle field to the other buffer set
#include "pdfmc_dev.h"
#include "pdfmc_sort.h"

namespace pdfmc {

__device__ inline void sort_runs(int key, bool& head, int& rank, int& len)
{
    const int lane = __lane_id();
    const int prev = __shfl_up(key, 1);
    head = (lane == 0) || (prev != key);
    const unsigned long long hm = __ballot(head);
    // first lane of my run, last lane of my run
    const unsigned long long below = hm & (~0ull >> (63 - lane));
    const int first = 63 - __clzll(below);
    const unsigned long long above = hm & ~(~0ull >> (63 - lane));
    const int next = above ? (__ffsll(above) - 1) : 64;
    rank = lane - first;
    len = next - first;
}

__global__ void k_sort_hist(SortArgs A)
{
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int tile = (int)(gid / TILE);
    if (tile >= A.ntiles) return;
    const CaseDev& C = A.cases[A.tile_case[tile]];
    const int64_t i = gid - C.poff;
    const bool valid = i >= 0 && i < C.np;
    const int key = valid ? A.elem[gid] : -1;
    bool head; int rank, len;
    sort_runs(key, head, rank, len);
    if (head && key >= 0) atomicAdd(A.count + key, len);
}

// exclusive scan of count[0..ne) into offset, then rebased per case so that
// offset[e] = poff(case) + sum of counts of the case's earlier elements;
// cursor[e] is reset to offset[e].
__global__ void __launch_bounds__(1024) k_sort_scan(SortArgs A)
{
    __shared__ int64_t part[1024];
    const int tid = threadIdx.x, nt = blockDim.x;
    const int64_t chunk = (A.ne + nt - 1) / nt;
    const int64_t lo = tid * chunk, hi = lo + chunk < A.ne ? lo + chunk : A.ne;
    int64_t s = 0;
    for (int64_t e = lo; e < hi; ++e) s += A.count[e];
    part[tid] = s;
    __syncthreads();
    for (int d = 1; d < nt; d <<= 1) {
        int64_t v = tid >= d ? part[tid - d] : 0;
        __syncthreads();
        part[tid] += v;
        __syncthreads();
    }
    int64_t run = part[tid] - s;
    for (int64_t e = lo; e < hi; ++e) {
        A.scan[e] = run;
        run += A.count[e];
    }
    __syncthreads();
    __threadfence_block();
    for (int64_t e = lo; e < hi; ++e) {
        const CaseDev& C = A.cases[A.elem_case[e]];
        const int64_t off = A.scan[e] - A.scan[C.eoff] + C.poff;
        A.cursor[e] = off;
    }
}

template <typename R>
__global__ void k_sort_scatter(SortArgs A, Particles<R> src, Particles<R> dst)
{
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int tile = (int)(gid / TILE);
    if (tile >= A.ntiles) return;
    const CaseDev& C = A.cases[A.tile_case[tile]];
    const int64_t i = gid - C.poff;
    const bool valid = i >= 0 && i < C.np;
    const int key = valid ? src.elem[gid] : -1;
    bool head; int rank, len;
    sort_runs(key, head, rank, len);
    unsigned long long base = 0;
    if (head && key >= 0) base = atomicAdd((unsigned long long*)(A.cursor + key), (unsigned long long)len);
    // broadcast the run head's base to the run
    const int lane = __lane_id();
    const int first = lane - rank;
    base = __shfl(base, first);
    if (!valid) return;
    const int64_t q = (int64_t)base + rank;
    const int64_t j = q - C.poff;
    dst.x[q] = src.x[gid]; dst.y[q] = src.y[gid];
    dst.u[q] = src.u[gid]; dst.v[q] = src.v[gid]; dst.w[q] = src.w[gid];
    dst.om[q] = src.om[gid]; dst.wt[q] = src.wt[gid];
    dst.elem[q] = key; dst.id[q] = src.id[gid]; dst.bin[q] = src.bin[gid];
    for (int a = 0; a < C.ns; ++a) dst.psi[C.psioff + (int64_t)a * C.cap + j] = src.psi[C.psioff + (int64_t)a * C.cap + i];
}
template __global__ void k_sort_scatter<double>(SortArgs, Particles<double>, Particles<double>);
template __global__ void k_sort_scatter<float>(SortArgs, Particles<float>, Particles<float>);

}  // namespace pdfmc
