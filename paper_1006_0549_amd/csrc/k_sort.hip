// Counting sort of the particle arrays by element (periodic re-sort).
//
// Keeping each case's particles grouped by element keeps the gathers of
// element records and nodal fields cache-resident and the runs of equal
// element long, which is what the particle kernel's segmented scatter
// relies on. Order inside an element is not kept (the run heads claim their
// slots with atomics); results do not depend on it beyond the summation
// order of the FP64 node sums.
//   k_sort_hist     per-element counts (one atomic per run of equal element)
//   k_sort_scan_*   exclusive scan of the counts (blocks, block totals), and
//   k_sort_cursor   the per-case slot cursors
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

// Exclusive scan of count[0..ne) in three passes: a scan inside each block of
// SCAN_B elements with its total, a scan of the block totals, and the
// cursors: cursor[e] = poff(case) + sum of the counts of the case's earlier
// elements.

__device__ inline int64_t block_excl_scan(int64_t v, int64_t& total)
{
    // SCAN_B threads: wave scans by shuffles, then the wave totals
    __shared__ int64_t wsum[SCAN_B / 64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    int64_t x = v;
    for (int d = 1; d < 64; d <<= 1) {
        const int64_t y = __shfl_up(x, d);
        if (lane >= d) x += y;
    }
    if (lane == 63) wsum[w] = x;
    __syncthreads();
    int64_t before = 0;
    total = 0;
    for (int k = 0; k < SCAN_B / 64; ++k) {
        if (k < w) before += wsum[k];
        total += wsum[k];
    }
    return before + x - v;
}

__global__ void __launch_bounds__(SCAN_B) k_sort_scan_blocks(SortArgs A)
{
    const int64_t e = (int64_t)blockIdx.x * SCAN_B + threadIdx.x;
    const int64_t v = e < A.ne ? A.count[e] : 0;
    int64_t total;
    const int64_t x = block_excl_scan(v, total);
    if (e < A.ne) A.scan[e] = x;
    if (threadIdx.x == 0) A.bsum[blockIdx.x] = total;
}

// one workgroup: exclusive scan of the nb block totals, SCAN_B at a time
__global__ void __launch_bounds__(SCAN_B) k_sort_scan_totals(SortArgs A, int nb)
{
    int64_t carry = 0;
    for (int b0 = 0; b0 < nb; b0 += SCAN_B) {
        const int b = b0 + threadIdx.x;
        const int64_t v = b < nb ? A.bsum[b] : 0;
        int64_t total;
        const int64_t x = block_excl_scan(v, total);
        __syncthreads();
        if (b < nb) A.bsum[b] = carry + x;
        carry += total;
        __syncthreads();
    }
}

__global__ void __launch_bounds__(SCAN_B) k_sort_cursor(SortArgs A)
{
    const int64_t e = (int64_t)blockIdx.x * SCAN_B + threadIdx.x;
    if (e >= A.ne) return;
    const CaseDev& C = A.cases[A.elem_case[e]];
    const int64_t here = A.scan[e] + A.bsum[e / SCAN_B];
    const int64_t first = A.scan[C.eoff] + A.bsum[C.eoff / SCAN_B];
    A.cursor[e] = here - first + C.poff;
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
