// Counting sort of the particle arrays by element (periodic re-sort), in a
// fixed order: by element, and inside an element by particle id (R-32), so
// the order after a sort depends only on which particles each element holds.
//
// Keeping each case's particles grouped by element keeps the gathers of
// element records and nodal fields cache-resident and the elements per
// workgroup few, which is what the particle kernel's scatter relies on.
//   k_sort_hist     per-element counts (one atomic per element per wavefront)
//   k_sort_scan_*   exclusive scan of the counts (blocks, block totals), and
//   k_sort_cursor   the per-case segment starts and slot cursors
//   k_sort_place    each particle's id and index into a slot of its element's
//                   segment (slots claimed with one atomic per element per
//                   wavefront, so their order inside a segment is arbitrary)
//   k_sort_order    one wavefront per segment: the rank of each id inside
//                   its segment gives the particle's final position
//   k_sort_gather   move every particle field to the other buffer set
#include "pdfmc_dev.h"
#include "pdfmc_sort.h"

namespace pdfmc {

// The lanes of the wavefront that hold the same key as this lane, wherever
// they sit (one ballot per distinct key: particles leave their element
// between sorts, so the lanes of one element are rarely contiguous by then).
// rank = this lane's position among them, len = their count, first = the
// lowest of them, head = this lane is first. Keys < 0 get len = 0.
__device__ inline void sort_sets(int key, bool& head, int& rank, int& len, int& first)
{
    const int lane = __lane_id();
    unsigned long long mine = 0;
    unsigned long long rem = __ballot(key >= 0);
    while (rem) {
        const int k = __shfl(key, __ffsll((long long)rem) - 1);
        const unsigned long long set = __ballot(key == k);
        if (key == k) mine = set;
        rem &= ~set;
    }
    first = mine ? __ffsll((long long)mine) - 1 : lane;
    head = mine != 0 && first == lane;
    rank = __popcll(mine & ((1ull << lane) - 1));
    len = __popcll(mine);
}

// the tile of a wavefront: block sizes are multiples of 64 and TILE of the
// block size, so a wavefront lies inside one tile
__device__ inline int wave_tile(int64_t gid) { return __builtin_amdgcn_readfirstlane((int)(gid / TILE)); }

__global__ void k_sort_hist(SortArgs A)
{
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int tile = wave_tile(gid);
    if (tile >= A.ntiles) return;
    const CaseDev& C = A.cases[__builtin_amdgcn_readfirstlane(A.tile_case[tile])];
    const int64_t i = gid - C.poff;
    const bool valid = i >= 0 && i < C.np;
    const int key = valid ? A.elem[gid] : -1;
    bool head; int rank, len, first;
    sort_sets(key, head, rank, len, first);
    if (head) atomicAdd(A.count + key, len);
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
    A.start[e] = here - first + C.poff;
}

__global__ void k_sort_place(SortArgs A, const uint32_t* __restrict__ ids)
{
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int tile = wave_tile(gid);
    if (tile >= A.ntiles) return;
    const CaseDev& C = A.cases[__builtin_amdgcn_readfirstlane(A.tile_case[tile])];
    const int64_t i = gid - C.poff;
    const bool valid = i >= 0 && i < C.np;
    const int key = valid ? A.elem[gid] : -1;
    bool head; int rank, len, first;
    sort_sets(key, head, rank, len, first);
    unsigned long long base = 0;
    if (head) base = atomicAdd((unsigned long long*)(A.cursor + key), (unsigned long long)len);
    // broadcast the head's base to the lanes of its element
    base = __shfl(base, first);
    if (!valid) return;
    const int64_t q = (int64_t)base + rank;
    A.tmp_id[q] = ids[gid];
    A.tmp_src[q] = gid;
}

// (id, source index) of slot j of a segment as one 64-bit key: source
// indices are below 2^32 (particle arrays of fewer than 4 G entries)
__device__ inline unsigned long long sort_key(const SortArgs& A, int64_t s0, int j)
{
    return ((unsigned long long)A.tmp_id[s0 + j] << 32) | (unsigned long long)A.tmp_src[s0 + j];
}

// one wavefront per element segment: the segment's (id, source index) pairs
// are sorted in LDS by a bitonic network, and the sorted source indices are
// the final order. ids are distinct within a case as uploaded (R-32); the
// source index breaks ties should they not be. Segments longer than SORT_SEG
// are listed for k_sort_order_big.
constexpr int SORT_SEG = 512;
__global__ void __launch_bounds__(256) k_sort_order(SortArgs A)
{
    __shared__ unsigned long long s_keys[4][SORT_SEG];
    const int wid = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t e = (int64_t)blockIdx.x * 4 + wid;
    if (e >= A.ne) return;
    const int64_t s0 = A.start[e];
    const int len = A.count[e];
    if (len > SORT_SEG) {
        if (lane == 0) A.big[atomicAdd(A.nbig, 1)] = (int32_t)e;
        return;
    }
    int P = 1;
    while (P < len) P <<= 1;
    unsigned long long* k = s_keys[wid];
    for (int i = lane; i < P; i += 64) k[i] = i < len ? sort_key(A, s0, i) : ~0ull;
    for (int kk = 2; kk <= P; kk <<= 1) {
        for (int j = kk >> 1; j > 0; j >>= 1) {
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            for (int i = lane; i < P; i += 64) {
                const int ixj = i ^ j;
                if (ixj > i) {
                    const unsigned long long a = k[i], b = k[ixj];
                    const bool up = (i & kk) == 0;
                    if ((a > b) == up) { k[i] = b; k[ixj] = a; }
                }
            }
        }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    for (int i = lane; i < len; i += 64) A.perm[s0 + i] = (int64_t)(k[i] & 0xffffffffull);
}

// The listed long segments, one 1024-thread workgroup at a time (the grid is
// fixed; workgroup w takes list entries w, w + gridDim, ...): a bitonic sort
// in LDS for up to SORT_BIG particles, else ranks from memory.
constexpr int SORT_BIG = 8192;
__global__ void __launch_bounds__(1024) k_sort_order_big(SortArgs A)
{
    __shared__ unsigned long long k[SORT_BIG];
    const int nb = *A.nbig;
    for (int b = blockIdx.x; b < nb; b += gridDim.x) {
        const int e = A.big[b];
        const int64_t s0 = A.start[e];
        const int len = A.count[e];
        if (len <= SORT_BIG) {
            int P = 1;
            while (P < len) P <<= 1;
            for (int i = threadIdx.x; i < P; i += blockDim.x) k[i] = i < len ? sort_key(A, s0, i) : ~0ull;
            for (int kk = 2; kk <= P; kk <<= 1) {
                for (int j = kk >> 1; j > 0; j >>= 1) {
                    __syncthreads();
                    for (int i = threadIdx.x; i < P; i += blockDim.x) {
                        const int ixj = i ^ j;
                        if (ixj > i) {
                            const unsigned long long a = k[i], c2 = k[ixj];
                            const bool up = (i & kk) == 0;
                            if ((a > c2) == up) { k[i] = c2; k[ixj] = a; }
                        }
                    }
                }
            }
            __syncthreads();
            for (int i = threadIdx.x; i < len; i += blockDim.x) A.perm[s0 + i] = (int64_t)(k[i] & 0xffffffffull);
            __syncthreads();
        } else {
            for (int j = threadIdx.x; j < len; j += blockDim.x) {
                const unsigned long long my = sort_key(A, s0, j);
                int r = 0;
                for (int i = 0; i < len; ++i) r += sort_key(A, s0, i) < my ? 1 : 0;
                A.perm[s0 + r] = (int64_t)(my & 0xffffffffull);
            }
        }
    }
}

template <typename R>
__global__ void k_sort_gather(SortArgs A, Particles<R> src, Particles<R> dst)
{
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int tile = wave_tile(q);
    if (tile >= A.ntiles) return;
    const CaseDev& C = A.cases[__builtin_amdgcn_readfirstlane(A.tile_case[tile])];
    const int64_t j = q - C.poff;
    if (j < 0 || j >= C.np) return;
    const int64_t p = A.perm[q];
    const int64_t i = p - C.poff;
    dst.x[q] = src.x[p]; dst.y[q] = src.y[p];
    dst.u[q] = src.u[p]; dst.v[q] = src.v[p]; dst.w[q] = src.w[p];
    dst.om[q] = src.om[p]; dst.wt[q] = src.wt[p];
    dst.elem[q] = src.elem[p]; dst.id[q] = src.id[p]; dst.bin[q] = src.bin[p];
    for (int a = 0; a < C.ns; ++a) dst.psi[C.psioff + (int64_t)a * C.cap + j] = src.psi[C.psioff + (int64_t)a * C.cap + i];
}
template __global__ void k_sort_gather<double>(SortArgs, Particles<double>, Particles<double>);
template __global__ void k_sort_gather<float>(SortArgs, Particles<float>, Particles<float>);

}  // namespace pdfmc
