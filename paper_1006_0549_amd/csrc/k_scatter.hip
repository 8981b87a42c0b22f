// The passes that turn the particle kernel's scatter records into grid
// statistics (Sec. I, grid role (i); estimator of reading R-11) and IECM cell
// means (R-23), in a fixed summation order, so that a step gives the same
// bits every time it runs on the same input.
//
//   k_scatter_register  one thread per record slot: lists each record written
//                  this step under its element (SC_K entries per element; up
//                  to SC_XK more go to one overflow list for the pass; beyond
//                  that, or with that list full, into FP64 overflow sums,
//                  counted as scatter overflow)
//   k_elem_reduce  one wavefront per element: the element's records (listed
//                  in any order) are sorted by key and summed in that order,
//                  plus the overflow sums when the element had any. Out: the
//                  element's three vertex sums of the node moments and, with
//                  cells, its cell counts and cell means with the residual
//                  rule of R-23.
//   k_node_reduce  one thread per statistics node: the vertex sums of the
//                  incident elements, in the order of the node's incidence
//                  list, give the node sums; then the weighted means,
//                  central moments and density of R-11, with the thin-node
//                  rule of R-34.
#include "pdfmc_dev.h"
#include "pdfmc_nodes.h"

namespace pdfmc {

// a wavefront's LDS writes made visible to all of its lanes
__device__ inline void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__global__ void k_scatter_register(NodeArgs A, int ntiles, int block, const int32_t* tile_case, const int32_t* pool_cnt,
                                   int pool_cap, unsigned long long* counters, int cells_on)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t nreg = (int64_t)ntiles * SC_RT;
    const double* rp = nullptr;
    int handle = 0;
    int c = 0;
    if (t < nreg) {
        // regular slot: tile, workgroup inside the tile, slot inside the workgroup
        const int tile = (int)(t / SC_RT), it = (int)(t % SC_RT);
        const int wg_slots = SC_RT * block / TILE;
        const int wg = tile * (TILE / block) + it / wg_slots, sl = it % wg_slots;
        if (sl >= A.wgcnt[wg]) return;
        c = tile_case[tile];
        const CaseDev& C = A.cases[c];
        handle = (int)((tile - C.poff / TILE) * SC_RT + it);
        rp = A.srec + C.rec_off + (int64_t)handle * C.rec_stride;
    } else {
        const int64_t pi = t - nreg;
        const int np = min(*pool_cnt, pool_cap);
        if (pi >= np) return;
        handle = -1 - (int)pi;
        rp = A.srec + A.pool_off + pi * A.pool_stride;
    }
    const long long key = __double_as_longlong(rp[0]);
    const int el = (int)__double_as_longlong(rp[1]);
    if (t >= nreg) c = A.elem_case[el];
    const int slot = atomicAdd(A.ecnt + el, 1);
    // the key travels with the handle, so the element pass ranks its records
    // without reading their headers
    const int64_t entry = (int64_t)((unsigned long long)key << 32 | (uint32_t)handle);
    if (slot < SC_K) {
        A.eslot[(int64_t)el * SC_K + slot] = entry;
        return;
    }
    if (slot < SC_K + SC_XK) {
        // beyond the element's list: the pass's overflow list, which the
        // element pass searches for the element's further records
        const int q = atomicAdd(A.ovl_n, 1);
        if (q < A.ovl_cap) {
            A.ovl[q] = entry;
            A.ovl_el[q] = el;
            return;
        }
    }
    // both lists full: the record's values go to the element's overflow sums
    const CaseDev& C = A.cases[c];
    const int ns = C.ns, nq = 12 + 2 * ns, nc = 2 + ns;
    const bool cells = cells_on && ns > 0;
    const int nv = sc_nvals(ns, cells);
    const long long mask = __double_as_longlong(rp[2]);
    double* eo = A.eo + (int64_t)el * SC_VMAX;
    for (int v = 0; v < nv; ++v)
        if (v < 3 * nq || ((mask >> ((v - 3 * nq) / nc)) & 1)) unsafeAtomicAdd(eo + v, rp[SC_HDR + v]);
    atomicExch(A.eof + el, 1);
    atomicAdd(counters + (int64_t)c * NCNT + C_SCATTER_OVERFLOW, 1ull);
}

template <typename R>
__global__ void __launch_bounds__(256) k_elem_reduce(NodeArgs A, R* __restrict__ cmean, int cells_on, int rebin_only)
{
    __shared__ double s_cell[4][8 * (2 + MAXS)];
    __shared__ int64_t s_xent[4][SC_XK];              // an element's records from the overflow list
    __shared__ int s_rank_h[4][SC_K + SC_XK];         // its records' handles in key order
    __shared__ int s_nx[4];
    const int wid = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t e = (int64_t)blockIdx.x * 4 + wid;
    if (e >= A.ne) return;            // whole wavefronts leave together
    const int c = A.elem_case[e];
    const CaseDev& C = A.cases[c];
    if (rebin_only && !C.rebin) return;   // a case that keeps the bins of its step (no records this pass)
    const int ns = C.ns, nq = 12 + 2 * ns, nc = 2 + ns;
    const bool cells = cells_on && ns > 0;
    const int nv = sc_nvals(ns, cells);
    // the list entries are read together with the count (entries past the
    // count are stale and unused); lane j < n: record j as listed, and its key
    const int64_t ent = A.eslot[e * SC_K + lane];
    const int cnt = A.ecnt[e];
    auto rec_of = [&](int h) -> const double* {
        return h >= 0 ? A.srec + C.rec_off + (int64_t)h * C.rec_stride
                      : A.srec + A.pool_off + (int64_t)(-1 - h) * A.pool_stride;
    };
    // the bin of each lane's cell values (-1: a vertex sum); a record's cell
    // values are valid for the bins in its mask only
    const int b0 = cells && lane >= 3 * nq && lane < nv ? (lane - 3 * nq) / nc : -1;
    const int b1 = cells && lane + 64 >= 3 * nq && lane + 64 < nv ? (lane + 64 - 3 * nq) / nc : -1;
    double acc0 = 0.0, acc1 = 0.0;
    if (cnt <= SC_K) {
        const int n = cnt;
        const double* rp = nullptr;
        long long key = 0x7fffffffffffffffll;
        if (lane < n) {
            rp = rec_of((int)(uint32_t)ent);
            key = (long long)((unsigned long long)ent >> 32);
        }
        // rank of the record among the element's records (keys are distinct)
        int rank = 0;
        for (int i = 0; i < n; ++i) rank += __shfl(key, i) < key ? 1 : 0;
        // four records at a time: their loads first, then the sums in rank order
        for (int r0 = 0; r0 < n; r0 += 4) {
            long long mk[4];
            double x0[4], x1[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                mk[u] = 0; x0[u] = 0.0; x1[u] = 0.0;
                if (r0 + u < n) {
                    const int src = __ffsll((long long)__ballot(lane < n && rank == r0 + u)) - 1;
                    const double* q = (const double*)__shfl((long long)rp, src);
                    mk[u] = __double_as_longlong(q[2]);
                    if (lane < nv) x0[u] = q[SC_HDR + lane];
                    if (lane + 64 < nv) x1[u] = q[SC_HDR + 64 + lane];
                }
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                if (r0 + u < n) {
                    if (lane < nv && (b0 < 0 || ((mk[u] >> b0) & 1))) acc0 += x0[u];
                    if (lane + 64 < nv && (b1 < 0 || ((mk[u] >> b1) & 1))) acc1 += x1[u];
                }
            }
        }
    } else {
        // more records than the list holds: the element's further records (up
        // to SC_XK) are in the pass's overflow list. They are gathered into
        // LDS, each record is ranked by key among all of the element's, and
        // the sums are taken in that order, as for a listed element.
        int64_t* xs = s_xent[wid];
        int* hs = s_rank_h[wid];
        if (lane == 0) s_nx[wid] = 0;
        wave_lds_sync();
        const int nov = min(*A.ovl_n, A.ovl_cap);
        for (int i = lane; i < nov; i += 64)
            if (A.ovl_el[i] == (int32_t)e) {
                const int q = atomicAdd(&s_nx[wid], 1);
                if (q < SC_XK) xs[q] = A.ovl[i];
            }
        wave_lds_sync();
        const int n = SC_K + min(s_nx[wid], SC_XK);
        constexpr int MR = (SC_K + SC_XK) / 64;
        long long kj[MR];
        int hj[MR], rk[MR];
#pragma unroll
        for (int m = 0; m < MR; ++m) {
            const int j = lane + 64 * m;
            const int64_t en = m == 0 ? ent : (j < n ? xs[j - SC_K] : 0);
            kj[m] = j < n ? (long long)((unsigned long long)en >> 32) : 0x7fffffffffffffffll;
            hj[m] = (int)(uint32_t)en;
            rk[m] = 0;
        }
        for (int i = 0; i < n; ++i) {
            const long long ki = i < SC_K ? __shfl(kj[0], i) : (long long)((unsigned long long)xs[i - SC_K] >> 32);
#pragma unroll
            for (int m = 0; m < MR; ++m) rk[m] += ki < kj[m] ? 1 : 0;
        }
#pragma unroll
        for (int m = 0; m < MR; ++m)
            if (lane + 64 * m < n) hs[rk[m]] = hj[m];
        wave_lds_sync();
        for (int r0 = 0; r0 < n; r0 += 4) {
            long long mk[4];
            double x0[4], x1[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                mk[u] = 0; x0[u] = 0.0; x1[u] = 0.0;
                if (r0 + u < n) {
                    const double* q = rec_of(hs[r0 + u]);
                    mk[u] = __double_as_longlong(q[2]);
                    if (lane < nv) x0[u] = q[SC_HDR + lane];
                    if (lane + 64 < nv) x1[u] = q[SC_HDR + 64 + lane];
                }
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                if (r0 + u < n) {
                    if (lane < nv && (b0 < 0 || ((mk[u] >> b0) & 1))) acc0 += x0[u];
                    if (lane + 64 < nv && (b1 < 0 || ((mk[u] >> b1) & 1))) acc1 += x1[u];
                }
            }
        }
    }
    if (A.eof[e]) {
        // sums that found no record slot or list entry (counted as scatter overflow)
        double* eo = A.eo + e * SC_VMAX;
        if (lane < nv) { acc0 += eo[lane]; eo[lane] = 0.0; }
        if (lane + 64 < nv) { acc1 += eo[lane + 64]; eo[lane + 64] = 0.0; }
        if (lane == 0) A.eof[e] = 0;
    }
    if (lane == 0) A.ecnt[e] = 0;
    // vertex sums: value v = k nq + q -> etot[e][k][q]
    double* et = A.etot + e * 3 * NQ;
    if (lane < 3 * nq) et[(lane / nq) * NQ + lane % nq] = acc0;
    if (lane + 64 < 3 * nq) et[((lane + 64) / nq) * NQ + (lane + 64) % nq] = acc1;
    if (!cells) return;
    // cells: value 3 nq + b nc + j: j = 0 particle count, 1 sum w, 2 + a sum w psi_a
    const int v0 = lane - 3 * nq, v1 = lane + 64 - 3 * nq;
    if (v0 >= 0 && v0 < 8 * nc) s_cell[wid][v0] = acc0;
    if (v1 >= 0 && v1 < 8 * nc) s_cell[wid][v1] = acc1;
    wave_lds_sync();
    if (lane < 8) A.ccnt[e * 8 + lane] = (int32_t)s_cell[wid][lane * nc];
    // lane (b, a): mean of scalar a in bin b; bins with fewer than n_min
    // particles share one residual cell, pooled in bin order
    if (lane < 8 * ns) {
        const int b = lane / ns, a = lane - b * ns;
        double rw = 0.0, rpa = 0.0;
        for (int bb = 0; bb < 8; ++bb) {
            const int cb = (int)s_cell[wid][bb * nc];
            if (cb > 0 && cb < C.nmin) {
                rw += s_cell[wid][bb * nc + 1];
                rpa += s_cell[wid][bb * nc + 2 + a];
            }
        }
        const int cb = (int)s_cell[wid][b * nc];
        double m = 0.0;
        if (cb >= C.nmin) m = s_cell[wid][b * nc + 2 + a] / s_cell[wid][b * nc + 1];
        else if (rw > 0.0) m = rpa / rw;
        cmean[C.cmoff + ((int64_t)(e - C.eoff) * 8 + b) * ns + a] = (R)m;
    }
}
template __global__ void k_elem_reduce<double>(NodeArgs, double*, int, int);
template __global__ void k_elem_reduce<float>(NodeArgs, float*, int, int);

__global__ void k_node_reduce(NodeArgs A)
{
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= A.nn) return;
    const int c = A.node_case[s];
    const CaseDev& C = A.cases[c];
    const int ns = C.ns, nq = 12 + 2 * ns;
    double r[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) r[q] = 0.0;
    for (int j = A.inc_ptr[s]; j < A.inc_ptr[s + 1]; ++j) {
        const int ent = A.inc[j];
        const double* et = A.etot + (int64_t)(ent / 3) * 3 * NQ + (ent % 3) * NQ;
#pragma unroll
        for (int q = 0; q < NQ; ++q)
            if (q < nq) r[q] += et[q];
    }
    double* ns_out = A.nsum + (int64_t)s * NQ;
#pragma unroll
    for (int q = 0; q < NQ; ++q)
        if (q < nq) ns_out[q] = r[q];
    double* st = A.stats + (int64_t)s * NST;
    const double W = r[0];
    // an empty node, or (once there are previous statistics) one whose
    // effective sample size W^2 / sum (w N)^2 is below n_eff_min, keeps its
    // previous moments (R-34)
    st[0] = W;
    st[1] = W / A.vol[s];
    double wsq = 0.0;
#pragma unroll
    for (int q = 0; q < NQ; ++q)
        if (q == 11 + 2 * ns) wsq = r[q];
    if (W > 0.0 && (A.first_stats || W * W >= C.neff_min * wsq)) {
        const double m1 = r[1] / W, m2 = r[2] / W, m3 = r[3] / W;
        st[2] = m1; st[3] = m2; st[4] = m3;
        st[5] = r[4] / W - m1 * m1;
        st[6] = r[5] / W - m2 * m2;
        st[7] = r[6] / W - m3 * m3;
        st[8] = r[7] / W - m1 * m2;
        st[9] = r[8] / W - m1 * m3;
        st[10] = r[9] / W - m2 * m3;
        st[11] = r[10] / W;
#pragma unroll
        for (int a = 0; a < MAXS; ++a) {
            if (a < ns) {
                double ps = 0.0, p2 = 0.0;
#pragma unroll
                for (int q = 0; q < NQ; ++q) {
                    if (q == 11 + a) ps = r[q];
                    if (q == 11 + ns + a) p2 = r[q];
                }
                const double m = ps / W;
                st[12 + a] = m;
                st[12 + ns + a] = p2 / W - m * m;
            }
        }
    } else {
        atomicAdd(A.counters + (int64_t)c * NCNT + C_EMPTY_NODE, 1ull);
    }
}

}  // namespace pdfmc
