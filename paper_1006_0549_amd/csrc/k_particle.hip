// Particle kernel: one forward-Euler step of every particle of every case in
// one launch, fused with the grid statistics of the new state.
//
// Per particle (order of reading R-08):
//   barycentric coordinates in its element (R-05) -> P1 interpolation of the
//   Eulerian fields (R-06) -> Wiener increments (R-09, R-10) -> IECM mixing,
//   Eq.(9) (R-23, R-24) -> velocity increment, Eq.(4) -> position increment,
//   Eq.(2), with the same dW_i -> frequency increment, Eq.(5) (R-21) ->
//   neighbour walk with wall reflection and periodic shift (R-12..R-15) ->
//   concentrated sources (R-26) -> velocity bin against the fields of this
//   step (R-23) -> shape-weighted sums of the new state at the element's
//   three vertices (R-11) and cell sums for the next mixing step.
//
// Layout: structure of arrays, one lane per particle, tiles of 256 particles
// that never straddle two cases. The scatter is deterministic and uses no
// floating-point atomics: each wavefront sorts its particles by (element,
// bin, lane), lane groups walk the sorted positions and sum each element's
// run in sorted order, and each element's sums go out as one record per
// (workgroup, element) with plain stores (the runs of an element that
// several wavefronts hold are first added in LDS, in wavefront order). The
// records of an element are summed in key order by the element pass, and the
// vertex sums of the elements around a node by the node pass (k_scatter.hip).
// Arithmetic of the FP64 instantiation follows the operation order of the
// readings exactly (no contraction; explicit fma only where the readings put
// one), so that it reproduces the CPU oracle bit for bit; only the summation
// order of the node and cell sums differs.
#include "pdfmc_dev.h"
#include "pdfmc_math.h"

namespace pdfmc {

template <typename R> __device__ inline R rfma(R a, R b, R c);
template <> __device__ inline double rfma<double>(double a, double b, double c) { return __builtin_fma(a, b, c); }
template <> __device__ inline float rfma<float>(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
// square root: correctly rounded in FP64 (required for bit parity), hardware in FP32
template <typename R> __device__ inline R r_sqrt(R a);
template <> __device__ inline double r_sqrt<double>(double a) { return __builtin_sqrt(a); }
template <> __device__ inline float r_sqrt<float>(float a) { return __builtin_sqrtf(a); }

// reaction rate constant a of the case, in the particle precision
template <typename R> __device__ inline R kr(const CaseDev& C, int a);
template <> __device__ inline double kr<double>(const CaseDev& C, int a) { return C.kr[a]; }
template <> __device__ inline float kr<float>(const CaseDev& C, int a) { return C.fkr[a]; }

__device__ inline int pick(const int4& v, int k) { return k == 0 ? v.x : (k == 1 ? v.y : v.z); }

// R-05: lambda_k = fma(c_k, dy, fma(b_k, dx, delta_k1)), dx = x - x1, dy = y - y1
template <typename R>
__device__ inline void bary(const R* __restrict__ rec, int e, R x, R y, R lam[3])
{
    const R* r = rec + 8 * (int64_t)e;
    R dx = x - r[0], dy = y - r[1];
    lam[0] = rfma<R>(r[5], dy, rfma<R>(r[2], dx, R(1)));
    lam[1] = rfma<R>(r[6], dy, rfma<R>(r[3], dx, R(0)));
    lam[2] = rfma<R>(r[7], dy, rfma<R>(r[4], dx, R(0)));
}

struct WalkCount { int refl, per, steps, fallback; };

// R-12..R-15 walk; returns the element holding (x, y) and its lambda.
// A step straight back into the element just left (rounding on their shared
// edge) ends the walk in whichever of the two has the larger min lambda.
// Fallback (cap reached): FP64 follows R-13 (brute force over the case);
// FP32, whose rounding near thin wall cells can make every element look
// slightly outside, keeps the visited element with the largest min lambda.
template <typename R>
__device__ int walk(const MeshDev<R>& M, const CaseDev& C, int e, R& x, R& y, R u3[3], R lam[3], WalkCount& wc,
                    const int4 nb_start)
{
    int nrefl = 0;
    int prev = -1;
    R prev_min = R(0), prev_x = R(0), prev_y = R(0);
    int best = e;
    R best_min = R(-1e30), best_x = x, best_y = y;
    int ring[4] = {-1, -1, -1, -1};   // FP32: recently left elements
    for (int it = 0; it < 64; ++it) {
        bary<R>(M.rec, e, x, y, lam);
        int k = 0;
        if (lam[1] < lam[k]) k = 1;
        if (lam[2] < lam[k]) k = 2;
        if (lam[k] >= R(0)) return e;
        if constexpr (sizeof(R) == 4) {
            if (lam[k] > best_min) { best = e; best_min = lam[k]; best_x = x; best_y = y; }
        }
        // the start element's neighbours were loaded with its other tables
        const int nb = pick(it == 0 ? nb_start : M.nbr[e], k);
        const BcDev* bc = nb >= 0 ? nullptr : &M.bc[-1 - nb];
        const int next = nb >= 0 ? nb : (bc->type == 1 ? pick(M.partner[e], k) : e);
        if constexpr (sizeof(R) == 4) {
            // a longer cycle (rounding around a vertex): stop in the best element seen
            if (next != e && next != prev && (next == ring[0] || next == ring[1] || next == ring[2] || next == ring[3]))
                break;
            ring[it & 3] = e;
        }
        if (next == prev && next != e) {
            if (prev_min > lam[k]) {
                x = prev_x; y = prev_y;
                bary<R>(M.rec, prev, x, y, lam);
                return prev;
            }
            return e;
        }
        wc.steps++;
        if (nb >= 0) { prev = e; prev_min = lam[k]; prev_x = x; prev_y = y; e = nb; continue; }
        if (bc->type == 1) {
            prev = e; prev_min = lam[k]; prev_x = x; prev_y = y;
            if constexpr (sizeof(R) == 8) { x = x + bc->shift[0]; y = y + bc->shift[1]; }
            else { x = x + bc->shiftf[0]; y = y + bc->shiftf[1]; }
            e = next;
            wc.per++;
            continue;
        }
        prev = -1;
        // a reflection turns the walk back: forget the cycle ring and the best
        // element seen so far, whose position predates the mirrored velocity
        if constexpr (sizeof(R) == 4) { ring[0] = ring[1] = ring[2] = ring[3] = -1; best_min = R(-1e30); }
        if (nrefl == 8) break;
        const R* v = M.exy + 6 * (int64_t)e;
        int ka = (k + 1) % 3, kb = (k + 2) % 3;
        R xa = v[2 * ka], ya = v[2 * ka + 1];
        R ex = v[2 * kb] - xa, ey = v[2 * kb + 1] - ya;
        R L = r_sqrt<R>(ex * ex + ey * ey);
        R nx = ey / L, ny = -ex / L;
        R d = (x - xa) * nx + (y - ya) * ny;
        x = x - (R(2) * d) * nx;
        y = y - (R(2) * d) * ny;
        for (int i = 0; i < 3; ++i) {
            R uw;
            if constexpr (sizeof(R) == 8) uw = bc->uw[i]; else uw = bc->uwf[i];
            u3[i] = R(2) * uw - u3[i];
        }
        nrefl++;
        wc.refl++;
    }
    wc.fallback++;
    if constexpr (sizeof(R) == 4) {
        x = best_x; y = best_y;
        bary<R>(M.rec, best, x, y, lam);
        return best;
    }
    // R-13: lowest-index containing element, else the one maximising min lambda
    int bf = -1;
    R bestv = R(0);
    for (int q = C.eoff; q < C.eoff + C.ne; ++q) {
        R l[3];
        bary<R>(M.rec, q, x, y, l);
        R mn = l[0];
        if (l[1] < mn) mn = l[1];
        if (l[2] < mn) mn = l[2];
        if (mn >= R(0)) { bf = q; break; }
        if (bf < 0 || mn > bestv) { bf = q; bestv = mn; }
    }
    bary<R>(M.rec, bf, x, y, lam);
    return bf;
}

// ---------------------------------------------------------------- wave helpers

__device__ inline int wave_sum_int(int v)
{
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d);
    return v;
}

// The value of lane (lane xor m) for the constant masks of a 64-lane bitonic
// sort, without a trip through LDS where the lane pattern allows: masks 1 and
// 2 by a quad permutation, 4 by reversing each quad and then each half-row
// (i -> 7 - (i xor 3) = i xor 4 within eight lanes), 8 by reversing each
// half-row and then each row (likewise within sixteen), 16 by the swizzle's
// bit-mask mode (xor 16 within 32 lanes), 32 by a permute through LDS.
__device__ inline unsigned lane_xor(unsigned v, int m)
{
    const int x = (int)v;
    switch (m) {
    case 1: return (unsigned)__builtin_amdgcn_mov_dpp(x, 0xB1, 0xF, 0xF, false);
    case 2: return (unsigned)__builtin_amdgcn_mov_dpp(x, 0x4E, 0xF, 0xF, false);
    case 4: return (unsigned)__builtin_amdgcn_mov_dpp(__builtin_amdgcn_mov_dpp(x, 0x1B, 0xF, 0xF, false), 0x141, 0xF,
                                                      0xF, false);
    case 8: return (unsigned)__builtin_amdgcn_mov_dpp(__builtin_amdgcn_mov_dpp(x, 0x141, 0xF, 0xF, false), 0x140, 0xF,
                                                      0xF, false);
    case 16: return (unsigned)__builtin_amdgcn_ds_swizzle(x, 0x401F);
    default: return (unsigned)__shfl_xor(x, m);
    }
}

// Lane moves of an FP64 value by a DPP control (row mask: the rows written;
// the others read 0).
template <int CTRL, int ROWS>
__device__ inline double dpp_f64(double v)
{
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, ROWS, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, ROWS, 0xF, false);
    return __hiloint2double(hi, lo);
}

// Inclusive sum of v over the lanes [st, lane] of the wavefront (st: the
// first lane of this lane's segment), every lane active: shifts by 1, 2, 4
// and 8 within each row of sixteen lanes, then the last lane of row 0 and of
// row 2 added to the rows after them, then lane 31 to rows 2 and 3, each step
// only where the segment reaches the lane it takes from.
__device__ inline double seg_scan(double v, int lane, int st)
{
    double y;
    y = dpp_f64<0x111, 0xF>(v);
    v = (lane & 15) >= 1 && lane - 1 >= st ? v + y : v;
    y = dpp_f64<0x112, 0xF>(v);
    v = (lane & 15) >= 2 && lane - 2 >= st ? v + y : v;
    y = dpp_f64<0x114, 0xF>(v);
    v = (lane & 15) >= 4 && lane - 4 >= st ? v + y : v;
    y = dpp_f64<0x118, 0xF>(v);
    v = (lane & 15) >= 8 && lane - 8 >= st ? v + y : v;
    y = dpp_f64<0x142, 0xA>(v);                  // rows 1 and 3 take lanes 15 and 47
    v = ((lane >> 4) & 1) && st <= (lane & ~15) - 1 ? v + y : v;
    y = dpp_f64<0x143, 0xC>(v);                  // rows 2 and 3 take lane 31
    v = lane >= 32 && st <= 31 ? v + y : v;
    return v;
}

// ---------------------------------------------------------------- scatter helpers

// per-lane record in LDS: lambda_0..2, w | U_1..3, omega | psi_0..3 | 1, 0
// (the constants stand in for absent factors of a vertex term), 16 slots so
// that the first four load as one vector
constexpr int NREC = 16;
constexpr int RI_ONE = 12, RI_ZERO = 13;

// ---------------------------------------------------------------- the kernel

template <typename R>
__device__ inline void load_field_row(const R* __restrict__ F, int stride, int s, R* out)
{
    const R* row = F + (int64_t)s * stride;
#pragma unroll
    for (int q = 0; q < NF; ++q) out[q] = row[q];
}

template <typename R>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) k_particle_step(StepArgs<R> A)
{
    __shared__ __align__(16) R s_rec[256 * NREC];   // per-lane records of the new state
    __shared__ int s_sorted[256];                    // each wavefront's elements, sorted
    __shared__ double s_stage[4 * SC_SQ * SC_VMAX];  // sums of shared elements, per wavefront
    __shared__ int s_sel[4 * SC_SQ];                 // their elements
    __shared__ int s_smask[4 * SC_SQ];               // their bin masks
    __shared__ int s_nst[4];                         // staged entries per wavefront
    __shared__ int s_mel[4 * 64], s_mfirst[4 * 64];  // shared elements each wavefront merges, first positions
    __shared__ int s_nmerge[4];
    __shared__ int s_slot;                           // record slots taken by the workgroup
    // XCD-aware order: the chip hands workgroups to its eight XCDs in turn
    // (hardware block b on XCD b mod 8), so logical block lb gives each XCD a
    // contiguous range of particle tiles, whose elements then meet in its L2
    const int lb = xcd_block((int)blockIdx.x, (int)gridDim.x);
    const int64_t gid = (int64_t)lb * blockDim.x + threadIdx.x;
    // block sizes are multiples of 64 and TILE of the block size, so a
    // wavefront lies inside one tile: the tile, the case and its constants
    // are the same for all lanes and are taken from the first lane (scalar
    // registers and loads)
    const int tile = __builtin_amdgcn_readfirstlane((int)(gid / TILE));
    const int c = __builtin_amdgcn_readfirstlane(A.tile_case[tile < A.ntiles ? tile : A.ntiles - 1]);
    const CaseDev& C = A.cases[c];
    // a rebinning pass skips the cases that keep the bins of their step: the
    // whole workgroup leaves (one case per workgroup), with no records
    if (A.rebin_only && !C.rebin) {
        if (threadIdx.x == 0) A.wgcnt[lb] = 0;
        return;
    }
    const int64_t i = gid - C.poff;
    const bool valid = tile < A.ntiles && (i >= 0) && (i < C.np);
    const int64_t p = gid;
    const int ns = C.ns;
    const uint32_t step = *A.step;

    int e = -1;
    R x = R(0), y = R(0), wt = R(0), om = R(0);
    R u3[3] = {R(0), R(0), R(0)};
    R psi[MAXS] = {R(0), R(0), R(0), R(0)};
    R lam[3] = {R(0), R(0), R(0)};
    int bin = 0;
    WalkCount wc = {0, 0, 0, 0};
    int flips = 0, nans = 0;

    if (valid) {
        e = A.P.elem[p];
        x = A.P.x[p]; y = A.P.y[p];
        u3[0] = A.P.u[p]; u3[1] = A.P.v[p]; u3[2] = A.P.w[p];
        om = A.P.om[p]; wt = A.P.wt[p];
        for (int a = 0; a < ns; ++a) psi[a] = A.P.psi[C.psioff + (int64_t)a * C.cap + i];
        bary<R>(A.M.rec, e, x, y, lam);
        if (A.advance) {
            {
                // R-27: the last projection corrects the velocity, U <- U - dt grad <P>(X),
                // before the step uses it (zero without a projection)
                const R* G0 = A.Fel + (int64_t)e * 3 * NFE;
                const R gpx = rfma<R>(lam[2], G0[2 * NFE + FE_GPX], rfma<R>(lam[1], G0[NFE + FE_GPX], lam[0] * G0[FE_GPX]));
                const R gpy = rfma<R>(lam[2], G0[2 * NFE + FE_GPY], rfma<R>(lam[1], G0[NFE + FE_GPY], lam[0] * G0[FE_GPY]));
                R dtc;
                if constexpr (sizeof(R) == 8) dtc = C.dt; else dtc = C.fdt;
                u3[0] = u3[0] - dtc * gpx;
                u3[1] = u3[1] - dtc * gpy;
            }
            // the element's field rows are not loaded above this point: loaded
            // together with the correction's, the FP32 kernel's registers
            // spilled (no spill, about 1% faster)
            __builtin_amdgcn_sched_barrier(0);
            const int4 nbe = A.M.nbr[e];
            // Wiener increments first: they need only the particle's id, so
            // their arithmetic overlaps the loads of the element's tables
            R xi[6];
            if constexpr (sizeof(R) == 8) gauss6_f64(C.seed_lo, C.seed_hi, A.P.id[p], step, C.stream, xi);
            else gauss6_f32(C.seed_lo, C.seed_hi, A.P.id[p], step, C.stream, xi);
            R f[NF];
            {
                // R-06, row by row: f = fma(l2, F2, fma(l1, F1, l0 F0)), so
                // only one vertex row is live at a time; the element's three
                // vertex rows lie together (element-major copy of the fields)
                const R* F0 = A.Fel + (int64_t)e * 3 * NFE;
                const R* F1 = F0 + NFE;
                const R* F2 = F1 + NFE;
                R om_n[3];
#pragma unroll
                for (int q = 0; q < NF; ++q) f[q] = lam[0] * F0[q];
                om_n[0] = F0[F_OMEGA];
#pragma unroll
                for (int q = 0; q < NF; ++q) f[q] = rfma<R>(lam[1], F1[q], f[q]);
                om_n[1] = F1[F_OMEGA];
#pragma unroll
                for (int q = 0; q < NF; ++q) f[q] = rfma<R>(lam[2], F2[q], f[q]);
                om_n[2] = F2[F_OMEGA];
                // Eq.(9) IECM with the cell means of this state (R-23, R-24),
                // plus the closed reaction source on the composition before
                // the step (R-35)
                if (ns > 0) {
                    R om_e = ((om_n[0] + om_n[1]) + om_n[2]) / R(3);
                    R hphi, dt;
                    if constexpr (sizeof(R) == 8) { hphi = C.hphi; dt = C.dt; } else { hphi = C.fhphi; dt = C.fdt; }
                    R fm = dt * (hphi * om_e);
                    if (fm > R(1)) fm = R(1);
                    const int b = A.P.bin[p];
                    const R* cm = A.cmean + C.cmoff + ((int64_t)(e - C.eoff) * 8 + b) * ns;
                    R s[MAXS] = {R(0), R(0), R(0), R(0)};
                    if (C.reaction == 1) {
                        for (int a = 0; a < ns; ++a) s[a] = -(kr<R>(C, a) * psi[a]);
                    } else if (C.reaction == 2) {
                        const R r = (kr<R>(C, 0) * psi[0]) * psi[1];
                        s[0] = -r;
                        s[1] = -r;
                        s[2] = r;
                    }
                    for (int a = 0; a < ns; ++a) psi[a] = (psi[a] - fm * (psi[a] - cm[a])) + dt * s[a];
                }
            }
            R dt, tnu, sq_nu, C3, c34;
            if constexpr (sizeof(R) == 8) { dt = C.dt; tnu = C.tnu; sq_nu = C.sq_nu; C3 = C.C3; c34 = C.c34; }
            else { dt = C.fdt; tnu = C.ftnu; sq_nu = C.fsq_nu; C3 = C.fC3; c34 = C.fc34; }
            // Eq.(4), generalized Langevin model; same dW_j as Eq.(2) (R-01)
            const R u = u3[0], v = u3[1], w = u3[2];
            const R d1 = u - f[F_U1], d2 = v - f[F_U2], d3 = w - f[F_U3];
            const R c0e = f[F_C0EPS] > R(0) ? f[F_C0EPS] : R(0);
            const R sq_c0 = r_sqrt<R>(c0e * dt);
            R du = dt * ((-f[F_DPX] + tnu * f[F_LAP1]) + (f[F_G11] * d1 + f[F_G12] * d2))
                 + sq_nu * (f[F_DU1X] * xi[0] + f[F_DU1Y] * xi[1]) + sq_c0 * xi[2];
            R dv = dt * ((-f[F_DPY] + tnu * f[F_LAP2]) + (f[F_G21] * d1 + f[F_G22] * d2))
                 + sq_nu * (f[F_DU2X] * xi[0] + f[F_DU2Y] * xi[1]) + sq_c0 * xi[3];
            R dw = dt * (tnu * f[F_LAP3] + f[F_G33] * d3)
                 + sq_nu * (f[F_DU3X] * xi[0] + f[F_DU3Y] * xi[1]) + sq_c0 * xi[4];
            // Eq.(2): X^{n+1} = X^n + U^n dt + (2 nu)^{1/2} dW
            x = (x + u * dt) + sq_nu * xi[0];
            y = (y + v * dt) + sq_nu * xi[1];
            u3[0] = u + du; u3[1] = v + dv; u3[2] = w + dw;
            // Eq.(5) with S_omega of Eq.(6) (R-17, R-21)
            const R W = f[F_OMEGA], S = f[F_SOMEGA];
            const R drift = ((-C3 * W) * (om - W)) - ((S * W) * om);
            const R omp = om > R(0) ? om : R(0);
            const R diff = r_sqrt<R>(((c34 * (W * W)) * omp) * dt);
            R omn = (om + dt * drift) + diff * xi[5];
            if (omn < R(0)) { omn = -omn; flips = 1; }
            om = omn;
            // tracking (R-12..R-15)
            if (__builtin_isfinite(x) && __builtin_isfinite(y)) {
                e = walk<R>(A.M, C, e, x, y, u3, lam, wc, nbe);
            } else {
                nans = 1;
            }
            // concentrated sources (R-26)
            for (int a = 0; a < ns; ++a) {
                R r, cx, cy, val;
                if constexpr (sizeof(R) == 8) { r = C.src[a][2]; cx = C.src[a][0]; cy = C.src[a][1]; val = C.src[a][3]; }
                else { r = C.srcf[a][2]; cx = C.srcf[a][0]; cy = C.srcf[a][1]; val = C.srcf[a][3]; }
                if (r > R(0)) {
                    R dx = x - cx, dy = y - cy;
                    if (dx * dx + dy * dy < r * r) psi[a] = val;
                }
            }
            A.P.x[p] = x; A.P.y[p] = y;
            A.P.u[p] = u3[0]; A.P.v[p] = u3[1]; A.P.w[p] = u3[2];
            A.P.om[p] = om; A.P.elem[p] = e;
            for (int a = 0; a < ns; ++a) A.P.psi[C.psioff + (int64_t)a * C.cap + i] = psi[a];
        }
        // R-23 bin: octant of U - <U>(X) with <U> from the fields of this step
        if (A.do_bins && C.nbins == 8) {
            const R* F0 = A.Fel + (int64_t)e * 3 * NFE;
            const R* F1 = F0 + NFE;
            const R* F2 = F1 + NFE;
            for (int q = 0; q < 3; ++q) {
                R m = rfma<R>(lam[2], F2[q], rfma<R>(lam[1], F1[q], lam[0] * F0[q]));
                if (u3[q] - m >= R(0)) bin += (1 << q);
            }
        }
        if (A.do_bins) A.P.bin[p] = (uint8_t)bin;
    }

    if (A.scatter) {
    // ---- shape-weighted sums of the new state at the element's vertices
    // (R-11) and cell sums (R-23), FP64, in an order fixed by the particle
    // order alone, with no floating-point atomics.
    //  1. Each wavefront sorts its lanes by (element, bin, lane); the
    //     particles of one element then form a run of sorted positions.
    //  2. Lane groups walk the sorted positions, a contiguous range per
    //     group, adding the vertex terms w lambda_k Q of one particle per
    //     step (lane q of a group holds term q); a run that crosses a range
    //     boundary is completed by a carry from group to group.
    //  3. Cell sums (count, w, w psi_a per element and bin) come from a
    //     segmented scan over the same sorted order.
    //  4. A run whose element no other wavefront of the workgroup holds goes
    //     out as a record; the runs of an element that several wavefronts
    //     hold are staged in LDS and, after a barrier, added in wavefront
    //     order by the lowest of those wavefronts.
    // Record keys derive from the workgroup, the wavefront and the run's
    // first sorted position, so the element pass sums an element's records
    // in an order that depends on the particle order only.
    const int nq = 12 + 2 * ns;
    const bool cells = A.do_bins && ns > 0;
    const int nv = sc_nvals(ns, cells);
    const int nc = 2 + ns;                       // cell values per bin
    const int lane = __lane_id(), wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
    // (1) sort key: case-local element << 9 | bin << 6 | lane (a case has
    // fewer than 2^23 elements); lanes without a particle last
    unsigned sk = valid ? ((unsigned)(e - C.eoff) << 9) | ((unsigned)(cells ? bin : 0) << 6) | (unsigned)lane : ~0u;
#pragma unroll
    for (int kk = 2; kk <= 64; kk <<= 1) {
#pragma unroll
        for (int jj = kk >> 1; jj > 0; jj >>= 1) {
            const unsigned o = lane_xor(sk, jj);
            const bool keep_min = ((lane & jj) == 0) == ((lane & kk) == 0);
            sk = keep_min ? min(o, sk) : max(o, sk);
        }
    }
    // sorted position = lane: its particle's lane, element and bin
    const bool pv = sk != ~0u;
    const int src = (int)(sk & 63);
    const int E = pv ? C.eoff + (int)(sk >> 9) : -1;
    const int sbin = (int)((sk >> 6) & 7);
    {
        R* my = s_rec + threadIdx.x * NREC;
        my[0] = lam[0]; my[1] = lam[1]; my[2] = lam[2]; my[3] = wt;
        my[4] = u3[0]; my[5] = u3[1]; my[6] = u3[2]; my[7] = om;
#pragma unroll
        for (int a = 0; a < MAXS; ++a) my[8 + a] = psi[a];
        my[RI_ONE] = R(1);
        my[RI_ZERO] = R(0);
        s_sorted[threadIdx.x] = pv ? E : 0x7fffffff;
        if (threadIdx.x == 0) s_slot = 0;
        if (threadIdx.x < 4) s_nmerge[threadIdx.x] = 0;
    }
    __syncthreads();
    // (2) runs of equal element among the sorted positions
    const int Ep = __shfl_up(E, 1), En = __shfl_down(E, 1);
    const bool head = pv && (lane == 0 || Ep != E);
    const bool tail = pv && (lane == 63 || En != E);
    const unsigned long long hm = __ballot(head);
    const unsigned long long before = (1ull << lane) - 1;          // positions < lane
    const unsigned long long upto = before | (1ull << lane);        // positions <= lane
    const int hpos = 63 - __clzll(hm & upto | 1ull);      // first position of this position's run
    // wavefronts of the workgroup that hold this position's element (binary
    // search in each one's sorted elements)
    int inw = 1 << wid;
    for (int t = 0; t < nw; ++t) {
        if (t == wid) continue;
        const int* L = s_sorted + t * 64;
        int lo = 0;
#pragma unroll
        for (int st = 32; st >= 1; st >>= 1)
            if (L[lo + st - 1] < E) lo += st;
        if (pv && L[lo] == E) inw |= 1 << t;
    }
    const bool shared_el = inw != (1 << wid);
    // destination of the run starting at each head: a stage entry (element
    // shared with another wavefront, while entries are left), else a record
    // slot (the workgroup's regular slots, then the pool), else the
    // element's overflow sums (FP64 atomics, counted)
    const unsigned long long shm = __ballot(head && shared_el);
    const int sidx = __popcll(shm & before);
    const bool staged = head && shared_el && sidx < SC_SQ;
    const bool needrec = head && !staged;
    const unsigned long long rm = __ballot(needrec);
    const int nrec = __popcll(rm), ridx = __popcll(rm & before);
    const int64_t ltile = gid / TILE - C.poff / TILE;     // the case's tile of this workgroup
    const int wg_slots = SC_RT * (int)blockDim.x / TILE;
    const int wg_first = (int)((lb * (int64_t)blockDim.x) % TILE) / (int)blockDim.x * wg_slots;
    const long long kbase = (long long)lb * 512;
    int base = 0;
    if (lane == 0 && nrec > 0) base = atomicAdd(&s_slot, nrec);
    base = __shfl(base, 0);
    const int nreg = max(0, min(nrec, wg_slots - base));
    int pbase = 0;
    if (lane == 0 && nrec > nreg) pbase = atomicAdd(A.pool_cnt, nrec - nreg);
    pbase = __shfl(pbase, 0);
    int kind = 2, dcode = E;             // 0 record (handle), 1 stage entry, 2 overflow (element)
    if (staged) {
        kind = 1;
        dcode = wid * SC_SQ + sidx;
    } else if (needrec) {
        if (ridx < nreg) {
            kind = 0;
            dcode = (int)(ltile * SC_RT) + wg_first + base + ridx;
        } else if (pbase + (ridx - nreg) < A.pool_cap) {
            kind = 0;
            dcode = -1 - (pbase + (ridx - nreg));
        }
    }
    double* const rec_base = A.srec + C.rec_off;
    double* const pool_base = A.srec + A.pool_off;
    const int64_t rec_stride = C.rec_stride, pool_stride = A.pool_stride;
    auto rec_ptr = [&](int h) -> double* {
        return h >= 0 ? rec_base + (int64_t)h * rec_stride : pool_base + (int64_t)(-1 - h) * pool_stride;
    };
    // bins present in the run starting at each head (cells only)
    long long mask = 0;
    if (cells) {
        const unsigned long long later = hm & ~upto;
        const unsigned long long vm = __ballot(pv);
        // last position of the run starting here: before the next head, else the last particle
        const int tpos = later ? __ffsll((long long)later) - 2 : 63 - __clzll(vm | 1ull);
        const unsigned long long runm = (tpos >= 63 ? ~0ull : ((1ull << (tpos + 1)) - 1)) & ~before;
#pragma unroll
        for (int b = 0; b < 8; ++b)
            if (__ballot(pv && sbin == b) & runm) mask |= 1ll << b;
    }
    // headers, stage entries and the merge list, from the head lanes
    if (head) {
        if (kind == 0) {
            double* dst = rec_ptr(dcode);
            dst[0] = __longlong_as_double(kbase + (shared_el ? 256 : 0) + wid * 64 + lane);
            dst[1] = __longlong_as_double((long long)E);
            dst[2] = __longlong_as_double(mask);
        } else if (kind == 1) {
            s_sel[dcode] = E;
            s_smask[dcode] = (int)mask;
        } else {
            atomicExch(A.eof + E, 1);
            atomicAdd(A.counters + (int64_t)c * NCNT + C_SCATTER_OVERFLOW, 1ull);
        }
    }
    {
        const bool merger = head && shared_el && (__ffs(inw) - 1) == wid;
        const unsigned long long mm = __ballot(merger);
        if (merger) {
            const int mi = __popcll(mm & before);
            s_mel[wid * 64 + mi] = E;
            s_mfirst[wid * 64 + mi] = lane;
        }
        if (lane == 0) {
            s_nmerge[wid] = __popcll(mm);
            s_nst[wid] = min(__popcll(shm), SC_SQ);
        }
    }
    // per position: its run's destination
    const int rkind = __shfl(kind, hpos), rdcode = __shfl(dcode, hpos);
    const R* wave_rec = s_rec + wid * 64 * NREC;
    // (3) vertex sums: G groups of GS lanes, group g walks sorted positions
    // [g P, g P + P); lane q of a group holds term q < nq:
    //   (w lambda_k) * fma(sqm, w lambda_k, fa fb),
    // fa, fb record values (or 1), and for the square term fa fb = 0, sqm = 1
    {
        const int G = nq <= 16 ? 4 : 3, GS = nq <= 16 ? 16 : 21, P = nq <= 16 ? 16 : 22;
        const int g = nq <= 16 ? lane >> 4 : (lane * 49) >> 10;      // lane / GS for lane < 64
        const int q = lane - g * GS;
        const bool glane = g < G;
        // factors of term q: record slots ia, ib (1 when absent, 0 for the square term)
        const int qs = q - 11;                     // scalar terms
        int ia, ib;
        if (q == 0) { ia = RI_ONE; ib = RI_ONE; }
        else if (q <= 3) { ia = 3 + q; ib = RI_ONE; }
        else if (q <= 6) { ia = q; ib = q; }
        else if (q <= 9) { ia = q == 9 ? 5 : 4; ib = q == 7 ? 5 : 6; }
        else if (q == 10) { ia = 7; ib = RI_ONE; }
        else if (qs < ns) { ia = 8 + qs; ib = RI_ONE; }
        else if (qs < 2 * ns) { ia = 8 + qs - ns; ib = ia; }
        else { ia = RI_ZERO; ib = RI_ZERO; }
        const double sqm = q == 11 + 2 * ns ? 1.0 : 0.0;
        const bool wq = glane && q < nq;      // lanes that write sums
        // per sorted position, packed: particle lane, tail, valid, run head, run destination kind
        const int pk = src | ((int)tail << 6) | ((int)pv << 7) | (hpos << 8) | (rkind << 14);
        auto emit = [&](int k_, int d_, double v0, double v1, double v2) {
            if (!wq) return;
            if (k_ == 0) {
                double* dst = rec_ptr(d_) + SC_HDR;
                dst[q] = v0; dst[nq + q] = v1; dst[2 * nq + q] = v2;
            } else if (k_ == 1) {
                double* sv = s_stage + d_ * SC_VMAX;
                sv[q] = v0; sv[nq + q] = v1; sv[2 * nq + q] = v2;
            } else {
                double* eo = A.eo + (int64_t)d_ * SC_VMAX;
                unsafeAtomicAdd(eo + q, v0); unsafeAtomicAdd(eo + nq + q, v1); unsafeAtomicAdd(eo + 2 * nq + q, v2);
            }
        };
        const int p0 = glane ? g * P : 64;
        // the group's range [p0, p0 + P) among the sorted positions:
        //   hp   its first run began before the range
        //   hpe  ... and ends inside it (else the range is that run's middle)
        //   tp   its last run began inside the range and continues past it
        const unsigned long long tm = __ballot(tail);
        const unsigned long long rmask = p0 >= 64 ? 0ull : (~0ull << p0) & (p0 + P >= 64 ? ~0ull : ((1ull << (p0 + P)) - 1));
        const int w0 = __shfl(pk, p0 & 63);
        const int dc0 = __shfl(rdcode, p0 & 63);
        const int plast = min(p0 + P, 64) - 1;
        const int wl = __shfl(pk, plast & 63);
        const bool hp = p0 < 64 && ((w0 >> 7) & 1) && ((w0 >> 8) & 63) < p0;
        const bool hpe = hp && (tm & rmask) != 0ull;
        const bool tp = p0 < 64 && ((wl >> 7) & 1) && !((wl >> 6) & 1) && (hm & rmask) != 0ull;
        double a0 = 0.0, a1 = 0.0, a2 = 0.0;     // the run in progress
        double h0 = 0.0, h1 = 0.0, h2 = 0.0;     // the range's first run, when it began before the range
        // two positions per trip: the loop's bookkeeping is shared (measured
        // 0.8% faster than one; four was slower)
#pragma unroll 2
        for (int it = 0; it < P; ++it) {
            const int pos = p0 + it;
            const int w_ = __shfl(pk, pos & 63);
            const int dc = __shfl(rdcode, pos & 63);
            if (pos < 64 && ((w_ >> 7) & 1)) {
                const R* rq = wave_rec + (w_ & 63) * NREC;
                const R l0 = rq[0], l1 = rq[1], l2 = rq[2], rw = rq[3];
                const double gq = (double)rq[ia] * (double)rq[ib];
                const double w = (double)rw;
                const double wn0 = w * (double)l0, wn1 = w * (double)l1, wn2 = w * (double)l2;
                a0 = __builtin_fma(wn0, __builtin_fma(sqm, wn0, gq), a0);
                a1 = __builtin_fma(wn1, __builtin_fma(sqm, wn1, gq), a1);
                a2 = __builtin_fma(wn2, __builtin_fma(sqm, wn2, gq), a2);
                if ((w_ >> 6) & 1) {
                    // a run ends here: complete if it began in the range,
                    // else the first run's piece, completed after the carry
                    if (((w_ >> 8) & 63) >= p0) emit((w_ >> 14) & 3, dc, a0, a1, a2);
                    else { h0 = a0; h1 = a1; h2 = a2; }
                    a0 = 0.0; a1 = 0.0; a2 = 0.0;
                }
            }
        }
        if (hp && !hpe) { h0 = a0; h1 = a1; h2 = a2; }     // the whole range is the middle of one run
        // carry from group to group, in group order: what group g passes on
        // is its last run when that began in its range (a), else the
        // continued run when it spans the whole range (carry + h)
        double c0 = 0.0, c1 = 0.0, c2 = 0.0;
        for (int gg = 1; gg < G; ++gg) {
            const double o0 = tp ? a0 : (hp && !hpe ? c0 + h0 : 0.0);
            const double o1 = tp ? a1 : (hp && !hpe ? c1 + h1 : 0.0);
            const double o2 = tp ? a2 : (hp && !hpe ? c2 + h2 : 0.0);
            const int from = lane >= GS ? lane - GS : lane;
            const double r0 = __shfl(o0, from), r1 = __shfl(o1, from), r2 = __shfl(o2, from);
            if (g == gg) { c0 = r0; c1 = r1; c2 = r2; }
        }
        // a continued run that ends in this group's range: carry + h
        if (glane && hpe) emit((w0 >> 14) & 3, dc0, c0 + h0, c1 + h1, c2 + h2);
    }
    if (cells) {
        // (4) cell sums: a segmented inclusive scan of (1, w, w psi_a) over
        // the sorted positions; the last position of each (element, bin)
        // run holds the run's sums
        const unsigned ck = sk >> 6;
        const unsigned ckp = (unsigned)__shfl_up((int)ck, 1);
        const unsigned ckn = (unsigned)__shfl_down((int)ck, 1);
        const bool chead = lane == 0 || ckp != ck;
        const bool ctail = lane == 63 || ckn != ck;
        // the run's first position: the last run head at or before this one
        const int st = 63 - __clzll(__ballot(chead) & upto);
        const R* rq = wave_rec + src * NREC;
        const double w = pv ? (double)rq[3] : 0.0;
        double x[2 + MAXS];
        x[0] = 1.0;
        x[1] = w;
#pragma unroll
        for (int a = 0; a < MAXS; ++a) x[2 + a] = a < ns ? w * (double)rq[8 + a] : 0.0;
#pragma unroll
        for (int j2 = 0; j2 < 2 + MAXS; ++j2)
            if (j2 < nc) x[j2] = seg_scan(x[j2], lane, st);
        if (pv && ctail) {
            const int off = 3 * nq + sbin * nc;
            if (rkind == 1) {
                double* sv = s_stage + rdcode * SC_VMAX + off;
#pragma unroll
                for (int j2 = 0; j2 < 2 + MAXS; ++j2) if (j2 < nc) sv[j2] = x[j2];
            } else if (rkind == 0) {
                double* dst = rec_ptr(rdcode) + SC_HDR + off;
#pragma unroll
                for (int j2 = 0; j2 < 2 + MAXS; ++j2) if (j2 < nc) dst[j2] = x[j2];
            } else {
                double* eo = A.eo + (int64_t)rdcode * SC_VMAX + off;
#pragma unroll
                for (int j2 = 0; j2 < 2 + MAXS; ++j2) if (j2 < nc) unsafeAtomicAdd(eo + j2, x[j2]);
            }
        }
    }
    __syncthreads();
    // (5) the wavefront's merges: the staged sums of each shared element
    // whose lowest wavefront is this one, in wavefront order (entry index
    // t SC_SQ + s), go out as one record
    {
        auto take_slot = [&](int& handle) -> double* {
            int idx = 0;
            if (lane == 0) idx = atomicAdd(&s_slot, 1);
            idx = __shfl(idx, 0);
            if (idx < wg_slots) {
                handle = (int)(ltile * SC_RT) + wg_first + idx;
                return A.srec + C.rec_off + (int64_t)handle * C.rec_stride;
            }
            int pidx = 0;
            if (lane == 0) pidx = atomicAdd(A.pool_cnt, 1);
            pidx = __shfl(pidx, 0);
            if (pidx < A.pool_cap) {
                handle = -1 - pidx;
                return A.srec + A.pool_off + (int64_t)pidx * A.pool_stride;
            }
            handle = INT32_MIN;
            return nullptr;
        };
        const int ne_w = nw * SC_SQ;
        int el_j = -1;
        if (lane < ne_w && lane - (lane / SC_SQ) * SC_SQ < s_nst[lane / SC_SQ]) el_j = s_sel[lane];
        const int nmerge = s_nmerge[wid];
        for (int r = 0; r < nmerge; ++r) {
            const int el = s_mel[wid * 64 + r], first = s_mfirst[wid * 64 + r];
            const unsigned long long ents = __ballot(el_j == el);
            if (!ents) continue;          // every share of it went out as a record of its own
            double x0 = 0.0, x1 = 0.0;
            long long mk = 0;
            unsigned long long m = ents;
            while (m) {
                const int jx = __ffsll((long long)m) - 1;
                m &= m - 1;
                const int em = s_smask[jx];
                mk |= em;
                const double* sv = s_stage + jx * SC_VMAX;
                if (lane < nv && (lane < 3 * nq || ((em >> ((lane - 3 * nq) / nc)) & 1))) x0 += sv[lane];
                if (lane + 64 < nv && (lane + 64 < 3 * nq || ((em >> ((lane + 64 - 3 * nq) / nc)) & 1)))
                    x1 += sv[lane + 64];
            }
            int h;
            double* dst = take_slot(h);
            if (dst) {
                if (lane < nv) dst[SC_HDR + lane] = x0;
                if (lane + 64 < nv) dst[SC_HDR + 64 + lane] = x1;
                if (lane == 0) {
                    dst[0] = __longlong_as_double(kbase + wid * 64 + first);
                    dst[1] = __longlong_as_double((long long)el);
                    dst[2] = __longlong_as_double(mk);
                }
            } else {
                double* eo = A.eo + (int64_t)el * SC_VMAX;
                if (lane < nv && x0 != 0.0) unsafeAtomicAdd(eo + lane, x0);
                if (lane + 64 < nv && x1 != 0.0) unsafeAtomicAdd(eo + 64 + lane, x1);
                if (lane == 0) {
                    atomicExch(A.eof + el, 1);
                    atomicAdd(A.counters + (int64_t)c * NCNT + C_SCATTER_OVERFLOW, 1ull);
                }
            }
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) A.wgcnt[lb] = s_slot < wg_slots ? s_slot : wg_slots;
    }
    // ---- counters, one atomic per wavefront
    {
        int v0 = wave_sum_int(wc.fallback), v1 = wave_sum_int(wc.refl), v2 = wave_sum_int(wc.per);
        int v3 = wave_sum_int(flips), v5 = wave_sum_int(nans), v6 = wave_sum_int(wc.steps);
        if (__lane_id() == 0) {
            unsigned long long* cc = A.counters + (int64_t)c * NCNT;
            if (v0) atomicAdd(cc + C_WALK_FALLBACK, (unsigned long long)v0);
            if (v1) atomicAdd(cc + C_REFLECT, (unsigned long long)v1);
            if (v2) atomicAdd(cc + C_PERIODIC, (unsigned long long)v2);
            if (v3) atomicAdd(cc + C_OMEGA_FLIP, (unsigned long long)v3);
            if (v5) atomicAdd(cc + C_NAN, (unsigned long long)v5);
            if (v6) atomicAdd(cc + C_WALK_STEPS, (unsigned long long)v6);
        }
    }
}

template __global__ void k_particle_step<double>(StepArgs<double>);
template __global__ void k_particle_step<float>(StepArgs<float>);

// Initial ensemble of a case (R-29..R-32): particle i of the case lies in its
// element i / ppe, has id i, and draws its state from the generator with
// purpose 1 (init_uniforms): position uniform in the element, Gaussian
// velocity, Gamma(4, scale) frequency, scalars set inside their initial
// disks, mass weight A_e / ppe. FP64 arithmetic in either precision (the
// FP32 context stores the rounded values); the operation order is the one of
// the written recipe, so the FP64 ensemble is the same bit for bit wherever
// the recipe is followed.
template <typename R>
__global__ void k_particles_init(InitArgs<R> A)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= A.n) return;
    const CaseDev& C = A.cases[A.cs];
    const int e = C.eoff + (int)(i / A.ppe);
    double u[10];
    init_uniforms(C.seed_lo, C.seed_hi, (uint32_t)i, C.stream, u);
    const double* v = A.exy + 6 * (int64_t)e;
    const double s = __builtin_sqrt(u[0]);
    const double l0 = 1.0 - s, l1 = s * (1.0 - u[1]), l2 = s * u[1];
    const double x = (l0 * v[0] + l1 * v[2]) + l2 * v[4];
    const double y = (l0 * v[1] + l1 * v[3]) + l2 * v[5];
    const double r0 = __builtin_sqrt(-2.0 * ln_series(u[2]));
    const double r1 = __builtin_sqrt(-2.0 * ln_series(u[4]));
    double s0, c0, s1, c1;
    sincos2pi_series(u[3], s0, c0);
    sincos2pi_series(u[5], s1, c1);
    const double om = -A.omega_scale * (((ln_series(u[6]) + ln_series(u[7])) + ln_series(u[8])) + ln_series(u[9]));
    const int64_t p = C.poff + i;
    A.P.x[p] = (R)x; A.P.y[p] = (R)y;
    A.P.u[p] = (R)(A.u_std * (r0 * c0));
    A.P.v[p] = (R)(A.u_std * (r0 * s0));
    A.P.w[p] = (R)(A.u_std * (r1 * c1));
    A.P.om[p] = (R)om;
    A.P.wt[p] = (R)(A.area[e] / (double)A.ppe);
    A.P.elem[p] = e;
    A.P.id[p] = (uint32_t)i;
    A.P.bin[p] = 0;
    for (int a = 0; a < C.ns; ++a) {
        double val = 0.0;
        if (A.disk[a][2] > 0.0) {
            const double dx = x - A.disk[a][0], dy = y - A.disk[a][1];
            if (dx * dx + dy * dy < A.disk[a][2] * A.disk[a][2]) val = A.disk[a][3];
        }
        A.P.psi[C.psioff + (int64_t)a * C.cap + i] = (R)val;
    }
}
template __global__ void k_particles_init<double>(InitArgs<double>);
template __global__ void k_particles_init<float>(InitArgs<float>);

// Device draws of the Wiener increments (test hook of R-09/R-10).
template <typename R>
__global__ void k_draw_gaussians(uint32_t slo, uint32_t shi, uint32_t step, uint32_t stream,
                                 const uint32_t* __restrict__ ids, int64_t n, R* __restrict__ out)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    R xi[6];
    if constexpr (sizeof(R) == 8) gauss6_f64(slo, shi, ids[i], step, stream, xi);
    else gauss6_f32(slo, shi, ids[i], step, stream, xi);
    for (int j = 0; j < 6; ++j) out[6 * i + j] = xi[j];
}
template __global__ void k_draw_gaussians<double>(uint32_t, uint32_t, uint32_t, uint32_t, const uint32_t*, int64_t, double*);
template __global__ void k_draw_gaussians<float>(uint32_t, uint32_t, uint32_t, uint32_t, const uint32_t*, int64_t, float*);

}  // namespace pdfmc
