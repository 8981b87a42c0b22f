// Internal layout shared by the library's host and kernel sources.
//
// Device data of a context are concatenations over its cases: particles,
// elements, statistics nodes (periodic images merged) and boundary records
// each carry a per-case offset. Element and node ids stored on the device are
// global (offset included); the host converts to case-local ids at the API.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pdfmc {

constexpr int NF = 22;         // Eulerian field slots per node
constexpr int NFE = 24;        // padded row of the element-major field copy (3 rows per element)
constexpr int MAXS = 4;        // scalars per case
constexpr int NQ = 20;         // node-sum stride: 12 + 2*MAXS
constexpr int NST = 20;        // statistics stride: 12 + 2*MAXS
constexpr int NCNT = 13;       // counters per case
constexpr int TILE = 256;      // particle ranges of cases are padded to this
constexpr int NER = 5;         // elliptic-relaxation components 11,12,21,22,33

enum Field {
    F_U1 = 0, F_U2, F_U3, F_DPX, F_DPY,
    F_DU1X, F_DU1Y, F_DU2X, F_DU2Y, F_DU3X, F_DU3Y,
    F_LAP1, F_LAP2, F_LAP3,
    F_G11, F_G12, F_G21, F_G22, F_G33,
    F_OMEGA, F_C0EPS, F_SOMEGA
};
// slots of the element-major copy past the fields: the recovered gradient of
// the mean pressure, i.e. the velocity correction of the next step (R-27)
constexpr int FE_GPX = 22, FE_GPY = 23;

// The logical block of hardware block b of a grid of nb blocks. The chip
// hands workgroups to its eight XCDs in turn (block b to XCD b mod 8), each
// with an L2 of its own; this bijection gives XCD x the contiguous logical
// blocks [x q + min(x, r), ...), q = nb / 8, r = nb mod 8, so that blocks
// working on neighbouring data share an L2.
__device__ inline int xcd_block(int b, int nb)
{
    const int q = nb >> 3, r = nb & 7, x = b & 7, i = b >> 3;
    return x < r ? x * (q + 1) + i : r * (q + 1) + (x - r) * q + i;
}

enum Counter {
    C_WALK_FALLBACK = 0, C_REFLECT, C_PERIODIC, C_OMEGA_FLIP, C_EMPTY_NODE, C_NAN,
    C_WALK_STEPS, C_CG_ER, C_CG_P, C_CG_FAIL, C_K_FLOOR, C_EPS_FLOOR, C_SCATTER_OVERFLOW
};

// Scatter records (reading R-11 and the cell sums of R-23). Each workgroup of
// the particle kernel writes one record per distinct element among its
// particles (more when the element's sums could not all be merged): the
// element's three vertex sums of the node moments and its cell sums, summed
// over the workgroup's particles in a fixed order. Record layout (doubles):
// [0] key (int64 bits: global workgroup index * 512 + the element's first
// lane in the workgroup, or 256 + a wavefront's first lane of it for a share
// that went out alone), [1] element (int64 bits), [2] mask of the bins with
// particles (int64 bits), [3 .. 3 + 3 nq) vertex sums (vertex-major), then,
// with cells, 8 bins x (2 + ns): particle count, sum w, sum w psi_a (valid
// for the bins in the mask only).
constexpr int SC_HDR = 3;
constexpr int SC_RT = 40;       // regular record slots per particle tile
constexpr int SC_SQ = 6;        // sums of shared elements a wavefront stages in LDS for the merge
constexpr int SC_K = 64;        // record handles listed per element per step (one per lane of the element pass)
constexpr int SC_VMAX = 3 * NQ + 8 * (2 + MAXS);   // values of a record
__device__ __host__ inline int sc_nvals(int ns, bool cells) { return 3 * (12 + 2 * ns) + (cells ? 8 * (2 + ns) : 0); }

struct BcDev {
    int32_t type;        // 0 wall, 1 periodic
    int32_t pad;
    double uw[3];
    double shift[2];
    float uwf[3];
    float shiftf[2];
};

struct CaseDev {
    int64_t poff, np;          // particle range [poff, poff+np)
    int64_t psioff;            // scalar block: psi[psioff + a*cap + i]
    int64_t cap;               // capacity (stride of the scalar block)
    int64_t cmoff;             // cell means [ne][8][ns] at cmean + cmoff
    int64_t csoff;             // cell sums  [ne][8][1+ns] at csum + csoff
    int32_t eoff, ne, noff, nsn, bcoff, nbc;
    int32_t ns, nbins, nmin, mode;
    uint32_t seed_lo, seed_hi, stream, pad0;
    int32_t ell_w, pad1;       // width of the case's Galerkin matrix in ELL form
    int64_t ell_off;           // its offset in the global ELL arrays
    int64_t inc_off;           // incidence list offset (entries 3*e+k, global e)
    // particle-step constants, computed on the host in FP64 (and rounded for FP32)
    double dt, tnu, sq_nu, C3, c34, hphi;
    float fdt, ftnu, fsq_nu, fC3, fc34, fhphi;
    double src[MAXS][4];
    float srcf[MAXS][4];
    // Eulerian constants
    double nu, C0, Cw1, Cw2, C1, C2, gamma5, Cv, CL, Ceta, nu34, k_floor, eps_floor;
    double dpdx[2];
    double cg_rtol;
    double neff_min;           // least effective sample size of a node estimate
    int32_t cg_maxit, reaction;  // reaction: closed scalar source kind (0, 1, 2)
    int32_t rebin;             // bins and cell means formed again at the end of a step (R-36)
    double kr[MAXS];           // reaction rate constants
    float fkr[MAXS];
    int64_t rec_off;           // scatter records of the case at srec + rec_off (doubles)
    int32_t rec_stride;        // doubles per record: SC_HDR + values with cells
    uint32_t freeze;           // field slots kept at their uploaded values (bit q: slot q)
};

template <typename R>
struct Particles {
    R *x, *y, *u, *v, *w, *om, *wt, *psi;
    int32_t* elem;
    uint32_t* id;
    uint8_t* bin;
};

template <typename R>
struct MeshDev {
    const R* rec;          // [8*NE]: x1, y1, b0, b1, b2, c0, c1, c2   (R-05)
    const int4* tri_s;     // statistics node per vertex (global), .w unused
    const int4* nbr;       // neighbour element (global) or -1 - global bc index
    const int4* partner;   // partner element across a periodic edge (global) or -1
    const R* exy;          // [6*NE]: vertex coordinates, for reflections
    const BcDev* bc;
};

// Everything a particle kernel needs, passed by value.
template <typename R>
struct StepArgs {
    Particles<R> P;
    MeshDev<R> M;
    const CaseDev* cases;
    const int32_t* tile_case;     // particle tile -> case
    const R* Fel;                 // fields at the element's vertices, [NE][3][NFE] (Real)
    const R* cmean;               // cell means (Real)
    double* srec;                 // scatter records (regular slots per case, then the pool)
    int64_t pool_off;             // pool records at srec + pool_off, pool_stride doubles each
    int32_t pool_stride, pool_cap;
    int32_t* pool_cnt;            // records taken from the pool this step
    int32_t* wgcnt;               // [workgroups] regular record slots used by each workgroup
    int32_t* eof;                 // [NE] 1: the element has values in the overflow sums
    double* eo;                   // [NE][SC_VMAX] overflow sums (FP64 atomics)
    unsigned long long* counters; // [ncase][NCNT]
    const uint32_t* step;         // device step index
    int32_t ntiles;
    int32_t advance;              // 1: advance then statistics; 0: statistics only
    int32_t do_bins;              // 1: bins + cell sums
    int32_t rebin_only;           // 1: only the cases with the end-of-step rebinning take part
    int32_t scatter;              // 1: statistics records of the new state; 0: none
};

// Arguments of the initial-ensemble kernel (R-29..R-32).
template <typename R>
struct InitArgs {
    Particles<R> P;
    const CaseDev* cases;
    const double* exy;         // [6*NE] FP64 vertex coordinates
    const double* area;        // [NE] element areas
    int64_t n;                 // particles: ne * ppe
    int32_t cs, ppe;
    double u_std, omega_scale;
    double disk[MAXS][4];
};

}  // namespace pdfmc
