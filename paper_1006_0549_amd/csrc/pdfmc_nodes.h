// Arguments of the node-level kernels (FP64 Eulerian side).
#pragma once
#include "pdfmc_dev.h"

namespace pdfmc {

// records of an element beyond its SC_K list entries that the element pass
// still sums in key order, through one overflow list per pass
constexpr int SC_XK = 192;

struct NodeArgs {
    int32_t nn, ne;                  // global statistics nodes and elements
    int32_t first_stats;             // 1: no previous node statistics exist yet
    int32_t pad;
    const CaseDev* cases;
    const int32_t* node_case;        // [nn]
    const int32_t* elem_case;        // [ne]
    const double* rec;               // [8*ne] FP64 element records
    const double* area;              // [ne]
    const double* vol;               // [nn] lumped node areas
    const int4* tri_s;               // [ne]
    const int32_t* inc_ptr;          // [nn+1] absolute offsets into inc
    const int32_t* inc;              // [3*ne] entries 3*e+k (global e)
    const int32_t* incpos;           // [3*3*ne] ELL positions of (row, vertex) per incidence entry
    const int32_t* ell_col;          // Galerkin pattern, ELL column-major per case, local columns
    const int32_t* ell_len;          // [nn] entries per row
    const int32_t* is_wall;          // [nn]
    const double* wnx;               // [nn]
    const double* wny;
    double* nsum;                    // [nn][NQ]
    double* stats;                   // [nn][NST]
    double* F;                       // [nn][NF]
    double* csum;
    int32_t* ccnt;                   // [ne][8]
    double* kf;                      // [nn] floored k
    double* ef;                      // [nn] floored eps
    double* L2;                      // [nn]
    double* er_r;                    // [nn][5] relaxation sources (a node's five together)
    double* er_dval;                 // [5][nn] wall values
    double* er_b;                    // [nn][5] right-hand sides (components interleaved)
    double* er_x;                    // [nn][5] relaxed tensor (warm start)
    double* er_val;                  // relaxation matrix (ELL)
    double* pk_val;                  // stiffness of the projection (ELL)
    double* pb;                      // [nn]
    double* phi;                     // [nn]
    double* P;                       // [nn] mean pressure (the last projection's phi)
    double* gphi;                    // [nn][2] its recovered gradient (the next step's velocity correction)
    unsigned long long* counters;    // [ncase][NCNT]
    // scatter records of the particle kernel (see pdfmc_dev.h)
    const double* srec;
    int64_t pool_off;
    int32_t pool_stride, pad2;
    int32_t* ecnt;                   // [ne] records listed per element
    int64_t* eslot;                  // [ne][SC_K] record key << 32 | handle (>= 0 regular, < 0 pool: -1 - index)
    int32_t* eof;                    // [ne] overflow flags
    double* eo;                      // [ne][SC_VMAX] overflow sums
    const int32_t* wgcnt;            // [workgroups] regular record slots used by each workgroup
    double* etot;                    // [ne][3][NQ] vertex sums of each element
    // an element's records beyond its SC_K list entries (up to SC_XK more):
    // appended to one list for the pass, which the element pass searches
    int64_t* ovl;                    // [ovl_cap] key << 32 | handle, as in eslot
    int32_t* ovl_el;                 // [ovl_cap] their elements
    int32_t* ovl_n;                  // entries appended in this pass (cleared before each particle kernel)
    int32_t ovl_cap, pad3;
};

constexpr int AMG_MAXL = 8;        // multigrid levels
constexpr int AMG_MAXC = 64;       // largest coarsest level (dense inverse in LDS)

// Square or rectangular matrix in ELL form, column-major (entry k of row i at
// k * n + i), local column indices, zero-valued padding.
struct EllDev {
    int32_t n, w;
    const int32_t* col;
    const double* val;
    const int32_t* len;            // entries of each row (padding after them), or null: w for every row
};

// One multigrid hierarchy; level 0 is the fine system of one case. Levels
// 0..nbig-1 are processed by row-parallel phase kernels over many
// workgroups; levels nbig.. by one workgroup per system.
struct AmgDev {
    int32_t nlev, nbig;
    int32_t n[AMG_MAXL];
    EllDev A[AMG_MAXL];
    EllDev P[AMG_MAXL];            // level l <- level l+1
    EllDev R[AMG_MAXL];            // level l+1 <- level l
    double* dinv[AMG_MAXL];        // inverse diagonals, refreshed every solve
    // two-step polynomial smoother in D^-1 A, from zero:
    //   y1 = sa D^-1 b,  y2 = se y1 + sc D^-1 (b - A y1)
    // and from y0: y1 = y0 + sa D^-1 (b - A y0),
    //   y2 = y1 + (se - 1)(y1 - y0) + sc D^-1 (b - A y1)
    double sa[AMG_MAXL], se[AMG_MAXL], sc[AMG_MAXL];
    double* ainv;                  // [AMG_MAXC * AMG_MAXC] inverse of the coarsest matrix
    double coarse_shift;           // relative diagonal shift of the coarsest inverse
};

// Galerkin update of one level of one hierarchy:
// dst[gdst[k]] = sum_j gcoef[j] src[gidx[j]], j in [gptr[k], gptr[k+1])
struct GalJob {
    int32_t nnz;
    int32_t lpe;                   // lanes per coarse entry: 1, 4 or 16 (from this hierarchy's lists)
    const int32_t* gptr;
    const int32_t* gidx;
    const double* gcoef;
    const int32_t* gdst;
    const double* src;
    double* dst;
};

// One linear system on the rows of one case; every pointer is offset to the
// case's first row (local indices). Preconditioned CG whose iterations are
// split into phases; scalars are accumulated per iteration in rotating slots.
constexpr int MG_SLOT = 32;        // doubles per accumulator slot: one 256-byte line per slot and column
constexpr int MG_NSLOT = 5;        // 4 iteration slots + 1 set-up slot
constexpr int MG_PART = 16;        // doubles per row block's partial sums (nv M <= 10)
struct MgJob {
    int32_t hier;                  // index of the hierarchy
    int32_t mean_free;             // singular system: solution and residual kept mean-free
    int32_t warm;                  // 1: start from the current x; 0: start from zero
    int32_t nv;                    // right-hand sides sharing the matrix (1 or NER)
    int32_t maxit, n;              // iteration cap, rows
    double tol;                    // relative residual tolerance
    // every vector below holds nv interleaved columns: entry v of row i at i * nv + v
    double* b;                     // right-hand side (made mean-free in place)
    double* x;                     // solution, warm start
    double* r[2];                  // residual, ping-pong by iteration parity
    double* p[2];                  // search direction, ping-pong
    double* q;                     // A p
    double* lb[AMG_MAXL];          // level right-hand sides (level 0 uses r)
    double* ly[AMG_MAXL];          // level corrections (level 0: z = M^-1 r)
    double* la[AMG_MAXL];          // smoothing intermediate
    double* lt[AMG_MAXL];          // residual, then the pre-smoothing copy
    double* acc;                   // [MG_NSLOT][nv][MG_SLOT]
    int32_t* state;                // [0] converged, [1] iteration count
    unsigned long long* iters;
    unsigned long long* fails;
    unsigned int* need;            // largest iteration count of this system since the host last read it
    double* part;                  // [nblk0][MG_PART] the row-parallel workgroups' sums of a phase
    int32_t nblk0;                 // row blocks of level 0
    int32_t ksw;                   // the row-parallel phases run iterations k < ksw (<= maxit); the
                                   // one-workgroup completion takes over at k = ksw. Set from this
                                   // system's own history, so its bits do not depend on the batch.
};

// One supernode of a case's projection factor (nested-dissection Cholesky of
// the constant projection matrix), with global unknown indices.
constexpr int DS_MAXS = 2048;      // largest supernode and reach the sweeps stage in LDS
constexpr int DS_SMALL = 256;      // LDS capacity of the sweep variant for small supernodes
struct DsNode {
    int32_t s, m;                  // own unknowns, later unknowns reached
    int64_t idx;                   // own unknowns at idx[idx .. idx+s), later ones at [idx+s .. idx+s+m)
    int64_t val;                   // L11^-1 (s x s, row-major, lower) at val, then L21 (m x s, row-major)
    int64_t cof;                   // its updates of the m later unknowns at contrib[cof .. cof+m)
};
// The forward sweep's updates of later unknowns, for a fixed summation order:
// unknown u (global index) subtracts contrib[clist[q]] for q in
// [cptr[u], cptr[u+1]), its contributors in supernode order.
struct DsUpd {
    const int32_t* cptr;
    const int32_t* clist;
    double* contrib;
};
struct DsCase {
    int32_t noff, n, pin, pad;     // first statistics node, unknowns, decoupled unknown (case-local)
};

}  // namespace pdfmc
