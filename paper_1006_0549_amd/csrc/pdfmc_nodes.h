// Arguments of the node-level kernels (FP64 Eulerian side).
#pragma once
#include "pdfmc_dev.h"

namespace pdfmc {

struct NodeArgs {
    int32_t nn, ne;                  // global statistics nodes and elements
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
    double* er_r;                    // [5][nn] relaxation sources
    double* er_dval;                 // [5][nn] wall values
    double* er_b;                    // [5][nn] right-hand sides
    double* er_x;                    // [5][nn] relaxed tensor (warm start)
    double* er_val;                  // relaxation matrix (ELL)
    double* pk_val;                  // stiffness of the projection (ELL)
    double* pb;                      // [nn]
    double* phi;                     // [nn]
    double* P;                       // [nn] mean pressure
    unsigned long long* counters;    // [ncase][NCNT]
};

constexpr int AMG_MAXL = 8;        // multigrid levels
constexpr int AMG_MAXC = 64;       // largest coarsest level (dense inverse in LDS)

// Square or rectangular matrix in ELL form, column-major (entry k of row i at
// k * n + i), local column indices, zero-valued padding.
struct EllDev {
    int32_t n, w;
    const int32_t* col;
    const double* val;
};

// One multigrid hierarchy; level 0 is the fine system of one case.
struct AmgDev {
    int32_t nlev, pad;
    int32_t n[AMG_MAXL];
    EllDev A[AMG_MAXL];
    EllDev P[AMG_MAXL];            // level l <- level l+1
    EllDev R[AMG_MAXL];            // level l+1 <- level l
    double omega[AMG_MAXL];        // Jacobi smoothing weight per level
    double coarse_shift;           // relative diagonal shift of the coarsest inverse
};

// Galerkin update of one level of one hierarchy:
// dst[gdst[k]] = sum_j gcoef[j] src[gidx[j]], j in [gptr[k], gptr[k+1])
struct GalJob {
    int32_t nnz;
    const int32_t* gptr;
    const int32_t* gidx;
    const double* gcoef;
    const int32_t* gdst;
    const double* src;
    double* dst;
};

// One linear system on the rows of one case; every pointer is offset to the
// case's first row (local indices).
struct CgJob {
    EllDev A;
    double* b;
    double* x;
    double* r;
    double* p;
    double* q;
    double* dinv;
    double tol;
    int32_t maxit, mean_free;
    unsigned long long* iters;
    unsigned long long* fails;
    const AmgDev* amg;             // multigrid preconditioner, or null for Jacobi
    double* amg_work;              // per-job vectors: 5 per level
};

}  // namespace pdfmc
