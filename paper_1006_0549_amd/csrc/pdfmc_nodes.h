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
    const int32_t* incpos;           // [3*3*ne] CSR positions of (row, vertex) per incidence entry
    const int32_t* csr_ptr;          // [nn+1]
    const int32_t* csr_col;          // [nnz]
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
    double* er_val;                  // [nnz]
    double* pk_val;                  // [nnz] stiffness of the projection
    double* pb;                      // [nn]
    double* phi;                     // [nn]
    double* P;                       // [nn] mean pressure
    unsigned long long* counters;    // [ncase][NCNT]
};

constexpr int AMG_MAXL = 8;        // multigrid levels
constexpr int AMG_MAXC = 64;       // largest coarsest level (dense inverse in LDS)

// One multigrid hierarchy. Level 0 is the fine system: its rows are the
// case's statistics nodes, A0 is a slice of the global CSR (row offset r0,
// global columns); coarser levels use local indices.
struct AmgDev {
    int32_t nlev, r0;
    int32_t n[AMG_MAXL];
    const int32_t* Aptr[AMG_MAXL];
    const int32_t* Acol[AMG_MAXL];
    double* Aval[AMG_MAXL];
    const int32_t* Pptr[AMG_MAXL];
    const int32_t* Pcol[AMG_MAXL];
    const double* Pval[AMG_MAXL];
    const int32_t* Rptr[AMG_MAXL];
    const int32_t* Rcol[AMG_MAXL];
    const double* Rval[AMG_MAXL];
    double omega[AMG_MAXL];        // Jacobi smoothing weight per level
    double coarse_shift;           // relative diagonal shift of the coarsest inverse
};

// Galerkin update of one level of one hierarchy: dst[k] = sum coef src[idx]
struct GalJob {
    int32_t nnz;
    const int32_t* gptr;
    const int32_t* gidx;           // positions relative to src
    const double* gcoef;
    const double* src;
    double* dst;
};

struct CgJob {
    int32_t r0, n;                   // global row range
    const int32_t* ptr;
    const int32_t* col;
    const double* val;
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
    double* amg_work;              // per-job vectors: dinv, x, b, t on every level
};

}  // namespace pdfmc
