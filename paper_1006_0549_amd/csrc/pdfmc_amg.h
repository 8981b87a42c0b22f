// Smoothed-aggregation multigrid hierarchy (host setup) for the P1 Galerkin
// systems of the Eulerian solves. The aggregates and prolongators come from
// the constant stiffness matrix of the mesh; the operator on every level is
// the Galerkin product P^T A P. For a matrix whose values change every step
// (the elliptic relaxation) the coarse values are recomputed on the device
// from per-level contribution lists: A_{l+1}[k] = sum_j coef_j A_l[idx_j].
#pragma once
#include <vector>

namespace pdfmc {

struct CsrH {
    int n = 0, m = 0;                   // rows, columns
    std::vector<int> ptr, col;
    std::vector<double> val;
};

struct AmgLevelH {
    CsrH A;                             // operator on this level
    CsrH P;                             // prolongator to this level from the next (n x n_next)
    CsrH R;                             // restriction = P^T
    std::vector<int> gptr, gidx;        // contributions to the next level's A values
    std::vector<double> gcoef;
};

struct AmgH {
    std::vector<AmgLevelH> lv;          // lv.back() is the coarsest (no P/R)
};

// ELL form of a CSR matrix, column-major: entry k of row i at k * n + i.
// The width is the longest row rounded up to a multiple of 4; shorter rows
// are padded with value 0 and column i itself (pad_self) or column 0.
struct EllH {
    int n = 0, w = 0;
    std::vector<int> col, len;
    std::vector<double> val;
    std::vector<int> map;               // CSR position -> ELL position
};

void to_ell(const CsrH& A, bool pad_self, EllH& E);

// Build the hierarchy of the symmetric matrix A0 (values used for strength,
// aggregation and prolongator smoothing). Rows flagged in `isolated` keep no
// strong connections (Dirichlet rows). Coarsening stops at <= max_coarse
// unknowns or max_levels levels.
void amg_setup(const CsrH& A0, const std::vector<int>& isolated, AmgH& H, int max_coarse, int max_levels);

}  // namespace pdfmc
