// Sparse Cholesky factor of a case's projection matrix by nested dissection
// (host side): the matrix is constant for the whole run, so it is factored
// once when the case is added and every projection solve (reading R-27) is
// two sweeps over the factor on the GPU.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "pdfmc_amg.h"

namespace pdfmc {

// One supernode: variables eliminated together (a separator, or a leaf of the
// dissection), the later variables its columns reach, the inverse of the
// Cholesky factor of its diagonal block and its off-diagonal block.
struct CholNode {
    std::vector<int> vars;      // s variables, in elimination order
    std::vector<int> str;       // m later variables (ancestors), in elimination order
    std::vector<double> linv;   // s x s, row-major, lower triangular: L11^-1
    std::vector<double> l21;    // m x s, row-major: L21
    std::vector<int> children;
    int height = 0;             // 0 for a node without children, else 1 + max over the children
};

struct CholFactor {
    int n = 0;
    int pin = -1;               // the variable whose row and column are decoupled
    int height = 0;             // height of the tallest node
    int max_s = 0, max_m = 0;
    int64_t n_idx = 0, n_val = 0;   // total variable indices and stored values
    std::vector<CholNode> nodes;    // children before their parent
};

// Factors the symmetric matrix K of a connected Neumann problem (constant null
// space) with the row and column of `pin` reduced to their diagonal, which
// makes it positive definite; a solution of K x = b for a b of zero sum is
// then the solution with x[pin] = 0. (x, y) are coordinates of the unknowns,
// used to bisect the graph; parts of at most `leaf` unknowns are not split.
// Returns false with a message when a pivot is not positive.
bool chol_factor(const CsrH& K, const std::vector<double>& x, const std::vector<double>& y, int pin, int leaf,
                 CholFactor& F, std::string& err);

}  // namespace pdfmc
