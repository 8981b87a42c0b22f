// Host-side mesh tables of one case (case-local ids).
#pragma once
#include <string>
#include <vector>

#include "../../include/pdfmc.h"

namespace pdfmc {

struct MeshHost {
    int nn = 0, ne = 0, nsn = 0;
    std::vector<double> x, y;
    std::vector<int> tri, tag;
    std::vector<pdfmc_bc> bc;
    std::vector<double> rec, area, vol;
    std::vector<int> nbr, partner, snode, rep, tri_s;
    std::vector<int> inc_ptr, inc;
    std::vector<int> is_wall;
    std::vector<double> wnx, wny;
    std::vector<int> csr_ptr, csr_col, incpos;
};

int derive_mesh(const pdfmc_mesh_desc& d, MeshHost& m, std::string& err);

}  // namespace pdfmc
