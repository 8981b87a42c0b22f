// Arguments of the particle sort kernels.
#pragma once
#include "pdfmc_dev.h"

namespace pdfmc {

struct SortArgs {
    const CaseDev* cases;
    const int32_t* tile_case;
    const int32_t* elem_case;
    int32_t ntiles, ne;
    const int32_t* elem;     // keys of the source buffer set (hist)
    int32_t* count;          // [ne]
    int64_t* scan;           // [ne] exclusive scan of the counts inside each block of SCAN_B elements
    int64_t* bsum;           // [ne / SCAN_B + 1] block totals, then their exclusive scan
    int64_t* cursor;         // [ne] next free slot of each element's segment
    int64_t* start;          // [ne] first slot of each element's segment
    uint32_t* tmp_id;        // [NP] ids placed in their segments (arbitrary order inside)
    int64_t* tmp_src;        // [NP] source index of each placed id
    int64_t* perm;           // [NP] source index of the particle at each final position
    int32_t* big;            // [ne] elements whose segments are sorted by k_sort_order_big
    int32_t* nbig;           // their count
};

constexpr int SCAN_B = 1024;     // elements per block of the count scan

}  // namespace pdfmc
