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
    int64_t* scan;           // [ne]
    int64_t* cursor;         // [ne]
};

}  // namespace pdfmc
