// Chebyshev-interpolation fast multipole method (Sec. 3.3): placeholder until
// the tree and translation kernels land.
#include "common.hpp"

namespace ertvie {

struct FmmData {
    int dummy;
};

ert_status fmm_apply(ert_plan_impl*, int, int, const double*, double*, int) { return ERT_EUNSUPPORTED; }

void fmm_destroy(FmmData* f) { delete f; }

}  // namespace ertvie
