// Discrete adjoint of the RK4 + kick schedule (placeholder until implemented).
#include "../../include/lll.h"
#include "lll_internal.hpp"

extern "C" lll_status lll_adjoint(lll_lattice*, const lll_params*, uint64_t, int64_t, int32_t,
                                  double, const double*, double*, double*, double*, void*, void*) {
    return LLL_EUNSUPPORTED;
}
