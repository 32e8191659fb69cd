// ILU(0) apply kernels for real vectors of 2 limbs (see apply.hpp).
#include "apply.hpp"

namespace mpk {
template int ilu0_apply_ck<1, 2>(const Ilu0 &, int, const double *, double *, int32_t *,
                                  int32_t *, const int32_t *, hipStream_t);
}
