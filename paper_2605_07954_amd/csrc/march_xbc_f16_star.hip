// Row-marching kernels with the periodic and framed boundary rules, F16 storage, star footprints
// (see march.hip).
#include "march_kern.h"

namespace st {

march_k::MarchFn march_lookup_xbc_f16_star(int mode, int r, int levels, bool periodic) {
    return march_k::march_lookup_shape_xbc<ST_F16, SHAPE_STAR>(mode, r, levels, periodic);
}

}  // namespace st
