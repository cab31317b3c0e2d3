// Row-marching kernels with the periodic and framed boundary rules, F32 storage, box footprints
// (see march.hip).
#include "march_kern.h"

namespace st {

march_k::MarchFn march_lookup_xbc_f32_box(int mode, int r, int levels, bool periodic) {
    return march_k::march_lookup_shape_xbc<ST_F32, SHAPE_BOX>(mode, r, levels, periodic);
}

}  // namespace st
