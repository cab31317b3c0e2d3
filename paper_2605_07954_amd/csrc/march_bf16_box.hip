// Row-marching kernels, BF16 storage, box footprints (see march.hip).
#include "march_kern.h"

namespace st {

march_k::MarchFn march_lookup_bf16_box(int mode, int r, int levels) {
    return march_k::march_lookup_shape<ST_BF16, SHAPE_BOX>(mode, r, levels);
}

}  // namespace st
