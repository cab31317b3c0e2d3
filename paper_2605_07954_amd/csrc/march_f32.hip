// Row-marching kernels with F32 storage (see march.hip).
#include "march_kern.h"

namespace st {

march_k::MarchFn march_lookup_f32(int V, int shape, int r, int levels) {
    return march_k::march_lookup_storage<ST_F32>(V, shape, r, levels);
}

}  // namespace st
