// Row-marching kernels with BF16 storage (see march.hip).
#include "march_kern.h"

namespace st {

march_k::MarchFn march_lookup_bf16(int V, int shape, int r, int levels) {
    return march_k::march_lookup_storage<ST_BF16>(V, shape, r, levels);
}

}  // namespace st
