// Where the backward of a submanifold layer keeps its bfloat16 dZ and its bias partials inside
// the workspace of npvs_sparse_conv_bwd (defined in backward.hip), for kernels of other files that
// form a layer's dZ in place.
#pragma once
#include "npvs_common.hpp"

namespace npvs {

// Byte offsets of dZ16 [cap][cout] and of the bias partials dbpart[kBwdDbBlocks][cout] in the
// BF16 backward workspace of a (cin -> cout) layer, and that workspace's size in bytes.
void bwd_ws_dz_parts(int32_t cin, int32_t cout, int32_t cap, size_t *o_dz16, size_t *o_dbpart, size_t *bytes);

}  // namespace npvs
