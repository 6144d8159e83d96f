// Patch-kernel variants of the 3D level list 7, 3, 1 (FP64, FP32, BF16 and split BF16).
#include "patch_kernels.hpp"

namespace pmgi {

const PatchVariant* variants_3d_q7_table(size_t* count) {
  static const PatchVariant table[] = {
      make_variant<double, 3, 7, 3, 1>(),
      make_variant<float, 3, 7, 3, 1>(),
      make_variant_bf16<false, 3, 7, 3, 1>(),
      make_variant_bf16<true, 3, 7, 3, 1>()};
  *count = sizeof(table) / sizeof(table[0]);
  return table;
}

hipError_t variants_3d_q7_upload() { return upload_tables(); }

}  // namespace pmgi
