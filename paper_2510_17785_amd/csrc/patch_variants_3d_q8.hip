// Patch-kernel variants of the 3D level list 8, 4, 2, 1.
#include "patch_kernels.hpp"

namespace pmgi {

const PatchVariant* variants_3d_q8_table(size_t* count) {
  static const PatchVariant table[] = {
      make_variant<double, 3, 8, 4, 2, 1>(),
      make_variant<float, 3, 8, 4, 2, 1>()};
  *count = sizeof(table) / sizeof(table[0]);
  return table;
}

hipError_t variants_3d_q8_upload() { return upload_tables(); }

}  // namespace pmgi
