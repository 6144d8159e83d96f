// Patch-kernel variants of the 3D level lists with tops of degree 2 to 4.
#include "patch_kernels.hpp"

namespace pmgi {

const PatchVariant* variants_3d_low_table(size_t* count) {
  static const PatchVariant table[] = {
      make_variant<double, 3, 2, 1>(),
      make_variant<double, 3, 3, 1>(),
      make_variant<double, 3, 3, 2, 1>(),
      make_variant<double, 3, 4, 2, 1>(),
      make_variant<float, 3, 2, 1>(),
      make_variant<float, 3, 3, 1>(),
      make_variant<float, 3, 3, 2, 1>(),
      make_variant<float, 3, 4, 2, 1>()};
  *count = sizeof(table) / sizeof(table[0]);
  return table;
}

hipError_t variants_3d_low_upload() { return upload_tables(); }

}  // namespace pmgi
