// Patch-kernel variants of the 2D level lists (degrees 2 to 15).
#include "patch_kernels.hpp"

namespace pmgi {

const PatchVariant* variants_2d_table(size_t* count) {
  static const PatchVariant table[] = {
      make_variant<double, 2, 2, 1>(),
      make_variant<double, 2, 3, 1>(),
      make_variant<double, 2, 3, 2, 1>(),
      make_variant<double, 2, 4, 2, 1>(),
      make_variant<double, 2, 7, 3, 1>(),
      make_variant<double, 2, 15, 7, 3, 1>(),
      make_variant<float, 2, 2, 1>(),
      make_variant<float, 2, 3, 1>(),
      make_variant<float, 2, 3, 2, 1>(),
      make_variant<float, 2, 4, 2, 1>(),
      make_variant<float, 2, 7, 3, 1>(),
      make_variant<float, 2, 15, 7, 3, 1>()};
  *count = sizeof(table) / sizeof(table[0]);
  return table;
}

hipError_t variants_2d_upload() { return upload_tables(); }

}  // namespace pmgi
