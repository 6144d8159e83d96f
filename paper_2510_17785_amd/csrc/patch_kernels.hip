// Registry of the patch-kernel variants (one table per patch_variants_*.hip
// file), the feature kernel of the bound-predicting network, the constant
// tables of every file and the device work array of the allocation-free
// patch CG.
#include "patch_kernels.hpp"

namespace pmgi {

namespace {

const VariantPart kParts[] = {
    {variants_2d_table, variants_2d_upload},       {variants_3d_low_table, variants_3d_low_upload},
    {variants_3d_q6_table, variants_3d_q6_upload}, {variants_3d_q7_table, variants_3d_q7_upload},
    {variants_3d_q8_table, variants_3d_q8_upload},
};

const PatchVariant* registry(size_t* count) {
  static const std::vector<PatchVariant> all = [] {
    std::vector<PatchVariant> v;
    for (const VariantPart& p : kParts) {
      size_t n = 0;
      const PatchVariant* t = p.table(&n);
      v.insert(v.end(), t, t + n);
    }
    return v;
  }();
  *count = all.size();
  return all.data();
}

}  // namespace

hipError_t launch_features(int dim, const PatchArgs& a, int n_patch, float* out, hipStream_t s) {
  if (n_patch <= 0) return hipSuccess;
  (void)hipGetLastError();
  if (dim == 3)
    hipLaunchKernelGGL(feature_kernel<3>, dim3(n_patch), dim3(64), 0, s, a, out);
  else
    hipLaunchKernelGGL(feature_kernel<2>, dim3(n_patch), dim3(64), 0, s, a, out);
  return hipGetLastError();
}

// Device work memory of pmg_patch_pcg_noalloc (the residual and search
// direction of every patch of the call), one array per GPU, held until the
// process ends.  Host code never uses the name `scratch` as an address: the
// device address comes from hipGetSymbolAddress, once per device.
constexpr size_t kPcgScratchDoubles = PMG_PCG_SCRATCH_BYTES / sizeof(double);
static __device__ __align__(256) double scratch[kPcgScratchDoubles];

hipError_t pcg_scratch(double** ptr, size_t* bytes) {
  constexpr int kMaxDevices = 64;
  static std::mutex mu;
  static double* addr[kMaxDevices] = {nullptr};
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(mu);
  if (!addr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    addr[dev] = static_cast<double*>(p);
  }
  *ptr = addr[dev];
  *bytes = kPcgScratchDoubles * sizeof(double);
  return hipSuccess;
}

hipError_t init_constant_tables() {
  hipError_t e = upload_tables();  // this file's copy
  for (const VariantPart& p : kParts)
    if (e == hipSuccess) e = p.upload();
  return e;
}

const PatchVariant* find_variant(int precision, int dim, int n_levels, const int* levels) {
  size_t n = 0;
  const PatchVariant* t = registry(&n);
  for (size_t i = 0; i < n; ++i) {
    if (t[i].precision != precision || t[i].dim != dim || t[i].n_levels != n_levels) continue;
    bool same = true;
    for (int l = 0; l < n_levels; ++l) same = same && t[i].levels[l] == levels[l];
    if (same) return &t[i];
  }
  return nullptr;
}

std::string list_variants() {
  size_t n = 0;
  const PatchVariant* t = registry(&n);
  std::string s;
  for (size_t i = 0; i < n; ++i) {
    if (t[i].precision == PMG_FP32) continue;  // same level lists as FP64
    if (t[i].precision == PMG_BF16X3_FP32ACC) continue;  // same level lists as BF16
    s += t[i].precision == PMG_BF16_FP32ACC ? "bf16 " : "";
    s += std::to_string(t[i].dim) + "D:";
    for (int l = 0; l < t[i].n_levels; ++l) s += (l ? "," : "") + std::to_string(t[i].levels[l]);
    s += " ";
  }
  return s;
}

}  // namespace pmgi
