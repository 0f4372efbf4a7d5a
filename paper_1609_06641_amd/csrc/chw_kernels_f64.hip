// Kernel variants for dtype F64 (verification and gradient checks): K = 12
// tiles only (a 2^12 FP64 tile is 33 KiB of LDS).
#include "chw_kernels.inc"

CHW_INST_ITEMS(chw::DT_F64, 12, 5, CHW_K12_CA, 3)
template __global__ void chw::chw_last_signed_kernel<chw::DT_F64, 12, 5, CHW_K12_CA, 3>(chw::LaunchArgs);
CHW_INST_PERSIST(chw::DT_F64, 5)
CHW_INST_TINY(chw::DT_F64)
CHW_INST_HAAR(chw::DT_F64)

#if !defined(__HIP_DEVICE_COMPILE__)
namespace chw {
extern const ItemsVariant items_variants_f64[] = {
    make_items_variant<DT_F64, 12, 5, CHW_K12_CA, 3, false>(),
    make_items_variant<DT_F64, 12, 5, CHW_K12_CA, 3, true>(),
};
extern const int n_items_variants_f64 = sizeof(items_variants_f64) / sizeof(items_variants_f64[0]);
extern const TinyVariant tiny_variants_f64[] = {CHW_TINY_VARIANTS(DT_F64)};
extern const HaarVariant haar_variants_f64[] = {CHW_HAAR_VARIANTS(DT_F64)};
}  // namespace chw
#endif
