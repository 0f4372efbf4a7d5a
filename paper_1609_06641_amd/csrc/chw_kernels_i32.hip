// Kernel variants for dtype I32.
#include "chw_kernels.inc"

CHW_INST_ITEMS_4(chw::DT_I32)
CHW_INST_TINY(chw::DT_I32)
CHW_INST_HAAR(chw::DT_I32)

#if !defined(__HIP_DEVICE_COMPILE__)
namespace chw {
extern const ItemsVariant items_variants_i32[] = {CHW_ITEMS_VARIANTS_4(DT_I32)};
extern const int n_items_variants_i32 = sizeof(items_variants_i32) / sizeof(items_variants_i32[0]);
extern const TinyVariant tiny_variants_i32[] = {CHW_TINY_VARIANTS(DT_I32)};
extern const HaarVariant haar_variants_i32[] = {CHW_HAAR_VARIANTS(DT_I32)};
}  // namespace chw
#endif
