// Kernel variants for dtype F32.
#include "chw_kernels.inc"

CHW_INST_ITEMS_4(chw::DT_F32)
CHW_INST_TINY(chw::DT_F32)
CHW_INST_HAAR(chw::DT_F32)

#if !defined(__HIP_DEVICE_COMPILE__)
namespace chw {
extern const ItemsVariant items_variants_f32[] = {CHW_ITEMS_VARIANTS_4(DT_F32)};
extern const int n_items_variants_f32 = sizeof(items_variants_f32) / sizeof(items_variants_f32[0]);
extern const TinyVariant tiny_variants_f32[] = {CHW_TINY_VARIANTS(DT_F32)};
extern const HaarVariant haar_variants_f32[] = {CHW_HAAR_VARIANTS(DT_F32)};
}  // namespace chw
#endif
