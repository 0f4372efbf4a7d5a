// Kernel variants for dtype F16.
#include "chw_kernels.inc"

CHW_INST_ITEMS_4(chw::DT_F16)
CHW_INST_TINY(chw::DT_F16)
CHW_INST_HAAR(chw::DT_F16)

#if !defined(__HIP_DEVICE_COMPILE__)
namespace chw {
extern const ItemsVariant items_variants_f16[] = {CHW_ITEMS_VARIANTS_4(DT_F16)};
extern const int n_items_variants_f16 = sizeof(items_variants_f16) / sizeof(items_variants_f16[0]);
extern const TinyVariant tiny_variants_f16[] = {CHW_TINY_VARIANTS(DT_F16)};
extern const HaarVariant haar_variants_f16[] = {CHW_HAAR_VARIANTS(DT_F16)};
}  // namespace chw
#endif
