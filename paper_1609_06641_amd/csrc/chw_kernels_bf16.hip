// Kernel variants for dtype BF16.
#include "chw_kernels.inc"

CHW_INST_ITEMS_4(chw::DT_BF16)
CHW_INST_TINY(chw::DT_BF16)
CHW_INST_HAAR(chw::DT_BF16)

#if !defined(__HIP_DEVICE_COMPILE__)
namespace chw {
extern const ItemsVariant items_variants_bf16[] = {CHW_ITEMS_VARIANTS_4(DT_BF16)};
extern const int n_items_variants_bf16 = sizeof(items_variants_bf16) / sizeof(items_variants_bf16[0]);
extern const TinyVariant tiny_variants_bf16[] = {CHW_TINY_VARIANTS(DT_BF16)};
extern const HaarVariant haar_variants_bf16[] = {CHW_HAAR_VARIANTS(DT_BF16)};
}  // namespace chw
#endif
