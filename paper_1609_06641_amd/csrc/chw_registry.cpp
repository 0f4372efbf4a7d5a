// chw_registry.cpp -- merges the per-dtype kernel variant tables.
#include <vector>

#include <hip/hip_runtime.h>

#include "chw_variants.h"

namespace chw {

extern const ItemsVariant items_variants_f32[], items_variants_bf16[], items_variants_f16[],
    items_variants_i32[], items_variants_f64[];
extern const int n_items_variants_f32, n_items_variants_bf16, n_items_variants_f16,
    n_items_variants_i32, n_items_variants_f64;
extern const TinyVariant tiny_variants_f32[], tiny_variants_bf16[], tiny_variants_f16[],
    tiny_variants_i32[], tiny_variants_f64[];
extern const HaarVariant haar_variants_f32[], haar_variants_bf16[], haar_variants_f16[],
    haar_variants_i32[], haar_variants_f64[];

namespace {
struct Registry {
    std::vector<ItemsVariant> items;
    std::vector<TinyVariant> tiny;
    std::vector<HaarVariant> haar;
    Registry()
    {
        const ItemsVariant *tabs[] = {items_variants_f32, items_variants_bf16, items_variants_f16,
                                      items_variants_i32, items_variants_f64};
        const int ns[] = {n_items_variants_f32, n_items_variants_bf16, n_items_variants_f16,
                          n_items_variants_i32, n_items_variants_f64};
        for (int d = 0; d < 5; ++d)
            for (int i = 0; i < ns[d]; ++i) items.push_back(tabs[d][i]);
        const TinyVariant *tt[] = {tiny_variants_f32, tiny_variants_bf16, tiny_variants_f16,
                                   tiny_variants_i32, tiny_variants_f64};
        for (int d = 0; d < 5; ++d)
            for (int i = 0; i < 2; ++i) tiny.push_back(tt[d][i]);
        const HaarVariant *hv[] = {haar_variants_f32, haar_variants_bf16, haar_variants_f16,
                                   haar_variants_i32, haar_variants_f64};
        for (int d = 0; d < 5; ++d)
            for (int i = 0; i < 2; ++i) haar.push_back(hv[d][i]);
    }
};
const Registry &reg()
{
    static Registry r;
    return r;
}
}  // namespace

const ItemsVariant *items_variants(int *count)
{
    *count = (int)reg().items.size();
    return reg().items.data();
}

const TinyVariant *tiny_variants(int *count)
{
    *count = (int)reg().tiny.size();
    return reg().tiny.data();
}

const ItemsVariant *find_items_variant(int dt, int K, int LR, int adj)
{
    for (const ItemsVariant &v : reg().items)
        if (v.dt == dt && v.K == K && v.LR == LR && v.adj == adj) return &v;
    return nullptr;
}

const HaarVariant *find_haar_variant(int dt, int adj)
{
    for (const HaarVariant &v : reg().haar)
        if (v.dt == dt && v.adj == adj) return &v;
    return nullptr;
}

const TinyVariant *find_tiny_variant(int dt, int adj)
{
    for (const TinyVariant &v : reg().tiny)
        if (v.dt == dt && v.adj == adj) return &v;
    return nullptr;
}

}  // namespace chw
