// chw_variants.h -- registry of compiled kernel variants (host side).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "chw_types.h"

namespace chw {

typedef hipError_t (*ItemsLauncher)(dim3 grid, hipStream_t s, const LaunchArgs &a);
typedef hipError_t (*TinyLauncher)(dim3 grid, dim3 block, hipStream_t s, const void *in,
                                   void *out, const int64_t *offs, const int32_t *ms,
                                   int n, int ortho, const uint32_t *signs, int sign_shared,
                                   int rounds, int64_t sign_words, int order);

// One compiled tile kernel: dtype, tile bits K, register bits LR, the two
// first-pass row counts (log2) CA and CB, direction.
struct ItemsVariant {
    int dt, K, LR, CA, CB, adj;
    int nt;                 // threads per workgroup
    size_t lds_bytes;       // static LDS
    ItemsLauncher launch;
    const void *fn;         // kernel symbol (occupancy queries)
    ItemsLauncher launch_persistent;  // persistent form (K = 12 only), or null
    const void *fn_persistent;
    ItemsLauncher launch_stream[kNumStreamSlots];  // prefetching form for items
    const void *fn_stream[kNumStreamSlots];        // of each kind, by stream_slot()
    ItemsLauncher launch_order[2];    // one workgroup per item, sequency and
                                      // natural coefficient order
    ItemsLauncher launch_stream_order[2][kNumStreamSlots];  // forward prefetching forms of
    const void *fn_stream_order[2][kNumStreamSlots];        // those orders (K = 15), by slot
    ItemsLauncher launch_turn;        // KIND_TURN items (K = 15), one workgroup
                                      // per item (forward or adjoint boundary)
    ItemsLauncher launch_turn_stream; // prefetching form (forward)
    const void *fn_turn_stream;
    ItemsLauncher launch_turn_adj_stream[4];  // prefetching adjoint form per
    const void *fn_turn_adj_stream[4];        // row count: 2^CA, 2^CM, 2^CB, 2^CD
    ItemsLauncher launch_last_signed; // forward last-pass tiles with a diagonal
                                      // at the store, one workgroup per tile
};

struct TinyVariant {
    int dt, adj;
    TinyLauncher launch;
};

// Haar pyramid tiles (2^12 elements, 2^5 registers per thread).
struct HaarVariant {
    int dt, adj;
    ItemsLauncher launch;
};

// All variants of all dtypes.
const ItemsVariant *items_variants(int *count);
const TinyVariant *tiny_variants(int *count);
const ItemsVariant *find_items_variant(int dt, int K, int LR, int adj);
const TinyVariant *find_tiny_variant(int dt, int adj);
const HaarVariant *find_haar_variant(int dt, int adj);

// Fills rounds x words sign words from Philox4x64-10 (chw_philox.hip):
// word w of round r at out[r * words + w].
hipError_t launch_philox_signs(uint32_t *out, int64_t words, int rounds, uint64_t seed,
                               int cus, hipStream_t s);

// One node of the factor-by-factor evaluation (chw_nodes.hip): factor r of
// eq. (3) (r = 0: Psi_m) on `batch` packed FP32 signals of 2^m, in -> out;
// `sums` holds batch * 2^{m-12} floats when m > 12.
hipError_t launch_node(const float *in, float *out, float *sums, int64_t batch, int m, int r,
                       int cus, hipStream_t st);

// Largest log2 size a tiny (one thread per signal) launch handles.
constexpr int TINY_MAX_LOG2 = 3;


}  // namespace chw
