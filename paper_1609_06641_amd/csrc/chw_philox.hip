// chw_philox.hip -- random-sign words from a counter-based generator.
//
// Philox4x64-10 (J. Salmon, M. Moraes, R. Dror, D. Shaw, "Parallel random
// numbers: as easy as 1, 2, 3", SC 2011): a 256-bit counter block
// (c0, c1, c2, c3) and a 128-bit key (k0, k1) go through ten rounds of
//     (c0, c1, c2, c3) <- (hi(M1 c2) ^ c1 ^ k0, lo(M1 c2), hi(M0 c0) ^ c3 ^ k1, lo(M0 c0))
// with 64 x 64 -> 128-bit products, the key bumped by the Weyl constants
// (W0, W1) after every round.  Every counter gives an independent block, so
// each thread makes its own words with no state shared between threads.
//
// Word w of round r is 32-bit word (w mod 8) of the block with counter
// (floor(w / 8), r, 0, 0) and key (seed, 0); block outputs o_0..o_3 give
// words 2i = low half of o_i and 2i + 1 = high half.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "chw_variants.h"

namespace chw {
namespace {

constexpr uint64_t PHILOX_M0 = 0xD2E7470EE14C6C93ull;
constexpr uint64_t PHILOX_M1 = 0xCA5A826395121157ull;
constexpr uint64_t PHILOX_W0 = 0x9E3779B97F4A7C15ull;
constexpr uint64_t PHILOX_W1 = 0xBB67AE8584CAA73Bull;

__device__ __forceinline__ void philox4x64_10(uint64_t c[4], uint64_t k0, uint64_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t hi0 = __umul64hi(PHILOX_M0, c[0]), lo0 = PHILOX_M0 * c[0];
        const uint64_t hi1 = __umul64hi(PHILOX_M1, c[2]), lo1 = PHILOX_M1 * c[2];
        c[0] = hi1 ^ c[1] ^ k0;
        c[1] = lo1;
        c[2] = hi0 ^ c[3] ^ k1;
        c[3] = lo0;
        k0 += PHILOX_W0;
        k1 += PHILOX_W1;
    }
}

// One thread per (round, block of 8 words); grid-stride over all of them.
__global__ void __launch_bounds__(256) chw_philox_kernel(uint32_t *out, int64_t words,
                                                         int64_t blocks, int64_t total,
                                                         uint64_t seed)
{
    for (int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; b < total;
         b += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r = b / blocks, g = b - r * blocks;
        uint64_t c[4] = {(uint64_t)g, (uint64_t)r, 0, 0};
        philox4x64_10(c, seed, 0);
        uint32_t w[8];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            w[2 * i] = (uint32_t)c[i];
            w[2 * i + 1] = (uint32_t)(c[i] >> 32);
        }
        uint32_t *dst = out + r * words + g * 8;
        const int64_t n = words - g * 8;  // words of this block inside the round
        if (n >= 8 && (reinterpret_cast<uintptr_t>(dst) & 15u) == 0) {
            uint4 *d4 = reinterpret_cast<uint4 *>(dst);
            d4[0] = make_uint4(w[0], w[1], w[2], w[3]);
            d4[1] = make_uint4(w[4], w[5], w[6], w[7]);
        } else {
#pragma unroll
            for (int i = 0; i < 8; ++i)
                if (i < n) dst[i] = w[i];
        }
    }
}

}  // namespace

hipError_t launch_philox_signs(uint32_t *out, int64_t words, int rounds, uint64_t seed,
                               int cus, hipStream_t s)
{
    const int64_t blocks = (words + 7) / 8;
    const int64_t total = blocks * rounds;
    if (total <= 0) return hipSuccess;
    const int64_t want = (total + 255) / 256;
    const int64_t cap = (int64_t)(cus > 0 ? cus : 256) * 16;
    const unsigned grid = (unsigned)(want < cap ? want : cap);
    hipLaunchKernelGGL(chw_philox_kernel, dim3(grid), dim3(256), 0, s, out, words, blocks, total,
                       seed);
    return hipGetLastError();
}

}  // namespace chw
