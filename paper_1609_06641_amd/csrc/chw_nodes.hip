// chw_nodes.hip -- the factor-by-factor ("node") evaluation of Sec. 4.
//
// The paper proposes m - 1 processing nodes, each dedicated to the Haar
// transforms of one size, with the data streaming from node to node.  This
// file evaluates the cascade of eq. (3) that way on the GPU, as a reference
// point for the stage-grouped kernels: one launch per node, node 0 applying
// Psi_m (eq. 2) to every signal and node r (1 <= r <= m - 1) applying
//     F_r = I_{r-1} (x) diag(I_{m-r}, Psi_{m-r}),
// i.e. the Haar transform of size 2^s, s = m - r, to the upper half of every
// block of 2^{s+1} elements and passing the lower halves through.  Each node
// reads and writes the whole vector (the stream); Haar levels scale by
// fl(2^{-1/2}) one level at a time, as eq. (2) writes them.
//
// A node runs on tiles of 2^12 contiguous elements in LDS:
//   s < 12   every tile holds whole sub-vectors (the upper halves of its
//            blocks, or whole signals for node 0): all their levels run in
//            the tile, the tile is stored back in place of the stream;
//   s >= 12  a tile is either a lower-half chunk (copied) or chunk c of one
//            sub-vector: its 12 finest levels run in the tile and their
//            details go to their final positions in eq. (2)'s order
//            (level l at [2^{s-l}, 2^{s-l+1}) of the sub-vector, chunk c's
//            part at offset c 2^{12-l}); the chunk's sum goes to the sums
//            array, whose own Haar transform (s - 12 <= 12 levels, second
//            launch) gives the coarse details and the scaling coefficient,
//            which sit at positions [0, 2^{s-12}) of the sub-vector.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "chw_variants.h"

namespace chw {
namespace {

constexpr int NODE_K = 12, NODE_N = 1 << NODE_K, NODE_T = 256;
constexpr int NODE_PAIRS = NODE_N / 2 / NODE_T;  // butterfly pairs per thread per level

// Haar levels on segments of 2^s elements of an LDS tile: segment q starts
// at q * seg_stride + seg_off, nseg segments; level l turns the current sum
// block [0, 2^{s-l+1}) of each segment into sums [0, 2^{s-l}) and details
// [2^{s-l}, 2^{s-l+1}) (first minus second), both scaled by c.
__device__ void node_haar_levels(float *lds, int s, int nseg, int seg_stride, int seg_off,
                                 float c, int t)
{
    for (int l = 1; l <= s; ++l) {
        const int half = 1 << (s - l);
        const int total = nseg * half;
        float a[NODE_PAIRS], b[NODE_PAIRS];
#pragma unroll
        for (int k = 0; k < NODE_PAIRS; ++k) {
            const int i = t + NODE_T * k;
            if (i < total) {
                const int q = i >> (s - l), p = i & (half - 1);
                const float *seg = lds + q * seg_stride + seg_off;
                a[k] = seg[2 * p];
                b[k] = seg[2 * p + 1];
            }
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < NODE_PAIRS; ++k) {
            const int i = t + NODE_T * k;
            if (i < total) {
                const int q = i >> (s - l), p = i & (half - 1);
                float *seg = lds + q * seg_stride + seg_off;
                seg[p] = (a[k] + b[k]) * c;
                seg[half + p] = (a[k] - b[k]) * c;
            }
        }
        __syncthreads();
    }
}

__device__ __forceinline__ float node_c() { return (float)0.70710678118654752440; }

// One node over tiles of the stream.  `total` elements (the batch, packed
// signals of 2^m); `whole` = node 0 (the sub-vector is the whole signal).
__global__ void __launch_bounds__(NODE_T) chw_node_tile_kernel(const float *in, float *out,
                                                               float *sums, int64_t total,
                                                               int m, int s, int whole)
{
    __shared__ float lds[NODE_N];
    const int t = threadIdx.x;
    const int64_t ntiles = (total + NODE_N - 1) / NODE_N;
    const float c = node_c();
    for (int64_t T = blockIdx.x; T < ntiles; T += gridDim.x) {
        const int64_t base = T * NODE_N;
        const int nvalid = (int)(total - base < NODE_N ? total - base : NODE_N);
        for (int i = t; i < NODE_N; i += NODE_T) lds[i] = i < nvalid ? in[base + i] : 0.f;
        __syncthreads();
        if (s < NODE_K) {
            // whole sub-vectors inside the tile
            if (whole) node_haar_levels(lds, s, NODE_N >> s, 1 << s, 0, c, t);
            else node_haar_levels(lds, s, NODE_N >> (s + 1), 1 << (s + 1), 1 << s, c, t);
            for (int i = t; i < nvalid; i += NODE_T) out[base + i] = lds[i];
        } else {
            const int64_t sig = base >> m;
            const int64_t pos = base & ((int64_t(1) << m) - 1);
            bool upper = true;
            int64_t sub_base, sub_id, chunk;
            if (whole) {
                sub_base = sig << m;
                sub_id = sig;
                chunk = pos >> NODE_K;
            } else {
                upper = ((pos >> s) & 1) != 0;
                const int64_t b = pos >> (s + 1);
                sub_base = (sig << m) + ((2 * b + 1) << s);
                sub_id = (sig << (m - s - 1)) + b;
                chunk = (pos & ((int64_t(1) << s) - 1)) >> NODE_K;
            }
            if (!upper) {
                for (int i = t; i < NODE_N; i += NODE_T) out[base + i] = lds[i];
            } else {
                node_haar_levels(lds, NODE_K, 1, 0, 0, c, t);
                // details of level l = 12 - h at LDS [2^h, 2^{h+1})
                for (int k = t; k < NODE_N; k += NODE_T) {
                    if (k == 0) continue;
                    const int h = 31 - __builtin_clz((unsigned)k);
                    const int64_t dst = sub_base + (int64_t(1) << (s - NODE_K + h)) +
                                        (chunk << h) + (k - (1 << h));
                    out[dst] = lds[k];
                }
                if (t == 0) {
                    if (s == NODE_K) out[sub_base] = lds[0];
                    else sums[(sub_id << (s - NODE_K)) + chunk] = lds[0];
                }
            }
        }
        __syncthreads();
    }
}

// The sums of every sub-vector of a node with s > 12: Psi_{s-12} of each
// sub-vector's 2^{s-12} chunk sums, stored at [0, 2^{s-12}) of the sub-vector.
__global__ void __launch_bounds__(NODE_T) chw_node_sums_kernel(const float *sums, float *out,
                                                               int64_t nsub, int m, int s,
                                                               int whole)
{
    __shared__ float lds[NODE_N];
    const int t = threadIdx.x;
    const int ls = s - NODE_K;                 // log2 sums per sub-vector (1..12)
    const int64_t nsums = nsub << ls;
    const int64_t ntiles = (nsums + NODE_N - 1) / NODE_N;
    const float c = node_c();
    for (int64_t T = blockIdx.x; T < ntiles; T += gridDim.x) {
        const int64_t base = T * NODE_N;
        const int nvalid = (int)(nsums - base < NODE_N ? nsums - base : NODE_N);
        for (int i = t; i < NODE_N; i += NODE_T) lds[i] = i < nvalid ? sums[base + i] : 0.f;
        __syncthreads();
        node_haar_levels(lds, ls, NODE_N >> ls, 1 << ls, 0, c, t);
        for (int i = t; i < nvalid; i += NODE_T) {
            const int64_t e = base + i;
            const int64_t sub = e >> ls;
            const int64_t j = e & ((int64_t(1) << ls) - 1);
            int64_t sub_base;
            if (whole) {
                sub_base = sub << m;
            } else {
                const int64_t sig = sub >> (m - s - 1);
                const int64_t b = sub & ((int64_t(1) << (m - s - 1)) - 1);
                sub_base = (sig << m) + ((2 * b + 1) << s);
            }
            out[sub_base + j] = lds[i];
        }
        __syncthreads();
    }
}

unsigned node_grid(int64_t ntiles, int cus)
{
    const int64_t cap = (int64_t)(cus > 0 ? cus : 256) * 32;
    return (unsigned)(ntiles < cap ? ntiles : cap);
}

}  // namespace

hipError_t launch_node(const float *in, float *out, float *sums, int64_t batch, int m, int r,
                       int cus, hipStream_t st)
{
    const int s = r == 0 ? m : m - r;
    const int whole = r == 0 ? 1 : 0;
    const int64_t total = batch << m;
    if (total <= 0) return hipSuccess;
    const int64_t ntiles = (total + NODE_N - 1) / NODE_N;
    hipLaunchKernelGGL(chw_node_tile_kernel, dim3(node_grid(ntiles, cus)), dim3(NODE_T), 0, st,
                       in, out, sums, total, m, s, whole);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || s <= NODE_K) return e;
    const int64_t nsub = whole ? batch : batch << (m - s - 1);
    const int64_t nsums = nsub << (s - NODE_K);
    hipLaunchKernelGGL(chw_node_sums_kernel, dim3(node_grid((nsums + NODE_N - 1) / NODE_N, cus)),
                       dim3(NODE_T), 0, st, sums, out, nsub, m, s, whole);
    return hipGetLastError();
}

}  // namespace chw
