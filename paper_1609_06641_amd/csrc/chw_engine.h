// chw_engine.h -- device tile engine of the CHW cascade for gfx950.
//
// One workgroup transforms one tile of 2^K elements staged in LDS:
//   1. a load phase streams 16-byte global vectors into LDS (widening BF16 /
//      FP16 to FP32 exactly),
//   2. register rounds apply the cascade's stages LR at a time: each thread
//      reads R = 2^LR elements that differ in the round's active bits, runs
//      the sum/difference butterflies of those stages in registers, and writes
//      them back,
//   3. a store phase streams the result out with 16-byte vectors, in the
//      dyadic (Paley) order of eq. (1) for a final pass, or in the cascade's
//      own layout after L1 stages for a first HBM pass.
//
// Butterflies are unnormalized (a+b, a-b); the orthonormal factor 2^{-m/2}
// (the product of the 1/sqrt(2) of every level of eqs. (1)-(2)) is applied
// once, at the final store, as an exact power of two times fl(1/sqrt(2)) for
// odd m.  The numbers therefore do not depend on the tiling or the pass split.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "chw_layout.h"
#include "chw_types.h"

namespace chw {

// ---------------------------------------------------------------------------
// element types and 16-byte vector I/O

struct bf16s { uint16_t v; };
struct f16s { uint16_t v; };

template <int DT> struct Types;
template <> struct Types<DT_F32>  { using S = float;    using C = float; };
template <> struct Types<DT_BF16> { using S = bf16s;    using C = float; };
template <> struct Types<DT_F16>  { using S = f16s;     using C = float; };
template <> struct Types<DT_I32>  { using S = uint32_t; using C = uint32_t; };
template <> struct Types<DT_F64>  { using S = double;   using C = double; };

typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef _Float16 f16x2 __attribute__((ext_vector_type(2)));

template <typename T> struct Vec;

template <> struct Vec<float> {
    static constexpr int V = 4;
    static __device__ __forceinline__ void load(const float *p, float *o)
    {
        float4 q = *reinterpret_cast<const float4 *>(p);
        o[0] = q.x; o[1] = q.y; o[2] = q.z; o[3] = q.w;
    }
    static __device__ __forceinline__ void store(float *p, const float *v)
    {
        *reinterpret_cast<float4 *>(p) = make_float4(v[0], v[1], v[2], v[3]);
    }
};

template <> struct Vec<uint32_t> {
    static constexpr int V = 4;
    static __device__ __forceinline__ void load(const uint32_t *p, uint32_t *o)
    {
        uint4 q = *reinterpret_cast<const uint4 *>(p);
        o[0] = q.x; o[1] = q.y; o[2] = q.z; o[3] = q.w;
    }
    static __device__ __forceinline__ void store(uint32_t *p, const uint32_t *v)
    {
        *reinterpret_cast<uint4 *>(p) = make_uint4(v[0], v[1], v[2], v[3]);
    }
};

template <> struct Vec<double> {
    static constexpr int V = 2;
    static __device__ __forceinline__ void load(const double *p, double *o)
    {
        double2 q = *reinterpret_cast<const double2 *>(p);
        o[0] = q.x; o[1] = q.y;
    }
    static __device__ __forceinline__ void store(double *p, const double *v)
    {
        *reinterpret_cast<double2 *>(p) = make_double2(v[0], v[1]);
    }
};

// bfloat16: widening is exact (the 16 bits are the top half of an FP32);
// narrowing rounds to nearest even (v_cvt_pk_bf16_f32).
template <> struct Vec<bf16s> {
    static constexpr int V = 8;
    static __device__ __forceinline__ void load(const bf16s *p, float *o)
    {
        uint4 q = *reinterpret_cast<const uint4 *>(p);
        uint32_t w[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            o[2 * i] = __uint_as_float(w[i] << 16);
            o[2 * i + 1] = __uint_as_float(w[i] & 0xffff0000u);
        }
    }
    static __device__ __forceinline__ void store(bf16s *p, const float *v)
    {
        uint32_t w[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            f32x2 f = {v[2 * i], v[2 * i + 1]};
            bf16x2 h = __builtin_convertvector(f, bf16x2);
            w[i] = __builtin_bit_cast(uint32_t, h);
        }
        *reinterpret_cast<uint4 *>(p) = make_uint4(w[0], w[1], w[2], w[3]);
    }
};

// float16: widening is exact; narrowing rounds to nearest even.
template <> struct Vec<f16s> {
    static constexpr int V = 8;
    static __device__ __forceinline__ void load(const f16s *p, float *o)
    {
        uint4 q = *reinterpret_cast<const uint4 *>(p);
        uint32_t w[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            f16x2 h = __builtin_bit_cast(f16x2, w[i]);
            o[2 * i] = (float)h.x;
            o[2 * i + 1] = (float)h.y;
        }
    }
    static __device__ __forceinline__ void store(f16s *p, const float *v)
    {
        uint32_t w[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            f32x2 f = {v[2 * i], v[2 * i + 1]};
            f16x2 h = __builtin_convertvector(f, f16x2);
            w[i] = __builtin_bit_cast(uint32_t, h);
        }
        *reinterpret_cast<uint4 *>(p) = make_uint4(w[0], w[1], w[2], w[3]);
    }
};

// Orthonormal factor 2^{-m/2}: exact power of two, times fl(2^{-1/2}) when m
// is odd.
template <typename C> __device__ __forceinline__ C ortho_scale(int m);
template <> __device__ __forceinline__ float ortho_scale<float>(int m)
{
    return ldexpf((m & 1) ? 0.70710678118654752440f : 1.0f, -(m >> 1));
}
template <> __device__ __forceinline__ double ortho_scale<double>(int m)
{
    return ldexp((m & 1) ? 0.70710678118654752440 : 1.0, -(m >> 1));
}
template <> __device__ __forceinline__ uint32_t ortho_scale<uint32_t>(int)
{
    return 1u;
}

template <typename C> __device__ __forceinline__ C scale_mul(C v, C s) { return v * s; }
template <> __device__ __forceinline__ uint32_t scale_mul<uint32_t>(uint32_t v, uint32_t) { return v; }

// ---------------------------------------------------------------------------
// the engine

template <int DT, int K, int LR, int CA, int CB>
struct Engine {
    using L = Layout<K, LR>;
    using S = typename Types<DT>::S;
    using C = typename Types<DT>::C;
    static constexpr int N = L::N, NT = L::NT, R = L::R, J = L::J;
    static_assert(CA >= 2 && CB >= 2 && CA < K && CB < K, "first-pass row counts");

    // ---- butterflies -------------------------------------------------------
    // One stage on register bit rb: v[i] (bit clear) and v[i | 1 << rb]
    // become their sum and difference (Haar pair: first + second, first -
    // second).
    static __device__ __forceinline__ void bfly(C *v, int rb)
    {
#pragma unroll
        for (int i = 0; i < R; ++i) {
            if (!(i & (1 << rb))) {
                C a = v[i], b = v[i | (1 << rb)];
                v[i] = a + b;
                v[i | (1 << rb)] = a - b;
            }
        }
    }

    template <int j, bool ADJ>
    static __device__ __forceinline__ void round(C *lds, int nst, int t)
    {
        constexpr int lo = L::flo(j), a0 = L::alo(j), a1 = L::ahi(j);
        if (a0 >= nst) return;  // no active stage in this round (uniform)
        C *base = lds + L::pad(L::round_tbase(j, t));
        C v[R];
#pragma unroll
        for (int i = 0; i < R; ++i) v[i] = base[L::pad(L::round_reg(j, i))];
        if constexpr (!ADJ) {
#pragma unroll
            for (int bit = a0; bit < a1; ++bit)
                if (bit < nst) bfly(v, bit - lo);
        } else {
#pragma unroll
            for (int bit = a1 - 1; bit >= a0; --bit)
                if (bit < nst) bfly(v, bit - lo);
        }
#pragma unroll
        for (int i = 0; i < R; ++i) base[L::pad(L::round_reg(j, i))] = v[i];
        __syncthreads();
    }

    template <bool ADJ, int j = 0>
    static __device__ __forceinline__ void rounds(C *lds, int nst, int t)
    {
        if constexpr (j < J) {
            if constexpr (!ADJ) {
                round<j, false>(lds, nst, t);
                rounds<false, j + 1>(lds, nst, t);
            } else {
                round<J - 1 - j, true>(lds, nst, t);
                rounds<true, j + 1>(lds, nst, t);
            }
        }
    }

    // ---- contiguous phases ---------------------------------------------------
    // Tile element e <-> memory element (block e >> bits at its base) + (e &
    // (2^bits - 1)).  Blocks are consecutive from `off` unless `list` gives
    // their bases.  Only the first `count` blocks exist.
    template <typename T>
    static __device__ __forceinline__ void load_contig(C *lds, const T *src, int64_t off,
                                                       int bits, int count,
                                                       const int64_t *list, int t)
    {
        constexpr int V = Vec<T>::V, NV = N / (V * NT);
        static_assert(NV >= 1, "tile too small for the vector width");
        C *lb = lds + L::pad(V * t);
        const bool full = (list == nullptr) && ((count << bits) >= N);
        C vals[NV][V];
        if (full) {
            const T *s = src + off + V * t;
#pragma unroll
            for (int k = 0; k < NV; ++k) Vec<T>::load(s + V * NT * k, vals[k]);
#pragma unroll
            for (int k = 0; k < NV; ++k)
#pragma unroll
                for (int u = 0; u < V; ++u) lb[L::pad(V * NT * k) + u] = vals[k][u];
        } else {
            const int mask = (1 << bits) - 1;
#pragma unroll
            for (int k = 0; k < NV; ++k) {
                const int e0 = V * t + V * NT * k;
                const int blk = e0 >> bits;
                if (blk < count) {
                    const int64_t g = list ? list[blk] + (e0 & mask) : off + e0;
                    Vec<T>::load(src + g, vals[k]);
#pragma unroll
                    for (int u = 0; u < V; ++u) lb[L::pad(V * NT * k) + u] = vals[k][u];
                }
            }
        }
    }

    template <typename T>
    static __device__ __forceinline__ void store_contig(const C *lds, T *dst, int64_t off,
                                                        int bits, int count,
                                                        const int64_t *list, int t,
                                                        C scale, bool do_scale)
    {
        constexpr int V = Vec<T>::V, NV = N / (V * NT);
        const C *lb = lds + L::pad(V * t);
        const bool full = (list == nullptr) && ((count << bits) >= N);
        const int mask = (1 << bits) - 1;
#pragma unroll
        for (int k = 0; k < NV; ++k) {
            const int e0 = V * t + V * NT * k;
            const int blk = e0 >> bits;
            if (full || blk < count) {
                C vals[V];
#pragma unroll
                for (int u = 0; u < V; ++u) {
                    vals[u] = lb[L::pad(V * NT * k) + u];
                    if (do_scale) vals[u] = scale_mul(vals[u], scale);
                }
                const int64_t g = (!full && list) ? list[blk] + (e0 & mask) : off + e0;
                Vec<T>::store(dst + g, vals);
            }
        }
    }

    // ---- Paley-order phases --------------------------------------------------
    // Memory position (blk << bits) | p holds tile element (blk << bits) |
    // bitrev_bits(p): the dyadic order of eq. (1) is the natural radix-2 order
    // read at bit-reversed positions.
    template <typename T>
    static __device__ __forceinline__ void store_paley(const C *lds, T *dst, int64_t off,
                                                       int bits, int count,
                                                       const int64_t *list, int t,
                                                       C scale, bool do_scale)
    {
        constexpr int V = Vec<T>::V, NV = N / (V * NT);
        if (bits == K) {
            const C *lb = lds + L::pad((int)rbrev((uint32_t)(V * t), K));
            T *d = dst + (list ? list[0] : off) + V * t;
#pragma unroll
            for (int k = 0; k < NV; ++k) {
                C vals[V];
#pragma unroll
                for (int u = 0; u < V; ++u) {
                    vals[u] = lb[L::pad((int)cbrev((uint32_t)(V * NT * k + u), K))];
                    if (do_scale) vals[u] = scale_mul(vals[u], scale);
                }
                Vec<T>::store(d + V * NT * k, vals);
            }
        } else {
            const int mask = (1 << bits) - 1;
#pragma unroll
            for (int k = 0; k < NV; ++k) {
                const int o0 = V * t + V * NT * k;
                const int blk = o0 >> bits;
                if (blk < count) {
                    const int p0 = o0 & mask;
                    C vals[V];
#pragma unroll
                    for (int u = 0; u < V; ++u) {
                        const int e = (blk << bits) | (int)rbrev((uint32_t)(p0 + u), bits);
                        vals[u] = lds[L::pad(e)];
                        if (do_scale) vals[u] = scale_mul(vals[u], scale);
                    }
                    const int64_t g = list ? list[blk] + p0 : off + o0;
                    Vec<T>::store(dst + g, vals);
                }
            }
        }
    }

    template <typename T>
    static __device__ __forceinline__ void load_paley(C *lds, const T *src, int64_t off,
                                                      int bits, int count,
                                                      const int64_t *list, int t)
    {
        constexpr int V = Vec<T>::V, NV = N / (V * NT);
        C vals[NV][V];
        if (bits == K) {
            C *lb = lds + L::pad((int)rbrev((uint32_t)(V * t), K));
            const T *s = src + (list ? list[0] : off) + V * t;
#pragma unroll
            for (int k = 0; k < NV; ++k) Vec<T>::load(s + V * NT * k, vals[k]);
#pragma unroll
            for (int k = 0; k < NV; ++k)
#pragma unroll
                for (int u = 0; u < V; ++u)
                    lb[L::pad((int)cbrev((uint32_t)(V * NT * k + u), K))] = vals[k][u];
        } else {
            const int mask = (1 << bits) - 1;
#pragma unroll
            for (int k = 0; k < NV; ++k) {
                const int o0 = V * t + V * NT * k;
                const int blk = o0 >> bits;
                if (blk < count) {
                    const int p0 = o0 & mask;
                    const int64_t g = list ? list[blk] + p0 : off + o0;
                    Vec<T>::load(src + g, vals[k]);
#pragma unroll
                    for (int u = 0; u < V; ++u) {
                        const int e = (blk << bits) | (int)rbrev((uint32_t)(p0 + u), bits);
                        lds[L::pad(e)] = vals[k][u];
                    }
                }
            }
        }
    }

    // ---- transposed phases of a first-pass tile -------------------------------
    // Tile = 2^CC rows of 2^L1 (L1 = K - CC) contiguous elements; element e =
    // (hl << L1) | lo of row h0 + hl sits, after stages 0..L1-1, at position
    // bitrev_L1(lo) * 2^rs + h0 + hl of the signal in the cascade's layout
    // (runs of 2^CC consecutive rows).
    template <int CC>
    static __device__ __forceinline__ void store_transp(const C *lds, C *dst, int64_t base,
                                                        int h0, int rs, int t)
    {
        constexpr int V = Vec<C>::V, NV = N / (V * NT);
        static_assert(V <= (1 << CC), "a vector must stay inside one run");
        const C *lb = lds + L::pad(L::template transp_e<V, CC>(t, 0, 0));
        C *d = dst + base + h0 + L::template transp_goff<CC>(V * t, rs);
#pragma unroll
        for (int k = 0; k < NV; ++k) {
            C vals[V];
#pragma unroll
            for (int u = 0; u < V; ++u)
                vals[u] = lb[L::pad(L::template transp_e<V, CC>(0, k, u))];
            Vec<C>::store(d + L::template transp_goff<CC>(V * NT * k, rs), vals);
        }
    }

    template <int CC>
    static __device__ __forceinline__ void load_transp(C *lds, const C *src, int64_t base,
                                                       int h0, int rs, int t)
    {
        constexpr int V = Vec<C>::V, NV = N / (V * NT);
        static_assert(V <= (1 << CC), "a vector must stay inside one run");
        C *lb = lds + L::pad(L::template transp_e<V, CC>(t, 0, 0));
        const C *s = src + base + h0 + L::template transp_goff<CC>(V * t, rs);
        C vals[NV][V];
#pragma unroll
        for (int k = 0; k < NV; ++k)
            Vec<C>::load(s + L::template transp_goff<CC>(V * NT * k, rs), vals[k]);
#pragma unroll
        for (int k = 0; k < NV; ++k)
#pragma unroll
            for (int u = 0; u < V; ++u)
                lb[L::pad(L::template transp_e<V, CC>(0, k, u))] = vals[k][u];
    }

    // ---- one work item -------------------------------------------------------
    template <int CC, bool ADJ>
    static __device__ __forceinline__ void first_item(const Item &it, const LaunchArgs &a,
                                                      C *lds, int t)
    {
        constexpr int L1 = K - CC;
        C *inter = static_cast<C *>(a.inter);
        const int64_t base = a.inter_is_io ? it.io_off - ((int64_t)it.h0 << L1) : it.ws_off;
        if constexpr (!ADJ) {
            load_contig<S>(lds, static_cast<const S *>(a.in), it.io_off, K, 1, nullptr, t);
            __syncthreads();
            rounds<false>(lds, L1, t);
            store_transp<CC>(lds, inter, base, it.h0, it.rs, t);
        } else {
            load_transp<CC>(lds, inter, base, it.h0, it.rs, t);
            __syncthreads();
            rounds<true>(lds, L1, t);
            store_contig<S>(lds, static_cast<S *>(a.out), it.io_off, K, 1, nullptr, t,
                            ortho_scale<C>(it.m), a.ortho != 0);
        }
    }

    template <bool ADJ>
    static __device__ __forceinline__ void run_item(const Item &it, const LaunchArgs &a,
                                                    C *lds, int t)
    {
        switch (it.kind) {
        case KIND_BLOCKS: {
            const int64_t *list = it.list >= 0 ? a.list + it.list : nullptr;
            if constexpr (!ADJ) {
                load_contig<S>(lds, static_cast<const S *>(a.in), it.io_off, it.bits,
                               it.count, list, t);
                __syncthreads();
                rounds<false>(lds, it.bits, t);
                store_paley<S>(lds, static_cast<S *>(a.out), it.io_off, it.bits, it.count,
                               list, t, ortho_scale<C>(it.m), a.ortho != 0);
            } else {
                load_paley<S>(lds, static_cast<const S *>(a.in), it.io_off, it.bits,
                              it.count, list, t);
                __syncthreads();
                rounds<true>(lds, it.bits, t);
                store_contig<S>(lds, static_cast<S *>(a.out), it.io_off, it.bits, it.count,
                                list, t, ortho_scale<C>(it.m), a.ortho != 0);
            }
            break;
        }
        case KIND_FIRST_A:
            first_item<CA, ADJ>(it, a, lds, t);
            break;
        case KIND_FIRST_B:
            first_item<CB, ADJ>(it, a, lds, t);
            break;
        case KIND_LAST: {
            C *inter = static_cast<C *>(a.inter);
            const int64_t woff = a.inter_is_io ? it.io_off : it.ws_off;
            if constexpr (!ADJ) {
                load_contig<C>(lds, inter, woff, it.bits, it.count, nullptr, t);
                __syncthreads();
                rounds<false>(lds, it.bits, t);
                store_paley<S>(lds, static_cast<S *>(a.out), it.io_off, it.bits, it.count,
                               nullptr, t, ortho_scale<C>(it.m), a.ortho != 0);
            } else {
                load_paley<S>(lds, static_cast<const S *>(a.in), it.io_off, it.bits,
                              it.count, nullptr, t);
                __syncthreads();
                rounds<true>(lds, it.bits, t);
                store_contig<C>(lds, inter, woff, it.bits, it.count, nullptr, t, C(1), false);
            }
            break;
        }
        default:
            break;
        }
    }
};

}  // namespace chw
