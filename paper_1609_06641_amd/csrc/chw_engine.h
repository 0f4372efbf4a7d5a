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

#include <type_traits>

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
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

// Every global access of the tile phases is one 16-byte vector.  Each element
// is read once and written once per HBM pass, so by default the accesses carry
// the non-temporal (streaming) hint; the three roles (input reads, output
// writes, intermediate reads and writes) can be switched separately.
#ifndef CHW_NT_IN
#define CHW_NT_IN 1
#endif
#ifndef CHW_NT_OUT
#define CHW_NT_OUT 1
#endif
#ifndef CHW_NT_INTER
#define CHW_NT_INTER 1
#endif

template <bool NT, typename P>
__device__ __forceinline__ u32x4 ld16(const P *p)
{
    const u32x4 *q = reinterpret_cast<const u32x4 *>(p);
    if constexpr (NT) return __builtin_nontemporal_load(q);
    else return *q;
}

template <bool NT, typename P>
__device__ __forceinline__ void st16(P *p, u32x4 v)
{
    u32x4 *q = reinterpret_cast<u32x4 *>(p);
    if constexpr (NT) __builtin_nontemporal_store(v, q);
    else *q = v;
}

// Vec<T>: V elements of storage type T per 16-byte vector; decode widens to
// the compute type, encode narrows from it.
template <typename T> struct Vec;

template <> struct Vec<float> {
    static constexpr int V = 4;
    static __device__ __forceinline__ void decode(u32x4 r, float *o)
    {
#pragma unroll
        for (int i = 0; i < 4; ++i) o[i] = __uint_as_float(r[i]);
    }
    static __device__ __forceinline__ u32x4 encode(const float *v)
    {
        return u32x4{__float_as_uint(v[0]), __float_as_uint(v[1]), __float_as_uint(v[2]),
                     __float_as_uint(v[3])};
    }
};

template <> struct Vec<uint32_t> {
    static constexpr int V = 4;
    static __device__ __forceinline__ void decode(u32x4 r, uint32_t *o)
    {
#pragma unroll
        for (int i = 0; i < 4; ++i) o[i] = r[i];
    }
    static __device__ __forceinline__ u32x4 encode(const uint32_t *v)
    {
        return u32x4{v[0], v[1], v[2], v[3]};
    }
};

template <> struct Vec<double> {
    static constexpr int V = 2;
    static __device__ __forceinline__ void decode(u32x4 r, double *o)
    {
        o[0] = __builtin_bit_cast(double, (uint64_t)r[0] | ((uint64_t)r[1] << 32));
        o[1] = __builtin_bit_cast(double, (uint64_t)r[2] | ((uint64_t)r[3] << 32));
    }
    static __device__ __forceinline__ u32x4 encode(const double *v)
    {
        const uint64_t a = __builtin_bit_cast(uint64_t, v[0]), b = __builtin_bit_cast(uint64_t, v[1]);
        return u32x4{(uint32_t)a, (uint32_t)(a >> 32), (uint32_t)b, (uint32_t)(b >> 32)};
    }
};

// bfloat16: widening is exact (the 16 bits are the top half of an FP32);
// narrowing rounds to nearest even (v_cvt_pk_bf16_f32).
template <> struct Vec<bf16s> {
    static constexpr int V = 8;
    static __device__ __forceinline__ void decode(u32x4 r, float *o)
    {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            o[2 * i] = __uint_as_float(r[i] << 16);
            o[2 * i + 1] = __uint_as_float(r[i] & 0xffff0000u);
        }
    }
    static __device__ __forceinline__ u32x4 encode(const float *v)
    {
        u32x4 w;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            f32x2 f = {v[2 * i], v[2 * i + 1]};
            bf16x2 h = __builtin_convertvector(f, bf16x2);
            w[i] = __builtin_bit_cast(uint32_t, h);
        }
        return w;
    }
};

// float16: widening is exact; narrowing rounds to nearest even.
template <> struct Vec<f16s> {
    static constexpr int V = 8;
    static __device__ __forceinline__ void decode(u32x4 r, float *o)
    {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            f16x2 h = __builtin_bit_cast(f16x2, (uint32_t)r[i]);
            o[2 * i] = (float)h.x;
            o[2 * i + 1] = (float)h.y;
        }
    }
    static __device__ __forceinline__ u32x4 encode(const float *v)
    {
        u32x4 w;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            f32x2 f = {v[2 * i], v[2 * i + 1]};
            f16x2 h = __builtin_convertvector(f, f16x2);
            w[i] = __builtin_bit_cast(uint32_t, h);
        }
        return w;
    }
};

template <bool NT, typename T, typename C>
__device__ __forceinline__ void vload(const T *p, C *o) { Vec<T>::decode(ld16<NT>(p), o); }
template <bool NT, typename T, typename C>
__device__ __forceinline__ void vstore(T *p, const C *v) { st16<NT>(p, Vec<T>::encode(v)); }

// one element (for scattered accesses), same conversions as Vec<T>
__device__ __forceinline__ float get1(const float *p) { return *p; }
__device__ __forceinline__ uint32_t get1(const uint32_t *p) { return *p; }
__device__ __forceinline__ double get1(const double *p) { return *p; }
__device__ __forceinline__ float get1(const bf16s *p) { return __uint_as_float((uint32_t)p->v << 16); }
__device__ __forceinline__ float get1(const f16s *p) { return (float)__builtin_bit_cast(_Float16, p->v); }
__device__ __forceinline__ void put1(float *p, float v) { *p = v; }
__device__ __forceinline__ void put1(uint32_t *p, uint32_t v) { *p = v; }
__device__ __forceinline__ void put1(double *p, double v) { *p = v; }
__device__ __forceinline__ void put1(bf16s *p, float v) { p->v = __builtin_bit_cast(uint16_t, (__bf16)v); }
__device__ __forceinline__ void put1(f16s *p, float v) { p->v = __builtin_bit_cast(uint16_t, (_Float16)v); }

__device__ __forceinline__ int gray_code(int x) { return x ^ (x >> 1); }
__device__ __forceinline__ int64_t inv_gray_code(int64_t x)
{
    x ^= x >> 32; x ^= x >> 16; x ^= x >> 8; x ^= x >> 4; x ^= x >> 2; x ^= x >> 1;
    return x;
}

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

// Multiplication by a diagonal entry d = +1 (bit 0) or -1 (bit 1): exact in
// every type (the float sign bit flips; int32 negates, wrapping).
__device__ __forceinline__ float apply_sign(float v, uint32_t bit)
{
    return __uint_as_float(__float_as_uint(v) ^ (bit << 31));
}
__device__ __forceinline__ double apply_sign(double v, uint32_t bit)
{
    return __builtin_bit_cast(double, __builtin_bit_cast(uint64_t, v) ^ ((uint64_t)bit << 63));
}
__device__ __forceinline__ uint32_t apply_sign(uint32_t v, uint32_t bit)
{
    return bit ? 0u - v : v;
}

// Sign bits of one contiguous 16-byte vector: the V bits starting at the
// vector's first element (signal position jbase + j when the diagonal is
// shared by the signals, buffer position g otherwise).  V divides 32 and
// vectors start at multiples of V, so the bits sit in one word.
struct SignCtx {
    const uint32_t *w;  // null: no diagonal
    int64_t jbase;
    int shared;
};
__device__ __forceinline__ uint32_t sign_bits(const SignCtx &sc, int64_t g, int64_t j)
{
    const int64_t b = sc.shared ? sc.jbase + j : g;
    return sc.w[b >> 5] >> (uint32_t)(b & 31);
}

// A per-thread LDS base for accesses at offsets that are compile-time
// constants once the loops are unrolled.  An LDS instruction carries a 16-bit
// byte offset, so in a tile larger than 64 KiB (2^15 FP32 elements) every
// access past 64 KiB from the base would otherwise get an address register of
// its own, and the optimizer hoists those out of the item loop, where they
// take registers for the whole kernel.  Offsets of 64 KiB and more go from a
// second base (the first plus 64 KiB), kept opaque so that it stays one
// register.  Offsets not known at compile time go from the first base.
template <typename C, int WORDS>
struct LdsAt {
    static constexpr int SPLIT = 65536 / (int)sizeof(C);
    C *lds;
    int b0, b1;
    __device__ __forceinline__ LdsAt(C *l, int b) : lds(l), b0(b), b1(0)
    {
        if constexpr (WORDS > SPLIT) {
            b1 = b + SPLIT;
            asm("" : "+v"(b1));
        }
    }
    __device__ __forceinline__ C &operator[](int off) const
    {
        if constexpr (WORDS > SPLIT) {
            if (__builtin_constant_p(off) && off >= SPLIT) return lds[b1 + (off - SPLIT)];
        }
        return lds[b0 + off];
    }
};

// ---------------------------------------------------------------------------
// the engine

template <int DT, int K, int LR, int CA, int CB>
struct Engine {
    using L = Layout<K, LR>;
    using S = typename Types<DT>::S;
    using C = typename Types<DT>::C;
    static constexpr int N = L::N, NT = L::NT, R = L::R, J = L::J;
    static constexpr bool NT_IN = CHW_NT_IN, NT_OUT = CHW_NT_OUT, NT_INTER = CHW_NT_INTER;
    using At = LdsAt<C, L::LDS_WORDS>;
    using CAt = LdsAt<const C, L::LDS_WORDS>;
    static constexpr int CM = mid_rows(K);
    static constexpr int CD = d_rows(K);
    static_assert(CA >= 2 && CB >= 2 && CA < K && CB < K, "first-pass row counts");
    // row count (log2) of a first-pass kind
    template <int KIND>
    static constexpr int rows_of()
    {
        return KIND == KIND_FIRST_A ? CA : KIND == KIND_FIRST_B ? CB : KIND == KIND_FIRST_D ? CD : CM;
    }

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

    // One register round with its first NA active stages known at compile
    // time: read, NA stages, write.  Each count is a whole round of its own,
    // so no value crosses a branch between the stages (a stage skipped at run
    // time inside one round would make the compiler carry both register
    // assignments and reconcile them with moves).
    template <int j, bool ADJ, int B0, int NA>
    static __device__ __forceinline__ void round_body(C *lds, int t)
    {
        constexpr int lo = L::flo(j, B0), a0 = L::alo(j, B0);
        const At base(lds, L::pad(L::round_tbase(j, t, B0)));
        C v[R];
#pragma unroll
        for (int i = 0; i < R; ++i) v[i] = base[L::pad(L::round_reg(j, i, B0))];
        if constexpr (!ADJ) {
#pragma unroll
            for (int bit = a0; bit < a0 + NA; ++bit) bfly(v, bit - lo);
        } else {
#pragma unroll
            for (int bit = a0 + NA - 1; bit >= a0; --bit) bfly(v, bit - lo);
        }
#pragma unroll
        for (int i = 0; i < R; ++i) base[L::pad(L::round_reg(j, i, B0))] = v[i];
    }

    // round j with each stage tested against nst: the form for a bound known
    // at compile time (the tests fold away)
    template <int j, bool ADJ, int B0>
    static __device__ __forceinline__ void round_nst(C *lds, int nst, int t)
    {
        constexpr int lo = L::flo(j, B0), a0 = L::alo(j, B0), a1 = L::ahi(j, B0);
        const At base(lds, L::pad(L::round_tbase(j, t, B0)));
        C v[R];
#pragma unroll
        for (int i = 0; i < R; ++i) v[i] = base[L::pad(L::round_reg(j, i, B0))];
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
        for (int i = 0; i < R; ++i) base[L::pad(L::round_reg(j, i, B0))] = v[i];
        __syncthreads();
    }

    // the active stages of round j are [a0, min(a1, nst)): dispatch their
    // count (uniform) to a compile-time round
    template <int j, bool ADJ, int B0, int NA>
    static __device__ __forceinline__ void round_count(C *lds, int na, int t)
    {
        if constexpr (NA >= 1) {
            if (na == NA) round_body<j, ADJ, B0, NA>(lds, t);
            else round_count<j, ADJ, B0, NA - 1>(lds, na, t);
        }
    }

    // 2^12-element tiles with 2^5 registers dispatch the stage count of a
    // round to a compile-time round (VALU: with the stages tested one by one,
    // the register moves that reconcile skipped and taken stages cost about a
    // third as much as the butterflies).  The other shapes test the stages
    // one by one: there the register allocator fits that form better (2^15
    // tiles' prefetching forms run at the register limit; 2^6 registers would
    // lose a wave per SIMD).
    template <int j, bool ADJ, int B0 = 0>
    static __device__ __forceinline__ void round(C *lds, int nst, int t)
    {
        constexpr int a0 = L::alo(j, B0), a1 = L::ahi(j, B0);
        if (a0 >= nst) return;  // no active stage in this round (uniform)
        if constexpr (K == 12 && LR == 5) {
            if (nst >= a1) round_body<j, ADJ, B0, a1 - a0>(lds, t);
            else round_count<j, ADJ, B0, a1 - a0 - 1>(lds, nst - a0, t);
            __syncthreads();
        } else {
            round_nst<j, ADJ, B0>(lds, nst, t);
        }
    }

    // the stages [B0, nst): increasing (forward) or decreasing (adjoint; the
    // stages below B0 then run on the stored vectors, see post_bits)
    template <bool ADJ, int j = 0, int B0 = 0>
    static __device__ __forceinline__ void rounds(C *lds, int nst, int t)
    {
        if constexpr (j < L::rounds_from(B0)) {
            if constexpr (!ADJ) {
                round<j, false, B0>(lds, nst, t);
                rounds<false, j + 1, B0>(lds, nst, t);
            } else {
                round<L::rounds_from(B0) - 1 - j, true, B0>(lds, nst, t);
                rounds<true, j + 1, B0>(lds, nst, t);
            }
        }
    }

    // rounds() with the stage bound known at compile time
    template <bool ADJ, int NST, int j = 0, int B0 = 0>
    static __device__ __forceinline__ void rounds_ct(C *lds, int t)
    {
        if constexpr (j < L::rounds_from(B0)) {
            constexpr int jj = ADJ ? L::rounds_from(B0) - 1 - j : j;
            constexpr int a0 = L::alo(jj, B0), a1 = L::ahi(jj, B0);
            if constexpr (a0 < NST) {
                if constexpr (K == 12 && LR == 5) {
                    round_body<jj, ADJ, B0, (a1 < NST ? a1 : NST) - a0>(lds, t);
                    __syncthreads();
                } else {
                    round_nst<jj, ADJ, B0>(lds, NST, t);
                }
            }
            rounds_ct<ADJ, NST, j + 1, B0>(lds, t);
        }
    }

    // ---- the Haar transform Psi_m alone (eq. 2) --------------------------------
    // Psi_m is the part of the stages that acts on sums only: at stage b the
    // pair (e, e | 2^b) belongs to Psi_m iff the low b bits of e are zero.
    // In register round j those bits are the thread bits below the register
    // field (one test per thread) and the low register bits (known at compile
    // time); threads whose test fails hold no pair of the round.
    template <int j, bool ADJ>
    static __device__ __forceinline__ void haar_round(C *lds, int nst, int t)
    {
        constexpr int lo = L::flo(j), a0 = L::alo(j), a1 = L::ahi(j);
        if (a0 >= nst) return;  // uniform
        if ((t & ((1 << lo) - 1)) == 0) {
            C *base = lds + L::pad(L::round_tbase(j, t));
            C v[R];
#pragma unroll
            for (int i = 0; i < R; ++i) v[i] = base[L::pad(L::round_reg(j, i))];
#pragma unroll
            for (int s = 0; s < a1 - a0; ++s) {
                const int bit = ADJ ? a1 - 1 - s : a0 + s;
                if (bit < nst) {
                    const int rb = bit - lo;
#pragma unroll
                    for (int i = 0; i < R; ++i)
                        if ((i & ((1 << (rb + 1)) - 1)) == 0) {
                            C a = v[i], b = v[i | (1 << rb)];
                            v[i] = a + b;
                            v[i | (1 << rb)] = a - b;
                        }
                }
            }
#pragma unroll
            for (int i = 0; i < R; ++i) base[L::pad(L::round_reg(j, i))] = v[i];
        }
        __syncthreads();
    }

    template <bool ADJ, int j = 0>
    static __device__ __forceinline__ void haar_rounds(C *lds, int nst, int t)
    {
        if constexpr (j < J) {
            if constexpr (!ADJ) {
                haar_round<j, false>(lds, nst, t);
                haar_rounds<false, j + 1>(lds, nst, t);
            } else {
                haar_round<J - 1 - j, true>(lds, nst, t);
                haar_rounds<true, j + 1>(lds, nst, t);
            }
        }
    }

    // ---- contiguous phases ---------------------------------------------------
    // Tile element e <-> memory element (block e >> bits at its base) + (e &
    // (2^bits - 1)).  Blocks are consecutive from `off` unless `list` gives
    // their bases.  Only the first `count` blocks exist.  PRE > 0: a loaded
    // vector holds every value of tile bits [0, PRE) of its block, and the
    // stages below min(PRE, pre_lim) run on it (after the signs) before it
    // goes to LDS.
    template <int V, int NB>
    static __device__ __forceinline__ void pre_stages_n(C *v)
    {
#pragma unroll
        for (int b = 0; b < NB; ++b) {
#pragma unroll
            for (int i = 0; i < V; ++i)
                if (!(i & (1 << b))) {
                    C x = v[i], y = v[i | (1 << b)];
                    v[i] = x + y;
                    v[i | (1 << b)] = x - y;
                }
        }
    }
    // stages 0 .. min(PRE, lim) - 1; the count (uniform) picks a
    // compile-time sequence, as round() does
    template <int V, int PRE>
    static __device__ __forceinline__ void pre_stages(C *v, int lim)
    {
        static_assert((1 << PRE) <= V && PRE <= 3, "pre-stages stay inside one vector");
        if constexpr (PRE >= 1) {
            if (lim >= PRE) pre_stages_n<V, PRE>(v);
            else if (lim == PRE - 1) pre_stages_n<V, PRE - 1>(v);
            else if constexpr (PRE >= 3) {
                if (lim == PRE - 2) pre_stages_n<V, PRE - 2>(v);
            }
        }
    }

    // The adjoint's last stages (tile bits POST - 1 .. 0, decreasing) on one
    // stored vector, below min(POST, lim): the counterpart of pre_stages
    template <int V, int NB>
    static __device__ __forceinline__ void post_stages_n(C *v)
    {
#pragma unroll
        for (int b = NB - 1; b >= 0; --b) {
#pragma unroll
            for (int i = 0; i < V; ++i)
                if (!(i & (1 << b))) {
                    C x = v[i], y = v[i | (1 << b)];
                    v[i] = x + y;
                    v[i | (1 << b)] = x - y;
                }
        }
    }
    template <int V, int POST>
    static __device__ __forceinline__ void post_stages(C *v, int lim)
    {
        static_assert((1 << POST) <= V && POST <= 3, "post-stages stay inside one vector");
        if constexpr (POST >= 1) {
            if (lim >= POST) post_stages_n<V, POST>(v);
            else if (lim == POST - 1) post_stages_n<V, POST - 1>(v);
            else if constexpr (POST >= 3) {
                if (lim == POST - 2) post_stages_n<V, POST - 2>(v);
            }
        }
    }

    template <bool H, typename T, int PRE = 0>
    static __device__ __forceinline__ void load_contig(C *lds, const T *src, int64_t off,
                                                       int bits, int count,
                                                       const int64_t *list, int t,
                                                       const SignCtx &sg = SignCtx{nullptr, 0, 0},
                                                       int pre_lim = 0)
    {
        constexpr int V = Vec<T>::V, NV = N / (V * NT);
        static_assert(NV >= 1, "tile too small for the vector width");
        const At lb(lds, L::pad(V * t));
        const bool full = (list == nullptr) && ((count << bits) >= N);
        const int mask = (1 << bits) - 1;
        C vals[NV][V];
        if (full) {
            const T *s = src + off + V * t;
#pragma unroll
            for (int k = 0; k < NV; ++k) vload<H>(s + V * NT * k, vals[k]);
            if (sg.w) {
#pragma unroll
                for (int k = 0; k < NV; ++k) {
                    const int e0 = V * t + V * NT * k;
                    const uint32_t sb = sign_bits(sg, off + e0, e0 & mask);
#pragma unroll
                    for (int u = 0; u < V; ++u) vals[k][u] = apply_sign(vals[k][u], (sb >> u) & 1u);
                }
            }
            if constexpr (PRE > 0) {
#pragma unroll
                for (int k = 0; k < NV; ++k) pre_stages<V, PRE>(vals[k], pre_lim);
            }
#pragma unroll
            for (int k = 0; k < NV; ++k)
#pragma unroll
                for (int u = 0; u < V; ++u) lb[L::pad(V * NT * k) + u] = vals[k][u];
        } else {
#pragma unroll
            for (int k = 0; k < NV; ++k) {
                const int e0 = V * t + V * NT * k;
                const int blk = e0 >> bits;
                if (blk < count) {
                    const int64_t g = list ? list[blk] + (e0 & mask) : off + e0;
                    vload<H>(src + g, vals[k]);
                    if (sg.w) {
                        const uint32_t sb = sign_bits(sg, g, e0 & mask);
#pragma unroll
                        for (int u = 0; u < V; ++u) vals[k][u] = apply_sign(vals[k][u], (sb >> u) & 1u);
                    }
                    if constexpr (PRE > 0) pre_stages<V, PRE>(vals[k], pre_lim);
#pragma unroll
                    for (int u = 0; u < V; ++u) lb[L::pad(V * NT * k) + u] = vals[k][u];
                }
            }
        }
    }

    template <bool H, typename T, int POST = 0>
    static __device__ __forceinline__ void store_contig(const C *lds, T *dst, int64_t off,
                                                        int bits, int count,
                                                        const int64_t *list, int t,
                                                        C scale, bool do_scale,
                                                        const SignCtx &sg = SignCtx{nullptr, 0, 0},
                                                        int post_lim = 0)
    {
        constexpr int V = Vec<T>::V, NV = N / (V * NT);
        const CAt lb(lds, L::pad(V * t));
        const bool full = (list == nullptr) && ((count << bits) >= N);
        const int mask = (1 << bits) - 1;
#pragma unroll
        for (int k = 0; k < NV; ++k) {
            const int e0 = V * t + V * NT * k;
            const int blk = e0 >> bits;
            if (full || blk < count) {
                C vals[V];
#pragma unroll
                for (int u = 0; u < V; ++u) vals[u] = lb[L::pad(V * NT * k) + u];
                if constexpr (POST > 0) post_stages<V, POST>(vals, post_lim);
                if (do_scale) {
#pragma unroll
                    for (int u = 0; u < V; ++u) vals[u] = scale_mul(vals[u], scale);
                }
                const int64_t g = (!full && list) ? list[blk] + (e0 & mask) : off + e0;
                if (sg.w) {
                    const uint32_t sb = sign_bits(sg, g, e0 & mask);
#pragma unroll
                    for (int u = 0; u < V; ++u) vals[u] = apply_sign(vals[u], (sb >> u) & 1u);
                }
                vstore<H>(dst + g, vals);
            }
        }
    }

    // ---- Paley-order phases --------------------------------------------------
    // brev_low(x, bits) reverses bits [0, bits) of x and keeps the others: a
    // bit permutation, so for the disjoint thread / iteration / lane fields of
    // an output position o = V t | V NT k | u the tile element is
    // brev_low(V t) | brev_low(V NT k) | brev_low(u), and its padded LDS word is
    // the sum of the three padded parts (the last two are wave-uniform).
    static __device__ __forceinline__ int brev_low(int x, int bits)
    {
        const int mask = (1 << bits) - 1;
        return (x & ~mask) | (int)rbrev((uint32_t)(x & mask), bits);
    }

    // Memory position (blk << bits) | p holds tile element (blk << bits) |
    // bitrev_bits(p): the dyadic order of eq. (1) is the natural radix-2 order
    // read at bit-reversed positions.  SG: the output also takes the diagonal
    // sg after the scale (position o of the tile is buffer element off + o,
    // signal position sg.jbase + o; no block list).
    template <bool H, typename T, bool SG = false>
    static __device__ __forceinline__ void store_paley(const C *lds, T *dst, int64_t off,
                                                       int bits, int count,
                                                       const int64_t *list, int t,
                                                       C scale, bool do_scale,
                                                       const SignCtx &sg = SignCtx{nullptr, 0, 0})
    {
        constexpr int V = Vec<T>::V, NV = N / (V * NT);
        if (bits == K) {
            const CAt lb(lds, L::pad((int)rbrev((uint32_t)(V * t), K)));
            T *d = dst + (list ? list[0] : off) + V * t;
#pragma unroll
            for (int k = 0; k < NV; ++k) {
                C vals[V];
#pragma unroll
                for (int u = 0; u < V; ++u) {
                    vals[u] = lb[L::pad((int)cbrev((uint32_t)(V * NT * k + u), K))];
                    if (do_scale) vals[u] = scale_mul(vals[u], scale);
                }
                if constexpr (SG) {
                    const int o = V * t + V * NT * k;
                    const uint32_t w = sign_bits(sg, off + o, o);
#pragma unroll
                    for (int u = 0; u < V; ++u) vals[u] = apply_sign(vals[u], (w >> u) & 1u);
                }
                vstore<H>(d + V * NT * k, vals);
            }
        } else {
            const int mask = (1 << bits) - 1;
            const C *lb = lds + L::pad(brev_low(V * t, bits));
            int ul[V];
#pragma unroll
            for (int u = 0; u < V; ++u) ul[u] = L::pad(brev_low(u, bits));
#pragma unroll
            for (int k = 0; k < NV; ++k) {
                const int o0 = V * t + V * NT * k;
                const int blk = o0 >> bits;
                if (blk < count) {
                    const int p0 = o0 & mask;
                    const int kl = L::pad(brev_low(V * NT * k, bits));
                    C vals[V];
#pragma unroll
                    for (int u = 0; u < V; ++u) {
                        vals[u] = lb[kl + ul[u]];
                        if (do_scale) vals[u] = scale_mul(vals[u], scale);
                    }
                    const int64_t g = list ? list[blk] + p0 : off + o0;
                    if constexpr (SG) {
                        const uint32_t w = sign_bits(sg, g, o0);
#pragma unroll
                        for (int u = 0; u < V; ++u) vals[u] = apply_sign(vals[u], (w >> u) & 1u);
                    }
                    vstore<H>(dst + g, vals);
                }
            }
        }
    }

    template <bool H, typename T>
    static __device__ __forceinline__ void load_paley(C *lds, const T *src, int64_t off,
                                                      int bits, int count,
                                                      const int64_t *list, int t)
    {
        constexpr int V = Vec<T>::V, NV = N / (V * NT);
        C vals[NV][V];
        if (bits == K) {
            const At lb(lds, L::pad((int)rbrev((uint32_t)(V * t), K)));
            const T *s = src + (list ? list[0] : off) + V * t;
#pragma unroll
            for (int k = 0; k < NV; ++k) vload<H>(s + V * NT * k, vals[k]);
#pragma unroll
            for (int k = 0; k < NV; ++k)
#pragma unroll
                for (int u = 0; u < V; ++u)
                    lb[L::pad((int)cbrev((uint32_t)(V * NT * k + u), K))] = vals[k][u];
        } else {
            const int mask = (1 << bits) - 1;
            C *lb = lds + L::pad(brev_low(V * t, bits));
            int ul[V];
#pragma unroll
            for (int u = 0; u < V; ++u) ul[u] = L::pad(brev_low(u, bits));
#pragma unroll
            for (int k = 0; k < NV; ++k) {
                const int o0 = V * t + V * NT * k;
                const int blk = o0 >> bits;
                if (blk < count) {
                    const int p0 = o0 & mask;
                    const int64_t g = list ? list[blk] + p0 : off + o0;
                    vload<H>(src + g, vals[k]);
                    const int kl = L::pad(brev_low(V * NT * k, bits));
#pragma unroll
                    for (int u = 0; u < V; ++u) lb[kl + ul[u]] = vals[k][u];
                }
            }
        }
    }

    // ---- coefficient orders other than dyadic --------------------------------
    // Every order is a permutation of the dyadic output: coefficient at output
    // position o of a block of 2^bits comes from tile element M(o) of the
    // block (natural storage holds the radix-2 (Sylvester) result):
    //   dyadic   M(o) = bitrev(o)
    //   sequency M(o) = bitrev(gray(o))   (dyadic row gray(o) has o sign changes)
    //   natural  M(o) = o
    // The adjoint gathers its input through the same map.
    template <int ORD>
    static __device__ __forceinline__ int block_src(int o, int bits)
    {
        if constexpr (ORD == ORDER_NATURAL) return o;
        else if constexpr (ORD == ORDER_SEQUENCY) return (int)rbrev((uint32_t)gray_code(o), bits);
        else return (int)rbrev((uint32_t)o, bits);
    }

    // single-pass tiles: store (forward) / gather (adjoint) in order ORD
    template <int ORD, bool LOAD, typename T>
    static __device__ __forceinline__ void blocks_ordered(C *lds, T *io, int64_t off, int bits,
                                                          int count, const int64_t *list, int t,
                                                          C scale, bool do_scale)
    {
        constexpr int V = Vec<T>::V, NV = N / (V * NT);
        const int mask = (1 << bits) - 1;
#pragma unroll
        for (int k = 0; k < NV; ++k) {
            const int o0 = V * t + V * NT * k;
            const int blk = o0 >> bits;
            if (blk >= count) continue;
            const int p0 = o0 & mask;
            const int64_t g = list ? list[blk] + p0 : off + o0;
            C vals[V];
            if constexpr (LOAD) {
                vload<NT_IN>(io + g, vals);
#pragma unroll
                for (int u = 0; u < V; ++u) lds[L::pad((blk << bits) | block_src<ORD>(p0 + u, bits))] = vals[u];
            } else {
#pragma unroll
                for (int u = 0; u < V; ++u) {
                    vals[u] = lds[L::pad((blk << bits) | block_src<ORD>(p0 + u, bits))];
                    if (do_scale) vals[u] = scale_mul(vals[u], scale);
                }
                vstore<NT_OUT>(io + g, vals);
            }
        }
    }

    // last-pass tiles of a two-pass signal in order ORD.  The tile holds
    // blocks bg0 .. bg0 + count - 1 of the signal's 2^L1 blocks of 2^bits.
    //   sequency: dyadic position P = (bg << bits) | q has sequency index
    //     invgray(P) = (invgray(bg) << bits) | (invgray(q) ^ (parity(bg) ? mask : 0)),
    //     so block bg lands as a whole on block invgray(bg);
    //   natural: the first pass kept block bg = its row element (no bit
    //     reversal), so element k of block bg is coefficient (k << L1) | bg:
    //     runs of `count` consecutive blocks, stride 2^L1.
    template <int ORD, bool LOAD, typename T>
    static __device__ __forceinline__ void last_ordered(C *lds, T *io, const Item &it, int t,
                                                        C scale, bool do_scale)
    {
        constexpr int V = Vec<T>::V, NV = N / (V * NT);
        const int b = it.bits, mask = (1 << b) - 1, L1 = it.m - b;
        const int64_t bg0 = (it.io_off - it.sig_off) >> b;
        if constexpr (ORD == ORDER_SEQUENCY) {
#pragma unroll
            for (int k = 0; k < NV; ++k) {
                const int o0 = V * t + V * NT * k;
                const int blk = o0 >> b, s0 = o0 & mask;
                const int64_t bg = bg0 + blk;
                const int flipm = (__builtin_popcountll((uint64_t)bg) & 1) ? mask : 0;
                T *p = io + it.sig_off + (inv_gray_code(bg) << b) + s0;
                C vals[V];
                if constexpr (LOAD) vload<NT_IN>(p, vals);
#pragma unroll
                for (int u = 0; u < V; ++u) {
                    const int e = (blk << b) | (int)rbrev((uint32_t)gray_code((s0 + u) ^ flipm), b);
                    if constexpr (LOAD) {
                        lds[L::pad(e)] = vals[u];
                    } else {
                        vals[u] = lds[L::pad(e)];
                        if (do_scale) vals[u] = scale_mul(vals[u], scale);
                    }
                }
                if constexpr (!LOAD) vstore<NT_OUT>(p, vals);
            }
        } else {
            // natural: compact output index o = kh * count + blk
            const int lnb = K - b;                     // log2 count (full tile)
            if (lnb >= (V == 8 ? 3 : V == 4 ? 2 : 1)) {
#pragma unroll
                for (int k = 0; k < NV; ++k) {
                    const int o0 = V * t + V * NT * k;
                    const int kh = o0 >> lnb, blk0 = o0 & ((1 << lnb) - 1);
                    T *p = io + it.sig_off + ((int64_t)kh << L1) + bg0 + blk0;
                    C vals[V];
                    if constexpr (LOAD) vload<NT_IN>(p, vals);
#pragma unroll
                    for (int u = 0; u < V; ++u) {
                        const int e = ((blk0 + u) << b) | kh;
                        if constexpr (LOAD) {
                            lds[L::pad(e)] = vals[u];
                        } else {
                            vals[u] = lds[L::pad(e)];
                            if (do_scale) vals[u] = scale_mul(vals[u], scale);
                        }
                    }
                    if constexpr (!LOAD) vstore<NT_OUT>(p, vals);
                }
            } else {
                // runs shorter than one vector: element by element
                for (int o = t; o < N; o += NT) {
                    const int kh = o >> lnb, blk = o & ((1 << lnb) - 1);
                    T *p = io + it.sig_off + ((int64_t)kh << L1) + bg0 + blk;
                    const int e = (blk << b) | kh;
                    if constexpr (LOAD) {
                        lds[L::pad(e)] = get1(p);
                    } else {
                        C v = lds[L::pad(e)];
                        if (do_scale) v = scale_mul(v, scale);
                        put1(p, v);
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
    template <int CC, bool BR = true>
    static __device__ __forceinline__ void store_transp(const C *lds, C *dst, int64_t base,
                                                        int h0, int rs, int t)
    {
        constexpr int V = Vec<C>::V, NV = N / (V * NT);
        static_assert(V <= (1 << CC), "a vector must stay inside one run");
        const CAt lb(lds, L::pad(L::template transp_e<V, CC, BR>(t, 0, 0)));
        C *d = dst + base + h0 + L::template transp_goff<CC>(V * L::template transp_q<V, CC>(t), rs);
#pragma unroll
        for (int k = 0; k < NV; ++k) {
            C vals[V];
#pragma unroll
            for (int u = 0; u < V; ++u)
                vals[u] = lb[L::pad(L::template transp_e<V, CC, BR>(0, k, u))];
            st16<NT_INTER>(d + L::template transp_goff<CC>(V * L::template transp_q<V, CC>(NT * k), rs),
                           Vec<C>::encode(vals));
        }
    }

    // First-pass store that runs the row's top nk = log2(R / V) stages: a
    // thread's vectors differ exactly in row-element bits L1 - nk .. L1 - 1
    // (the low run-index bits), so those stages, in increasing order, pair
    // whole vectors in registers; the element whose bit is clear (the earlier
    // one in the row) takes the sum.  The global layout is the one of
    // store_transp; only which thread writes which vector differs.  Used for
    // 2^15-element tiles of 2^7 rows (L1 = 8) with 2^5 registers, where it
    // leaves one register round (stages 0 .. 4) instead of two, and of 2^6
    // rows (L1 = 9), where the loaded vectors also run the row's first stages
    // (first_pre) and one register round is left as well (stages 2 .. 5 for
    // FP32 input).
    template <int CC, bool BR>
    static constexpr bool merge_ok()
    {
        return BR && K == 15 && LR == 5 && (CC == 7 || CC == 6) && sizeof(C) == 4;
    }
    template <int CC>
    static constexpr int merge_stages() { return LR - pre_bits<C>(); }
    // stages 0 .. first_pre - 1 of a forward first-pass tile run on its loaded
    // 16-byte vectors (storage type S) before they reach LDS: where the merged
    // store leaves more stages than one register round holds
    template <int CC, bool BR>
    static constexpr int first_pre()
    {
        if constexpr (merge_ok<CC, BR>())
            return K - CC - merge_stages<CC>() > LR ? pre_bits<S>() : 0;
        else
            return 0;
    }

    template <int CC>
    static __device__ __forceinline__ void store_transp_merged(const C *lds, C *dst,
                                                               int64_t base, int h0, int rs,
                                                               int t)
    {
        constexpr int V = Vec<C>::V, NV = N / (V * NT), L1 = K - CC, nk = merge_stages<CC>();
        static_assert((1 << nk) == NV && nk < L1, "one vector per value of the merged bits");
        const CAt lb(lds, L::pad(L::template transpm_e<V, CC>(t, 0, 0)));
        C vals[NV][V];
#pragma unroll
        for (int k = 0; k < NV; ++k)
#pragma unroll
            for (int u = 0; u < V; ++u)
                vals[k][u] = lb[L::pad(L::template transpm_e<V, CC>(0, k, u))];
#pragma unroll
        for (int b = L1 - nk; b < L1; ++b) {
            const int kb = L1 - 1 - b;  // row-element bit b is run-index bit L1 - 1 - b
#pragma unroll
            for (int k = 0; k < NV; ++k)
                if (!(k & (1 << kb))) {
#pragma unroll
                    for (int u = 0; u < V; ++u) {
                        C x = vals[k][u], y = vals[k | (1 << kb)][u];
                        vals[k][u] = x + y;
                        vals[k | (1 << kb)][u] = x - y;
                    }
                }
        }
        C *d = dst + base + h0 +
               L::template transp_goff<CC>(V * L::template transpm_q<V, CC>(t, 0), rs);
#pragma unroll
        for (int k = 0; k < NV; ++k)
            st16<NT_INTER>(d + L::template transp_goff<CC>(V * L::template transpm_q<V, CC>(0, k), rs),
                           Vec<C>::encode(vals[k]));
    }

    // ---- transposed gather of the adjoint first pass -------------------------
    // Where the merged map applies (merge_ok), a thread's vectors differ in
    // row-element bits L1 - nk .. L1 - 1 and the adjoint's first stages (those
    // bits, in decreasing order) run on them right after the gather, before the
    // LDS write; the rounds then start below them.  gather_q(t, k): vector index
    // of thread t's k-th vector; the split gather_q(t, 0) | gather_q(0, k) holds.
    template <int CC, bool BR>
    static __device__ __forceinline__ int gather_q(int t, int k)
    {
        constexpr int V = Vec<C>::V;
        if constexpr (merge_ok<CC, BR>()) return L::template transpm_q<V, CC>(t, k);
        else return L::template transp_q<V, CC>(t + NT * k);
    }
    template <int CC, bool BR>
    static __device__ __forceinline__ int gather_e(int t, int k, int u)
    {
        constexpr int V = Vec<C>::V;
        if constexpr (merge_ok<CC, BR>()) return L::template transpm_e<V, CC>(t, k, u);
        else return L::template transp_e<V, CC, BR>(t, k, u);
    }
    // stages the gather leaves to the register rounds: row-element bits below
    template <int CC, bool BR>
    static constexpr int gather_nst() { return K - CC - (merge_ok<CC, BR>() ? merge_stages<CC>() : 0); }

    // the gathered vectors (decoded) -> merged stages -> LDS
    template <int CC, bool BR>
    static __device__ __forceinline__ void put_gather(C *lds, C (*vals)[Vec<C>::V], int t)
    {
        constexpr int V = Vec<C>::V, NV = N / (V * NT), L1 = K - CC;
        if constexpr (merge_ok<CC, BR>()) {
            constexpr int nk = merge_stages<CC>();
            static_assert((1 << nk) == NV, "one vector per value of the merged bits");
#pragma unroll
            for (int b = L1 - 1; b >= L1 - nk; --b) {
                const int kb = L1 - 1 - b;
#pragma unroll
                for (int k = 0; k < NV; ++k)
                    if (!(k & (1 << kb))) {
#pragma unroll
                        for (int u = 0; u < V; ++u) {
                            C x = vals[k][u], y = vals[k | (1 << kb)][u];
                            vals[k][u] = x + y;
                            vals[k | (1 << kb)][u] = x - y;
                        }
                    }
            }
        }
        const At lb(lds, L::pad(gather_e<CC, BR>(t, 0, 0)));
#pragma unroll
        for (int k = 0; k < NV; ++k)
#pragma unroll
            for (int u = 0; u < V; ++u) lb[L::pad(gather_e<CC, BR>(0, k, u))] = vals[k][u];
    }

    template <int CC, bool BR = true>
    static __device__ __forceinline__ void load_transp(C *lds, const C *src, int64_t base,
                                                       int h0, int rs, int t)
    {
        constexpr int V = Vec<C>::V, NV = N / (V * NT);
        static_assert(V <= (1 << CC), "a vector must stay inside one run");
        const C *s = src + base + h0 + L::template transp_goff<CC>(V * gather_q<CC, BR>(t, 0), rs);
        C vals[NV][V];
#pragma unroll
        for (int k = 0; k < NV; ++k)
            vload<NT_INTER>(s + L::template transp_goff<CC>(V * gather_q<CC, BR>(0, k), rs), vals[k]);
        put_gather<CC, BR>(lds, vals, t);
    }

    // ---- one work item -------------------------------------------------------
    // run_item = load_item, barrier, finish_item.  load_item stages the tile in
    // LDS; finish_item runs the tile's stages and its store phase.
    template <int CC>
    static __device__ __forceinline__ int64_t first_base(const Item &it, const LaunchArgs &a)
    {
        return a.inter_is_io ? it.io_off - ((int64_t)it.h0 << (K - CC)) : it.ws_off;
    }
    static __device__ __forceinline__ int64_t last_base(const Item &it, const LaunchArgs &a)
    {
        return a.inter_is_io ? it.io_off : it.ws_off;
    }
    // sign context of a first-pass tile: its rows start at signal position
    // h0 * 2^(K - CC)
    template <int CC>
    static __device__ __forceinline__ SignCtx first_signs(const Item &it, const LaunchArgs &a)
    {
        return SignCtx{a.signs, (int64_t)it.h0 << (K - CC), a.sign_shared};
    }

    template <bool ADJ, int ORD = ORDER_DYADIC>
    static __device__ __forceinline__ void load_item(const Item &it, const LaunchArgs &a,
                                                     C *lds, int t)
    {
        constexpr bool BR = ORD != ORDER_NATURAL;  // first-pass runs bit-reversed
        const S *in = static_cast<const S *>(a.in);
        const C *inter = static_cast<const C *>(a.inter);
        switch (it.kind) {
        case KIND_BLOCKS: {
            const int64_t *list = it.list >= 0 ? a.list + it.list : nullptr;
            if constexpr (!ADJ)
                load_contig<NT_IN, S>(lds, in, it.io_off, it.bits, it.count, list, t,
                                      SignCtx{a.signs, 0, a.sign_shared});
            else if constexpr (ORD == ORDER_DYADIC)
                load_paley<NT_IN, S>(lds, in, it.io_off, it.bits, it.count, list, t);
            else
                blocks_ordered<ORD, true>(lds, const_cast<S *>(in), it.io_off, it.bits, it.count,
                                          list, t, C(1), false);
            break;
        }
        case KIND_FIRST_A:
            if constexpr (!ADJ)
                load_contig<NT_IN, S, first_pre<CA, BR>()>(lds, in, it.io_off, K, 1, nullptr, t,
                                                          first_signs<CA>(it, a), K);
            else load_transp<CA, BR>(lds, inter, first_base<CA>(it, a), it.h0, it.rs, t);
            break;
        case KIND_FIRST_B:
            if constexpr (!ADJ)
                load_contig<NT_IN, S, first_pre<CB, BR>()>(lds, in, it.io_off, K, 1, nullptr, t,
                                                          first_signs<CB>(it, a), K);
            else load_transp<CB, BR>(lds, inter, first_base<CB>(it, a), it.h0, it.rs, t);
            break;
        case KIND_FIRST_C:
            if constexpr (!ADJ)
                load_contig<NT_IN, S, first_pre<CM, BR>()>(lds, in, it.io_off, K, 1, nullptr, t,
                                                          first_signs<CM>(it, a), K);
            else load_transp<CM, BR>(lds, inter, first_base<CM>(it, a), it.h0, it.rs, t);
            break;
        case KIND_FIRST_D:
            if constexpr (!ADJ)
                load_contig<NT_IN, S, first_pre<CD, BR>()>(lds, in, it.io_off, K, 1, nullptr, t,
                                                          first_signs<CD>(it, a), K);
            else load_transp<CD, BR>(lds, inter, first_base<CD>(it, a), it.h0, it.rs, t);
            break;
        case KIND_LAST:
            if constexpr (!ADJ) load_contig<NT_INTER, C>(lds, inter, last_base(it, a), it.bits, it.count, nullptr, t);
            else if constexpr (ORD == ORDER_DYADIC)
                load_paley<NT_IN, S>(lds, in, it.io_off, it.bits, it.count, nullptr, t);
            else
                last_ordered<ORD, true>(lds, const_cast<S *>(in), it, t, C(1), false);
            break;
        default:
            break;
        }
    }

    // ---- several signed rounds inside one single-pass tile ---------------------
    // y = H D_k ... H D_1 x (adjoint: D_1 H^T ... D_k H^T g) without leaving
    // LDS.  After a round the tile holds the round's dyadic-ordered output either
    // at natural positions or at bit-reversed ones ("flipped").  A round on a
    // natural tile runs the stages in increasing tile-bit order, on a flipped
    // tile in decreasing order: both pair the same elements in the same order
    // as a separate launch would after reloading the output, so the numbers
    // equal those of one launch per round (FP32 between the rounds).
    // Multiply every element of the tile's blocks by the scale and by the
    // sign of the diagonal at its signal position j (the element's position in
    // its block, bit-reversed when the tile is flipped).  A thread takes 32
    // consecutive positions j of one block: their sign bits come from one
    // 64-bit window of the sign words (two 32-bit loads).
    static __device__ __forceinline__ void lds_sign_scale(const Item &it, const LaunchArgs &a,
                                                          const uint32_t *w, bool flip,
                                                          C scale, bool do_scale, C *lds, int t)
    {
        const int bits = it.bits;
        const int gl = bits >= 5 ? 5 : bits;          // log2 positions per group
        const int groups = N >> gl;
        for (int q = t; q < groups; q += NT) {
            const int e0 = q << gl;                   // first tile element of the group
            const int blk = e0 >> bits;
            if (blk >= it.count) continue;
            const int j0 = e0 & ((1 << bits) - 1);
            const int64_t base = it.list >= 0 ? a.list[it.list + blk]
                                              : it.io_off + ((int64_t)blk << bits);
            const int64_t b0 = a.sign_shared ? (int64_t)j0 : base + j0;
            // the second word only when the group's bits reach into it
            const bool two = (int)(b0 & 31) + (1 << gl) > 32;
            const uint64_t win = (uint64_t)w[b0 >> 5] |
                                 (two ? (uint64_t)w[(b0 >> 5) + 1] << 32 : 0ull);
            const uint32_t sb = (uint32_t)(win >> (uint32_t)(b0 & 31));
            // independent reads, then the flips, then the writes
            int ad[32];
            C v[32];
#pragma unroll
            for (int u = 0; u < 32; ++u) {
                const int j = j0 + u;
                const int e = (blk << bits) | (flip ? (int)rbrev((uint32_t)j, bits) : j);
                ad[u] = L::pad(e);
                if (u < (1 << gl)) v[u] = lds[ad[u]];
            }
#pragma unroll
            for (int u = 0; u < 32; ++u) {
                if (do_scale) v[u] = scale_mul(v[u], scale);
                v[u] = apply_sign(v[u], (sb >> u) & 1u);
            }
#pragma unroll
            for (int u = 0; u < 32; ++u)
                if (u < (1 << gl)) lds[ad[u]] = v[u];
        }
        __syncthreads();
    }

    template <bool ADJ>
    static __device__ __forceinline__ void blocks_rounds(const Item &it, const LaunchArgs &a,
                                                         C *lds, int t)
    {
        S *out = static_cast<S *>(a.out);
        const int64_t *list = it.list >= 0 ? a.list + it.list : nullptr;
        const C sc = ortho_scale<C>(it.m);
        const bool ortho = a.ortho != 0;
        const int k = a.rounds;
        bool flip = ADJ;  // the adjoint's tile starts Paley-gathered
        for (int i = 0; i < k; ++i) {
            if (!flip) rounds<false>(lds, it.bits, t);
            else rounds<true>(lds, it.bits, t);
            flip = !flip;
            if constexpr (!ADJ) {
                // the next round's diagonal (round 0's was applied as the tile loaded)
                if (i + 1 < k)
                    lds_sign_scale(it, a, a.signs + (int64_t)(i + 1) * a.sign_words, flip, sc,
                                   ortho, lds, t);
            } else {
                // this round's diagonal: rounds run k-1, ..., 0
                lds_sign_scale(it, a, a.signs + (int64_t)(k - 1 - i) * a.sign_words, flip, sc,
                               ortho, lds, t);
            }
        }
        // forward: the last round's scale goes with the store; adjoint: done
        const bool last_scale = !ADJ && ortho;
        if (flip) store_paley<NT_OUT, S>(lds, out, it.io_off, it.bits, it.count, list, t, sc, last_scale);
        else store_contig<NT_OUT, S>(lds, out, it.io_off, it.bits, it.count, list, t, sc, last_scale);
    }

    // Stages below post_bits() of an adjoint tile run on its stored 16-byte
    // vectors (after the register rounds, before the scale and the diagonal),
    // so the adjoint's rounds stop at that bit: with 2^5 registers and 4-byte
    // elements 12 stages take two rounds instead of three, 7 one instead of
    // two, and no count grows.
    static constexpr int post_bits() { return LR == 5 && sizeof(C) == 4 ? pre_bits<C>() : 0; }

    // stages and store phase of one item of a kind known at compile time
    template <bool ADJ, int KIND, int ORD = ORDER_DYADIC>
    static __device__ __forceinline__ void finish_kind(const Item &it, const LaunchArgs &a,
                                                       C *lds, int t)
    {
        constexpr bool BR = ORD != ORDER_NATURAL;  // first-pass runs bit-reversed
        S *out = static_cast<S *>(a.out);
        C *inter = static_cast<C *>(a.inter);
        const C sc = ortho_scale<C>(it.m);
        const bool ortho = a.ortho != 0;
        if constexpr (KIND == KIND_TURN) {
            if constexpr (!ADJ && ORD == ORDER_DYADIC) finish_turn(it, a, lds, t);
        } else if constexpr (KIND == KIND_BLOCKS) {
            const int64_t *list = it.list >= 0 ? a.list + it.list : nullptr;
            if constexpr (ORD == ORDER_DYADIC) {
                if (a.rounds > 1) {
                    blocks_rounds<ADJ>(it, a, lds, t);
                    return;
                }
            }
            if constexpr (!ADJ) rounds<false>(lds, it.bits, t);
            else rounds<true, 0, post_bits()>(lds, it.bits, t);
            if constexpr (!ADJ && ORD == ORDER_DYADIC)
                store_paley<NT_OUT, S>(lds, out, it.io_off, it.bits, it.count, list, t, sc, ortho);
            else if constexpr (!ADJ)
                blocks_ordered<ORD, false>(lds, out, it.io_off, it.bits, it.count, list, t, sc, ortho);
            else store_contig<NT_OUT, S, post_bits()>(lds, out, it.io_off, it.bits, it.count, list, t,
                                                      sc, ortho, SignCtx{a.signs, 0, a.sign_shared},
                                                      it.bits);
        } else if constexpr (is_first_kind(KIND)) {
            constexpr int CC = rows_of<KIND>();
            if constexpr (!ADJ && merge_ok<CC, BR>()) {
                constexpr int P = first_pre<CC, BR>();
                static_assert(L::rounds_from(P) >= 1 && K - CC - merge_stages<CC>() - P <= LR,
                              "one register round between the loaded vectors and the store");
                rounds_ct<false, K - CC - merge_stages<CC>(), 0, P>(lds, t);
                store_transp_merged<CC>(lds, inter, first_base<CC>(it, a), it.h0, it.rs, t);
                return;
            }
            if constexpr (!ADJ) {
                rounds_ct<false, K - CC>(lds, t);
                store_transp<CC, BR>(lds, inter, first_base<CC>(it, a), it.h0, it.rs, t);
            } else {
                rounds_ct<true, gather_nst<CC, BR>(), 0, post_bits()>(lds, t);
                store_contig<NT_OUT, S, post_bits()>(lds, out, it.io_off, K, 1, nullptr, t, sc, ortho,
                                                     first_signs<CC>(it, a), K);
            }
        } else {
            if constexpr (!ADJ) rounds<false>(lds, it.bits, t);
            else rounds<true, 0, post_bits()>(lds, it.bits, t);
            if constexpr (!ADJ && ORD == ORDER_DYADIC)
                store_paley<NT_OUT, S>(lds, out, it.io_off, it.bits, it.count, nullptr, t, sc, ortho);
            else if constexpr (!ADJ)
                last_ordered<ORD, false>(lds, out, it, t, sc, ortho);
            else store_contig<NT_INTER, C, post_bits()>(lds, inter, last_base(it, a), it.bits, it.count,
                                                        nullptr, t, C(1), false, SignCtx{nullptr, 0, 0},
                                                        it.bits);
        }
    }

    // ---- a round boundary of a two-pass signal (signed rounds, forward) -------
    // A 2^15-element tile of consecutive last-pass blocks of round r holds,
    // after the round's remaining stages, round r's output for 2^15
    // consecutive positions -- 2^CC whole first-pass rows of round r + 1.
    // turn_round0 takes round r + 1's first register round straight from that
    // state: thread t reads the 2^LR consecutive output positions its register
    // round covers through the last pass's Paley map, runs round r's last LR
    // stages, scales the values, applies round r + 1's diagonal, runs round
    // r + 1's first stages and writes the values back in natural order; the
    // remaining register rounds and the transposed store follow as in a
    // first-pass tile.  Operands and their order are those of a last-pass
    // store, a reload and a first-pass load, so the numbers are the same, with
    // one HBM pass fewer.

    // Sign bits of n <= 64 consecutive positions starting at bit b0 of the
    // diagonal (as many words as the window touches).
    static __device__ __forceinline__ uint64_t sign_window(const uint32_t *w, int64_t b0, int n)
    {
        const int64_t w0 = b0 >> 5, w1 = (b0 + n - 1) >> 5;
        uint64_t lo = w[w0];
        if (w1 > w0) lo |= (uint64_t)w[w0 + 1] << 32;
        const int sh = (int)(b0 & 31);
        uint64_t r = lo >> sh;
        if (w1 > w0 + 1) r |= (uint64_t)w[w0 + 2] << (64 - sh);
        return r;
    }

    // Register i of thread t holds tile element brev_low(o0 + i, bits): its
    // register bits b are tile bits bits - 1 - b, so the last LR stages of
    // round r (tile bits bits - LR .. bits - 1, in that order) run here too,
    // on register bits LR - 1 .. 0, before the scale and the diagonal.
    // B > 0: the block size is 2^B, known at compile time (the register
    // offsets become immediates); B = 0: it.bits at run time.
    template <int B = 0>
    static __device__ __forceinline__ void turn_round0(const Item &it, const LaunchArgs &a,
                                                       int nst, C *lds, int t)
    {
        const int bits = B ? B : it.bits;
        const int o0 = t << LR;  // register round 0: positions o0 .. o0 + R - 1
        const At rb(lds, L::pad(brev_low(o0, bits)));
        C v[R];
#pragma unroll
        for (int i = 0; i < R; ++i) v[i] = rb[L::pad(brev_low(i, bits))];
        __syncthreads();
#pragma unroll
        for (int b = LR - 1; b >= 0; --b) bfly(v, b);
        const C sc = ortho_scale<C>(it.m);
        const bool ortho = a.ortho != 0;
        const uint64_t sb = a.signs ? sign_window(a.signs, a.sign_shared ? it.io_off - it.sig_off + o0
                                                                         : it.io_off + o0, R)
                                    : 0ull;
#pragma unroll
        for (int i = 0; i < R; ++i) {
            C x = v[i];
            if (ortho) x = scale_mul(x, sc);
            v[i] = apply_sign(x, (uint32_t)(sb >> i) & 1u);
        }
#pragma unroll
        for (int bit = 0; bit < LR; ++bit)
            if (bit < nst) bfly(v, bit);
        C *wb = lds + L::pad(o0);
#pragma unroll
        for (int i = 0; i < R; ++i) wb[L::pad(i)] = v[i];
        __syncthreads();
    }

    // A round-boundary tile loads the intermediate contiguously and runs the
    // stages below min(turn_pre(), bits - LR) on the loaded vectors (both
    // load forms), so round r's remaining early stages start at that bit:
    // with 2^5 registers and 2^12-element last-pass blocks, stages 2 .. 6 in
    // one register round instead of 0 .. 6 in two.  (With 2^6 registers those
    // stages fit one round from bit 0 already.)
    static constexpr int turn_pre() { return LR == 5 ? pre_bits<C>() : 0; }

    template <int CC, int B>
    static __device__ __forceinline__ void finish_turn_cc(const Item &it, const LaunchArgs &a,
                                                          C *lds, int t)
    {
        static_assert(L::flo(0) == 0 && L::J >= 2, "register round 0 covers tile bits 0 .. LR - 1");
        // round r's stages below the last LR
        if constexpr (B > 0) rounds_ct<false, B - LR, 0, turn_pre()>(lds, t);
        else rounds<false, 0, turn_pre()>(lds, it.bits - LR, t);
        turn_round0<B>(it, a, K - CC, lds, t);
        const int64_t base = a.inter2_is_io ? it.sig_off
                                            : it.ws_off - ((int64_t)it.h0 << (K - CC));
        if constexpr (merge_ok<CC, true>()) {
            // round r + 1's stages LR .. L1 - 1: a register round for those
            // below the merged ones (2^6 rows: stage 5), then the merged store
            if constexpr (K - CC - merge_stages<CC>() > LR)
                rounds_ct<false, K - CC - merge_stages<CC>(), 1>(lds, t);
            store_transp_merged<CC>(lds, static_cast<C *>(a.inter2), base, it.h0, it.rs, t);
        } else {
            rounds_ct<false, K - CC, 1>(lds, t);
            store_transp<CC, true>(lds, static_cast<C *>(a.inter2), base, it.h0, it.rs, t);
        }
    }

    // The adjoint's round boundary runs the other way: round r's adjoint
    // first pass (transposed gather from the intermediate, stages L1 - 1 .. 0)
    // leaves round r's output for 2^15 consecutive positions in natural order;
    // scaled and multiplied by D_r, it moves to the tile elements the last
    // pass's Paley gather would have put it at, and the tile continues as
    // round r - 1's adjoint last-pass tile (stages down to L1, contiguous store
    // to the next intermediate).

    // Register rounds J - 1 .. 1 of an adjoint pass (register round 0, tile
    // bits 0 .. LR - 1, left out).
    template <int j>
    static __device__ __forceinline__ void rounds_down_to1(C *lds, int nst, int t)
    {
        if constexpr (j >= 1) {
            round<j, true>(lds, nst, t);
            rounds_down_to1<j - 1>(lds, nst, t);
        }
    }

    // The middle of the adjoint's round boundary in one register round: thread
    // t takes the 2^LR consecutive positions of register round 0, runs round
    // r's last adjoint first-pass stages (tile bits LR - 1 .. 0), scales and
    // applies D_r, runs round r - 1's first adjoint last-pass stages (tile bits
    // bits - 1 .. bits - LR of the Paley-gathered tile, which are register bits
    // 0 .. LR - 1) and writes the values at their Paley-gathered places.
    template <int B = 0>
    static __device__ __forceinline__ void turn_round_adj(const Item &it, const LaunchArgs &a,
                                                          C *lds, int t)
    {
        const int bits = B ? B : it.bits;
        const int o0 = t << LR;
        const C *nb = lds + L::pad(o0);
        C v[R];
#pragma unroll
        for (int i = 0; i < R; ++i) v[i] = nb[L::pad(i)];
        __syncthreads();
#pragma unroll
        for (int b = LR - 1; b >= 0; --b) bfly(v, b);
        const C sc = ortho_scale<C>(it.m);
        const bool ortho = a.ortho != 0;
        const uint64_t sb = a.signs ? sign_window(a.signs, a.sign_shared ? it.io_off - it.sig_off + o0
                                                                         : it.io_off + o0, R)
                                    : 0ull;
#pragma unroll
        for (int i = 0; i < R; ++i) {
            C x = v[i];
            if (ortho) x = scale_mul(x, sc);
            v[i] = apply_sign(x, (uint32_t)(sb >> i) & 1u);
        }
#pragma unroll
        for (int b = 0; b < LR; ++b) bfly(v, b);
        const At wb(lds, L::pad(brev_low(o0, bits)));
#pragma unroll
        for (int i = 0; i < R; ++i) wb[L::pad(brev_low(i, bits))] = v[i];
        __syncthreads();
    }

    // signal base of the intermediate the adjoint boundary gathers from
    template <int CC>
    static __device__ __forceinline__ int64_t turn_adj_src(const Item &it, const LaunchArgs &a)
    {
        return a.inter_is_io ? it.sig_off : it.ws_off - ((int64_t)it.h0 << (K - CC));
    }

    template <int CC>
    static __device__ __forceinline__ void run_turn_adj_cc(const Item &it, const LaunchArgs &a,
                                                           C *lds, int t)
    {
        load_transp<CC, true>(lds, static_cast<const C *>(a.inter), turn_adj_src<CC>(it, a),
                              it.h0, it.rs, t);
        __syncthreads();
        finish_turn_adj<CC>(it, a, lds, t);
    }

    // the adjoint boundary after its transposed gather (B as in turn_round0)
    template <int CC, int B>
    static __device__ __forceinline__ void finish_turn_adj_b(const Item &it, const LaunchArgs &a,
                                                             C *lds, int t)
    {
        static_assert(L::flo(0) == 0 && L::J >= 2, "register round 0 covers tile bits 0 .. LR - 1");
        const int bits = B ? B : it.bits;
        // round r: stages L1 - 1 .. LR, those the gather left (none for 2^7
        // rows, whose merged stages are exactly these)
        if constexpr (gather_nst<CC, true>() > LR) rounds_down_to1<J - 1>(lds, gather_nst<CC, true>(), t);
        turn_round_adj<B>(it, a, lds, t);
        // round r - 1: stages bits - LR - 1 .. 0, those below post_bits() on
        // the stored vectors
        if constexpr (B > 0) rounds_ct<true, B - LR, 0, post_bits()>(lds, t);
        else rounds<true, 0, post_bits()>(lds, bits - LR, t);
        store_contig<NT_INTER, C, post_bits()>(lds, static_cast<C *>(a.inter2),
                                               a.inter2_is_io ? it.io_off : it.ws_off, bits,
                                               it.count, nullptr, t, C(1), false,
                                               SignCtx{nullptr, 0, 0}, bits - LR);
    }

    // Round-boundary tiles with block sizes known at compile time.  A tile
    // of 2^CC rows has L1 = K - CC and blocks of 2^bits = 2^(m - L1) with
    // 8 <= bits <= K (the planner makes no other round-boundary tile, and the
    // plan check rejects others), so with 2^7 rows (the
    // default split of signals of 2^16 .. 2^23) every block size has a form
    // of its own; with 2^6 and 2^5 rows, the default splits' 2^15 (signals of
    // 2^24 and 2^25) has one and other sizes take it at run time; 2^3 rows
    // (forced splits only) take it at run time.
    template <int CC>
    static constexpr int turn_bits_lo() { return CC == CA ? 8 : (CC == CD || CC == CM) ? K : K + 1; }
    template <int CC, int B = turn_bits_lo<CC>()>
    static __device__ __forceinline__ void finish_turn_adj(const Item &it, const LaunchArgs &a,
                                                           C *lds, int t)
    {
        if constexpr (B > K) {
            finish_turn_adj_b<CC, 0>(it, a, lds, t);
        } else if constexpr (B == K && CC == CA) {
            finish_turn_adj_b<CC, K>(it, a, lds, t);  // bits 8 .. K - 1 taken above
        } else {
            if (it.bits == B) finish_turn_adj_b<CC, B>(it, a, lds, t);
            else finish_turn_adj<CC, B + 1>(it, a, lds, t);
        }
    }
    template <int CC, int B = turn_bits_lo<CC>()>
    static __device__ __forceinline__ void finish_turn_bits(const Item &it, const LaunchArgs &a,
                                                            C *lds, int t)
    {
        if constexpr (B > K) {
            finish_turn_cc<CC, 0>(it, a, lds, t);
        } else if constexpr (B == K && CC == CA) {
            finish_turn_cc<CC, K>(it, a, lds, t);  // bits 8 .. K - 1 taken above
        } else {
            if (it.bits == B) finish_turn_cc<CC, B>(it, a, lds, t);
            else finish_turn_bits<CC, B + 1>(it, a, lds, t);
        }
    }

    static __device__ __forceinline__ void run_turn_adj(const Item &it, const LaunchArgs &a,
                                                        C *lds, int t)
    {
        if constexpr (K >= 15) {
            const int cc = K - (it.m - it.bits);
            if (cc == CA) run_turn_adj_cc<CA>(it, a, lds, t);
            else if (cc == CM) run_turn_adj_cc<CM>(it, a, lds, t);
            else if (cc == CD) run_turn_adj_cc<CD>(it, a, lds, t);
            else if (cc == CB) run_turn_adj_cc<CB>(it, a, lds, t);
        }
    }

    static __device__ __forceinline__ void finish_turn(const Item &it, const LaunchArgs &a,
                                                       C *lds, int t)
    {
        if constexpr (K >= 15) {
            const int cc = K - (it.m - it.bits);
            if (cc == CA) finish_turn_bits<CA>(it, a, lds, t);
            else if (cc == CM) finish_turn_bits<CM>(it, a, lds, t);
            else if (cc == CD) finish_turn_bits<CD>(it, a, lds, t);
            else if (cc == CB) finish_turn_bits<CB>(it, a, lds, t);
        }
    }

    // A forward last-pass tile whose output takes the diagonal a.signs at the
    // store, after the scale: the last launch of a signed adjoint run through
    // the forward launches (D_1 H D_2 H ... D_k H g, the last H's output
    // times D_1).  One workgroup per tile.
    static __device__ __forceinline__ void last_signed(const Item &it, const LaunchArgs &a,
                                                       C *lds, int t)
    {
        load_contig<NT_INTER, C>(lds, static_cast<const C *>(a.inter), last_base(it, a), it.bits,
                                 it.count, nullptr, t);
        __syncthreads();
        rounds<false>(lds, it.bits, t);
        store_paley<NT_OUT, S, true>(lds, static_cast<S *>(a.out), it.io_off, it.bits, it.count,
                                     nullptr, t, ortho_scale<C>(it.m), a.ortho != 0,
                                     SignCtx{a.signs, it.io_off - it.sig_off, a.sign_shared});
    }

    template <bool ADJ, int ORD = ORDER_DYADIC>
    static __device__ __forceinline__ void finish_item(const Item &it, const LaunchArgs &a,
                                                       C *lds, int t)
    {
        switch (it.kind) {
        case KIND_BLOCKS: finish_kind<ADJ, KIND_BLOCKS, ORD>(it, a, lds, t); break;
        case KIND_FIRST_A: finish_kind<ADJ, KIND_FIRST_A, ORD>(it, a, lds, t); break;
        case KIND_FIRST_B: finish_kind<ADJ, KIND_FIRST_B, ORD>(it, a, lds, t); break;
        case KIND_FIRST_C: finish_kind<ADJ, KIND_FIRST_C, ORD>(it, a, lds, t); break;
        case KIND_FIRST_D: finish_kind<ADJ, KIND_FIRST_D, ORD>(it, a, lds, t); break;
        case KIND_LAST: finish_kind<ADJ, KIND_LAST, ORD>(it, a, lds, t); break;
        default: break;
        }
    }

    // ---- single-pass 2^12-element tiles with 2^5 registers ---------------------
    // A 16-byte vector of the contiguous load holds every value of tile bits
    // [0, lv), lv = log2 of its element count: stages 0 .. lv - 1 run on the
    // loaded vectors and the register rounds cover bits [lv, 12) -- two rounds
    // instead of three, one LDS round trip fewer.  Same stages, operands and
    // order as the plain rounds, so the same bits.  (The forward round-boundary
    // tiles do the same with their first two stages, see turn_pre; other tile
    // shapes would keep their round count, so they load plainly.)

    // log2 of the elements of type T in one 16-byte vector
    template <typename T>
    static constexpr int pre_bits()
    {
        return Vec<T>::V == 8 ? 3 : Vec<T>::V == 4 ? 2 : Vec<T>::V == 2 ? 1 : 0;
    }
    template <bool ADJ, int ORD>
    static constexpr bool pre_ok()
    {
        return !ADJ && ORD == ORDER_DYADIC && K == 12 && LR == 5 && sizeof(C) == 4 &&
               L::rounds_from(pre_bits<S>()) < J;
    }

    static __device__ __forceinline__ void blocks_pre(const Item &it, const LaunchArgs &a,
                                                      C *lds, int t)
    {
        constexpr int P = pre_bits<S>();
        const int64_t *list = it.list >= 0 ? a.list + it.list : nullptr;
        load_contig<NT_IN, S, P>(lds, static_cast<const S *>(a.in), it.io_off, it.bits, it.count,
                                 list, t, SignCtx{a.signs, 0, a.sign_shared}, it.bits);
        __syncthreads();
        rounds<false, 0, P>(lds, it.bits, t);
        store_paley<NT_OUT, S>(lds, static_cast<S *>(a.out), it.io_off, it.bits, it.count, list, t,
                               ortho_scale<C>(it.m), a.ortho != 0);
    }

    template <bool ADJ, int ORD = ORDER_DYADIC>
    static __device__ __forceinline__ void run_item(const Item &it, const LaunchArgs &a,
                                                    C *lds, int t)
    {
        if constexpr (pre_ok<ADJ, ORD>()) {
            if (it.kind == KIND_BLOCKS && a.rounds <= 1) {
                blocks_pre(it, a, lds, t);
                return;
            }
        }
        load_item<ADJ, ORD>(it, a, lds, t);
        __syncthreads();
        finish_item<ADJ, ORD>(it, a, lds, t);
    }

    // ---- prefetching (streaming) form ------------------------------------------
    // A launch whose items are all full tiles of one kind (no block lists) can
    // fetch the next item's 16-byte vectors into registers while the current
    // item runs its stages and stores.  The tile's source is either the input
    // (storage type S) or the intermediate (compute type C):
    //   forward BLOCKS / FIRST : input, contiguous        -> LDS contiguous
    //   forward LAST / TURN    : intermediate, contiguous -> LDS contiguous
    //   adjoint BLOCKS / LAST  : input, contiguous        -> LDS Paley positions
    //   adjoint FIRST          : intermediate, transposed -> LDS transposed
    // and the LDS placement is exactly the one of load_item.  Global addresses
    // are a uniform base per vector iteration plus one 32-bit per-thread offset.
    template <bool ADJ, int KIND>
    static constexpr bool src_inter()
    {
        return ADJ ? is_first_kind(KIND) : (KIND == KIND_LAST || KIND == KIND_TURN);
    }
    template <bool ADJ, int KIND>
    using SrcT = typename std::conditional<src_inter<ADJ, KIND>(), C, S>::type;
    template <bool ADJ, int KIND>
    static constexpr int nraw() { return N / (Vec<SrcT<ADJ, KIND>>::V * NT); }

    template <bool ADJ, int KIND>
    static __device__ __forceinline__ void stream_fetch(const Item &it, const LaunchArgs &a,
                                                        u32x4 *raw, uint32_t *sw, int t)
    {
        using T = SrcT<ADJ, KIND>;
        constexpr int V = Vec<T>::V, NV = nraw<ADJ, KIND>();
        if constexpr (ADJ && src_inter<ADJ, KIND>()) {
            constexpr int CC = rows_of<KIND>();
            const C *base = static_cast<const C *>(a.inter) + first_base<CC>(it, a) + it.h0;
            const uint32_t toff =
                (uint32_t)L::template transp_goff<CC>(V * gather_q<CC, true>(t, 0), it.rs);
#pragma unroll
            for (int k = 0; k < NV; ++k) {
                const C *pk = base + L::template transp_goff<CC>(V * gather_q<CC, true>(0, k), it.rs);
                raw[k] = ld16<NT_INTER>(pk + toff);
            }
        } else {
            const T *base;
            if constexpr (src_inter<ADJ, KIND>()) base = static_cast<const C *>(a.inter) + last_base(it, a);
            else base = static_cast<const S *>(a.in) + it.io_off;
            const uint32_t toff = (uint32_t)(V * t);
#pragma unroll
            for (int k = 0; k < NV; ++k) raw[k] = ld16<src_inter<ADJ, KIND>() ? NT_INTER : NT_IN>(base + V * NT * k + toff);
            if constexpr (!ADJ && !src_inter<ADJ, KIND>()) {
                // forward input tiles: sign bits of the diagonal, if any
                if (a.signs) {
                    const int bits = KIND == KIND_BLOCKS ? it.bits : K;
                    const SignCtx sg{a.signs, KIND == KIND_BLOCKS ? 0 : (int64_t)it.h0 << (K - rows_of<KIND>()),
                                     a.sign_shared};
#pragma unroll
                    for (int k = 0; k < NV; ++k) {
                        const int e0 = V * t + V * NT * k;
                        sw[k] = sign_bits(sg, it.io_off + e0, e0 & ((1 << bits) - 1));
                    }
                }
            }
        }
    }

    template <bool ADJ, int KIND, int ORD = ORDER_DYADIC>
    static __device__ __forceinline__ void stream_put(const Item &it, const LaunchArgs &a,
                                                      const u32x4 *raw, const uint32_t *sw,
                                                      C *lds, int t)
    {
        using T = SrcT<ADJ, KIND>;
        constexpr int V = Vec<T>::V, NV = nraw<ADJ, KIND>();
        if constexpr (!ADJ) {
            const At lb(lds, L::pad(V * t));
#pragma unroll
            for (int k = 0; k < NV; ++k) {
                C vals[V];
                Vec<T>::decode(raw[k], vals);
                if constexpr (!src_inter<ADJ, KIND>()) {
                    if (a.signs) {
#pragma unroll
                        for (int u = 0; u < V; ++u) vals[u] = apply_sign(vals[u], (sw[k] >> u) & 1u);
                    }
                }
                if constexpr (KIND == KIND_TURN) pre_stages<V, turn_pre()>(vals, it.bits - LR);
                if constexpr (is_first_kind(KIND)) {
                    constexpr int P = first_pre<rows_of<KIND>(), ORD != ORDER_NATURAL>();
                    if constexpr (P > 0) pre_stages_n<V, P>(vals);
                }
#pragma unroll
                for (int u = 0; u < V; ++u) lb[L::pad(V * NT * k) + u] = vals[u];
            }
        } else if constexpr (src_inter<ADJ, KIND>()) {
            constexpr int CC = rows_of<KIND>();
            C vals[NV][V];
#pragma unroll
            for (int k = 0; k < NV; ++k) Vec<C>::decode(raw[k], vals[k]);
            put_gather<CC, true>(lds, vals, t);
        } else {
            const int bits = it.bits;
            if (bits == K) {
                const At lb(lds, L::pad((int)rbrev((uint32_t)(V * t), K)));
#pragma unroll
                for (int k = 0; k < NV; ++k) {
                    C vals[V];
                    Vec<T>::decode(raw[k], vals);
#pragma unroll
                    for (int u = 0; u < V; ++u)
                        lb[L::pad((int)cbrev((uint32_t)(V * NT * k + u), K))] = vals[u];
                }
            } else {
                C *lb = lds + L::pad(brev_low(V * t, bits));
                int ul[V];
#pragma unroll
                for (int u = 0; u < V; ++u) ul[u] = L::pad(brev_low(u, bits));
#pragma unroll
                for (int k = 0; k < NV; ++k) {
                    C vals[V];
                    Vec<T>::decode(raw[k], vals);
                    const int kl = L::pad(brev_low(V * NT * k, bits));
#pragma unroll
                    for (int u = 0; u < V; ++u) lb[kl + ul[u]] = vals[u];
                }
            }
        }
    }
};

}  // namespace chw
