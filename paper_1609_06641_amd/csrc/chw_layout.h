// chw_layout.h -- index maps of the CHW tile engine (host and device).
//
// A tile is N = 2^K elements held in LDS as the compute type (FP32, int32 or
// FP64), at padded word address pad(e) = e + (e >> P1) + (e >> P2), e = tile
// element.  A workgroup of NT = 2^(K-LR) threads processes it; in each
// "round" a thread holds R = 2^LR elements in registers.
//
// The two padding shifts and the lane order of the transposed phase were
// chosen with the bank rule measured on gfx950 for 4-byte LDS accesses: 32
// banks (word address mod 32), each half-wave (lanes 0-31, 32-63) served on
// its own.  With one word of padding every 2^5 and every 2^10 elements, no
// half-wave access of any phase of a compiled FP32 / int32 tile (register
// rounds, contiguous, Paley, transposed) puts two distinct words into one bank
// (the self-check reports the figures for every phase).
//
// Stage t of the cascade is the set of Haar levels at depth t: after stages
// 0..t-1 every element has been combined over input index bits 0..t-1, and
// stage t pairs the elements that differ in bit t (the element with the bit
// clear takes the sum, the other the difference), exactly the butterflies the
// Haar transforms of Sec. 2 / Theorem 1 perform at that depth.  Stages run
// in increasing t (forward) or decreasing t (adjoint).  Inside a tile, tile
// bit b is signal bit b (single-pass tiles, first-pass rows) or signal bit
// L1 + b (last-pass blocks).
//
// Every map below is a bit permutation of (thread, register/vector, unrolled
// iteration) fields that occupy disjoint bits, so
//     pad(a | b) = pad(a) + pad(b)   for disjoint a, b
// and each LDS access is one per-thread base plus a compile-time offset.
#pragma once
#include <stdint.h>

#if defined(__HIPCC__) || defined(__HIP__)
#define CHW_HD __host__ __device__ __forceinline__
#else
#define CHW_HD inline
#endif

// Padding shifts of the tile layout (pad() below); overridable at build time
// to compare layouts.
#ifndef CHW_PAD1
#define CHW_PAD1 5
#endif
#ifndef CHW_PAD2_15
#define CHW_PAD2_15 10
#endif
#ifndef CHW_PAD2_12
#define CHW_PAD2_12 10
#endif

namespace chw {

constexpr uint32_t cbrev(uint32_t v, int bits)
{
    uint32_t r = 0;
    for (int i = 0; i < bits; ++i) r = (r << 1) | ((v >> i) & 1u);
    return r;
}

CHW_HD uint32_t rbrev(uint32_t v, int bits)
{
#if defined(__HIP_DEVICE_COMPILE__)
    return bits ? (__builtin_bitreverse32(v) >> (32 - bits)) : 0u;
#else
    return cbrev(v, bits);
#endif
}

template <int K_, int LR_>
struct Layout {
    static constexpr int K = K_, LR = LR_;
    static constexpr int N = 1 << K, R = 1 << LR;
    static constexpr int LNT = K - LR, NT = 1 << LNT;
    static constexpr int J = (K + LR - 1) / LR;          // register rounds (from bit 0)
    // padding shifts: one word after every 2^P1 and every 2^P2 elements
    static constexpr int P1 = CHW_PAD1, P2 = K >= 15 ? CHW_PAD2_15 : CHW_PAD2_12;
    static_assert(LR >= 3 && LNT >= 6, "tile needs >= 8 registers and >= 1 wave");

    static CHW_HD constexpr int pad(int e) { return e + (e >> P1) + (e >> P2); }
    static constexpr int LDS_WORDS = pad(N - 1) + 1;

    // ---- register rounds -------------------------------------------------
    // Round j makes active the tile bits [alo(j), ahi(j)); the register field
    // is [flo(j), flo(j) + LR) (the last round's field is moved down so that it
    // stays inside the tile and holds R elements).  With B0 > 0 the rounds
    // start at tile bit B0: the stages below it ran on the loaded vectors
    // before the tile reached LDS.
    static CHW_HD constexpr int rounds_from(int B0) { return (K - B0 + LR - 1) / LR; }
    static CHW_HD constexpr int alo(int j, int B0 = 0) { return B0 + j * LR; }
    static CHW_HD constexpr int ahi(int j, int B0 = 0)
    {
        return B0 + (j + 1) * LR < K ? B0 + (j + 1) * LR : K;
    }
    static CHW_HD constexpr int flo(int j, int B0 = 0)
    {
        return B0 + j * LR < K - LR ? B0 + j * LR : K - LR;
    }
    // tile element of (thread t, register 0) in round j: thread bits fill the
    // tile bits outside the register field, low to high
    static CHW_HD constexpr int round_tbase(int j, int t, int B0 = 0)
    {
        return (t & ((1 << flo(j, B0)) - 1)) | ((t >> flo(j, B0)) << (flo(j, B0) + LR));
    }
    static CHW_HD constexpr int round_reg(int j, int i, int B0 = 0) { return i << flo(j, B0); }

    // ---- contiguous phase (16-byte vectors of V elements) -----------------
    // vector q = t + NT*k covers tile elements [q*V, q*V + V)
    template <int V>
    static CHW_HD constexpr int contig_e(int t, int k, int u) { return V * t + V * NT * k + u; }

    // ---- bit-reversed phase: output position o = (blk << bits) | p holds
    // tile element (blk << bits) | bitrev_bits(p) ----------------------------
    template <int V>
    static CHW_HD int bitrev_e(int t, int k, int u, int bits)
    {
        int o = V * t + V * NT * k + u;
        int blk = o >> bits;
        int p = o & ((1 << bits) - 1);
        return (blk << bits) | (int)rbrev((uint32_t)p, bits);
    }

    // ---- transposed phase of a first-pass tile: 2^C rows of 2^L1 elements,
    // tile element e = (hl << L1) | lo; output o (within the tile) = (rho << C)
    // | hl where rho = bitrev_L1(lo) indexes the output run of 2^C elements.
    // Output vector q = o / V is handled by thread t, iteration k with
    // q = transp_q(t + NT * k): the low transp_keep lane bits keep consecutive
    // vectors (eight: a 128-byte line, one run of 32 FP32 rows; sixteen for
    // runs of 64 FP32 rows, so that a wave stores four whole 256-byte runs),
    // and the bits above are rotated by transp_rot so that one wave access
    // spreads over the LDS banks.  A bit permutation keeps q(t | NT k) = q(t)
    // | q(NT k). ---
    template <int V, int C>
    static CHW_HD constexpr int transp_keep() { return V == 4 && C == 6 ? 4 : 3; }
    template <int V, int C>
    static CHW_HD constexpr int transp_rot()
    {
        // (K, V, C) -> rotation found with the bank rule above for the
        // compiled row counts (V = 2: the FP64 tiles, 2^12 elements only)
        if constexpr (K >= 15)
            return V == 4 ? (C == 6 ? 3 : C == 5 ? 3 : C == 3 ? 1 : 0) : 0;
        else
            return V == 4 ? (C == 6 ? 3 : C == 4 ? 2 : C == 3 ? 1 : 0) : (C == 4 ? 4 : 0);
    }
    template <int V, int C>
    static CHW_HD constexpr int transp_q(int n)
    {
        constexpr int lv = V == 8 ? 3 : V == 4 ? 2 : V == 2 ? 1 : 0;
        constexpr int kb = transp_keep<V, C>();
        constexpr int W = K - lv - kb, r = transp_rot<V, C>();
        if constexpr (W <= 0 || r == 0 || r >= W) {
            return n;
        } else {
            const int f = (n >> kb) & ((1 << W) - 1);
            const int g = ((f << r) | (f >> (W - r))) & ((1 << W) - 1);
            return (n & ((1 << kb) - 1)) | (g << kb);
        }
    }
    // BR = false: the natural-order variant, run rho holds row element rho
    // itself (no bit reversal)
    template <int V, int C, bool BR = true>
    static CHW_HD int transp_e(int t, int k, int u)
    {
        constexpr int L1 = K - C;
        int o = V * transp_q<V, C>(t + NT * k) + u;
        int hl = o & ((1 << C) - 1);
        int rho = o >> C;
        return (hl << L1) | (BR ? (int)rbrev((uint32_t)rho, L1) : rho);
    }
    // Merged variant (first-pass store that also runs the row's top stages):
    // the R / V vectors of a thread differ in the low run-index bits, i.e. in
    // row-element bits L1 - 1 .. L1 - log2(R / V), so the stages on those bits
    // run in registers before the store.  Thread bits below C - lv pick the
    // vector inside a run (lanes keep whole runs); the thread bits above go
    // above the run-index bits that k takes.
    template <int V, int C>
    static CHW_HD constexpr int transpm_q(int t, int k)
    {
        constexpr int lv = V == 8 ? 3 : V == 4 ? 2 : V == 2 ? 1 : 0;
        constexpr int wr = C - lv, nk = LR - lv;
        return (t & ((1 << wr) - 1)) | (k << wr) | ((t >> wr) << (wr + nk));
    }
    template <int V, int C>
    static CHW_HD int transpm_e(int t, int k, int u)
    {
        constexpr int L1 = K - C;
        int o = V * transpm_q<V, C>(t, k) + u;
        int hl = o & ((1 << C) - 1);
        int rho = o >> C;
        return (hl << L1) | (int)rbrev((uint32_t)rho, L1);
    }
    // element offset (relative to the signal base + h0) of output o, given the
    // run stride 2^rs of the transposed layout
    template <int C>
    static CHW_HD int64_t transp_goff(int o, int rs)
    {
        return ((int64_t)(o >> C) << rs) + (o & ((1 << C) - 1));
    }
};

}  // namespace chw
