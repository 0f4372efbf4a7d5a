// chw_types.h -- plain structs shared by the host planner and the kernels.
#pragma once
#include <stdint.h>

namespace chw {

enum DType : int { DT_F32 = 0, DT_BF16 = 1, DT_F16 = 2, DT_I32 = 3, DT_F64 = 4 };

// Work item kinds.  A work item is one tile (one workgroup's worth of work).
enum ItemKind : int32_t {
    // Whole signals (or last-pass blocks) of 2^bits <= 2^K elements, 2^(K-bits)
    // of them per tile: all stages of the block, Paley-ordered store.
    KIND_BLOCKS = 0,
    // First HBM pass of a large signal with the tile's variant-A row count:
    // 2^CA rows of 2^(K-CA) contiguous elements, stages 0..K-CA-1, stored in
    // the cascade's own layout after those stages (transposed, FP32/compute
    // type intermediate).
    KIND_FIRST_A = 1,
    // Same with the variant-B row count 2^CB.
    KIND_FIRST_B = 2,
    // Last HBM pass: blocks of 2^bits contiguous intermediate elements (the
    // remaining CHW_{m-L1} on each block), Paley-ordered store.
    KIND_LAST = 3,
    // First HBM pass with the middle row count 2^CM (K15_CM / K12_CM below).
    KIND_FIRST_C = 4,
    // Persistent launch: a whole multi-pass signal (first-pass tiles with the
    // variant-A / variant-B row count, then its last-pass tiles) run by one
    // workgroup.
    KIND_SIGNAL_A = 5,
    KIND_SIGNAL_B = 6,
    // Round boundary of a signed multi-round call (forward, 2^15-element
    // tiles): the last pass of round r on 2^(15-bits) consecutive blocks of the
    // intermediate `inter`, then, on the same 2^15 output positions, round
    // r + 1's diagonal and first pass (2^CC rows, CC = 15 - (m - bits)),
    // stored transposed into `inter2`.  Fields as KIND_LAST, plus h0 (first
    // row of the tile) and rs (= bits).
    KIND_TURN = 7,
    // First HBM pass with 2^6 rows in 2^15-element tiles (256-byte FP32
    // runs): the split of 2^24 signals, whose blocks the 2^7-row tiles would
    // leave larger than a last-pass tile.
    KIND_FIRST_D = 8,
    // Persistent launch: a whole multi-pass signal whose first-pass tiles
    // have the middle row count (2^4 rows of 2^8 elements in 2^12-element
    // tiles: 64-byte FP32 runs, against 32 with the 2^3 rows of
    // KIND_SIGNAL_B), then its last-pass tiles, run by one workgroup.
    KIND_SIGNAL_C = 9,
};

constexpr bool is_signal_kind(int kind)
{
    return kind == KIND_SIGNAL_A || kind == KIND_SIGNAL_B || kind == KIND_SIGNAL_C;
}

// Coefficient order of the transform's output (forward) / input (adjoint).
// Dyadic (Paley) is the order of eq. (1); sequency (Walsh) lists the rows by
// their number of sign changes, which is the Paley row index read through the
// inverse Gray code (row p of eq. (1) has invgray(p) sign changes); natural
// (Sylvester) is the radix-2 Kronecker order, the Paley index bit-reversed.
enum Order : int { ORDER_DYADIC = 0, ORDER_SEQUENCY = 1, ORDER_NATURAL = 2 };

constexpr bool is_first_kind(int kind)
{
    return kind == KIND_FIRST_A || kind == KIND_FIRST_B || kind == KIND_FIRST_C ||
           kind == KIND_FIRST_D;
}

// Middle row count (log2) of the first-pass tiles: 2^5 rows in 2^15-element
// tiles, 2^4 rows in 2^12-element tiles (128- and 64-byte FP32 runs), for the
// splits the wide variant cannot take.
constexpr int K15_CM = 5, K12_CM = 4;
constexpr int mid_rows(int K) { return K >= 15 ? K15_CM : K12_CM; }
// Row count (log2) of the KIND_FIRST_D tiles (2^15-element tiles only; the
// 2^12-element kernels compile the kind with their middle row count and the
// planner never gives it to them).
constexpr int K15_CD = 6;
constexpr int d_rows(int K) { return K >= 15 ? K15_CD : K12_CM; }

// Slot of a prefetching kernel in a variant's tables, by item kind (BLOCKS,
// FIRST_A, FIRST_B, LAST, FIRST_C, FIRST_D); -1 for the others.
constexpr int kNumStreamSlots = 6;
constexpr int stream_slot(int kind)
{
    return kind >= KIND_BLOCKS && kind <= KIND_FIRST_C ? kind : kind == KIND_FIRST_D ? 5 : -1;
}

// 64-byte work item.  Offsets are element offsets:
//   io_off : start of the tile's contiguous chunk in x / g / y space
//            (BLOCKS, LAST: the blocks; FIRST: rows h0 .. h0 + 2^C - 1)
//   ws_off : BLOCKS: unused; FIRST: base of the signal in the intermediate
//            buffer; LAST: start of the tile's blocks in the intermediate.
// Roles by direction:
//   forward  BLOCKS : x[io] -> y[io]                (all stages, Paley store)
//            FIRST  : x[io] -> inter[ws] transposed (stages 0..L1-1)
//            LAST   : inter[ws] -> y[io]            (stages L1..m-1, Paley)
//   adjoint  BLOCKS : g[io] -> y[io]                (Paley gather, stages down)
//            LAST   : g[io] -> inter[ws]            (Paley gather, top stages)
//            FIRST  : inter[ws] transposed -> y[io] (stages L1-1..0)
// When the intermediate is y itself (out-of-place forward, no workspace) the
// kernel derives its offsets from io_off instead of ws_off.
// For BLOCKS items with list >= 0 the blocks are not consecutive: block i of
// the tile starts at element list_base[list + i] of x and y alike.
struct Item {
    int64_t io_off;
    int64_t ws_off;
    int64_t sig_off;    // first element of the item's signal (the first
                        // signal of a BLOCKS tile)
    int32_t kind;
    int32_t bits;       // BLOCKS/LAST: log2 block size (stage bits per block)
    int32_t count;      // BLOCKS/LAST: valid blocks in the tile (>= 1)
    int32_t list;       // BLOCKS: index into the block-offset list, or -1
    int32_t rs;         // FIRST: log2 stride of the transposed runs (m - L1)
    int32_t h0;         // FIRST: first row (of 2^L1 elements) of the tile
    int32_t m;          // log2 size of the whole signal (sets the scale)
    int32_t pad_[3];
};
static_assert(sizeof(Item) == 64, "Item must stay 64 bytes");

// Arguments of one launch of the item kernels.
struct LaunchArgs {
    const void *in;          // x (forward) or g (adjoint)
    void *out;               // y
    void *inter;             // intermediate between passes (workspace or y)
    int32_t inter_is_io;     // 1: inter == y, offsets follow io_off
    int32_t inter2_is_io;    // KIND_TURN: 1 when inter2 == y
    void *inter2;            // KIND_TURN: the next round's intermediate
    const Item *items;       // device array
    const int64_t *list;     // device array of block offsets (ragged BLOCKS)
    int32_t nitems;
    int32_t ortho;           // 1: scale by 2^{-m/2} at the final store
    // Random-sign diagonal D of this call's round, as packed bits (bit set:
    // the element's sign flips), or null.  Forward: y = H D x, the sign is
    // applied to the input as it is loaded; adjoint: y = D H^T g, applied to
    // the output as it is stored.  sign_shared = 1: bit j applies to element
    // j of every signal; 0: bit e applies to element e of the buffer.
    const uint32_t *signs;
    int32_t sign_shared;
    // Rounds that single-pass tiles, whole-signal (persistent) items and the
    // tiny kernel run inside this launch (>= 1; more than 1 only with signs):
    // round r uses the diagonal at signs + r * sign_words.  Two-pass tiles
    // always run one round per launch.
    int32_t rounds;
    int64_t sign_words;
};

}  // namespace chw
