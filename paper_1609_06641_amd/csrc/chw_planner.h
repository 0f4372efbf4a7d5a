// chw_planner.h -- host planner: turns a batch description into work items
// and launch ranges for the tile kernels (no device needed).
#pragma once
#include <stddef.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "chw_types.h"

namespace chw {

// Tunable choices.  Every choice computes bitwise-identical results: the
// stages always run in the same order with the same operands, and the scale is
// applied once at the final store.
struct PlanConfig {
    int lr12 = 0;       // register bits of the 2^12-element tile kernels (5, 6;
                        // 0 = 5 in single-pass launches, 6 in the others)
    int lr15 = 5;       // register bits of the 2^15-element tile kernels (5, 6)
    int single15 = 1;   // signals with 13 <= m <= 15 in one pass of a 2^15 tile
    int split_l1 = -1;  // forced first-pass level count of multi-pass signals
    int exec = 0;       // 0 = one launch per pass; 2 = one persistent launch
                        // (a workgroup runs both passes of a multi-pass
                        // signal)
    int ptile = 0;      // tile bits of the persistent launch: 12 (m <= 21,
                        // several workgroups per CU), 15 (m <= 23, one
                        // workgroup per CU, 2^7-row first passes; not FP64)
                        // or 0 = 15 where it exists, else 12
    int64_t chunk = 0;  // elements of multi-pass signals per pass pair (0 = all):
                        // the batch runs as first pass, last pass on each chunk
                        // in turn, so a chunk's intermediate can stay in the
                        // memory-side cache between its two passes
    int pipeline = 0;   // 1 (with chunk > 0): overlap the passes of successive
                        // chunks: launch j runs the last pass of chunk j - 1
                        // and the first pass of chunk j together (2^15-element
                        // tiles for both), and the chunks' intermediates take
                        // turns in two workspace slots, so a chunk's
                        // intermediate is read back soon after it is written
    int order = 0;      // coefficient order (Order): set from the plan's
                        // flags, not a tuning choice
    int spread = 1;     // 1: a launch of single-pass 2^15-element tiles that
                        // would fill fewer than kSpreadTiles tiles puts its
                        // signals one or a few per tile (partly filled tiles,
                        // more CUs busy)
    int adjoint = 0;    // chw_backward of a dyadic-order plan: 0 runs the
                        // forward launches (the Paley-ordered H is symmetric
                        // and the adjoint cascade adds the same operands in
                        // the same order, so the bits are the same); 1 runs
                        // the synthesis cascade (transposed factors, reverse
                        // order).  Signed and other-order calls always take
                        // the synthesis cascade.
    int turn = 1;       // 1: signed multi-round forward calls join round r's
                        // last pass and round r + 1's first pass in one launch
                        // of KIND_TURN tiles where the plan qualifies
    int stream = 1;     // 1: launches of full 2^15-element tiles of one kind
                        // run the prefetching kernel (a workgroup loops over
                        // items and fetches the next tile while the current
                        // one runs; one such workgroup fills a CU's LDS)
    int three_min = 26; // signals of 2^three_min elements or more run in three
                        // HBM passes (set from the plan's flags, not a tuning
                        // choice: the workspace bound depends on it).  2^26
                        // and 2^27 could take two, but only with first-pass
                        // runs of 32 bytes: 2.40 / 2.26 ms per 2^28 elements
                        // against 1.09 / 1.10 ms in three passes (2^24 and
                        // 2^25: 0.90 / 0.85 ms in two, 1.10 in three)
    int occupancy = 0;  // workgroups per CU of the looping launches (the
                        // persistent kernel, the prefetching kernels): their
                        // grid is min(items, occupancy x CUs); 0 = as many as
                        // can be resident
};

// Items [begin, end) of the plan's table run in one launch of the tile kernel
// with tile bits K and register bits LR.  Launches run in list order on one
// stream; a launch may depend on any earlier one.
struct LaunchRange {
    int K, LR;
    int begin, end;
    int persistent = 0;  // 1: one persistent launch over the range
    int stream = 0;      // prefetching launch over items of kind stream - 1
                         // (all full tiles, no block lists); 0 = one
                         // workgroup per item
    int single_pass = 0; // 1: single-pass tiles only (all rounds of a signed
                         // call run inside the launch)
    int role = 0;        // 0: tiles read / write x, y and the workspace as
                         // their kind says; 1: the middle pass of three-pass
                         // signals, whose first-pass tiles read the first
                         // intermediate (offsets io_off, in the workspace)
                         // and write the second (adjoint: the other way),
                         // in the compute type, with no scale and no signs
};

// Smallest launch of single-pass 2^15-element tiles that runs the prefetching
// form.
constexpr int kStreamBlocksMin = 1024;

// A launch of single-pass 2^15-element tiles that would fill fewer tiles than
// this (the CU count of the part) puts its signals one or a few per tile
// instead, up to this many tiles per size.
constexpr int kSpreadTiles = 256;

// Prefetching form of a launch of items [begin, end): 0 when the items are not
// all full tiles of one kind without block lists, else 1 + that kind.
int stream_source(const std::vector<Item> &items, int begin, int end, int K, bool adj);

// Two-pass split of one signal size.
struct Split {
    int m, L1, K1, CC, kind, K2;
};

// Three-pass split: a first pass over rows of 2^L1 (split `outer`, whose
// blocks of 2^(m - L1) are then too large for one last-pass tile), after which
// every block is an independent signal of 2^(m - L1) elements taken through
// the two passes of split `inner`.
struct Split3 {
    int m;
    Split outer, inner;
};

// Compute type of a dtype's kernels (the type of the intermediates): the
// middle pass of three-pass signals runs the kernels of this type.
int compute_dt(int dt);

struct BuiltPlan {
    PlanConfig cfg;
    std::vector<Item> items;
    std::vector<int64_t> list;        // block offsets of ragged BLOCKS items
    std::vector<int64_t> tiny_off;    // signals below one 16-byte vector
    std::vector<int32_t> tiny_m;
    std::vector<LaunchRange> fwd;     // launches of a forward call, in order
    std::vector<LaunchRange> adj;     // launches of a backward call, in order
    // round boundaries of signed multi-round forward calls: KIND_TURN items of
    // every two-pass signal (2^15-element tiles); empty when the plan does not
    // qualify (other orders, persistent or chunked launches, a dtype whose
    // storage is narrower than its compute type, or a two-pass signal whose
    // first pass is not in 2^15-element tiles)
    std::vector<LaunchRange> turn;
    std::vector<Split> splits;        // distinct splits in use
    std::vector<Split3> splits3;      // distinct three-pass splits in use
    size_t ws_elems = 0;              // compact intermediate of this configuration
    size_t ws_bound = 0;              // intermediate bound over every configuration
    int64_t n_single = 0, n_multi = 0, n_tiny = 0;
    int64_t n_three = 0;              // signals in three passes (counted in n_multi too)
    size_t ws3_first = 0;             // workspace element where the three-pass
                                      // signals' first intermediates begin
    size_t ws3_elems = 0;             // their elements (the second
                                      // intermediates follow at ws3_first + ws3_elems)
};

// Row counts (log2) of the first-pass variants compiled for each tile size.
// The wide variants (A) give the first pass's transposed store runs of 2^7
// (2^15-element tiles) and 2^6 (2^12-element tiles) rows: 512- and 256-byte
// runs of FP32.  The narrow variants (B) cover the splits the wide ones cannot.
#ifndef CHW_K15_CA
#define CHW_K15_CA 7
#endif
#ifndef CHW_K12_CA
#define CHW_K12_CA 6
#endif
constexpr int K12_CA = CHW_K12_CA, K12_CB = 3, K15_CA = CHW_K15_CA, K15_CB = 3;

// Storage / compute element sizes of a dtype.
int elem_bytes(int dt);
int compute_bytes(int dt);

// Choose the two-pass split for a signal of 2^m elements; false when none of
// the compiled variants covers m.
bool choose_split(int m, int dt, int forced_l1, int whole, int order, bool last15,
                  Split *out);

// Choose the three-pass split of a dyadic-order signal of 2^m elements: the
// widest first-pass runs whose blocks have a two-pass split; false when none.
bool choose_split3(int m, int dt, Split3 *out);

// Build items and launch ranges.  Throws std::bad_alloc on allocation failure,
// std::invalid_argument when a signal cannot be planned.
void build_plan(const std::vector<int32_t> &m, const std::vector<int64_t> &off, int dt,
                const PlanConfig &cfg, BuiltPlan *out);

// Host-side invariants of a built plan (coverage, bounds, launch order,
// persistent dependencies); false with a reason in *err.
bool check_plan(const std::vector<int32_t> &ms, const std::vector<int64_t> &off, int dt,
                const BuiltPlan &p, std::string *err);

// The Haar transform Psi_m alone: level passes of 2^12-element tiles (see
// chw_haar_kernel).  passes[p] covers the tiles of pass p of every signal;
// the forward runs them in order, the adjoint in reverse.
struct HaarPlan {
    std::vector<Item> items;
    std::vector<LaunchRange> passes;
    size_t ws_elems = 0;   // tile sums between passes (compute type)
};
void build_haar_plan(const std::vector<int32_t> &ms, const std::vector<int64_t> &off,
                     HaarPlan *out);

// JSON description of a built plan.
std::string describe_plan(const BuiltPlan &p);

}  // namespace chw
