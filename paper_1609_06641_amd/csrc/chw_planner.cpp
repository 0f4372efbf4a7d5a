// chw_planner.cpp -- host planner for the CHW tile kernels.
//
// Signals are classified by size:
//   * tiny   : fewer bytes than one 16-byte vector -> one thread per signal;
//   * single : 2^m fits one tile (m <= 12 in 2^12-element tiles, 13..15 in
//              2^15-element tiles) -> one pass, 2^(K-m) signals per tile;
//   * multi  : two HBM passes split along the level structure of the cascade.
//              The proof of Theorem 1 (Sec. 5) shows that after the first
//              level the rest is I_1 (x) CHW_{m-1} on the two halves; applied
//              L1 times, the first pass runs stages 0..L1-1 on contiguous rows
//              of 2^L1 elements and leaves 2^L1 independent contiguous blocks
//              of 2^(m-L1) elements, on each of which the second pass runs the
//              whole CHW_{m-L1}.
#include "chw_planner.h"

#include <algorithm>
#include <cstdio>
#include <stdexcept>

namespace chw {

int elem_bytes(int dt)
{
    switch (dt) {
    case DT_F32: case DT_I32: return 4;
    case DT_BF16: case DT_F16: return 2;
    case DT_F64: return 8;
    default: return 0;
    }
}

int compute_bytes(int dt) { return dt == DT_F64 ? 8 : 4; }

bool choose_split(int m, int dt, int forced_l1, int whole, int order, bool last15,
                  Split *out)
{
    // whole = 12 / 15: both passes of the signal run in one workgroup of
    // 2^whole-element tiles (the persistent launch); its first-pass kinds are
    // the whole-signal ones (2^CA, 2^CM or 2^CB rows)
    const bool k12_only = whole == 12, k15_only = whole == 15;
    struct Opt { int K1, CC, kind; };
    // preference: the widest transposed runs first (2^7 rows = 512-byte runs
    // of FP32 in the first pass's store)
    const Opt opts[] = {{15, K15_CA, KIND_FIRST_A}, {15, K15_CD, KIND_FIRST_D},
                        {12, K12_CA, KIND_FIRST_A}, {15, K15_CM, KIND_FIRST_C},
                        {12, K12_CM, KIND_FIRST_C}, {15, K15_CB, KIND_FIRST_B},
                        {12, K12_CB, KIND_FIRST_B}};
    const int kmax2 = (dt == DT_F64 || k12_only) ? 12 : 15;
    if (k15_only) {
        if (dt == DT_F64) return false;  // no FP64 2^15-element tiles
        last15 = true;                  // the last pass runs in the same tile kernel
    }
    // the natural order's last pass also stores runs, of 2^(K2 - b) blocks:
    // it takes the larger last-pass tile and the split whose shorter run is
    // longest; pipelined chunks run both passes in 2^15-element tiles
    const bool natural = order == ORDER_NATURAL;
    bool found = false;
    int best_score = -1;
    for (const Opt &o : opts) {
        if (o.K1 == 15 && (dt == DT_F64 || k12_only)) continue;
        if (o.K1 == 12 && k15_only) continue;
        if (o.kind == KIND_FIRST_D && whole) continue;  // whole-signal items: A, C or B
        const int L1 = o.K1 - o.CC;
        if (forced_l1 > 0 && L1 != forced_l1) continue;
        const int b = m - L1;                 // levels left for the second pass
        if (b < o.CC || b > kmax2) continue;  // each first-pass tile needs 2^CC rows
        const int K2 = (b <= 12 && !((natural || last15) && kmax2 == 15)) ? 12 : 15;
        const int score = natural ? std::min(o.CC, K2 - b) : 0;
        if (found && score <= best_score) continue;
        found = true;
        best_score = score;
        out->m = m;
        out->L1 = L1;
        out->K1 = o.K1;
        out->CC = o.CC;
        out->kind = o.kind;
        out->K2 = K2;
        if (!natural) break;  // first valid option in preference order
    }
    return found;
}

int compute_dt(int dt)
{
    return dt == DT_BF16 || dt == DT_F16 ? DT_F32 : dt;
}

bool choose_split3(int m, int dt, Split3 *out)
{
    // The first pass over rows of 2^L1 leaves 2^L1 blocks of 2^(m - L1)
    // elements, each an independent signal (the induction step of the proof
    // of Theorem 1, applied L1 times); a block larger than a last-pass tile
    // takes two more passes of its own.  The outer first pass prefers the
    // widest transposed runs, as the two-pass split does.
    if (dt == DT_F64) return false;
    struct Opt { int K1, CC, kind; };
    const Opt opts[] = {{15, K15_CA, KIND_FIRST_A}, {12, K12_CA, KIND_FIRST_A},
                        {15, K15_CM, KIND_FIRST_C}, {12, K12_CM, KIND_FIRST_C},
                        {15, K15_CB, KIND_FIRST_B}, {12, K12_CB, KIND_FIRST_B}};
    for (const Opt &o : opts) {
        const int L1 = o.K1 - o.CC, b = m - L1;
        if (b < o.CC) continue;
        Split inner;
        if (!choose_split(b, compute_dt(dt), -1, 0, ORDER_DYADIC, false, &inner)) continue;
        out->m = m;
        out->outer = Split{m, L1, o.K1, o.CC, o.kind, 0};
        out->inner = inner;
        return true;
    }
    return false;
}

namespace {


Item blank_item()
{
    Item it{};
    it.list = -1;
    it.count = 1;
    return it;
}

int tiny_max_log2(int dt)
{
    // fewer bytes than one 16-byte vector
    int m = 0;
    while (((int64_t)1 << (m + 1)) * elem_bytes(dt) < 16) ++m;
    return m;  // F32: 1, BF16: 2, F64: 0
}

}  // namespace

void build_plan(const std::vector<int32_t> &ms, const std::vector<int64_t> &off, int dt,
                const PlanConfig &cfg, BuiltPlan *out)
{
    BuiltPlan p;
    p.cfg = cfg;
    if (p.cfg.order != ORDER_DYADIC && p.cfg.exec == 2)
        throw std::invalid_argument("the persistent launch computes the dyadic order only");
    if (dt == DT_F64) {  // FP64 has only the 2^12-element, 32-register tile kernels
        p.cfg.lr12 = 5;
        p.cfg.single15 = 0;
    }
    const int64_t batch = (int64_t)ms.size();
    const int tiny_max = tiny_max_log2(dt);
    const bool persistent = p.cfg.exec == 2;
    // the persistent launch runs one tile size for everything
    // (measured on the ragged batch, 2^30 elements: BF16 2.60 ms in
    // 2^15-element tiles against 3.26 ms in 2^12-element ones, FP32 3.17
    // against 4.16 ms)
    if (persistent && p.cfg.ptile == 15 && dt == DT_F64)
        throw std::invalid_argument("no FP64 2^15-element tiles for the persistent launch");
    const int ptile = !persistent              ? 0
                      : p.cfg.ptile == 12      ? 12
                      : p.cfg.ptile == 15      ? 15
                      : dt == DT_F64           ? 12
                                               : 15;
    const int single_max = ptile ? ptile : (p.cfg.single15 ? 15 : 12);
    // signals that take three HBM passes: from 2^three_min in the dyadic
    // order; the other orders keep two passes up to 2^27 (the only sizes they
    // support)
    auto three_pass = [&](int m) {
        return m >= p.cfg.three_min && m > 15 && !persistent &&
               (p.cfg.order == ORDER_DYADIC || m > 27);
    };

    // item lists: single-pass BLOCKS per tile size; multi-pass FIRST / LAST
    // per chunk and tile size
    auto kidx = [](int K) { return K == 12 ? 0 : 1; };
    std::vector<Item> blocks[2];
    struct Chunk { std::vector<Item> first[2], last[2]; };
    std::vector<Chunk> chunks(1);
    int64_t chunk_fill = 0;

    // ---- single-pass signals, grouped by size ---------------------------
    std::vector<int64_t> order;
    order.reserve(batch);
    for (int64_t i = 0; i < batch; ++i) {
        const int m = ms[i];
        if (m <= tiny_max) {
            p.tiny_off.push_back(off[i]);
            p.tiny_m.push_back(m);
            ++p.n_tiny;
        } else if (m <= single_max) {
            order.push_back(i);
            ++p.n_single;
        }
    }
    std::stable_sort(order.begin(), order.end(),
                     [&](int64_t a, int64_t b) { return ms[a] < ms[b]; });
    // packed 2^15-element single-pass tiles of the launch (all sizes): only a
    // launch that would fill fewer than kSpreadTiles of them spreads its groups
    int64_t packed15 = 0;
    for (size_t s = 0, g; s < order.size(); s = g) {
        g = s;
        while (g < order.size() && ms[order[g]] == ms[order[s]]) ++g;
        if (ms[order[s]] > 12) {
            const int64_t per = (int64_t)1 << (15 - ms[order[s]]);
            packed15 += ((int64_t)(g - s) + per - 1) / per;
        }
    }
    const bool spread15 = p.cfg.spread && !persistent && packed15 < kSpreadTiles;
    size_t group_end = 0;  // end of the current size group in `order`
    int per = 0;           // signals per tile in the current size group
    for (size_t s = 0; s < order.size();) {
        const int m = ms[order[s]];
        const int K = ptile ? ptile : m <= 12 ? 12 : 15;
        if (s >= group_end) {
            // a launch of 2^15-element tiles (one workgroup fills a CU) that
            // would fill fewer tiles than there are CUs spreads its size groups
            // over more, partly filled tiles, so that it occupies more CUs
            // (256 x 2^13: 11.3 -> 9.7 us; 2^12-element tiles share CUs and
            // gain nothing)
            group_end = s;
            while (group_end < order.size() && ms[order[group_end]] == m) ++group_end;
            const int64_t nm = (int64_t)(group_end - s);
            per = 1 << (K - m);
            if (spread15 && K == 15)
                per = (int)std::min<int64_t>(per, std::max<int64_t>(1, (nm + kSpreadTiles - 1) / kSpreadTiles));
        }
        size_t e = s;
        while (e < order.size() && ms[order[e]] == m && (int)(e - s) < per) ++e;
        Item it = blank_item();
        it.kind = KIND_BLOCKS;
        it.bits = m;
        it.m = m;
        it.count = (int32_t)(e - s);
        bool consecutive = true;
        for (size_t q = s + 1; q < e; ++q)
            if (off[order[q]] != off[order[s]] + ((int64_t)(q - s) << m)) consecutive = false;
        it.io_off = off[order[s]];
        it.sig_off = off[order[s]];
        if (!consecutive) {
            it.list = (int32_t)p.list.size();
            for (size_t q = s; q < e; ++q) p.list.push_back(off[order[q]]);
        }
        blocks[kidx(K)].push_back(it);
        s = e;
    }

    // ---- multi-pass signals --------------------------------------------------
    int64_t wsb = 0;
    std::vector<Item> turn_items;
    bool turn_ok = p.cfg.turn && p.cfg.order == ORDER_DYADIC && (dt == DT_F32 || dt == DT_I32);
    for (int64_t i = 0; i < batch; ++i) {
        const int m = ms[i];
        if (m <= single_max) continue;
        if (three_pass(m)) continue;  // three passes, below
        Split sp;
        const bool pipe = p.cfg.pipeline && p.cfg.chunk > 0 && !persistent;
        if (!choose_split(m, dt, p.cfg.split_l1, ptile, p.cfg.order, pipe, &sp))
            throw std::invalid_argument("no two-pass split covers log2 size " +
                                        std::to_string(m));
        ++p.n_multi;
        bool seen = false;
        for (const Split &q : p.splits)
            if (q.m == sp.m && q.L1 == sp.L1 && q.K1 == sp.K1 && q.K2 == sp.K2) seen = true;
        if (!seen) p.splits.push_back(sp);
        if (p.cfg.chunk > 0 && chunk_fill > 0 && chunk_fill + ((int64_t)1 << m) > p.cfg.chunk) {
            chunks.emplace_back();
            chunk_fill = 0;
        }
        chunk_fill += (int64_t)1 << m;
        Chunk &ch = chunks.back();
        const int L1 = sp.L1, b = m - L1;
        const int64_t rows = (int64_t)1 << b;
        for (int64_t h0 = 0; h0 < rows; h0 += (int64_t)1 << sp.CC) {
            Item it = blank_item();
            it.kind = sp.kind;
            it.bits = L1;
            it.m = m;
            it.rs = b;
            it.h0 = (int32_t)h0;
            it.io_off = off[i] + (h0 << L1);
            it.ws_off = wsb;
            it.sig_off = off[i];
            ch.first[kidx(sp.K1)].push_back(it);
        }
        const int bpt = 1 << (sp.K2 - b);  // blocks per last-pass tile
        const int64_t tiles = ((int64_t)1 << L1) / bpt;
        for (int64_t tl = 0; tl < tiles; ++tl) {
            Item it = blank_item();
            it.kind = KIND_LAST;
            it.bits = b;
            it.m = m;
            it.count = bpt;
            it.io_off = off[i] + (tl << sp.K2);
            it.ws_off = wsb + (tl << sp.K2);
            it.sig_off = off[i];
            ch.last[kidx(sp.K2)].push_back(it);
        }
        // round boundary tiles: 2^15 consecutive positions = 2^CC first-pass
        // rows of the next round (first pass in 2^15-element tiles only, and
        // last-pass blocks of at least 2^8, which the tile's first register
        // round needs)
        if (sp.K1 != 15 || b < 8) turn_ok = false;
        if (turn_ok) {
            for (int64_t tl = 0; tl < ((int64_t)1 << (m - 15)); ++tl) {
                Item it = blank_item();
                it.kind = KIND_TURN;
                it.bits = b;
                it.m = m;
                it.count = 1 << (15 - b);
                it.io_off = off[i] + (tl << 15);
                it.ws_off = wsb + (tl << 15);
                it.sig_off = off[i];
                it.h0 = (int32_t)(tl << sp.CC);
                it.rs = b;
                turn_items.push_back(it);
            }
        }
        wsb += (int64_t)1 << m;
    }
    // ---- three-pass signals ------------------------------------------------
    // Pass 1: first-pass tiles on x, into the first intermediate W1 (the
    // signal's blocks of 2^b, b = m - L1, contiguous).  Pass 2 ("middle"):
    // every block of W1 is a signal of 2^b whose first pass runs from W1 into
    // the second intermediate W2.  Pass 3: the blocks' last-pass tiles from
    // W2 into y, block g of the signal landing on y's block g.  Same stages in
    // the same order as any other split, so the same numbers.
    struct Three { std::vector<Item> first[2], mid[2], last[2]; } three;
    int64_t tot3 = 0;
    for (int64_t i = 0; i < batch; ++i)
        if (three_pass(ms[i])) {
            if (p.cfg.order != ORDER_DYADIC)
                throw std::invalid_argument("signals above 2^27 (three passes) compute the dyadic "
                                            "order only");
            tot3 += (int64_t)1 << ms[i];
        }
    const int64_t w1 = wsb, w2 = wsb + tot3;
    int64_t acc3 = 0;
    for (int64_t i = 0; i < batch && tot3 > 0; ++i) {
        const int m = ms[i];
        if (!three_pass(m)) continue;
        Split3 s3;
        if (!choose_split3(m, dt, &s3))
            throw std::invalid_argument("no three-pass split covers log2 size " + std::to_string(m));
        ++p.n_multi;
        ++p.n_three;
        bool seen = false;
        for (const Split3 &q : p.splits3)
            if (q.m == m) seen = true;
        if (!seen) p.splits3.push_back(s3);
        const Split &o = s3.outer, &in = s3.inner;
        const int L1 = o.L1, b = m - L1, L2 = in.L1, b3 = b - L2;
        const int64_t a = w1 + acc3, c = w2 + acc3;  // the signal in W1 and W2
        for (int64_t h0 = 0; h0 < ((int64_t)1 << b); h0 += (int64_t)1 << o.CC) {
            Item it = blank_item();
            it.kind = o.kind;
            it.bits = L1;
            it.m = m;
            it.rs = b;
            it.h0 = (int32_t)h0;
            it.io_off = off[i] + (h0 << L1);
            it.ws_off = a;
            it.sig_off = off[i];
            three.first[kidx(o.K1)].push_back(it);
        }
        const int bpt = 1 << (in.K2 - b3);  // blocks per last-pass tile
        for (int64_t g = 0; g < ((int64_t)1 << L1); ++g) {
            const int64_t blk = g << b;      // block g within the signal
            for (int64_t h0 = 0; h0 < ((int64_t)1 << b3); h0 += (int64_t)1 << in.CC) {
                Item it = blank_item();
                it.kind = in.kind;
                it.bits = L2;
                it.m = m;
                it.rs = b3;
                it.h0 = (int32_t)h0;
                it.io_off = a + blk + (h0 << L2);  // in the workspace (W1)
                it.ws_off = c + blk;               // the block's base in W2
                it.sig_off = a + blk;
                three.mid[kidx(in.K1)].push_back(it);
            }
            for (int64_t tl = 0; tl < ((int64_t)1 << L2) / bpt; ++tl) {
                Item it = blank_item();
                it.kind = KIND_LAST;
                it.bits = b3;
                it.m = m;  // the orthonormal scale of the whole signal
                it.count = bpt;
                it.io_off = off[i] + blk + (tl << in.K2);
                it.ws_off = c + blk + (tl << in.K2);
                it.sig_off = off[i] + blk;
                three.last[kidx(in.K2)].push_back(it);
            }
        }
        acc3 += (int64_t)1 << m;
    }
    if (tot3 > 0) turn_ok = false;
    p.ws3_first = (size_t)w1;
    p.ws3_elems = (size_t)tot3;
    wsb += 2 * tot3;
    p.ws_elems = (size_t)wsb;
    // every configuration runs a subset of the signals above 2^12 in two passes
    // (and those of 2^three_min or more in three, with two intermediates), so
    // this bounds the workspace of all of them (the size a caller allocates
    // must not change when the plan is tuned)
    for (int64_t i = 0; i < batch; ++i) {
        if (ms[i] > 12) p.ws_bound += (size_t)1 << ms[i];
        if (ms[i] >= p.cfg.three_min && ms[i] > 15 && (p.cfg.order == ORDER_DYADIC || ms[i] > 27))
            p.ws_bound += (size_t)1 << ms[i];
    }
    if (p.ws_elems > p.ws_bound) throw std::logic_error("workspace bound");

    // ---- table and launch order ----------------------------------------------
    if (persistent) {
        // one launch; single-pass tiles and whole multi-pass signals, sorted by
        // decreasing work (the kernel hands items out grid-stride)
        std::vector<Item> all(blocks[kidx(ptile)]);
        for (const Chunk &ch : chunks)
            for (const Item &f : ch.first[kidx(ptile)]) {
                if (f.h0 != 0) continue;  // one item per signal
                Item it = blank_item();
                it.kind = f.kind == KIND_FIRST_A   ? KIND_SIGNAL_A
                          : f.kind == KIND_FIRST_C ? KIND_SIGNAL_C
                                                   : KIND_SIGNAL_B;
                it.m = f.m;
                it.bits = f.bits;          // L1
                it.io_off = f.io_off;      // signal base (h0 = 0)
                it.ws_off = f.ws_off;
                it.sig_off = f.sig_off;
                all.push_back(it);
            }
        auto work = [](const Item &it) {
            return (it.kind == KIND_BLOCKS) ? ((int64_t)it.count << it.bits)
                                            : ((int64_t)2 << it.m);
        };
        std::stable_sort(all.begin(), all.end(),
                         [&](const Item &x, const Item &y) { return work(x) > work(y); });
        LaunchRange r;
        r.K = ptile;
        r.LR = ptile == 15 ? 5 : p.cfg.lr12 ? p.cfg.lr12 : 6;  // compiled forms
        r.persistent = 1;
        r.begin = (int)p.items.size();
        p.items.insert(p.items.end(), all.begin(), all.end());
        r.end = (int)p.items.size();
        if (p.items.size() > (size_t)0x7fffffff) throw std::bad_alloc();
        if (r.end > r.begin) {
            p.fwd.push_back(r);
            p.adj.push_back(r);
        }
        *out = std::move(p);
        return;
    }
    // measured: 2^5 registers per thread are faster for single-pass 2^12
    // tiles (8192 x 2^12: 28.7 against 30.9 us in BF16, 44.7 against 47.0 us
    // in FP32), 2^6 for the last pass of two-pass signals
    auto append = [&](const std::vector<Item> &v, int K, LaunchRange *r, bool single = false) {
        r->K = K;
        r->LR = K == 12 ? (p.cfg.lr12 ? p.cfg.lr12 : single ? 5 : 6) : p.cfg.lr15;
        r->begin = (int)p.items.size();
        p.items.insert(p.items.end(), v.begin(), v.end());
        r->end = (int)p.items.size();
        if (p.items.size() > (size_t)0x7fffffff) throw std::bad_alloc();
    };
    for (int k = 0; k < 2; ++k) {
        LaunchRange r;
        append(blocks[k], k == 0 ? 12 : 15, &r, true);
        r.single_pass = 1;
        if (r.end > r.begin) {
            p.fwd.push_back(r);
            p.adj.push_back(r);
        }
    }
    // pipelined chunks: launch 0 = first pass of chunk 0; launch j = last pass
    // of chunk j - 1 with the first pass of chunk j; the last launch = last
    // pass of the final chunk.  The adjoint pairs the adjoint first pass of
    // chunk j - 1 with the adjoint last pass of chunk j; its items are copies
    // laid out in that order.  Chunk j's intermediate lives in slot j % 2.
    if (p.cfg.pipeline && p.cfg.chunk > 0 && !persistent && chunks.size() > 1 && tot3 == 0) {
        int64_t slot = 0;
        std::vector<int64_t> start(chunks.size(), -1);
        for (size_t j = 0; j < chunks.size(); ++j) {
            int64_t lo = INT64_MAX, hi = 0;
            for (int k = 0; k < 2; ++k)
                for (const Item &it : chunks[j].last[k]) {
                    lo = std::min(lo, it.ws_off);
                    hi = std::max(hi, it.ws_off + ((int64_t)it.count << it.bits));
                }
            start[j] = lo == INT64_MAX ? 0 : lo;
            slot = std::max(slot, hi - start[j]);
        }
        if (2 * slot <= (int64_t)p.ws_bound) {
            for (size_t j = 0; j < chunks.size(); ++j) {
                const int64_t shift = (int64_t)(j & 1) * slot - start[j];
                for (int k = 0; k < 2; ++k) {
                    for (Item &it : chunks[j].first[k]) it.ws_off += shift;
                    for (Item &it : chunks[j].last[k]) it.ws_off += shift;
                }
            }
            p.ws_elems = (size_t)(2 * slot);
            auto merged = [&](const std::vector<Item> &a, const std::vector<Item> &b) {
                std::vector<Item> v(a);
                v.insert(v.end(), b.begin(), b.end());
                return v;
            };
            const size_t n = chunks.size();
            for (int dir = 0; dir < 2; ++dir) {
                for (size_t j = 0; j <= n; ++j) {
                    // forward: last(j-1) + first(j); adjoint: first(j-1) + last(j)
                    for (int k = 0; k < 2; ++k) {
                        const std::vector<Item> none;
                        const std::vector<Item> &prev = j > 0 ? (dir ? chunks[j - 1].first[k] : chunks[j - 1].last[k]) : none;
                        const std::vector<Item> &next = j < n ? (dir ? chunks[j].last[k] : chunks[j].first[k]) : none;
                        LaunchRange r;
                        append(merged(prev, next), k == 0 ? 12 : 15, &r);
                        if (r.end > r.begin) (dir ? p.adj : p.fwd).push_back(r);
                    }
                }
            }
            *out = std::move(p);
            return;
        }
    }
    for (const Chunk &ch : chunks) {
        LaunchRange f[2], l[2];
        for (int k = 0; k < 2; ++k) append(ch.first[k], k == 0 ? 12 : 15, &f[k]);
        for (int k = 0; k < 2; ++k) append(ch.last[k], k == 0 ? 12 : 15, &l[k]);
        for (int k = 0; k < 2; ++k)
            if (f[k].end > f[k].begin) p.fwd.push_back(f[k]);
        for (int k = 0; k < 2; ++k)
            if (l[k].end > l[k].begin) {
                p.fwd.push_back(l[k]);
                p.adj.push_back(l[k]);  // adjoint: the last pass's blocks come first
            }
        for (int k = 0; k < 2; ++k)
            if (f[k].end > f[k].begin) p.adj.push_back(f[k]);
    }
    if (tot3 > 0) {
        LaunchRange f[2], md[2], l[2];
        for (int k = 0; k < 2; ++k) append(three.first[k], k == 0 ? 12 : 15, &f[k]);
        for (int k = 0; k < 2; ++k) {
            append(three.mid[k], k == 0 ? 12 : 15, &md[k]);
            md[k].role = 1;
        }
        for (int k = 0; k < 2; ++k) append(three.last[k], k == 0 ? 12 : 15, &l[k]);
        for (const LaunchRange *g : {f, md, l})
            for (int k = 0; k < 2; ++k)
                if (g[k].end > g[k].begin) p.fwd.push_back(g[k]);
        for (const LaunchRange *g : {l, md, f})
            for (int k = 0; k < 2; ++k)
                if (g[k].end > g[k].begin) p.adj.push_back(g[k]);
    }
    if (turn_ok && chunks.size() == 1 && !turn_items.empty()) {
        // one launch per first-pass row count (the adjoint's prefetching form is
        // compiled per row count)
        for (int cc : {K15_CA, K15_CD, K15_CM, K15_CB}) {
            std::vector<Item> v;
            for (const Item &it : turn_items)
                if (15 - (it.m - it.bits) == cc) v.push_back(it);
            if (v.empty()) continue;
            LaunchRange r;
            append(v, 15, &r);
            r.stream = p.cfg.stream ? 1 + KIND_TURN : 0;
            p.turn.push_back(r);
        }
    }
    if (p.cfg.stream) {
        // 2^12-element tiles keep several workgroups per CU, which overlap
        // loads and work by themselves; only 2^15-element tiles prefetch.
        // In mode 1 single-pass tiles prefetch only when the launch has many
        // of them (measured for 2^28 elements: 2^15 signals 0.41 against
        // 0.43 ms, 2^14 0.42 against 0.46, 2^13 0.42 against 0.47, and 1024
        // tiles of 2^14 signals 55 against 61 us; launches of a few hundred
        // tiles do better with one workgroup per tile); mode 2 prefetches in
        // every launch that can.  The forward first pass of 2^6-row tiles (2^24
        // signals) runs one workgroup per tile in mode 1: 0.40 against 0.42 ms
        // per 2^28 elements prefetching (2^7 rows: 0.38-0.39 either way; 2^5
        // rows: 0.49 against 0.50, prefetching)
        auto form = [&](const LaunchRange &r, bool adj) {
            if (r.K != 15) return 0;
            const int s = stream_source(p.items, r.begin, r.end, r.K, adj);
            if (s == 1 + KIND_BLOCKS && p.cfg.stream == 1 && r.end - r.begin < kStreamBlocksMin)
                return 0;
            if (s == 1 + KIND_FIRST_D && !adj && p.cfg.stream == 1) return 0;
            return s;
        };
        // the adjoint of the other orders gathers by the order's map: one
        // workgroup per tile
        for (LaunchRange &r : p.fwd) r.stream = form(r, false);
        for (LaunchRange &r : p.adj) r.stream = p.cfg.order == ORDER_DYADIC ? form(r, true) : 0;
    }
    *out = std::move(p);
}

void build_haar_plan(const std::vector<int32_t> &ms, const std::vector<int64_t> &off,
                     HaarPlan *out)
{
    HaarPlan h;
    std::vector<std::vector<Item>> by_pass;
    int64_t wsb = 0;
    for (size_t s = 0; s < ms.size(); ++s) {
        int n = ms[s], p = 0;
        int64_t src = off[s];  // the pass's vector: x for p = 0, then the workspace
        while (true) {
            if ((int)by_pass.size() <= p) by_pass.emplace_back();
            if (n > 12) {
                const int64_t tiles = (int64_t)1 << (n - 12);
                const int64_t next = wsb;
                wsb += (tiles + 7) & ~(int64_t)7;  // every sums array 32-byte aligned
                for (int64_t tl = 0; tl < tiles; ++tl) {
                    Item it = blank_item();
                    it.kind = p == 0 ? 0 : 1;
                    it.io_off = src + (tl << 12);
                    it.sig_off = off[s];
                    it.m = ms[s];
                    it.bits = 12;
                    it.h0 = 12 * p;
                    it.count = (int32_t)tl;
                    it.ws_off = next + tl;
                    by_pass[p].push_back(it);
                }
                src = next;
                n -= 12;
                ++p;
            } else {
                Item it = blank_item();
                it.kind = p == 0 ? 0 : 1;
                it.io_off = src;
                it.sig_off = off[s];
                it.m = ms[s];
                it.bits = n;
                it.h0 = 12 * p;
                it.count = 0;
                it.ws_off = -1;
                by_pass[p].push_back(it);
                break;
            }
        }
    }
    for (const std::vector<Item> &v : by_pass) {
        LaunchRange r;
        r.K = 12;
        r.LR = 5;
        r.begin = (int)h.items.size();
        h.items.insert(h.items.end(), v.begin(), v.end());
        r.end = (int)h.items.size();
        if (h.items.size() > (size_t)0x7fffffff) throw std::bad_alloc();
        if (r.end > r.begin) h.passes.push_back(r);
    }
    h.ws_elems = (size_t)wsb;
    *out = std::move(h);
}

int stream_source(const std::vector<Item> &items, int begin, int end, int K, bool adj)
{
    (void)adj;  // the kernel derives its source (input or intermediate) from the kind
    if (begin >= end) return 0;
    const int kind = items[begin].kind;
    if (kind != KIND_BLOCKS && !is_first_kind(kind) && kind != KIND_LAST) return 0;
    for (int i = begin; i < end; ++i) {
        const Item &it = items[i];
        if (it.kind != kind) return 0;
        if ((kind == KIND_BLOCKS || kind == KIND_LAST) &&
            (it.list >= 0 || ((int64_t)it.count << it.bits) != ((int64_t)1 << K)))
            return 0;
    }
    return 1 + kind;
}

std::string describe_plan(const BuiltPlan &p)
{
    std::string s = "{";
    char buf[256];
    int64_t tiny_elements = 0;
    for (int32_t m : p.tiny_m) tiny_elements += (int64_t)1 << m;
    std::snprintf(buf, sizeof buf,
                  "\"items\": %zu, \"list\": %zu, \"tiny\": %lld, \"tiny_elements\": %lld, "
                  "\"single\": %lld, \"multi\": %lld, \"ws_elems\": %zu, ",
                  p.items.size(), p.list.size(), (long long)p.n_tiny, (long long)tiny_elements,
                  (long long)p.n_single, (long long)p.n_multi, p.ws_elems);
    s += buf;
    std::snprintf(buf, sizeof buf,
                  "\"config\": {\"lr12\": %d, \"lr15\": %d, \"single15\": %d, \"split_l1\": %d, "
                  "\"exec\": %d, \"ptile\": %d, \"chunk\": %lld, \"stream\": %d, \"pipeline\": %d, "
                  "\"order\": %d, \"turn\": %d, \"adjoint\": %d, \"spread\": %d, \"occupancy\": %d}, ",
                  p.cfg.lr12, p.cfg.lr15, p.cfg.single15, p.cfg.split_l1, p.cfg.exec, p.cfg.ptile,
                  (long long)p.cfg.chunk, p.cfg.stream, p.cfg.pipeline, p.cfg.order, p.cfg.turn,
                  p.cfg.adjoint, p.cfg.spread, p.cfg.occupancy);
    s += buf;
    s += "\"splits\": [";
    for (size_t i = 0; i < p.splits.size(); ++i) {
        const Split &q = p.splits[i];
        std::snprintf(buf, sizeof buf, "%s{\"m\": %d, \"L1\": %d, \"K1\": %d, \"rows_log2\": %d, \"K2\": %d}",
                      i ? ", " : "", q.m, q.L1, q.K1, q.CC, q.K2);
        s += buf;
    }
    s += "], \"splits3\": [";
    for (size_t i = 0; i < p.splits3.size(); ++i) {
        const Split3 &q = p.splits3[i];
        std::snprintf(buf, sizeof buf,
                      "%s{\"m\": %d, \"L1\": %d, \"K1\": %d, \"rows_log2\": %d, \"L2\": %d, "
                      "\"K2\": %d, \"rows2_log2\": %d, \"K3\": %d}",
                      i ? ", " : "", q.m, q.outer.L1, q.outer.K1, q.outer.CC, q.inner.L1,
                      q.inner.K1, q.inner.CC, q.inner.K2);
        s += buf;
    }
    s += "], ";
    std::snprintf(buf, sizeof buf, "\"three\": %lld, ", (long long)p.n_three);
    s += buf;
    // elements a launch takes through its part of the transform: every
    // element of its tiles (a whole-signal item counts its signal once)
    auto elements = [&](const LaunchRange &r) {
        int64_t n = 0;
        for (int k = r.begin; k < r.end; ++k) {
            const Item &it = p.items[k];
            if (it.kind == KIND_BLOCKS || it.kind == KIND_LAST) n += (int64_t)it.count << it.bits;
            else if (is_signal_kind(it.kind)) n += (int64_t)1 << it.m;
            else n += (int64_t)1 << r.K;  // first-pass and round-boundary tiles
        }
        return n;
    };
    auto ranges = [&](const char *name, const std::vector<LaunchRange> &v) {
        s += "\"";
        s += name;
        s += "\": [";
        for (size_t i = 0; i < v.size(); ++i) {
            const LaunchRange &r = v[i];
            std::snprintf(buf, sizeof buf,
                          "%s{\"K\": %d, \"LR\": %d, \"begin\": %d, \"end\": %d, \"persistent\": %d, "
                          "\"stream\": %d, \"role\": %d, \"elements\": %lld}",
                          i ? ", " : "", r.K, r.LR, r.begin, r.end, r.persistent, r.stream, r.role,
                          (long long)elements(r));
            s += buf;
        }
        s += "]";
    };
    ranges("forward", p.fwd);
    s += ", ";
    ranges("backward", p.adj);
    s += ", ";
    ranges("turn", p.turn);
    s += "}";
    return s;
}

}  // namespace chw
