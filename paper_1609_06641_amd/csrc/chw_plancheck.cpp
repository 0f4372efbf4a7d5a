// chw_plancheck.cpp -- host-side invariants of a built plan (no device).
//
//   * every element of every signal is covered exactly once per pass: by one
//     single-pass tile, or by one first-pass and one last-pass tile;
//   * every tile stays inside its signal (and the workspace);
//   * multi-launch order: a signal's last-pass launch comes after its
//     first-pass launch (forward) or before it (adjoint);
//   * persistent tables: a whole-signal item covers its signal in both passes
//     and its split fits the 2^12-element tiles;
//   * a prefetching launch holds only full tiles of one kind without block
//     lists, and reads them from the source its code names.
#include <algorithm>
#include <cstdio>
#include <string>
#include <vector>

#include "chw_planner.h"

namespace chw {

namespace {

struct Iv {
    int64_t lo, hi;
    int pass;  // 0 single, 1 first, 2 last
    int launch;
};

bool check_cover(const std::vector<int32_t> &ms, const std::vector<int64_t> &off,
                 std::vector<Iv> &iv, std::string *err, int want_pass, bool is_multi_pass)
{
    // intervals of `want_pass` must tile exactly the signals of that class
    std::vector<std::pair<int64_t, int64_t>> sig;
    (void)is_multi_pass;
    std::vector<Iv> mine;
    for (const Iv &v : iv)
        if (v.pass == want_pass) mine.push_back(v);
    std::sort(mine.begin(), mine.end(), [](const Iv &a, const Iv &b) { return a.lo < b.lo; });
    for (size_t i = 1; i < mine.size(); ++i)
        if (mine[i].lo < mine[i - 1].hi) {
            *err = "tiles of pass " + std::to_string(want_pass) + " overlap at element " +
                   std::to_string(mine[i].lo);
            return false;
        }
    (void)ms;
    (void)off;
    return true;
}

}  // namespace

bool check_plan(const std::vector<int32_t> &ms, const std::vector<int64_t> &off, int dt,
                const BuiltPlan &p, std::string *err)
{
    (void)dt;
    const size_t batch = ms.size();
    if (p.ws_elems > p.ws_bound) {
        *err = "configuration workspace exceeds the reported bound";
        return false;
    }
    // classify signals exactly as the plan did: a signal is multi-pass iff it
    // has first-pass tiles
    auto tile_intervals = [&](const std::vector<LaunchRange> &launches, std::vector<Iv> &iv) {
        for (size_t li = 0; li < launches.size(); ++li) {
            const LaunchRange &r = launches[li];
            if (r.role == 1) continue;  // middle passes work in the workspace (below)
            for (int k = r.begin; k < r.end; ++k) {
                const Item &it = p.items[k];
                const int K = r.K;
                if (it.kind == KIND_BLOCKS) {
                    for (int b = 0; b < it.count; ++b) {
                        const int64_t base = it.list >= 0 ? p.list[it.list + b]
                                                          : it.io_off + ((int64_t)b << it.bits);
                        iv.push_back({base, base + ((int64_t)1 << it.bits), 0, (int)li});
                    }
                    if (((int64_t)it.count << it.bits) > ((int64_t)1 << K)) {
                        *err = "single-pass tile larger than its kernel's tile";
                        return false;
                    }
                } else if (is_signal_kind(it.kind)) {
                    const int CC = it.kind == KIND_SIGNAL_A   ? (K == 15 ? K15_CA : K12_CA)
                                   : it.kind == KIND_SIGNAL_C ? mid_rows(K)
                                                              : (K == 15 ? K15_CB : K12_CB);
                    const int L1 = K - CC, b = it.m - L1;
                    if (!r.persistent || (K != 12 && K != 15) || b < CC || b > K || it.bits != L1) {
                        *err = "whole-signal item with an invalid split";
                        return false;
                    }
                    if (it.ws_off < 0 || (size_t)(it.ws_off + ((int64_t)1 << it.m)) > p.ws_elems) {
                        *err = "whole-signal item outside the workspace";
                        return false;
                    }
                    const int64_t n = (int64_t)1 << it.m;
                    iv.push_back({it.io_off, it.io_off + n, 1, (int)li});
                    iv.push_back({it.io_off, it.io_off + n, 2, (int)li});
                } else if (is_first_kind(it.kind)) {
                    iv.push_back({it.io_off, it.io_off + ((int64_t)1 << K), 1, (int)li});
                } else if (it.kind == KIND_LAST) {
                    iv.push_back({it.io_off, it.io_off + ((int64_t)it.count << it.bits), 2, (int)li});
                    if (((int64_t)it.count << it.bits) != ((int64_t)1 << K)) {
                        *err = "last-pass tile does not fill its kernel's tile";
                        return false;
                    }
                    if (it.ws_off < 0 ||
                        (size_t)(it.ws_off + ((int64_t)it.count << it.bits)) > p.ws_elems) {
                        *err = "last-pass tile outside the workspace";
                        return false;
                    }
                } else {
                    *err = "unknown item kind";
                    return false;
                }
            }
        }
        return true;
    };
    // round-boundary tiles: each a full 2^15-element tile of one two-pass
    // signal whose first pass has a compiled 2^15-element row count, inside
    // its signal and the workspace; together they cover every two-pass
    // signal exactly once
    if (!p.turn.empty()) {
        std::vector<std::pair<int64_t, int64_t>> tv;
        for (const LaunchRange &r : p.turn) {
            if (r.K != 15 || r.persistent || (r.stream != 0 && r.stream != 1 + KIND_TURN)) {
                *err = "round-boundary launch with the wrong tile or form";
                return false;
            }
            for (int k = r.begin; k < r.end; ++k) {
                const Item &it = p.items[k];
                const int L1 = it.m - it.bits, cc = 15 - L1;
                const Item &first = p.items[r.begin];
                if (L1 != first.m - first.bits) {
                    *err = "round-boundary launch mixes first-pass row counts";
                    return false;
                }
                if (it.kind != KIND_TURN || it.bits < 8 ||
                    ((int64_t)it.count << it.bits) != ((int64_t)1 << 15) ||
                    (cc != K15_CA && cc != K15_CM && cc != K15_CB && cc != K15_CD) ||
                    it.rs != it.bits ||
                    ((it.io_off - it.sig_off) & 32767) != 0 ||
                    (int64_t)it.h0 != ((it.io_off - it.sig_off) >> L1)) {
                    *err = "malformed round-boundary tile";
                    return false;
                }
                if (it.ws_off < 0 || (size_t)(it.ws_off + 32768) > p.ws_elems ||
                    it.io_off + 32768 > it.sig_off + ((int64_t)1 << it.m)) {
                    *err = "round-boundary tile outside its signal or the workspace";
                    return false;
                }
                tv.push_back({it.io_off, it.io_off + 32768});
            }
        }
        std::sort(tv.begin(), tv.end());
        int64_t need = 0, have = 0;
        for (size_t i = 0; i < tv.size(); ++i) {
            if (i && tv[i].first < tv[i - 1].second) {
                *err = "round-boundary tiles overlap";
                return false;
            }
            have += tv[i].second - tv[i].first;
        }
        for (size_t i = 0; i < batch; ++i)
            if (ms[i] > 15) need += (int64_t)1 << ms[i];
        if (have != need || p.n_multi == 0) {
            *err = "round-boundary tiles do not cover the two-pass signals";
            return false;
        }
    }
    // three-pass signals: the middle pass's first-pass tiles tile the first
    // intermediate [ws3_first, ws3_first + ws3_elems) exactly once, each
    // writes inside the second one, and in each direction the middle launches
    // sit between the launches of the outer passes that touch the
    // intermediates (forward: after every first-pass tile into W1, before
    // every last-pass tile from W2)
    if (p.n_three > 0 || p.ws3_elems > 0) {
        const int64_t w1 = (int64_t)p.ws3_first, n3 = (int64_t)p.ws3_elems, w2 = w1 + n3;
        if (w2 + n3 > (int64_t)p.ws_elems) {
            *err = "three-pass intermediates outside the workspace";
            return false;
        }
        for (int dir = 0; dir < 2; ++dir) {
            const std::vector<LaunchRange> &L = dir ? p.adj : p.fwd;
            std::vector<std::pair<int64_t, int64_t>> cover;
            int mid_lo = 1 << 30, mid_hi = -1;
            int first_lo = 1 << 30, first_hi = -1, last_lo = 1 << 30, last_hi = -1;
            for (size_t li = 0; li < L.size(); ++li) {
                const LaunchRange &r = L[li];
                for (int k = r.begin; k < r.end; ++k) {
                    const Item &it = p.items[k];
                    if (r.role == 1) {
                        if (!is_first_kind(it.kind) || r.persistent) {
                            *err = "middle pass with an item that is not a first-pass tile";
                            return false;
                        }
                        const int64_t n = (int64_t)1 << r.K;
                        const int64_t blk = (int64_t)1 << (it.bits + it.rs);  // the block's size
                        if (it.io_off < w1 || it.io_off + n > w2 || it.ws_off < w2 ||
                            it.ws_off + blk > w2 + n3 || it.io_off < it.sig_off ||
                            it.io_off + n > it.sig_off + blk) {
                            *err = "middle-pass tile outside its block or the intermediates";
                            return false;
                        }
                        cover.push_back({it.io_off, it.io_off + n});
                        mid_lo = std::min(mid_lo, (int)li);
                        mid_hi = std::max(mid_hi, (int)li);
                    } else if (is_first_kind(it.kind) && it.ws_off >= w1 && it.ws_off < w2) {
                        first_lo = std::min(first_lo, (int)li);  // outer first pass: W1
                        first_hi = std::max(first_hi, (int)li);
                    } else if (it.kind == KIND_LAST && it.ws_off >= w2) {
                        last_lo = std::min(last_lo, (int)li);    // outer last pass: W2
                        last_hi = std::max(last_hi, (int)li);
                    }
                }
            }
            std::sort(cover.begin(), cover.end());
            int64_t have = 0;
            for (size_t i = 0; i < cover.size(); ++i) {
                if (i && cover[i].first < cover[i - 1].second) {
                    *err = "middle-pass tiles overlap";
                    return false;
                }
                have += cover[i].second - cover[i].first;
            }
            const bool order_ok = first_hi >= 0 && last_hi >= 0 &&
                                  (dir == 0 ? (first_hi < mid_lo && mid_hi < last_lo)
                                            : (last_hi < mid_lo && mid_hi < first_lo));
            if (have != n3 || mid_hi < 0 || !order_ok) {
                *err = "middle pass does not cover the first intermediate between the outer passes";
                return false;
            }
        }
    }
    for (int dir = 0; dir < 2; ++dir) {
        const std::vector<LaunchRange> &L = dir ? p.adj : p.fwd;
        for (const LaunchRange &r : L) {
            if (r.stream != 0 && (r.persistent || r.K != 15 ||
                                  (dir == 1 && p.cfg.order != ORDER_DYADIC) ||
                                  r.stream != stream_source(p.items, r.begin, r.end, r.K, dir == 1))) {
                *err = "prefetching launch over items that are not full tiles of one kind";
                return false;
            }
        }
        std::vector<Iv> iv;
        if (!tile_intervals(L, iv)) return false;
        for (int pass = 0; pass < 3; ++pass)
            if (!check_cover(ms, off, iv, err, pass, pass > 0)) return false;
        // per signal: covered exactly once by single, or once by first and last
        std::vector<std::pair<int64_t, int>> starts;  // (lo, index into iv)
        std::sort(iv.begin(), iv.end(), [](const Iv &a, const Iv &b) {
            return a.lo != b.lo ? a.lo < b.lo : a.pass < b.pass;
        });
        size_t tiny_seen = 0;
        for (size_t i = 0; i < batch; ++i) {
            const int64_t lo = off[i], hi = off[i] + ((int64_t)1 << ms[i]);
            // tiles starting inside the signal
            auto first_it = std::lower_bound(iv.begin(), iv.end(), lo,
                                             [](const Iv &a, int64_t v) { return a.lo < v; });
            int64_t cov[3] = {0, 0, 0};
            int first_launch = -1, last_launch = -1;
            for (auto it = first_it; it != iv.end() && it->lo < hi; ++it) {
                if (it->hi > hi) {
                    *err = "tile crosses the end of signal " + std::to_string(i);
                    return false;
                }
                cov[it->pass] += it->hi - it->lo;
                if (it->pass == 1) first_launch = std::max(first_launch, it->launch);
                if (it->pass == 2) last_launch = last_launch < 0 ? it->launch : std::min(last_launch, it->launch);
            }
            const int64_t n = hi - lo;
            const bool single = cov[0] == n && cov[1] == 0 && cov[2] == 0;
            const bool multi = cov[0] == 0 && cov[1] == n && cov[2] == n;
            const bool tiny = cov[0] == 0 && cov[1] == 0 && cov[2] == 0;
            if (tiny) {
                ++tiny_seen;
                continue;
            }
            if (!single && !multi) {
                char b[200];
                std::snprintf(b, sizeof b, "signal %zu (m=%d) covered %lld/%lld/%lld of %lld", i, ms[i],
                              (long long)cov[0], (long long)cov[1], (long long)cov[2], (long long)n);
                *err = b;
                return false;
            }
            if (multi && L.size() > 0 && !L[0].persistent) {
                const bool ok = dir == 0 ? first_launch < last_launch : last_launch < first_launch;
                if (!ok) {
                    *err = "launch order of the two passes of signal " + std::to_string(i);
                    return false;
                }
            }
        }
        if (tiny_seen != p.tiny_off.size()) {
            *err = "signals without tiles do not match the tiny list";
            return false;
        }
    }
    return true;
}

}  // namespace chw
