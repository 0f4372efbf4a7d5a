// chw_selfcheck.cpp -- host-side check of the tile engine's index maps.
//
// Runs the same Layout<K, LR> formulas the kernels use, on the CPU, for every
// compiled (K, LR) pair and vector width, and checks that
//   * every phase touches each tile element exactly once (bijective maps),
//   * every padded LDS address stays below the tile's LDS allocation,
//   * the per-thread-base + compile-time-offset split the kernels rely on
//     equals the padded address of the intended element,
//   * the transposed first-pass store hits each global element of the tile's
//     runs exactly once.
// It also reports the worst LDS bank multiplicity of each phase for one
// 64-lane wave under a 64-bank and a 32-bank (per half wave) model.
#include <algorithm>
#include <cstdio>
#include <cstring>
#include <set>
#include <string>
#include <vector>

#include "chw.h"
#include "chw_layout.h"

using namespace chw;

namespace {

struct Stats {
    bool ok = true;
    int worst64 = 0, worst32 = 0;
    std::string err;
    void fail(const std::string &e)
    {
        if (ok) err = e;
        ok = false;
    }
};

// worst number of distinct addresses sharing a bank among `lanes` addresses
int bank_ways(const std::vector<int> &addr, int banks, int group)
{
    int worst = 0;
    for (size_t g0 = 0; g0 < addr.size(); g0 += group) {
        std::vector<std::set<int>> per(banks);
        for (size_t l = g0; l < std::min(addr.size(), g0 + group); ++l)
            per[((addr[l] % banks) + banks) % banks].insert(addr[l]);
        for (auto &s : per) worst = std::max(worst, (int)s.size());
    }
    return worst;
}

void bank_account(Stats &st, const std::vector<int> &wave_addr)
{
    st.worst64 = std::max(st.worst64, bank_ways(wave_addr, 64, 64));
    st.worst32 = std::max(st.worst32, bank_ways(wave_addr, 32, 32));
}

template <int K, int LR>
std::string check_variant()
{
    using L = Layout<K, LR>;
    constexpr int N = L::N, NT = L::NT, R = L::R;
    std::string out;
    char buf[512];

    // ---- rounds (from tile bit B0: B0 > 0 after stages on the loaded vectors)
    auto rounds_phase = [&](int B0) {
        Stats rs;
        int covered = 0;
        for (int j = 0; j < L::rounds_from(B0); ++j) {
            if (L::flo(j, B0) > L::alo(j, B0) || L::alo(j, B0) >= L::ahi(j, B0) ||
                L::ahi(j, B0) > L::flo(j, B0) + LR || L::alo(j, B0) != B0 + covered)
                rs.fail("round active bits outside the register field");
            covered = L::ahi(j, B0) - B0;
            std::vector<int> seen(N, 0);
            for (int t = 0; t < NT; ++t)
                for (int i = 0; i < R; ++i) {
                    const int tb = L::round_tbase(j, t, B0), ri = L::round_reg(j, i, B0);
                    if (tb & ri) rs.fail("round fields overlap");
                    const int e = tb | ri;
                    if (e < 0 || e >= N) { rs.fail("round element out of range"); continue; }
                    ++seen[e];
                    if (L::pad(tb) + L::pad(ri) != L::pad(e)) rs.fail("round offset split");
                    if (L::pad(e) >= L::LDS_WORDS) rs.fail("round LDS address out of range");
                }
            for (int e = 0; e < N; ++e)
                if (seen[e] != 1) { rs.fail("round map not bijective"); break; }
            for (int w = 0; w < NT / 64; ++w)
                for (int i = 0; i < R; ++i) {
                    std::vector<int> a;
                    for (int l = 0; l < 64; ++l)
                        a.push_back(L::pad(L::round_tbase(j, 64 * w + l, B0) | L::round_reg(j, i, B0)));
                    bank_account(rs, a);
                }
        }
        if (covered != K - B0) rs.fail("rounds do not cover the tile bits");
        std::snprintf(buf, sizeof buf, "%s{\"K\": %d, \"LR\": %d, \"phase\": \"%s\", \"B0\": %d, \"rounds\": %d, \"ok\": %s, \"ways64\": %d, \"ways32\": %d%s%s}",
                      B0 ? ", " : "", K, LR, B0 ? "rounds_from_bit" : "rounds", B0, L::rounds_from(B0),
                      rs.ok ? "true" : "false", rs.worst64, rs.worst32,
                      rs.ok ? "" : ", \"error\": \"", rs.ok ? "" : (rs.err + "\"").c_str());
        out += buf;
    };
    rounds_phase(0);
    // rounds after the stages on the loaded 16-byte vectors: single-pass
    // 2^12-element tiles with 2^5 registers start at bit 2 (4-byte elements)
    // or bit 3 (2-byte elements), the round-boundary 2^15-element tiles with
    // 2^5 registers at bit 2 (4-byte intermediate)
    if (K == 12 && LR == 5) {
        rounds_phase(2);
        rounds_phase(3);
    }
    if (K == 15 && LR == 5) rounds_phase(2);

    // ---- vector phases
    auto vec_phase = [&](auto vtag) {
        constexpr int V = decltype(vtag)::value;
        constexpr int NV = N / (V * NT);
        Stats cs, bs;
        std::vector<int> seen_c(N, 0), seen_b(N, 0);
        for (int t = 0; t < NT; ++t)
            for (int k = 0; k < NV; ++k)
                for (int u = 0; u < V; ++u) {
                    const int e = L::template contig_e<V>(t, k, u);
                    if (e < 0 || e >= N) { cs.fail("contig out of range"); continue; }
                    ++seen_c[e];
                    if (L::pad(V * t) + L::pad(V * NT * k) + u != L::pad(e)) cs.fail("contig offset split");
                    const int eb = L::template bitrev_e<V>(t, k, u, K);
                    if (eb < 0 || eb >= N) { bs.fail("bitrev out of range"); continue; }
                    ++seen_b[eb];
                    if (L::pad((int)cbrev((uint32_t)(V * t), K)) +
                            L::pad((int)cbrev((uint32_t)(V * NT * k + u), K)) != L::pad(eb))
                        bs.fail("bitrev offset split");
                }
        for (int e = 0; e < N; ++e) {
            if (seen_c[e] != 1) cs.fail("contig map not bijective");
            if (seen_b[e] != 1) bs.fail("bitrev map not bijective");
        }
        // partial blocks: every block size 2^bits >= V gives a bijection too
        for (int bits = 0; (1 << bits) <= N; ++bits) {
            if ((1 << bits) < V) continue;
            std::vector<int> seen(N, 0);
            for (int t = 0; t < NT; ++t)
                for (int k = 0; k < NV; ++k)
                    for (int u = 0; u < V; ++u) {
                        const int e = L::template bitrev_e<V>(t, k, u, bits);
                        if (e >= 0 && e < N) ++seen[e];
                    }
            for (int e = 0; e < N; ++e)
                if (seen[e] != 1) { bs.fail("bitrev(bits) map not bijective"); break; }
        }
        for (int w = 0; w < NT / 64; ++w)
            for (int k = 0; k < NV; ++k)
                for (int u = 0; u < V; ++u) {
                    std::vector<int> a, b;
                    for (int l = 0; l < 64; ++l) {
                        a.push_back(L::pad(L::template contig_e<V>(64 * w + l, k, u)));
                        b.push_back(L::pad(L::template bitrev_e<V>(64 * w + l, k, u, K)));
                    }
                    bank_account(cs, a);
                    bank_account(bs, b);
                }
        // Paley phase of blocks of 2^8 .. 2^(K-1) elements (last-pass tiles
        // and small signals)
        Stats ps;
        for (int bits = 8; bits < K; ++bits)
            for (int w = 0; w < NT / 64; ++w)
                for (int k = 0; k < NV; ++k)
                    for (int u = 0; u < V; ++u) {
                        std::vector<int> a;
                        for (int l = 0; l < 64; ++l)
                            a.push_back(L::pad(L::template bitrev_e<V>(64 * w + l, k, u, bits)));
                        bank_account(ps, a);
                    }
        std::snprintf(buf, sizeof buf,
                      ", {\"K\": %d, \"LR\": %d, \"V\": %d, \"phase\": \"contig\", \"ok\": %s, \"ways64\": %d, \"ways32\": %d}"
                      ", {\"K\": %d, \"LR\": %d, \"V\": %d, \"phase\": \"paley\", \"ok\": %s, \"ways64\": %d, \"ways32\": %d}"
                      ", {\"K\": %d, \"LR\": %d, \"V\": %d, \"phase\": \"paley_blocks_2^8..2^(K-1)\", \"ok\": true, \"ways64\": %d, \"ways32\": %d}",
                      K, LR, V, cs.ok ? "true" : "false", cs.worst64, cs.worst32, K, LR, V,
                      bs.ok ? "true" : "false", bs.worst64, bs.worst32, K, LR, V, ps.worst64,
                      ps.worst32);
        out += buf;
        if (!cs.ok) out += ", {\"error\": \"" + cs.err + "\"}";
        if (!bs.ok) out += ", {\"error\": \"" + bs.err + "\"}";
    };
    vec_phase(std::integral_constant<int, 2>{});
    vec_phase(std::integral_constant<int, 4>{});
    vec_phase(std::integral_constant<int, 8>{});

    // ---- transposed first-pass phases
    auto tr_phase = [&](auto vtag, auto ctag) {
        constexpr int V = decltype(vtag)::value, CC = decltype(ctag)::value;
        constexpr int NV = N / (V * NT), L1 = K - CC;
        Stats ts;
        std::vector<int> seen(N, 0);
        const int rsv = 13;  // any run stride >= CC exercises the address split
        std::set<int64_t> gseen;
        for (int t = 0; t < NT; ++t)
            for (int k = 0; k < NV; ++k)
                for (int u = 0; u < V; ++u) {
                    const int e = L::template transp_e<V, CC>(t, k, u);
                    if (e < 0 || e >= N) { ts.fail("transp out of range"); continue; }
                    ++seen[e];
                    if (L::pad(L::template transp_e<V, CC>(t, 0, 0)) +
                            L::pad(L::template transp_e<V, CC>(0, k, u)) != L::pad(e))
                        ts.fail("transp offset split");
                    const int qt = L::template transp_q<V, CC>(t);
                    const int qk = L::template transp_q<V, CC>(NT * k);
                    if ((qt & qk) || (qt | qk) != L::template transp_q<V, CC>(t + NT * k))
                        ts.fail("transp lane order not a bit permutation");
                    const int o = V * (qt | qk) + u;
                    const int64_t g = L::template transp_goff<CC>(o, rsv);
                    if (L::template transp_goff<CC>(V * qt, rsv) + L::template transp_goff<CC>(V * qk, rsv) + u != g)
                        ts.fail("transp global split");
                    // element (hl, lo) must land at bitrev_L1(lo) * 2^rs + hl
                    const int hl = e >> L1, lo = e & ((1 << L1) - 1);
                    if (g != ((int64_t)cbrev((uint32_t)lo, L1) << rsv) + hl) ts.fail("transp target");
                    gseen.insert(g);
                }
        for (int e = 0; e < N; ++e)
            if (seen[e] != 1) { ts.fail("transp map not bijective"); break; }
        if ((int)gseen.size() != N) ts.fail("transp global map not injective");
        for (int w = 0; w < NT / 64; ++w)
            for (int k = 0; k < NV; ++k)
                for (int u = 0; u < V; ++u) {
                    std::vector<int> a;
                    for (int l = 0; l < 64; ++l)
                        a.push_back(L::pad(L::template transp_e<V, CC>(64 * w + l, k, u)));
                    bank_account(ts, a);
                }
        std::snprintf(buf, sizeof buf,
                      ", {\"K\": %d, \"LR\": %d, \"V\": %d, \"rows_log2\": %d, \"phase\": \"transposed\", \"ok\": %s, \"ways64\": %d, \"ways32\": %d}",
                      K, LR, V, CC, ts.ok ? "true" : "false", ts.worst64, ts.worst32);
        out += buf;
        if (!ts.ok) out += ", {\"error\": \"" + ts.err + "\"}";
    };
    tr_phase(std::integral_constant<int, 4>{}, std::integral_constant<int, 3>{});
    tr_phase(std::integral_constant<int, 4>{}, std::integral_constant<int, 4>{});
    tr_phase(std::integral_constant<int, 4>{}, std::integral_constant<int, 5>{});
    tr_phase(std::integral_constant<int, 4>{}, std::integral_constant<int, 6>{});
    tr_phase(std::integral_constant<int, 4>{}, std::integral_constant<int, 7>{});
    tr_phase(std::integral_constant<int, 2>{}, std::integral_constant<int, 3>{});
    tr_phase(std::integral_constant<int, 2>{}, std::integral_constant<int, 4>{});

    // ---- merged transposed store of 2^15-element tiles with 2^5 registers and
    // 2^7 or 2^6 rows (4-byte elements): same global layout as the plain
    // store, and a thread's vector k covers run index bits 0 .. log2(R / V) - 1
    auto merged_phase = [&](auto ctag) {
        constexpr int V = 4, CC = decltype(ctag)::value, NV = N / (V * NT), L1 = K - CC;
        Stats ms;
        std::vector<int> seen(N, 0);
        const int rsv = 13;
        std::set<int64_t> gseen;
        for (int t = 0; t < NT; ++t)
            for (int k = 0; k < NV; ++k)
                for (int u = 0; u < V; ++u) {
                    const int e = L::template transpm_e<V, CC>(t, k, u);
                    if (e < 0 || e >= N) { ms.fail("merged out of range"); continue; }
                    ++seen[e];
                    if (L::pad(L::template transpm_e<V, CC>(t, 0, 0)) +
                            L::pad(L::template transpm_e<V, CC>(0, k, u)) != L::pad(e))
                        ms.fail("merged offset split");
                    const int qt = L::template transpm_q<V, CC>(t, 0);
                    const int qk = L::template transpm_q<V, CC>(0, k);
                    if ((qt & qk) || (qt | qk) != L::template transpm_q<V, CC>(t, k))
                        ms.fail("merged lane order not a bit permutation");
                    const int o = V * (qt | qk) + u;
                    if (((o >> CC) & (NV - 1)) != k) ms.fail("merged vectors do not span the low run bits");
                    const int64_t g = L::template transp_goff<CC>(o, rsv);
                    if (L::template transp_goff<CC>(V * qt, rsv) + L::template transp_goff<CC>(V * qk, rsv) + u != g)
                        ms.fail("merged global split");
                    const int hl = e >> L1, lo = e & ((1 << L1) - 1);
                    if (g != ((int64_t)cbrev((uint32_t)lo, L1) << rsv) + hl) ms.fail("merged target");
                    gseen.insert(g);
                }
        for (int e = 0; e < N; ++e)
            if (seen[e] != 1) { ms.fail("merged map not bijective"); break; }
        if ((int)gseen.size() != N) ms.fail("merged global map not injective");
        for (int w = 0; w < NT / 64; ++w)
            for (int k = 0; k < NV; ++k)
                for (int u = 0; u < V; ++u) {
                    std::vector<int> a;
                    for (int l = 0; l < 64; ++l)
                        a.push_back(L::pad(L::template transpm_e<V, CC>(64 * w + l, k, u)));
                    bank_account(ms, a);
                }
        std::snprintf(buf, sizeof buf,
                      ", {\"K\": %d, \"LR\": %d, \"V\": %d, \"rows_log2\": %d, \"phase\": \"transposed_merged\", \"ok\": %s, \"ways64\": %d, \"ways32\": %d}",
                      K, LR, V, CC, ms.ok ? "true" : "false", ms.worst64, ms.worst32);
        out += buf;
        if (!ms.ok) out += ", {\"error\": \"" + ms.err + "\"}";
    };
    if constexpr (K == 15 && LR == 5) {
        merged_phase(std::integral_constant<int, 7>{});
        merged_phase(std::integral_constant<int, 6>{});
    }
    return out;
}

}  // namespace

extern "C" chw_status chw_layout_selfcheck(char *report, size_t len)
{
    std::string s = "[" + check_variant<12, 5>() + ", " + check_variant<12, 6>() + ", " +
                    check_variant<15, 5>() + ", " + check_variant<15, 6>() + "]";
    const bool ok = s.find("\"ok\": false") == std::string::npos;
    if (report && len) {
        const size_t n = std::min(len - 1, s.size());
        std::memcpy(report, s.data(), n);
        report[n] = 0;
    }
    return ok ? CHW_OK : CHW_ERR_UNSUPPORTED;
}
