// chw_api.cpp -- the C ABI of libchw: validation, device state, launches,
// hipGraph replay and the autotuner.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cerrno>
#include <cstdint>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <stdexcept>
#include <string>
#include <vector>

#include "chw.h"
#include "chw_planner.h"
#include "chw_scratch.h"
#include "chw_types.h"
#include "chw_variants.h"

using namespace chw;

namespace {

thread_local std::string t_last_error;

bool log_enabled()
{
    static const bool on = std::getenv("CHW_LOG") != nullptr;
    return on;
}

chw_status fail(chw_status s, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    std::vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    t_last_error = buf;
    if (log_enabled()) std::fprintf(stderr, "[libchw] %s: %s\n", chw_status_string(s), buf);
    return s;
}

chw_status hip_fail(hipError_t e, const char *what)
{
    return fail(CHW_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
}

// ---- per-device resources of a plan -----------------------------------------

struct GraphEntry {
    int adj;
    const void *x;
    void *y;
    void *ws;
    const uint32_t *signs;
    int sign_shared;
    int rounds;
    hipGraphExec_t exec;
};

// Random-sign diagonals of a call: `rounds` diagonals of `words` packed
// words each (none when w is null).
struct SignArgs {
    const uint32_t *w = nullptr;
    int shared = 0;
    int rounds = 1;
    size_t words = 0;
};

struct DeviceState {
    int version = -1;              // plan build the tables belong to
    Item *haar_items = nullptr;    // Haar pyramid table (built once per plan)
    Item *items = nullptr;
    int64_t *list = nullptr;
    int64_t *tiny_off = nullptr;
    int32_t *tiny_m = nullptr;
    hipStream_t cap = nullptr;     // private stream for graph capture
    std::vector<GraphEntry> graphs;
    // per looping kernel: resident workgroups per CU, CUs of the device
    std::map<const void *, std::pair<int, int>> grid_cap;
    std::vector<hipEvent_t> ev;    // per-launch timing events (option "timing")
    int ev_used = 0;               // events recorded by the last call

    void free_haar()
    {
        if (haar_items) (void)hipFree(haar_items);
        haar_items = nullptr;
    }
    void free_tables()
    {
        if (items) (void)hipFree(items);
        if (list) (void)hipFree(list);
        if (tiny_off) (void)hipFree(tiny_off);
        if (tiny_m) (void)hipFree(tiny_m);
        items = nullptr;
        list = nullptr;
        tiny_off = nullptr;
        tiny_m = nullptr;
        drop_graphs();
    }
    void drop_graphs()
    {
        for (GraphEntry &g : graphs) (void)hipGraphExecDestroy(g.exec);
        graphs.clear();
    }
    void free_events()
    {
        for (hipEvent_t e : ev) (void)hipEventDestroy(e);
        ev.clear();
        ev_used = 0;
    }
};

struct DeviceInfo {
    bool ok = false;
    std::string arch;
    int cus = 0;
};

std::mutex g_dev_mu;
std::map<int, DeviceInfo> g_dev_info;

}  // namespace

struct chw_plan_s {
    int64_t batch = 0;
    int dt = 0;
    chw_norm norm = CHW_ORTHONORMAL;
    uint32_t flags = 0;
    std::vector<int32_t> m;
    std::vector<int64_t> off;  // [batch]
    int64_t extent = 0;        // elements
    PlanConfig cfg;
    BuiltPlan built;
    int version = 0;
    bool used = false;
    bool timing = false;       // record a HIP event around every launch
    int last_dev = -1;         // device of the last call (for timings)
    bool tuned = false;        // configuration taken from the tuning cache
    bool haar_built = false;   // the Haar pyramid table (independent of tuning)
    HaarPlan haar;
    std::mutex mu;
    std::map<int, DeviceState> dev;
};

namespace {

// ---- tuning cache ------------------------------------------------------------
// Configurations found by chw_autotune, kept for the rest of the process (and
// written to / read from text files by chw_tuning_save / chw_tuning_load).
// A plan made without CHW_FLAG_NO_AUTOTUNE starts from the entry whose key
// matches it.  The key holds what decides the tuned choices: the dtype, the
// coefficient order, the launch form the flags fix, and the size mix (every
// log2 size present with the bit length of its signal count, so batches of
// the same sizes and similar counts share an entry).

std::mutex g_tune_mu;
std::map<std::string, PlanConfig> g_tune;

std::string tuning_key(int dt, int order, uint32_t flags, const std::vector<int32_t> &ms)
{
    int64_t cnt[31] = {0};
    for (int32_t m : ms)
        if (m >= 0 && m <= 30) ++cnt[m];
    std::string k = "dt" + std::to_string(dt) + "/order" + std::to_string(order) + "/form" +
                    std::to_string((flags & CHW_FLAG_PERSISTENT) ? 2 :
                                   (flags & CHW_FLAG_MULTI_LAUNCH) ? 1 : 0) +
                    ((flags & CHW_FLAG_THREE_PASS) ? "/three" : "") + "/m";
    for (int m = 0; m <= 30; ++m) {
        if (!cnt[m]) continue;
        int bl = 0;
        for (int64_t c = cnt[m]; c; c >>= 1) ++bl;
        k += "," + std::to_string(m) + ":" + std::to_string(bl);
    }
    return k;
}

// the tuned choices of a configuration (the others are the caller's)
void copy_tunables(const PlanConfig &from, PlanConfig *to)
{
    to->lr12 = from.lr12;
    to->lr15 = from.lr15;
    to->single15 = from.single15;
    to->split_l1 = from.split_l1;
    to->exec = from.exec;
    to->ptile = from.ptile;
    to->chunk = from.chunk;
    to->stream = from.stream;
    to->pipeline = from.pipeline;
    to->spread = from.spread;
    to->occupancy = from.occupancy;
}

struct TunableField {
    const char *name;
    int64_t lo, hi;
    int64_t PlanConfig::*i64;
    int PlanConfig::*i32;
};
const TunableField kTunables[] = {
    {"lr12", 0, 6, nullptr, &PlanConfig::lr12},
    {"lr15", 5, 6, nullptr, &PlanConfig::lr15},
    {"single15", 0, 1, nullptr, &PlanConfig::single15},
    {"split_l1", -1, 30, nullptr, &PlanConfig::split_l1},
    {"exec", 0, 2, nullptr, &PlanConfig::exec},
    {"ptile", 0, 15, nullptr, &PlanConfig::ptile},
    {"chunk", 0, INT64_MAX, &PlanConfig::chunk, nullptr},
    {"stream", 0, 2, nullptr, &PlanConfig::stream},
    {"pipeline", 0, 1, nullptr, &PlanConfig::pipeline},
    {"spread", 0, 1, nullptr, &PlanConfig::spread},
    {"occupancy", 0, 32, nullptr, &PlanConfig::occupancy},
};

chw_status rebuild(chw_plan_t p, const PlanConfig &cfg)
{
    try {
        BuiltPlan b;
        build_plan(p->m, p->off, p->dt, cfg, &b);
        p->built = std::move(b);
        p->cfg = cfg;
        ++p->version;
    } catch (const std::bad_alloc &) {
        return fail(CHW_ERR_OUT_OF_MEMORY, "host allocation failed while planning");
    } catch (const std::exception &e) {
        return fail(CHW_ERR_UNSUPPORTED, "%s", e.what());
    }
    return CHW_OK;
}

chw_status device_check(int *dev_out)
{
    int n = 0;
    hipError_t e = hipGetDeviceCount(&n);
    if (e != hipSuccess || n <= 0) {
        (void)hipGetLastError();
        return fail(CHW_ERR_NO_DEVICE, "no HIP device visible to this process");
    }
    int dev = 0;
    e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    std::lock_guard<std::mutex> lk(g_dev_mu);
    auto it = g_dev_info.find(dev);
    if (it == g_dev_info.end()) {
        DeviceInfo info;
        hipDeviceProp_t prop;
        e = hipGetDeviceProperties(&prop, dev);
        if (e != hipSuccess) return hip_fail(e, "hipGetDeviceProperties");
        info.arch = prop.gcnArchName;
        info.cus = prop.multiProcessorCount;
        info.ok = info.arch.rfind("gfx950", 0) == 0;
        it = g_dev_info.emplace(dev, info).first;
    }
    if (!it->second.ok)
        return fail(CHW_ERR_UNSUPPORTED, "device %d is %s; libchw is built for gfx950", dev,
                    it->second.arch.c_str());
    *dev_out = dev;
    return CHW_OK;
}

template <typename T>
chw_status upload(T **dst, const std::vector<T> &src)
{
    *dst = nullptr;
    if (src.empty()) return CHW_OK;
    hipError_t e = hipMalloc(reinterpret_cast<void **>(dst), src.size() * sizeof(T));
    if (e != hipSuccess) {
        *dst = nullptr;
        (void)hipGetLastError();
        return fail(CHW_ERR_OUT_OF_MEMORY, "hipMalloc of %zu bytes failed", src.size() * sizeof(T));
    }
    e = hipMemcpy(*dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpy of plan tables");
    return CHW_OK;
}

// Caller holds p->mu.
chw_status ensure_tables(chw_plan_t p, int dev, DeviceState **out)
{
    DeviceState &ds = p->dev[dev];
    if (ds.version != p->version) {
        ds.free_tables();
        chw_status s;
        if ((s = upload(&ds.items, p->built.items)) != CHW_OK) return s;
        if ((s = upload(&ds.list, p->built.list)) != CHW_OK) return s;
        if ((s = upload(&ds.tiny_off, p->built.tiny_off)) != CHW_OK) return s;
        if ((s = upload(&ds.tiny_m, p->built.tiny_m)) != CHW_OK) return s;
        ds.version = p->version;
    }
    *out = &ds;
    return CHW_OK;
}

// Grid of a looping kernel (persistent or prefetching): the workgroups that
// can be resident at once, or `occupancy` per CU when the plan sets it lower.
int looping_grid(DeviceState &ds, const void *fn, int nt, int occupancy, int nitems)
{
    std::pair<int, int> &cap = ds.grid_cap[fn];
    if (cap.first == 0) {
        int per_cu = 0, dev = 0, cus = 0;
        (void)hipGetDevice(&dev);
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, nt, 0) != hipSuccess ||
            per_cu < 1) {
            (void)hipGetLastError();
            per_cu = 1;
        }
        (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        cap = {per_cu, std::max(1, cus)};
    }
    const int per = occupancy > 0 ? std::min(cap.first, occupancy) : cap.first;
    return std::max(1, std::min(nitems, per * cap.second));
}

// Record timing event number `i` of this call (option "timing").
chw_status mark(chw_plan_t p, DeviceState &ds, int i, hipStream_t stream)
{
    if (!p->timing) return CHW_OK;
    while ((int)ds.ev.size() <= i) {
        hipEvent_t e;
        hipError_t err = hipEventCreate(&e);
        if (err != hipSuccess) return hip_fail(err, "hipEventCreate");
        ds.ev.push_back(e);
    }
    hipError_t err = hipEventRecord(ds.ev[i], stream);
    if (err != hipSuccess) return hip_fail(err, "hipEventRecord");
    ds.ev_used = i + 1;
    return CHW_OK;
}

// Enqueue the launches of one round (iteration `ri` of `sg.rounds`) on
// `stream`.  Single-pass launches, the tiny kernel and the persistent launch
// run every round inside themselves, so they are enqueued with iteration 0
// only; two-pass launches run one round each.  Timing events continue from
// the call's previous ones unless `fresh`.
// `phase` selects launches: 0 all; 1 the tiny kernel, single-pass launches
// and the pass a two-pass signal starts with (forward: first pass; adjoint:
// last pass); 2 the pass it ends with; 3 the tiny kernel and single-pass
// launches only; 4 the starting passes of two-pass signals only.
// `last_signed` (forward, phase 2): the last pass applies the iteration's
// diagonal to its output at the store.
chw_status enqueue(chw_plan_t p, DeviceState &ds, int adj, const void *x, void *y, void *inter,
                   int inter_is_io, hipStream_t stream, const SignArgs &sg = SignArgs{},
                   int ri = 0, bool fresh = true, int phase = 0, bool last_signed = false)
{
    const BuiltPlan &b = p->built;
    chw_status ms;
    if (fresh) {
        ds.ev_used = 0;
        if ((ms = mark(p, ds, 0, stream)) != CHW_OK) return ms;
    }
    int nev = p->timing ? ds.ev_used : 0;
    const int k = sg.w ? sg.rounds : 1;
    // diagonal of this iteration for two-pass launches (the adjoint runs the
    // rounds backwards)
    const uint32_t *w_round =
        sg.w ? sg.w + (size_t)(adj ? k - 1 - ri : ri) * sg.words : nullptr;
    LaunchArgs a{};
    a.in = x;
    a.out = y;
    a.inter = inter;
    a.inter_is_io = inter_is_io;
    a.list = ds.list;
    a.ortho = p->norm == CHW_ORTHONORMAL ? 1 : 0;
    a.sign_shared = sg.shared;
    a.sign_words = (int64_t)sg.words;
    // the dyadic order runs every round of single-pass work inside one launch;
    // the other orders run one launch per round for every launch
    const int order = b.cfg.order;
    const bool fuse = order == ORDER_DYADIC;
    if (!b.tiny_off.empty() && (ri == 0 || !fuse) && phase != 2 && phase != 4) {
        const TinyVariant *tv = find_tiny_variant(p->dt, adj);
        if (!tv) return fail(CHW_ERR_UNSUPPORTED, "no tiny kernel for this dtype");
        const int n = (int)b.tiny_off.size();
        hipError_t e = tv->launch(dim3((n + 255) / 256), dim3(256), stream, x, y, ds.tiny_off,
                                  ds.tiny_m, n, a.ortho, fuse ? sg.w : w_round, sg.shared,
                                  fuse ? k : 1, (int64_t)sg.words, order);
        if (e != hipSuccess) return hip_fail(e, "tiny kernel launch");
        if ((ms = mark(p, ds, nev++, stream)) != CHW_OK) return ms;
    }
    for (const LaunchRange &r : adj ? b.adj : b.fwd) {
        const bool in_launch_rounds = fuse && (r.persistent || r.single_pass);
        if (in_launch_rounds && ri > 0) continue;
        if (phase != 0) {
            const int kind = b.items[r.begin].kind;
            const bool start = r.single_pass || (adj ? kind == KIND_LAST : is_first_kind(kind));
            if ((phase != 2) != start) continue;
            if ((phase == 3 && !r.single_pass) || (phase == 4 && r.single_pass)) continue;
        }
        a.signs = in_launch_rounds ? sg.w : w_round;
        a.rounds = in_launch_rounds ? k : 1;
        // the middle pass of three-pass signals: first-pass tiles from one
        // intermediate to the other, in the compute type, no scale, no signs
        // (adjoint: from the second back to the first)
        const bool mid = r.role == 1;
        a.in = mid ? inter : x;
        a.out = mid ? inter : y;
        a.inter_is_io = mid ? 0 : inter_is_io;
        a.ortho = mid ? 0 : (p->norm == CHW_ORTHONORMAL ? 1 : 0);
        if (mid) {
            a.signs = nullptr;
            a.rounds = 1;
        }
        const ItemsVariant *v = find_items_variant(mid ? compute_dt(p->dt) : p->dt, r.K, r.LR, adj);
        if (!v || (r.persistent && !v->launch_persistent))
            return fail(CHW_ERR_UNSUPPORTED, "no tile kernel for dtype %d, K=%d, LR=%d", p->dt,
                        r.K, r.LR);
        a.items = ds.items + r.begin;
        a.nitems = r.end - r.begin;
        hipError_t e;
        const int occ = b.cfg.occupancy;
        if (last_signed) {
            if (!v->launch_last_signed)
                return fail(CHW_ERR_UNSUPPORTED, "no last-pass kernel with a store-side diagonal "
                            "for %d-bit tiles", r.K);
            e = v->launch_last_signed(dim3(a.nitems), stream, a);
        } else if (r.persistent) {
            if (!v->launch_persistent || !v->fn_persistent)
                return fail(CHW_ERR_UNSUPPORTED, "no persistent kernel for %d-bit tiles with %d registers",
                            r.K, r.LR);
            e = v->launch_persistent(dim3(looping_grid(ds, v->fn_persistent, v->nt, occ, a.nitems)),
                                     stream, a);
        } else if (r.stream > 0) {
            // every prefetching launch runs its kernel or fails: no silent
            // fallback to one workgroup per tile
            const bool dy = order == ORDER_DYADIC;
            const int slot = stream_slot(r.stream - 1);
            const void *fn = slot < 0 ? nullptr
                             : dy ? v->fn_stream[slot] : v->fn_stream_order[order - 1][slot];
            const ItemsLauncher lf = slot < 0 ? nullptr
                                     : dy ? v->launch_stream[slot]
                                          : v->launch_stream_order[order - 1][slot];
            if (!fn || !lf)
                return fail(CHW_ERR_UNSUPPORTED,
                            "no prefetching kernel for %d-bit tiles of kind %d in order %d", r.K,
                            r.stream - 1, order);
            e = lf(dim3(looping_grid(ds, fn, v->nt, occ, a.nitems)), stream, a);
        } else if (order != ORDER_DYADIC) {
            e = v->launch_order[order - 1](dim3(a.nitems), stream, a);
        } else {
            e = v->launch(dim3(a.nitems), stream, a);
        }
        if (e != hipSuccess) return hip_fail(e, "tile kernel launch");
        if ((ms = mark(p, ds, nev++, stream)) != CHW_OK) return ms;
    }
    return CHW_OK;
}

// The round-boundary launch between rounds ri - 1 and ri of a signed forward
// call: KIND_TURN tiles read round ri - 1's intermediate `src` and write round
// ri's intermediate `dst` (the workspace and y take turns).
chw_status enqueue_turn(chw_plan_t p, DeviceState &ds, int adj, void *src, int src_io,
                        void *dst, int dst_io, void *y, hipStream_t stream, const SignArgs &sg,
                        int ri)
{
    const BuiltPlan &b = p->built;
    int nev = p->timing ? ds.ev_used : 0;
    chw_status ms;
    for (const LaunchRange &r : b.turn) {
        const ItemsVariant *v = find_items_variant(p->dt, r.K, r.LR, adj);
        if (!v || !v->launch_turn)
            return fail(CHW_ERR_UNSUPPORTED, "no round-boundary kernel for dtype %d, LR=%d", p->dt,
                        r.LR);
        LaunchArgs a{};
        a.out = y;
        a.inter = src;
        a.inter_is_io = src_io;
        a.inter2 = dst;
        a.inter2_is_io = dst_io;
        a.items = ds.items + r.begin;
        a.nitems = r.end - r.begin;
        a.list = ds.list;
        a.ortho = p->norm == CHW_ORTHONORMAL ? 1 : 0;
        a.signs = sg.w + (size_t)ri * sg.words;
        a.sign_shared = sg.shared;
        a.sign_words = (int64_t)sg.words;
        a.rounds = 1;
        hipError_t e;
        // prefetching form: the forward's handles every row count; the adjoint's
        // is compiled per row count (the launch's items share one)
        ItemsLauncher sl = nullptr;
        const void *sfn = nullptr;
        if (r.stream) {
            if (!adj) {
                sl = v->launch_turn_stream;
                sfn = v->fn_turn_stream;
            } else {
                const Item &f = b.items[r.begin];
                const int cc = 15 - (f.m - f.bits);
                const int i = cc == K15_CA ? 0 : cc == K15_CM ? 1 : cc == K15_CB ? 2 : cc == K15_CD ? 3 : -1;
                if (i >= 0) {
                    sl = v->launch_turn_adj_stream[i];
                    sfn = v->fn_turn_adj_stream[i];
                }
            }
        }
        if (sl && sfn) {
            e = sl(dim3(looping_grid(ds, sfn, v->nt, b.cfg.occupancy, a.nitems)), stream, a);
        } else {
            e = v->launch_turn(dim3(a.nitems), stream, a);
        }
        if (e != hipSuccess) return hip_fail(e, "round-boundary kernel launch");
        if ((ms = mark(p, ds, nev++, stream)) != CHW_OK) return ms;
    }
    return CHW_OK;
}

// Every round of a call: iteration 0 runs all launches (single-pass tiles
// do every round); iterations 1.. run the two-pass launches again, reading y
// in place.  The adjoint walks the rounds backwards.  A signed forward call
// whose plan has round-boundary tiles instead runs: the first pass of round
// 0 (with the single-pass work), one round-boundary launch per later round,
// and the last pass of the final round -- k + 1 passes over the two-pass
// signals instead of 2k.  The adjoint does the same backwards: round k - 1's
// adjoint last pass, boundaries that end round r and start round r - 1, and
// round 0's adjoint first pass.
// A signed adjoint of a dyadic plan (one round, or several with round-boundary
// tiles) can run the forward launches: the Paley-ordered matrix is symmetric and its adjoint
// cascade performs the forward's additions in the forward's order, so
// D_1 H D_2 H ... D_k H g has the same bits either way.  Run forward, the
// chain is round 0 without a diagonal, boundary i applying D_{k+1-i}, and
// the last pass's output times D_1 -- its boundaries read their intermediate
// contiguously and write runs, where the adjoint's gather strided runs.
// Needs a store-side kernel for every last-pass launch, no persistent launch
// and no three-pass signal; option "adjoint" keeps the synthesis kernels.  A
// one-round call needs no boundary: first pass, then the last pass with D_1.
static bool adjoint_by_forward(chw_plan_t p)
{
    const BuiltPlan &b = p->built;
    if (b.cfg.order != ORDER_DYADIC || b.cfg.adjoint || b.n_three > 0) return false;
    for (const LaunchRange &r : b.fwd) {
        if (r.persistent) return false;
        if (r.single_pass || b.items[r.begin].kind != KIND_LAST) continue;
        const ItemsVariant *v = find_items_variant(p->dt, r.K, r.LR, 0);
        if (!v || !v->launch_last_signed) return false;
    }
    return true;
}

chw_status enqueue_rounds(chw_plan_t p, DeviceState &ds, int adj, const void *x, void *y,
                          void *ws, void *inter0, int inter_is_io0, hipStream_t stream,
                          const SignArgs &sg)
{
    const int k = sg.w ? sg.rounds : 1;
    if (sg.w && (k == 1 || !p->built.turn.empty()) && ws && adj && adjoint_by_forward(p)) {
        // single-pass work through the synthesis kernels (every round inside
        // the launch), then the forward chain of the two-pass signals; its
        // buffers alternate as in the forward call below
        auto buf = [&](int i) { return i % 2 != 0 ? y : ws; };
        chw_status s = enqueue(p, ds, 1, x, y, buf(0), 0, stream, sg, 0, true, 3);
        if (s == CHW_OK) s = enqueue(p, ds, 0, x, y, buf(0), 0, stream, SignArgs{}, 0, false, 4);
        for (int i = 1; i < k && s == CHW_OK; ++i)
            s = enqueue_turn(p, ds, 0, buf(i - 1), (i - 1) % 2, buf(i), i % 2, y, stream, sg, k - i);
        if (s != CHW_OK) return s;
        return enqueue(p, ds, 0, y, y, buf(k - 1), (k - 1) % 2, stream, sg, 0, false, 2, true);
    }
    if (k > 1 && !p->built.turn.empty() && ws) {
        // Intermediates 0 .. k-1 of the chain take turns between the workspace
        // and y.  A pass that reads transposed runs from all over a signal
        // must not write the buffer it reads: the forward's first pass reads x
        // (which may be y), so its chain starts in the workspace and ends with
        // the last pass in place on y; the adjoint's final first pass reads
        // the last intermediate, so its chain ends in the workspace (its
        // opening last pass, which reads and writes each tile's own range, may
        // write y).
        auto on_y = [&](int i) { return adj ? ((k - 1 - i) % 2 != 0) : (i % 2 != 0); };
        auto buf = [&](int i) { return on_y(i) ? y : ws; };
        chw_status s = enqueue(p, ds, adj, x, y, buf(0), on_y(0) ? 1 : 0, stream, sg, 0, true, 1);
        for (int i = 1; i < k && s == CHW_OK; ++i)
            s = enqueue_turn(p, ds, adj, buf(i - 1), on_y(i - 1) ? 1 : 0, buf(i), on_y(i) ? 1 : 0,
                             y, stream, sg, adj ? k - i : i);
        if (s != CHW_OK) return s;
        return enqueue(p, ds, adj, y, y, buf(k - 1), on_y(k - 1) ? 1 : 0, stream, sg, k - 1,
                       false, 2);
    }
    // later iterations have work when some launch runs one round at a time
    bool repeat = p->built.cfg.order != ORDER_DYADIC;
    for (const LaunchRange &r : p->built.fwd)
        if (!r.persistent && !r.single_pass) repeat = true;
    for (int i = 0; i < k; ++i) {
        if (i > 0 && !repeat) break;
        chw_status s = enqueue(p, ds, adj, i == 0 ? x : y, y, i == 0 ? inter0 : ws,
                               i == 0 ? inter_is_io0 : 0, stream, sg, i, i == 0);
        if (s != CHW_OK) return s;
    }
    return CHW_OK;
}

bool intervals_overlap(const void *a, size_t alen, const void *b, size_t blen)
{
    const char *x = static_cast<const char *>(a), *y = static_cast<const char *>(b);
    return x < y + blen && y < x + alen;
}

chw_status run(chw_plan_t p, int adj, const void *x, void *y, void *ws, void *stream_v,
               const SignArgs &sg = SignArgs{})
{
    if (!p) return fail(CHW_ERR_INVALID_ARGUMENT, "plan is NULL");
    if (p->batch == 0 || p->extent == 0) return CHW_OK;
    if (!x || !y) return fail(CHW_ERR_INVALID_ARGUMENT, "x and y must be device pointers");
    if ((reinterpret_cast<uintptr_t>(x) | reinterpret_cast<uintptr_t>(y)) & 15u)
        return fail(CHW_ERR_MISALIGNED, "x and y must be 16-byte aligned");
    const size_t bytes = (size_t)p->extent * (size_t)elem_bytes(p->dt);
    if (x != y && intervals_overlap(x, bytes, y, bytes))
        return fail(CHW_ERR_INVALID_ARGUMENT, "x and y overlap partially");
    void *inter = nullptr;
    int inter_is_io = 0;
    if (p->built.ws_elems > 0) {
        const bool narrow = p->dt == DT_BF16 || p->dt == DT_F16;
        if (ws) {
            if (reinterpret_cast<uintptr_t>(ws) & 15u)
                return fail(CHW_ERR_MISALIGNED, "workspace must be 16-byte aligned");
            const size_t wsb = p->built.ws_bound * (size_t)compute_bytes(p->dt);
            if (intervals_overlap(ws, wsb, x, bytes))
                return fail(CHW_ERR_INVALID_ARGUMENT, "workspace overlaps x");
            if (intervals_overlap(ws, wsb, y, bytes))
                return fail(CHW_ERR_INVALID_ARGUMENT, "workspace overlaps y");
            inter = ws;
        } else if (!adj && !narrow && x != y && p->built.n_three == 0 &&
                   p->built.cfg.order == ORDER_DYADIC) {
            // out-of-place forward: the intermediate goes through y.  Only in
            // the dyadic order, whose last-pass tiles store into the blocks
            // they loaded; the other orders' last passes store into other
            // blocks (sequency: block g to block invgray(g); natural: runs
            // across the signal) that tiles not yet run still have to load.
            inter = y;
            inter_is_io = 1;
            if (sg.w && sg.rounds > 1)
                return fail(CHW_ERR_INVALID_ARGUMENT,
                            "several rounds run in place on y and need a workspace of "
                            "chw_workspace_size() bytes");
        } else {
            return fail(CHW_ERR_INVALID_ARGUMENT,
                        "this call needs a workspace of chw_workspace_size() bytes");
        }
    }
    int dev = 0;
    chw_status s = device_check(&dev);
    if (s != CHW_OK) return s;
    hipStream_t stream = static_cast<hipStream_t>(stream_v);
    std::lock_guard<std::mutex> lk(p->mu);
    p->used = true;
    p->last_dev = dev;
    DeviceState *ds = nullptr;
    if ((s = ensure_tables(p, dev, &ds)) != CHW_OK) return s;
    if (!(p->flags & CHW_FLAG_GRAPH) || p->timing)
        return enqueue_rounds(p, *ds, adj, x, y, ws, inter, inter_is_io, stream, sg);

    // graph replay: capture once per (direction, buffers, diagonals) on a
    // private stream
    GraphEntry *ge = nullptr;
    for (GraphEntry &g : ds->graphs)
        if (g.adj == adj && g.x == x && g.y == y && g.ws == ws && g.signs == sg.w &&
            g.sign_shared == sg.shared && g.rounds == sg.rounds)
            ge = &g;
    if (!ge) {
        hipError_t e;
        if (!ds->cap) {
            e = hipStreamCreateWithFlags(&ds->cap, hipStreamNonBlocking);
            if (e != hipSuccess) return hip_fail(e, "hipStreamCreate");
        }
        if (ds->graphs.size() >= 16) {
            (void)hipGraphExecDestroy(ds->graphs.front().exec);
            ds->graphs.erase(ds->graphs.begin());
        }
        e = hipStreamBeginCapture(ds->cap, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) return hip_fail(e, "hipStreamBeginCapture");
        chw_status es = enqueue_rounds(p, *ds, adj, x, y, ws, inter, inter_is_io, ds->cap, sg);
        hipGraph_t graph = nullptr;
        e = hipStreamEndCapture(ds->cap, &graph);
        if (es != CHW_OK) {
            if (graph) (void)hipGraphDestroy(graph);
            return es;
        }
        if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
        hipGraphExec_t exec = nullptr;
        e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (e != hipSuccess) return hip_fail(e, "hipGraphInstantiate");
        ds->graphs.push_back(GraphEntry{adj, x, y, ws, sg.w, sg.shared, sg.rounds, exec});
        ge = &ds->graphs.back();
    }
    hipError_t e = hipGraphLaunch(ge->exec, stream);
    if (e != hipSuccess) return hip_fail(e, "hipGraphLaunch");
    return CHW_OK;
}

}  // namespace

extern "C" {

const char *chw_status_string(chw_status s)
{
    switch (s) {
    case CHW_OK: return "CHW_OK";
    case CHW_ERR_INVALID_ARGUMENT: return "CHW_ERR_INVALID_ARGUMENT";
    case CHW_ERR_UNSUPPORTED: return "CHW_ERR_UNSUPPORTED";
    case CHW_ERR_MISALIGNED: return "CHW_ERR_MISALIGNED";
    case CHW_ERR_OUT_OF_MEMORY: return "CHW_ERR_OUT_OF_MEMORY";
    case CHW_ERR_NO_DEVICE: return "CHW_ERR_NO_DEVICE";
    case CHW_ERR_HIP: return "CHW_ERR_HIP";
    case CHW_ERR_DEVICE: return "CHW_ERR_DEVICE";
    }
    return "CHW_ERR_UNKNOWN";
}

const char *chw_last_error(void) { return t_last_error.c_str(); }

const char *chw_version(void) { return "libchw 0.1 (gfx950)"; }

chw_status chw_plan(chw_plan_t *plan, int64_t batch, const int32_t *log2_sizes,
                    const int64_t *offsets, chw_dtype dtype, chw_norm norm, uint32_t flags)
{
    t_last_error.clear();
    if (!plan) return fail(CHW_ERR_INVALID_ARGUMENT, "plan output pointer is NULL");
    *plan = nullptr;
    if (batch < 0) return fail(CHW_ERR_INVALID_ARGUMENT, "batch %lld < 0", (long long)batch);
    if (batch > 0 && !log2_sizes) return fail(CHW_ERR_INVALID_ARGUMENT, "log2_sizes is NULL");
    if ((int)dtype < 0 || (int)dtype > 4) return fail(CHW_ERR_INVALID_ARGUMENT, "bad dtype %d", (int)dtype);
    if ((int)norm < 0 || (int)norm > 1) return fail(CHW_ERR_INVALID_ARGUMENT, "bad norm %d", (int)norm);
    if (dtype == CHW_I32 && norm != CHW_UNNORMALIZED)
        return fail(CHW_ERR_UNSUPPORTED, "the integer type has only the unnormalized form");
    const uint32_t known = CHW_FLAG_GRAPH | CHW_FLAG_NO_AUTOTUNE | CHW_FLAG_PERSISTENT |
                           CHW_FLAG_MULTI_LAUNCH | CHW_FLAG_ORDER_SEQUENCY |
                           CHW_FLAG_ORDER_NATURAL | CHW_FLAG_THREE_PASS;
    if (flags & ~known) return fail(CHW_ERR_INVALID_ARGUMENT, "unknown flag bits 0x%x", flags & ~known);
    if ((flags & CHW_FLAG_PERSISTENT) && (flags & CHW_FLAG_MULTI_LAUNCH))
        return fail(CHW_ERR_INVALID_ARGUMENT, "PERSISTENT and MULTI_LAUNCH are exclusive");
    if ((flags & CHW_FLAG_ORDER_SEQUENCY) && (flags & CHW_FLAG_ORDER_NATURAL))
        return fail(CHW_ERR_INVALID_ARGUMENT, "ORDER_SEQUENCY and ORDER_NATURAL are exclusive");
    if ((flags & (CHW_FLAG_ORDER_SEQUENCY | CHW_FLAG_ORDER_NATURAL)) && (flags & CHW_FLAG_PERSISTENT))
        return fail(CHW_ERR_UNSUPPORTED, "the persistent launch computes the dyadic order only");
    if ((flags & CHW_FLAG_THREE_PASS) && (flags & CHW_FLAG_PERSISTENT))
        return fail(CHW_ERR_INVALID_ARGUMENT, "THREE_PASS and PERSISTENT are exclusive");
    if ((flags & CHW_FLAG_THREE_PASS) && (flags & (CHW_FLAG_ORDER_SEQUENCY | CHW_FLAG_ORDER_NATURAL)))
        return fail(CHW_ERR_UNSUPPORTED, "three-pass signals compute the dyadic order only");
    const int dt = (int)dtype;
    const int maxm = dtype == CHW_F64 ? CHW_MAX_LOG2_F64 : CHW_MAX_LOG2;
    const int es = elem_bytes(dt);
    chw_plan_s *p = nullptr;
    try {
        p = new chw_plan_s();
        p->batch = batch;
        p->dt = dt;
        p->norm = norm;
        p->flags = flags;
        p->m.assign(log2_sizes, log2_sizes + batch);
        p->off.resize((size_t)batch);
    } catch (const std::bad_alloc &) {
        delete p;
        return fail(CHW_ERR_OUT_OF_MEMORY, "host allocation failed");
    }
    auto bad = [&](chw_status s) {
        delete p;
        return s;
    };
    int64_t pos = 0;
    for (int64_t i = 0; i < batch; ++i) {
        const int m = log2_sizes[i];
        if (m < 0 || m > 30)
            return bad(fail(CHW_ERR_INVALID_ARGUMENT, "log2_sizes[%lld] = %d outside [0, 30]",
                            (long long)i, m));
        if (m > maxm)
            return bad(fail(CHW_ERR_UNSUPPORTED, "log2_sizes[%lld] = %d exceeds %d for this dtype",
                            (long long)i, m, maxm));
        const int64_t n = (int64_t)1 << m;
        int64_t o;
        if (offsets) {
            o = offsets[i];
            if (o < 0 || o < pos)
                return bad(fail(CHW_ERR_INVALID_ARGUMENT,
                                "offsets[%lld] = %lld is negative or overlaps the previous signal",
                                (long long)i, (long long)o));
            if (o > (((int64_t)1 << 62) - n))
                return bad(fail(CHW_ERR_OUT_OF_MEMORY, "offsets[%lld] overflows", (long long)i));
        } else {
            o = pos;
            if (o > (((int64_t)1 << 62) - n))
                return bad(fail(CHW_ERR_OUT_OF_MEMORY, "packed batch overflows"));
        }
        if (n * es >= 16 && ((o * es) & 15))
            return bad(fail(CHW_ERR_MISALIGNED, "signal %lld starts at element %lld, not 16-byte aligned",
                            (long long)i, (long long)o));
        p->off[(size_t)i] = o;
        pos = o + n;
    }
    if (offsets) {
        if (offsets[batch] < pos)
            return bad(fail(CHW_ERR_INVALID_ARGUMENT, "offsets[batch] = %lld is below the end of the last signal",
                            (long long)offsets[batch]));
        p->extent = offsets[batch];
    } else {
        p->extent = pos;
    }
    if (p->extent > (((int64_t)1 << 62) / 8)) return bad(fail(CHW_ERR_OUT_OF_MEMORY, "extent overflows"));
    PlanConfig cfg;
    if (flags & CHW_FLAG_PERSISTENT) cfg.exec = 2;
    if (flags & CHW_FLAG_THREE_PASS) cfg.three_min = 20;
    if (flags & CHW_FLAG_ORDER_SEQUENCY) cfg.order = ORDER_SEQUENCY;
    if (flags & CHW_FLAG_ORDER_NATURAL) cfg.order = ORDER_NATURAL;
    if (!(flags & CHW_FLAG_NO_AUTOTUNE)) {
        bool hit = false;
        PlanConfig tuned = cfg;
        {
            std::lock_guard<std::mutex> lk(g_tune_mu);
            auto it = g_tune.find(tuning_key(dt, cfg.order, flags, p->m));
            if (it != g_tune.end()) {
                copy_tunables(it->second, &tuned);
                hit = true;
            }
        }
        // an entry the planner cannot take leaves the plan untuned
        if (hit && rebuild(p, tuned) == CHW_OK) {
            p->tuned = true;
            t_last_error.clear();
            *plan = p;
            return CHW_OK;
        }
    }
    chw_status s = rebuild(p, cfg);
    if (s != CHW_OK) return bad(s);
    t_last_error.clear();
    *plan = p;
    return CHW_OK;
}

chw_status chw_plan_haar_walsh(chw_plan_t *plan, int64_t batch, int32_t m, chw_dtype dtype,
                               chw_norm norm, uint32_t flags)
{
    if (!plan) return fail(CHW_ERR_INVALID_ARGUMENT, "plan output pointer is NULL");
    *plan = nullptr;
    if (batch < 0) return fail(CHW_ERR_INVALID_ARGUMENT, "batch %lld < 0", (long long)batch);
    if (m < 0 || m > 30) return fail(CHW_ERR_INVALID_ARGUMENT, "m = %d outside [0, 30]", m);
    // blocks of one signal: w_0 (H_0 = 1), then H_k on [2^k, 2^{k+1}) for
    // k = 0 .. m-1
    const int64_t per = m == 0 ? 1 : (int64_t)m + 1;
    if (batch > ((int64_t)1 << 40) / per) return fail(CHW_ERR_OUT_OF_MEMORY, "batch too large");
    std::vector<int32_t> sizes;
    std::vector<int64_t> offs;
    try {
        sizes.reserve((size_t)(batch * per));
        offs.reserve((size_t)(batch * per + 1));
    } catch (const std::bad_alloc &) {
        return fail(CHW_ERR_OUT_OF_MEMORY, "host allocation failed");
    }
    for (int64_t i = 0; i < batch; ++i) {
        const int64_t base = i << m;
        sizes.push_back(0);
        offs.push_back(base);
        for (int k = 0; k < m; ++k) {
            sizes.push_back(k);
            offs.push_back(base + ((int64_t)1 << k));
        }
    }
    offs.push_back(batch << m);
    return chw_plan(plan, (int64_t)sizes.size(), sizes.data(), offs.data(), dtype, norm, flags);
}

chw_status chw_workspace_size(chw_plan_t plan, size_t *bytes)
{
    if (!plan || !bytes) return fail(CHW_ERR_INVALID_ARGUMENT, "NULL argument");
    // the bound over every configuration, so that tuning or options can never
    // need more than what a caller sized from this call
    *bytes = plan->built.ws_bound * (size_t)compute_bytes(plan->dt);
    return CHW_OK;
}

chw_status chw_forward(chw_plan_t plan, const void *x, void *y, void *workspace, void *stream)
{
    return run(plan, 0, x, y, workspace, stream);
}

chw_status chw_forward_noalloc(chw_plan_t plan, const void *x, void *y, void *stream_v)
{
    chw_plan_t p = plan;
    if (!p) return fail(CHW_ERR_INVALID_ARGUMENT, "plan is NULL");
    if (p->batch == 0 || p->extent == 0) return CHW_OK;
    if (!x || !y) return fail(CHW_ERR_INVALID_ARGUMENT, "x and y must be device pointers");
    if ((reinterpret_cast<uintptr_t>(x) | reinterpret_cast<uintptr_t>(y)) & 15u)
        return fail(CHW_ERR_MISALIGNED, "x and y must be 16-byte aligned");
    const size_t bytes = (size_t)p->extent * (size_t)elem_bytes(p->dt);
    if (x != y && intervals_overlap(x, bytes, y, bytes))
        return fail(CHW_ERR_INVALID_ARGUMENT, "x and y overlap partially");
    // the intermediate of the plan's current configuration goes to the static
    // scratch; every other byte the call touches is the caller's
    const size_t need = p->built.ws_elems * (size_t)compute_bytes(p->dt);
    if (need > SCRATCH_BYTES)
        return fail(CHW_ERR_UNSUPPORTED,
                    "the plan's intermediate needs %zu bytes; the static scratch of "
                    "chw_forward_noalloc holds %zu (use chw_forward with a workspace)",
                    need, (size_t)SCRATCH_BYTES);
    int dev = 0;
    chw_status s = device_check(&dev);
    if (s != CHW_OK) return s;
    std::lock_guard<std::mutex> lk(p->mu);
    if (p->timing)
        return fail(CHW_ERR_UNSUPPORTED,
                    "option \"timing\" creates events; chw_forward_noalloc records none");
    auto it = p->dev.find(dev);
    if (it == p->dev.end() || it->second.version != p->version)
        return fail(CHW_ERR_UNSUPPORTED,
                    "the plan's work tables are not on device %d yet (one chw_forward or "
                    "chw_backward call on this device uploads them)", dev);
    void *ws = nullptr;
    if (need > 0) {
        hipError_t e = scratch_address(dev, &ws);
        if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress of the static scratch");
    }
    p->used = true;
    p->last_dev = dev;
    // launched directly (no graph capture, which would allocate)
    return enqueue_rounds(p, it->second, 0, x, y, ws, ws, 0, static_cast<hipStream_t>(stream_v),
                          SignArgs{});
}

chw_status chw_backward(chw_plan_t plan, const void *g, void *y, void *workspace, void *stream)
{
    // dyadic order: H^T = H, and the forward launches give the adjoint
    // cascade's bits (option "adjoint" selects the synthesis kernels)
    const bool synth = !plan || plan->cfg.order != ORDER_DYADIC || plan->cfg.adjoint;
    return run(plan, synth ? 1 : 0, g, y, workspace, stream);
}

static chw_status run_haar(chw_plan_t p, int adj, const void *x, void *y, void *ws,
                           void *stream_v)
{
    if (!p) return fail(CHW_ERR_INVALID_ARGUMENT, "plan is NULL");
    if (p->batch == 0 || p->extent == 0) return CHW_OK;
    if (!x || !y) return fail(CHW_ERR_INVALID_ARGUMENT, "x and y must be device pointers");
    if ((reinterpret_cast<uintptr_t>(x) | reinterpret_cast<uintptr_t>(y)) & 15u)
        return fail(CHW_ERR_MISALIGNED, "x and y must be 16-byte aligned");
    const size_t bytes = (size_t)p->extent * (size_t)elem_bytes(p->dt);
    if (intervals_overlap(x, bytes, y, bytes))
        return fail(CHW_ERR_INVALID_ARGUMENT, "the Haar transform needs distinct x and y");
    {
        std::lock_guard<std::mutex> lk(p->mu);
        if (!p->haar_built) {
            try {
                build_haar_plan(p->m, p->off, &p->haar);
            } catch (const std::bad_alloc &) {
                return fail(CHW_ERR_OUT_OF_MEMORY, "host allocation failed while planning");
            }
            p->haar_built = true;
        }
    }
    if (p->haar.ws_elems > 0) {
        if (!ws)
            return fail(CHW_ERR_INVALID_ARGUMENT,
                        "signals above 2^12 need a workspace of chw_workspace_size() bytes");
        if (reinterpret_cast<uintptr_t>(ws) & 15u)
            return fail(CHW_ERR_MISALIGNED, "workspace must be 16-byte aligned");
        const size_t wsb = p->haar.ws_elems * (size_t)compute_bytes(p->dt);
        if (intervals_overlap(ws, wsb, x, bytes) || intervals_overlap(ws, wsb, y, bytes))
            return fail(CHW_ERR_INVALID_ARGUMENT, "workspace overlaps x or y");
    }
    int dev = 0;
    chw_status s = device_check(&dev);
    if (s != CHW_OK) return s;
    const HaarVariant *hv = find_haar_variant(p->dt, adj);
    if (!hv) return fail(CHW_ERR_UNSUPPORTED, "no Haar kernel for this dtype");
    hipStream_t stream = static_cast<hipStream_t>(stream_v);
    std::lock_guard<std::mutex> lk(p->mu);
    p->used = true;
    p->last_dev = dev;
    DeviceState &ds = p->dev[dev];
    if (!ds.haar_items && !p->haar.items.empty())
        if ((s = upload(&ds.haar_items, p->haar.items)) != CHW_OK) return s;
    ds.ev_used = 0;
    if ((s = mark(p, ds, 0, stream)) != CHW_OK) return s;
    int nev = 1;
    LaunchArgs a{};
    a.in = x;
    a.out = y;
    a.inter = ws;
    a.ortho = p->norm == CHW_ORTHONORMAL ? 1 : 0;
    a.rounds = 1;
    const int np = (int)p->haar.passes.size();
    for (int i = 0; i < np; ++i) {
        const LaunchRange &r = p->haar.passes[adj ? np - 1 - i : i];
        a.items = ds.haar_items + r.begin;
        a.nitems = r.end - r.begin;
        hipError_t e = hv->launch(dim3(a.nitems), stream, a);
        if (e != hipSuccess) return hip_fail(e, "Haar kernel launch");
        if ((s = mark(p, ds, nev++, stream)) != CHW_OK) return s;
    }
    return CHW_OK;
}

chw_status chw_haar_forward(chw_plan_t plan, const void *x, void *y, void *workspace,
                            void *stream)
{
    return run_haar(plan, 0, x, y, workspace, stream);
}

chw_status chw_haar_backward(chw_plan_t plan, const void *g, void *y, void *workspace,
                             void *stream)
{
    return run_haar(plan, 1, g, y, workspace, stream);
}

chw_status chw_sign_words(chw_plan_t plan, chw_sign_mode mode, size_t *words)
{
    if (!plan || !words) return fail(CHW_ERR_INVALID_ARGUMENT, "NULL argument");
    if (mode != CHW_SIGNS_PER_ELEMENT && mode != CHW_SIGNS_SHARED)
        return fail(CHW_ERR_INVALID_ARGUMENT, "bad sign mode %d", (int)mode);
    int64_t bits = 0;
    if (mode == CHW_SIGNS_SHARED) {
        for (int32_t m : plan->m) bits = std::max(bits, (int64_t)1 << m);
    } else {
        bits = plan->extent;
    }
    *words = (size_t)((bits + 31) / 32);
    return CHW_OK;
}

chw_status chw_philox_signs(chw_plan_t plan, chw_sign_mode mode, uint64_t seed, int rounds,
                            uint32_t *signs, void *stream)
{
    if (!plan) return fail(CHW_ERR_INVALID_ARGUMENT, "plan is NULL");
    if (!signs) return fail(CHW_ERR_INVALID_ARGUMENT, "signs is NULL");
    if (reinterpret_cast<uintptr_t>(signs) & 3u)
        return fail(CHW_ERR_MISALIGNED, "signs must be 4-byte aligned");
    if (rounds < 1 || rounds > CHW_MAX_ROUNDS)
        return fail(CHW_ERR_INVALID_ARGUMENT, "rounds = %d outside [1, %d]", rounds, CHW_MAX_ROUNDS);
    size_t words = 0;
    chw_status s = chw_sign_words(plan, mode, &words);
    if (s != CHW_OK) return s;
    if (words == 0) return CHW_OK;
    int dev = 0;
    if ((s = device_check(&dev)) != CHW_OK) return s;
    int cus = 0;
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    hipError_t e = launch_philox_signs(signs, (int64_t)words, rounds, seed, cus,
                                       static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "Philox sign kernel launch");
    return CHW_OK;
}

// ---- the factor-by-factor node evaluation (Sec. 4) ----------------------------

static chw_status nodes_shape(chw_plan_t p, int *m_out)
{
    if (!p) return fail(CHW_ERR_INVALID_ARGUMENT, "plan is NULL");
    if (p->dt != DT_F32 || p->norm != CHW_ORTHONORMAL || p->cfg.order != ORDER_DYADIC)
        return fail(CHW_ERR_UNSUPPORTED,
                    "the node evaluation takes orthonormal dyadic CHW_F32 plans only");
    const int m = p->batch > 0 ? p->m[0] : 1;
    if (m < 1 || m > 24) return fail(CHW_ERR_UNSUPPORTED, "the node evaluation takes 1 <= m <= 24");
    for (int64_t i = 0; i < p->batch; ++i)
        if (p->m[i] != m || p->off[i] != (i << m))
            return fail(CHW_ERR_UNSUPPORTED,
                        "the node evaluation takes equal sizes packed back to back");
    *m_out = m;
    return CHW_OK;
}

static size_t nodes_ws_elems(int64_t signals, int m)
{
    return (size_t)(signals << m) + (m > 12 ? (size_t)(signals << (m - 12)) : 0);
}

chw_status chw_nodes_workspace_size(chw_plan_t plan, size_t *bytes)
{
    if (!bytes) return fail(CHW_ERR_INVALID_ARGUMENT, "bytes is NULL");
    int m = 0;
    chw_status s = nodes_shape(plan, &m);
    if (s != CHW_OK) return s;
    *bytes = nodes_ws_elems(plan->batch, m) * sizeof(float);
    return CHW_OK;
}

chw_status chw_nodes_forward(chw_plan_t plan, const void *x, void *y, void *workspace,
                             int64_t chunk, void *stream)
{
    int m = 0;
    chw_status s = nodes_shape(plan, &m);
    if (s != CHW_OK) return s;
    if (chunk < 0) return fail(CHW_ERR_INVALID_ARGUMENT, "chunk = %lld < 0", (long long)chunk);
    const int64_t batch = plan->batch;
    if (batch == 0) return CHW_OK;
    if (!x || !y || !workspace)
        return fail(CHW_ERR_INVALID_ARGUMENT, "x, y and workspace must be device pointers");
    if ((reinterpret_cast<uintptr_t>(x) | reinterpret_cast<uintptr_t>(y) |
         reinterpret_cast<uintptr_t>(workspace)) & 3u)
        return fail(CHW_ERR_MISALIGNED, "x, y and workspace must be 4-byte aligned");
    const int64_t per = chunk > 0 && chunk < batch ? chunk : batch;
    const size_t bytes = (size_t)(batch << m) * sizeof(float);
    const size_t wsb = nodes_ws_elems(per, m) * sizeof(float);
    if (intervals_overlap(x, bytes, y, bytes) || intervals_overlap(workspace, wsb, x, bytes) ||
        intervals_overlap(workspace, wsb, y, bytes))
        return fail(CHW_ERR_INVALID_ARGUMENT, "x, y and workspace must not overlap");
    int dev = 0;
    if ((s = device_check(&dev)) != CHW_OK) return s;
    int cus = 0;
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    hipStream_t st = static_cast<hipStream_t>(stream);
    float *ws = static_cast<float *>(workspace);
    float *sums = ws + (per << m);
    for (int64_t c0 = 0; c0 < batch; c0 += per) {
        const int64_t nb = std::min(per, batch - c0);
        const float *in = static_cast<const float *>(x) + (c0 << m);
        float *yc = static_cast<float *>(y) + (c0 << m);
        // node r writes y when m - 1 - r is even, else the workspace, so that
        // the last node lands in y and no node reads what it writes
        for (int r = 0; r < m; ++r) {
            float *out = ((m - 1 - r) % 2 == 0) ? yc : ws;
            hipError_t e = launch_node(in, out, sums, nb, m, r, cus, st);
            if (e != hipSuccess) return hip_fail(e, "node kernel launch");
            in = out;
        }
    }
    return CHW_OK;
}

static chw_status run_signed(chw_plan_t plan, int adj, const void *x, void *y, void *workspace,
                             const uint32_t *signs, chw_sign_mode mode, int rounds, void *stream)
{
    if (!plan) return fail(CHW_ERR_INVALID_ARGUMENT, "plan is NULL");
    if (!signs) return fail(CHW_ERR_INVALID_ARGUMENT, "signs is NULL");
    if (reinterpret_cast<uintptr_t>(signs) & 3u)
        return fail(CHW_ERR_MISALIGNED, "signs must be 4-byte aligned");
    if (rounds < 1 || rounds > CHW_MAX_ROUNDS)
        return fail(CHW_ERR_INVALID_ARGUMENT, "rounds = %d outside [1, %d]", rounds, CHW_MAX_ROUNDS);
    SignArgs sg;
    chw_status s = chw_sign_words(plan, mode, &sg.words);
    if (s != CHW_OK) return s;
    sg.w = signs;
    sg.shared = mode == CHW_SIGNS_SHARED ? 1 : 0;
    sg.rounds = rounds;
    return run(plan, adj, x, y, workspace, stream, sg);
}

chw_status chw_forward_signed(chw_plan_t plan, const void *x, void *y, void *workspace,
                              const uint32_t *signs, chw_sign_mode mode, int rounds, void *stream)
{
    return run_signed(plan, 0, x, y, workspace, signs, mode, rounds, stream);
}

chw_status chw_backward_signed(chw_plan_t plan, const void *g, void *y, void *workspace,
                               const uint32_t *signs, chw_sign_mode mode, int rounds, void *stream)
{
    return run_signed(plan, 1, g, y, workspace, signs, mode, rounds, stream);
}

chw_status chw_plan_destroy(chw_plan_t plan)
{
    if (!plan) return CHW_OK;
    {
        std::lock_guard<std::mutex> lk(plan->mu);
        int cur = -1;
        (void)hipGetDevice(&cur);
        for (auto &kv : plan->dev) {
            if (kv.first != cur) (void)hipSetDevice(kv.first);
            kv.second.free_tables();
            kv.second.free_haar();
            kv.second.free_events();
            if (kv.second.cap) (void)hipStreamDestroy(kv.second.cap);
        }
        if (cur >= 0) (void)hipSetDevice(cur);
    }
    delete plan;
    return CHW_OK;
}

chw_status chw_plan_set_option(chw_plan_t plan, const char *key, int64_t value)
{
    if (!plan || !key) return fail(CHW_ERR_INVALID_ARGUMENT, "NULL argument");
    std::lock_guard<std::mutex> lk(plan->mu);
    const std::string k = key;
    if (k == "timing" && (value == 0 || value == 1)) {  // instrumentation only
        plan->timing = value != 0;
        return CHW_OK;
    }
    if (plan->used) return fail(CHW_ERR_INVALID_ARGUMENT, "plan already used; options are fixed");
    PlanConfig cfg = plan->cfg;
    if (k == "lr12" && (value == 0 || value == 5 || value == 6)) cfg.lr12 = (int)value;
    else if (k == "lr15" && (value == 5 || value == 6)) cfg.lr15 = (int)value;
    else if (k == "single15" && (value == 0 || value == 1)) cfg.single15 = (int)value;
    else if (k == "split_l1" && value >= -1 && value <= 30) cfg.split_l1 = (int)value;
    else if (k == "exec" && value == 1)
        return fail(CHW_ERR_UNSUPPORTED,
                    "exec 1 (dependency-counter work queue) is disabled");
    else if (k == "exec" && (value == 0 || value == 2)) cfg.exec = (int)value;
    else if (k == "ptile" && (value == 0 || value == 12 || value == 15)) cfg.ptile = (int)value;
    else if (k == "chunk" && value >= 0) cfg.chunk = value;
    else if (k == "stream" && value >= 0 && value <= 2) cfg.stream = (int)value;
    else if (k == "pipeline" && (value == 0 || value == 1)) cfg.pipeline = (int)value;
    else if (k == "turn" && (value == 0 || value == 1)) cfg.turn = (int)value;
    else if (k == "adjoint" && (value == 0 || value == 1)) cfg.adjoint = (int)value;
    else if (k == "spread" && (value == 0 || value == 1)) cfg.spread = (int)value;
    else if (k == "occupancy" && value >= 0 && value <= 32) cfg.occupancy = (int)value;
    else return fail(CHW_ERR_INVALID_ARGUMENT, "unknown option %s = %lld", key, (long long)value);
    const chw_status s = rebuild(plan, cfg);
    if (s == CHW_OK) plan->tuned = false;  // the caller's choice now
    return s;
}

chw_status chw_launch_times(chw_plan_t plan, float *ms, int *n)
{
    if (!plan || !n || (*n > 0 && !ms)) return fail(CHW_ERR_INVALID_ARGUMENT, "NULL argument");
    std::lock_guard<std::mutex> lk(plan->mu);
    if (!plan->timing || plan->last_dev < 0)
        return fail(CHW_ERR_INVALID_ARGUMENT, "option \"timing\" is off or the plan was not run");
    DeviceState &ds = plan->dev[plan->last_dev];
    const int launches = ds.ev_used > 0 ? ds.ev_used - 1 : 0;
    if (launches == 0) {
        *n = 0;
        return CHW_OK;
    }
    hipError_t e = hipEventSynchronize(ds.ev[launches]);
    if (e != hipSuccess) return hip_fail(e, "hipEventSynchronize");
    const int k = std::min(*n, launches);
    for (int i = 0; i < k; ++i) {
        e = hipEventElapsedTime(&ms[i], ds.ev[i], ds.ev[i + 1]);
        if (e != hipSuccess) return hip_fail(e, "hipEventElapsedTime");
    }
    *n = launches;
    return CHW_OK;
}

chw_status chw_plan_check(chw_plan_t plan)
{
    if (!plan) return fail(CHW_ERR_INVALID_ARGUMENT, "plan is NULL");
    std::lock_guard<std::mutex> lk(plan->mu);
    std::string err;
    if (!check_plan(plan->m, plan->off, plan->dt, plan->built, &err))
        return fail(CHW_ERR_UNSUPPORTED, "plan check failed: %s", err.c_str());
    return CHW_OK;
}

chw_status chw_plan_describe(chw_plan_t plan, char *buf, size_t len)
{
    if (!plan || !buf || len == 0) return fail(CHW_ERR_INVALID_ARGUMENT, "NULL argument");
    std::lock_guard<std::mutex> lk(plan->mu);
    char head[256];
    std::snprintf(head, sizeof head, "{\"batch\": %lld, \"dtype\": %d, \"norm\": %d, \"extent\": %lld, "
                  "\"tuned\": %d, \"plan\": ",
                  (long long)plan->batch, plan->dt, (int)plan->norm, (long long)plan->extent,
                  plan->tuned ? 1 : 0);
    std::string s = head + describe_plan(plan->built) + ", \"tuning_key\": \"" +
                    tuning_key(plan->dt, plan->cfg.order, plan->flags, plan->m) + "\"}";
    if (s.size() + 1 > len) return fail(CHW_ERR_INVALID_ARGUMENT, "buffer of %zu bytes too small (%zu needed)", len, s.size() + 1);
    std::memcpy(buf, s.c_str(), s.size() + 1);
    return CHW_OK;
}

chw_status chw_autotune(chw_plan_t plan, const void *x, void *y, void *workspace, void *stream,
                        int iters)
{
    if (!plan) return fail(CHW_ERR_INVALID_ARGUMENT, "plan is NULL");
    if (iters < 1) return fail(CHW_ERR_INVALID_ARGUMENT, "iters must be >= 1");
    if (plan->batch == 0 || plan->extent == 0) return CHW_OK;
    int dev = 0;
    chw_status s = device_check(&dev);
    if (s != CHW_OK) return s;
    hipStream_t st = static_cast<hipStream_t>(stream);
    // candidate configurations; a launch form fixed by the plan's flags
    // (CHW_FLAG_PERSISTENT: one persistent launch; CHW_FLAG_MULTI_LAUNCH: one
    // launch per pass) is kept, the other choices are searched
    const bool only_persistent = (plan->flags & CHW_FLAG_PERSISTENT) != 0;
    const bool only_multi = (plan->flags & CHW_FLAG_MULTI_LAUNCH) != 0;
    std::vector<PlanConfig> cands;
    bool has15 = false, has_multi = false;
    int maxm = 0;
    for (int32_t m : plan->m) {
        if (m >= 13 && m <= 15) has15 = true;
        if (m > 15) has_multi = true;
        maxm = std::max(maxm, (int)m);
    }
    std::vector<int> l1s = {-1};
    if (has_multi)
        for (int l1 : {15 - K15_CA, 15 - K15_CD, 12 - K12_CA, 15 - K15_CM, 12 - K12_CM, 15 - K15_CB,
                       12 - K12_CB}) {
            Split sp;
            bool ok = true;
            for (int32_t m : plan->m)
                if (m > 15 && !choose_split(m, plan->dt, l1, 0, plan->cfg.order, false, &sp)) ok = false;
            if (ok) l1s.push_back(l1);
        }
    if (!only_persistent) {
        for (int lr12 : {5, 6})
            for (int lr15 : {5, 6})
                for (int s15 : {0, 1}) {
                    if (!has15 && s15 == 0) continue;
                    if (plan->dt == DT_F64 && (lr12 != 5 || lr15 != 5 || s15 != 1)) continue;
                    for (int l1 : l1s)
                        for (int stream_mode : {0, 1, 2}) {
                            PlanConfig c = plan->cfg;
                            c.lr12 = lr12;
                            c.lr15 = lr15;
                            c.single15 = s15;
                            c.split_l1 = l1;
                            c.exec = 0;
                            c.chunk = 0;
                            c.pipeline = 0;
                            c.stream = stream_mode;
                            c.occupancy = 0;
                            cands.push_back(c);
                        }
                }
        // pipelined chunks of 8, 16 or 32 MiB-signals' worth of elements
        if (has_multi && plan->cfg.order == ORDER_DYADIC)
            for (int64_t ch : {(int64_t)1 << 23, (int64_t)1 << 24, (int64_t)1 << 25}) {
                PlanConfig c = plan->cfg;
                c.exec = 0;
                c.split_l1 = -1;
                c.chunk = ch;
                c.pipeline = 1;
                c.occupancy = 0;
                cands.push_back(c);
            }
    }
    // the persistent launch computes the dyadic order only (the planner
    // refuses it for the others) and takes signals up to 2^21 in 2^12-element
    // tiles, 2^23 in 2^15-element tiles (not FP64)
    const bool can_persist = maxm <= 23 && plan->cfg.order == ORDER_DYADIC && !only_multi;
    if (can_persist) {
        for (int lr12 : {5, 6})
            for (int occ : {0, 1, 2, 4}) {
                if (maxm > 21 || (plan->dt == DT_F64 && lr12 != 5)) continue;
                PlanConfig c = plan->cfg;
                c.lr12 = lr12;
                c.exec = 2;
                c.ptile = 12;
                c.split_l1 = -1;
                c.chunk = 0;
                c.pipeline = 0;
                c.stream = 0;
                c.occupancy = occ;
                cands.push_back(c);
            }
        if (plan->dt != DT_F64) {
            PlanConfig c = plan->cfg;
            c.lr15 = 5;
            c.exec = 2;
            c.ptile = 15;
            c.split_l1 = -1;
            c.chunk = 0;
            c.pipeline = 0;
            c.stream = 0;
            c.occupancy = 0;
            cands.push_back(c);
        }
    }
    // the plan's own configuration first: another one replaces the best so far
    // only when it is more than 1% faster, so near-ties keep the default and
    // repeated tunings pick the same kernels
    cands.insert(cands.begin(), plan->cfg);
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
        return fail(CHW_ERR_HIP, "hipEventCreate failed");
    const PlanConfig saved = plan->cfg;
    float best_ms = 1e30f;
    PlanConfig best = saved;
    const bool was_used = plan->used;
    int timed = 0;
    s = CHW_OK;
    for (const PlanConfig &c : cands) {
        {
            // a candidate the planner cannot take is skipped; it does not
            // decide the call's status
            std::lock_guard<std::mutex> lk(plan->mu);
            if (rebuild(plan, c) != CHW_OK) continue;
        }
        if ((s = run(plan, 0, x, y, workspace, stream)) != CHW_OK) break;  // warm-up
        if (hipEventRecord(e0, st) != hipSuccess) { s = fail(CHW_ERR_HIP, "hipEventRecord"); break; }
        for (int i = 0; i < iters && s == CHW_OK; ++i) s = run(plan, 0, x, y, workspace, stream);
        if (s != CHW_OK) break;
        if (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) {
            s = fail(CHW_ERR_HIP, "event timing failed");
            break;
        }
        float ms = 0;
        (void)hipEventElapsedTime(&ms, e0, e1);
        ++timed;
        if (log_enabled())
            std::fprintf(stderr, "[libchw] tune exec=%d lr12=%d lr15=%d single15=%d split_l1=%d stream=%d chunk=%lld pipeline=%d occupancy=%d: %.4f ms\n",
                         c.exec, c.lr12, c.lr15, c.single15, c.split_l1, c.stream, (long long)c.chunk, c.pipeline, c.occupancy, ms / iters);
        if (ms < 0.99f * best_ms) {
            best_ms = ms;
            best = c;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (s == CHW_OK && timed == 0)
        s = fail(CHW_ERR_UNSUPPORTED, "no candidate configuration could be planned");
    std::lock_guard<std::mutex> lk(plan->mu);
    chw_status s2 = rebuild(plan, s == CHW_OK ? best : saved);
    plan->used = was_used || s == CHW_OK;
    if (s == CHW_OK && s2 == CHW_OK && !(plan->flags & CHW_FLAG_NO_AUTOTUNE)) {
        std::lock_guard<std::mutex> tk(g_tune_mu);
        PlanConfig entry;
        copy_tunables(best, &entry);
        g_tune[tuning_key(plan->dt, plan->cfg.order, plan->flags, plan->m)] = entry;
        plan->tuned = true;
    }
    return s != CHW_OK ? s : s2;
}

chw_status chw_tuning_clear(void)
{
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune.clear();
    return CHW_OK;
}

chw_status chw_tuning_count(size_t *n)
{
    if (!n) return fail(CHW_ERR_INVALID_ARGUMENT, "n is NULL");
    std::lock_guard<std::mutex> lk(g_tune_mu);
    *n = g_tune.size();
    return CHW_OK;
}

chw_status chw_tuning_save(const char *path, const char *comment)
{
    if (!path) return fail(CHW_ERR_INVALID_ARGUMENT, "path is NULL");
    std::string text = "# libchw tuning cache (chw_tuning_save): key, then the tuned planner options\n";
    if (comment) {
        std::string line;
        for (const char *c = comment;; ++c) {
            if (*c == '\n' || *c == '\0') {
                text += "# " + line + "\n";
                line.clear();
                if (*c == '\0') break;
            } else {
                line += *c;
            }
        }
    }
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        for (const auto &kv : g_tune) {
            text += kv.first;
            for (const TunableField &f : kTunables) {
                const long long v = f.i64 ? (long long)(kv.second.*f.i64) : (long long)(kv.second.*f.i32);
                text += " " + std::string(f.name) + "=" + std::to_string(v);
            }
            text += "\n";
        }
    }
    FILE *fp = std::fopen(path, "w");
    if (!fp) return fail(CHW_ERR_INVALID_ARGUMENT, "cannot open %s for writing", path);
    const size_t w = std::fwrite(text.data(), 1, text.size(), fp);
    const int c = std::fclose(fp);
    if (w != text.size() || c != 0) return fail(CHW_ERR_INVALID_ARGUMENT, "cannot write %s", path);
    return CHW_OK;
}

chw_status chw_tuning_load(const char *path)
{
    if (!path) return fail(CHW_ERR_INVALID_ARGUMENT, "path is NULL");
    FILE *fp = std::fopen(path, "r");
    if (!fp) return fail(CHW_ERR_INVALID_ARGUMENT, "cannot open %s", path);
    std::map<std::string, PlanConfig> found;
    std::string line;
    int lineno = 0;
    chw_status s = CHW_OK;
    auto parse = [&](const std::string &ln) -> bool {
        size_t i = 0;
        while (i < ln.size() && (ln[i] == ' ' || ln[i] == '\t' || ln[i] == '\r')) ++i;
        if (i == ln.size() || ln[i] == '#') return true;
        size_t j = i;
        while (j < ln.size() && ln[j] != ' ' && ln[j] != '\t') ++j;
        const std::string key = ln.substr(i, j - i);
        PlanConfig cfg;
        bool seen[sizeof kTunables / sizeof kTunables[0]] = {};
        while (j < ln.size()) {
            while (j < ln.size() && (ln[j] == ' ' || ln[j] == '\t' || ln[j] == '\r')) ++j;
            if (j == ln.size()) break;
            size_t e = j;
            while (e < ln.size() && ln[e] != ' ' && ln[e] != '\t' && ln[e] != '\r') ++e;
            const std::string tok = ln.substr(j, e - j);
            j = e;
            const size_t eq = tok.find('=');
            if (eq == std::string::npos || eq == 0 || eq + 1 == tok.size()) return false;
            const std::string name = tok.substr(0, eq), val = tok.substr(eq + 1);
            char *endp = nullptr;
            errno = 0;
            const long long v = std::strtoll(val.c_str(), &endp, 10);
            if (errno != 0 || !endp || *endp != '\0') return false;
            size_t k = 0;
            for (; k < sizeof kTunables / sizeof kTunables[0]; ++k)
                if (name == kTunables[k].name) break;
            if (k == sizeof kTunables / sizeof kTunables[0] || seen[k]) return false;
            if (v < kTunables[k].lo || v > kTunables[k].hi) return false;
            seen[k] = true;
            if (kTunables[k].i64) cfg.*(kTunables[k].i64) = (int64_t)v;
            else cfg.*(kTunables[k].i32) = (int)v;
        }
        for (bool b : seen)
            if (!b) return false;
        found[key] = cfg;
        return true;
    };
    for (int ch = std::fgetc(fp);; ch = std::fgetc(fp)) {
        if (ch == '\n' || ch == EOF) {
            ++lineno;
            if (!parse(line)) {
                s = fail(CHW_ERR_INVALID_ARGUMENT, "%s:%d: malformed tuning entry", path, lineno);
                break;
            }
            line.clear();
            if (ch == EOF) break;
        } else {
            line += (char)ch;
            if (line.size() > 4096) {
                s = fail(CHW_ERR_INVALID_ARGUMENT, "%s:%d: line too long", path, lineno + 1);
                break;
            }
        }
    }
    std::fclose(fp);
    if (s != CHW_OK) return s;
    std::lock_guard<std::mutex> lk(g_tune_mu);
    for (const auto &kv : found) g_tune[kv.first] = kv.second;
    return CHW_OK;
}

}  // extern "C"
