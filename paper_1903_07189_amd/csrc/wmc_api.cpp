// wmc_api.cpp -- host side of libwmc: the C ABI declared in include/wmc.h.
//
// Validates arguments on the host (before any HIP call), plans launch
// sequences (temporal blocking depth per launch, ping-pong buffers,
// checkpoints), captures them into cached hipGraphs, runs the autotuner and
// drives the adjoint.  All device work is in wmc_stream.hip / wmc_adjoint.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <map>
#include <memory>
#include <mutex>
#include <sstream>
#include <string>
#include <vector>

#include <sys/stat.h>
#include <sys/types.h>

#include "wmc.h"
#include "wmc_internal.h"

using namespace wmc;

namespace {

thread_local std::string g_err;

int fail(int code, const std::string& msg) {
    g_err = msg;
    return code;
}

int hip_fail(hipError_t e, const char* what) {
    return fail(WMC_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}

#define WMC_HIP(call, what)                         \
    do {                                            \
        hipError_t _e = (call);                     \
        if (_e != hipSuccess) return hip_fail(_e, what); \
    } while (0)

// WMC_FAULT_INJECT=launch|graph|alloc makes the named stage report a HIP
// failure without touching the device (host-side error-path testing).
bool injected(const char* stage) {
    const char* v = std::getenv("WMC_FAULT_INJECT");
    return v && std::strcmp(v, stage) == 0;
}

// ---------------------------------------------------------------------------
// device checks
// ---------------------------------------------------------------------------
std::mutex g_mu;
std::map<int, int> g_arch_ok;  // device -> 1 gfx950, 0 other
std::map<int, int> g_num_cu;

int check_device(int* dev_out) {
    if (injected("launch")) return fail(WMC_EHIP, "injected launch failure (WMC_FAULT_INJECT)");
    int dev = 0;
    WMC_HIP(hipGetDevice(&dev), "hipGetDevice");
    {
        std::lock_guard<std::mutex> lk(g_mu);
        auto it = g_arch_ok.find(dev);
        if (it == g_arch_ok.end()) {
            hipDeviceProp_t prop;
            WMC_HIP(hipGetDeviceProperties(&prop, dev), "hipGetDeviceProperties");
            const bool ok = std::strncmp(prop.gcnArchName, "gfx950", 6) == 0;
            g_arch_ok[dev] = ok ? 1 : 0;
            g_num_cu[dev] = prop.multiProcessorCount;
            it = g_arch_ok.find(dev);
        }
        if (!it->second) return fail(WMC_EUNSUPPORTED, "libwmc runs on gfx950 (MI355X) only");
    }
    if (dev_out) *dev_out = dev;
    return WMC_OK;
}

int num_cu(int dev) {
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_num_cu.find(dev);
    return it == g_num_cu.end() ? 256 : it->second;
}

// ---------------------------------------------------------------------------
// validation helpers
// ---------------------------------------------------------------------------
constexpr int64_t kMaxSide = (int64_t)1 << 30;

int64_t extent_elems(const wmc_shape& s) { return (s.n - 1) * s.ps + (s.h - 1) * s.ld + s.w; }

// Elements between consecutive plane sets in workspace / checkpoint buffers:
// n*ps, or the extent of one plane set if that is larger.
int64_t set_stride_elems(const wmc_shape& s) {
    const int64_t e = extent_elems(s), np = s.n * s.ps;
    return np >= e ? np : e;
}

int check_shape(const wmc_shape& s) {
    if (s.n < 1 || s.h < 1 || s.w < 1) return fail(WMC_EINVAL, "shape: n, h and w must be >= 1");
    if (s.h >= kMaxSide || s.w >= kMaxSide) return fail(WMC_EINVAL, "shape: h and w must be < 2^30");
    if (s.n > 65535) return fail(WMC_EINVAL, "shape: at most 65535 planes per call");
    if (s.ld < s.w) return fail(WMC_EINVAL, "shape: ld must be >= w");
    if (s.n > 1 && s.ps < (s.h - 1) * s.ld + s.w)
        return fail(WMC_EINVAL, "shape: ps must be >= (h-1)*ld + w when n > 1");
    if (s.ps < 0) return fail(WMC_EINVAL, "shape: ps must be >= 0");
    return WMC_OK;
}

struct Range {
    uintptr_t lo, hi;  // [lo, hi)
};

Range range_of(const void* p, int64_t elems, int64_t elem_bytes) {
    const uintptr_t lo = reinterpret_cast<uintptr_t>(p);
    return {lo, lo + (uintptr_t)(elems * elem_bytes)};
}

bool overlaps(const Range& a, const Range& b) {
    if (!a.lo || !b.lo) return false;
    return a.lo < b.hi && b.lo < a.hi;
}

hipStream_t as_stream(void* s) { return reinterpret_cast<hipStream_t>(s); }

bool aligned_for(const void* p, int C) { return (reinterpret_cast<uintptr_t>(p) % (4 * C)) == 0; }

// Largest C in {4, 2, 1} for which every buffer row starts 4C-aligned.
int vec_cols(std::initializer_list<const void*> ptrs, int64_t ld, int64_t ps) {
    for (int C : {4, 2}) {
        bool ok = (ld % C == 0) && (ps % C == 0);
        for (const void* p : ptrs)
            if (p && !aligned_for(p, C)) ok = false;
        if (ok) return C;
    }
    return 1;
}

bool valid_T(int T) { return T == 1 || T == 2 || T == 3 || T == 4 || T == 6 || T == 8; }

// Splits a run of `len` sweeps into launches of at most T sweeps each, every
// one a compiled depth.
void split_run(int len, int T, std::vector<int>& out) {
    static const int depths[] = {8, 6, 4, 3, 2, 1};
    while (len > 0) {
        int t = std::min(len, T);
        for (int d : depths)
            if (d <= t) {
                t = d;
                break;
            }
        out.push_back(t);
        len -= t;
    }
}

// Output rows per work item.  A launch of the streaming kernel is a set of
// equal work items (one wave each); when their number is just above a
// multiple of the waves the device holds at once, the last round runs
// nearly empty and the launch takes a whole extra round.  So R is chosen to
// make the items fill k complete rounds: nseg = floor(k * slots / (planes *
// strips)), R = ceil(h / nseg) -- the smallest k whose R is at least
// max(8, 4T) rows (segment overlap costs T rows per sweep depth).  slots =
// resident waves of this kernel variant (occupancy API) times the CUs.
// Whether a launch over planes w columns wide takes the vector-only build
// (see vector_only), assuming aligned rows, the usual case.
bool likely_vector_only(int64_t w, int C, int T) {
    return strip_count((int)w, C, T) >= 2 && (w - 64 * C) % C == 0;
}

int64_t resident_waves(int dev, int C, int T, int mode, bool traj = false, int64_t w = 0) {
    const bool vo = w > 0 && likely_vector_only(w, C, T);
    int per_cu = traj ? stream_traj_blocks_per_cu(C, T, mode, vo)
                      : stream_single_blocks_per_cu(C, T, mode, false, vo);
    if (per_cu <= 0) per_cu = 1;
    return (int64_t)num_cu(dev) * per_cu * 4;  // 4 waves per 256-thread block
}

int rows_for_rounds(int64_t planes, int64_t h, int64_t w, int C, int T, int64_t slots, int k) {
    const int64_t strips = strip_count((int)w, C, T);
    const int64_t nseg = std::max<int64_t>(1, (k * slots) / std::max<int64_t>(1, strips * planes));
    const int64_t R = (h + nseg - 1) / nseg;
    return (int)std::max<int64_t>(1, std::min<int64_t>(R, h));
}

int default_rows(int64_t planes, int64_t h, int64_t w, int C, int T, int dev, int mode,
                 bool traj = false) {
    const int64_t slots = resident_waves(dev, C, T, mode, traj, w);
    const int64_t rmin = std::min<int64_t>(h, std::max<int64_t>(8, 4 * (int64_t)T));
    for (int k = 1; k <= 64; ++k) {
        const int R = rows_for_rounds(planes, h, w, C, T, slots, k);
        if (R < rmin) break;
        if (R <= 512) return R;
    }
    return (int)rmin;
}

// Row counts worth timing for (C, T): the first three round-filling values
// and two plain ones.
std::vector<int> candidate_rows(int64_t planes, int64_t h, int64_t w, int C, int T, int dev,
                                int mode) {
    const int64_t slots = resident_waves(dev, C, T, mode, false, w);
    std::vector<int> out;
    auto add = [&](int R) {
        if (R < 1 || R > 512) return;
        if (std::find(out.begin(), out.end(), R) == out.end()) out.push_back(R);
    };
    const int64_t rmin = std::min<int64_t>(h, std::max<int64_t>(4, 2 * (int64_t)T));
    for (int k = 1, got = 0; k <= 64 && got < 3; ++k) {
        const int R = rows_for_rounds(planes, h, w, C, T, slots, k);
        if (R < rmin) break;
        if (R <= 512) {
            add(R);
            ++got;
        }
    }
    add(16);
    add(32);
    // a problem too small to fill one round of resident waves even at a
    // few rows per item: its launches last about one item's serial latency,
    // so short items win despite their recomputed ramp rows (256 x 256,
    // 50 iterations: 0.27 ms at 16 rows per item, 0.11 ms at 2)
    if (rows_for_rounds(planes, h, w, C, T, slots, 1) < 16) {
        add(std::min<int>((int)h, 2));
        add(std::min<int>((int)h, 4));
        add(std::min<int>((int)h, 8));
    }
    return out;
}

// ---------------------------------------------------------------------------
// cached launch plans: device-side work tables and hipGraphs
// ---------------------------------------------------------------------------
struct PlanEntry {
    hipGraphExec_t exec = nullptr;
    hipGraph_t graph = nullptr;
    std::vector<void*> owned;   // device buffers owned by this entry
    std::shared_ptr<void> data;  // host-side description of `owned`
    uint64_t last_use = 0;
    ~PlanEntry() {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        for (void* p : owned) (void)hipFree(p);
    }
};

std::mutex g_plan_mu;
std::map<std::string, std::unique_ptr<PlanEntry>> g_plans;
std::map<int, hipStream_t> g_capture_stream;
uint64_t g_use_clock = 0;
constexpr size_t kMaxPlans = 64;

int capture_stream(int dev, hipStream_t* out) {
    auto it = g_capture_stream.find(dev);
    if (it != g_capture_stream.end()) {
        *out = it->second;
        return WMC_OK;
    }
    hipStream_t s = nullptr;
    WMC_HIP(hipStreamCreateWithFlags(&s, hipStreamNonBlocking), "hipStreamCreateWithFlags");
    g_capture_stream[dev] = s;
    *out = s;
    return WMC_OK;
}

void evict_plans() {
    while (g_plans.size() > kMaxPlans) {
        auto oldest = g_plans.begin();
        for (auto it = g_plans.begin(); it != g_plans.end(); ++it)
            if (it->second->last_use < oldest->second->last_use) oldest = it;
        g_plans.erase(oldest);
    }
}

// Enqueue function: (stream, entry) -> status.  With use_graph the sequence
// is recorded once per key on a private capture stream and replayed on st;
// without, it is enqueued on st directly (the entry still owns its tables).
// `prepare` runs once when the entry is created (uploads work tables).
template <class Prep, class Enq>
int run_plan(const std::string& key, int dev, hipStream_t st, bool use_graph, Prep&& prepare,
             Enq&& enqueue) {
    std::lock_guard<std::mutex> lk(g_plan_mu);
    const std::string full = (use_graph ? "G|" : "D|") + key;
    auto it = g_plans.find(full);
    if (it == g_plans.end()) {
        auto e = std::make_unique<PlanEntry>();
        int rc = prepare(*e);
        if (rc) return rc;
        if (use_graph) {
            if (injected("graph")) return fail(WMC_EHIP, "injected graph failure (WMC_FAULT_INJECT)");
            hipStream_t cs;
            rc = capture_stream(dev, &cs);
            if (rc) return rc;
            WMC_HIP(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal),
                    "hipStreamBeginCapture");
            const int erc = enqueue(cs, *e);
            hipGraph_t g = nullptr;
            const hipError_t ce = hipStreamEndCapture(cs, &g);
            if (erc) {
                if (g) (void)hipGraphDestroy(g);
                return erc;
            }
            if (ce != hipSuccess) return hip_fail(ce, "hipStreamEndCapture");
            e->graph = g;
            WMC_HIP(hipGraphInstantiate(&e->exec, g, nullptr, nullptr, 0), "hipGraphInstantiate");
        }
        it = g_plans.emplace(full, std::move(e)).first;
    }
    PlanEntry& e = *it->second;
    e.last_use = ++g_use_clock;
    int rc = WMC_OK;
    if (use_graph) {
        const hipError_t le = hipGraphLaunch(e.exec, st);
        if (le != hipSuccess) rc = hip_fail(le, "hipGraphLaunch");
    } else {
        rc = enqueue(st, e);
    }
    evict_plans();
    return rc;
}

int device_alloc(PlanEntry& e, size_t bytes, void** out) {
    if (injected("alloc")) return fail(WMC_EHIP, "injected allocation failure (WMC_FAULT_INJECT)");
    void* p = nullptr;
    WMC_HIP(hipMalloc(&p, bytes < 256 ? 256 : bytes), "hipMalloc");
    e.owned.push_back(p);
    *out = p;
    return WMC_OK;
}

template <class T>
void key_add(std::string& k, const T& v) {
    k.append(reinterpret_cast<const char*>(&v), sizeof(T));
}

// ---------------------------------------------------------------------------
// tuning
// ---------------------------------------------------------------------------
struct Tuned {
    int C, T, R;
};

std::mutex g_tune_mu;
std::map<std::string, Tuned> g_tune;
bool g_tune_loaded = false;

std::string tune_path() {
    if (const char* p = std::getenv("WMC_TUNE_CACHE")) return p;
    const char* home = std::getenv("HOME");
    return std::string(home ? home : "/tmp") + "/.cache/wmc/tune.json";
}

// The cache file is a flat JSON object {"key": [C, T, R], ...}.
void load_tune_file() {
    if (g_tune_loaded) return;
    g_tune_loaded = true;
    std::ifstream in(tune_path());
    if (!in) return;
    std::stringstream ss;
    ss << in.rdbuf();
    const std::string txt = ss.str();
    size_t pos = 0;
    while (true) {
        const size_t q0 = txt.find('"', pos);
        if (q0 == std::string::npos) break;
        const size_t q1 = txt.find('"', q0 + 1);
        if (q1 == std::string::npos) break;
        const std::string key = txt.substr(q0 + 1, q1 - q0 - 1);
        const size_t b0 = txt.find('[', q1);
        if (b0 == std::string::npos) break;
        const size_t b1 = txt.find(']', b0);
        if (b1 == std::string::npos) break;
        int C = 0, T = 0, R = 0;
        if (std::sscanf(txt.c_str() + b0 + 1, "%d , %d , %d", &C, &T, &R) == 3 &&
            (C == 1 || C == 2 || C == 4) && valid_T(T) && R >= 1)
            g_tune[key] = {C, T, R};
        pos = b1 + 1;
    }
}

void save_tune_file() {
    const std::string path = tune_path();
    for (size_t i = 1; i < path.size(); ++i)
        if (path[i] == '/') (void)mkdir(path.substr(0, i).c_str(), 0755);
    std::ofstream out(path + ".tmp");
    if (!out) return;
    out << "{\n";
    size_t i = 0;
    for (auto& kv : g_tune)
        out << "  \"" << kv.first << "\": [" << kv.second.C << ", " << kv.second.T << ", "
            << kv.second.R << "]" << (++i < g_tune.size() ? "," : "") << "\n";
    out << "}\n";
    out.close();
    (void)std::rename((path + ".tmp").c_str(), path.c_str());
}

int ilog2_ceil(int64_t v) {
    int r = 0;
    while (((int64_t)1 << r) < v) ++r;
    return r;
}

// ---------------------------------------------------------------------------
// batches (also used for single plane sets by the tuner)
// ---------------------------------------------------------------------------
struct BatchImg {
    const float* src;  // u0 or f
    const float* f;
    float* out;
    float* tmp;        // ping-pong partner in the workspace
    int64_t h, w, ld, ps;
    int channels;
    int lam_index;
    int lam_stride;
};

int64_t img_extent(const BatchImg& b) { return (b.channels - 1) * b.ps + (b.h - 1) * b.ld + b.w; }

// Work table for one launch depth T: descriptors with strip/segment counts and
// item bases.  Returns the number of work items.
// Descriptor table of a batched launch and, if `owner` is given, the image of
// every work item.  Returns the number of work items.
int64_t build_table(const std::vector<BatchImg>& imgs, int C, int T, int R,
                    std::vector<ImageDesc>& tab, std::vector<int32_t>* owner = nullptr) {
    tab.clear();
    if (owner) owner->clear();
    int64_t base = 0;
    for (const BatchImg& b : imgs) {
        ImageDesc d{};
        d.src0 = b.src;
        d.f = b.f;
        d.bufA = b.out;
        d.bufB = b.tmp;
        d.amap = nullptr;
        d.ld = b.ld;
        d.ps = b.ps;
        d.H = (int32_t)b.h;
        d.W = (int32_t)b.w;
        d.channels = b.channels;
        d.lam_index = b.lam_index;
        d.lam_stride = b.lam_stride;
        d.nstrip = strip_count((int)b.w, C, T);
        d.nseg = seg_count((int)b.h, R);
        d.vec = vec_cols({b.src, b.f, b.out, b.tmp}, b.ld, b.channels > 1 ? b.ps : 0) >= C ? 1 : 0;
        d.item_base = base;
        const int64_t n = (int64_t)d.channels * d.nseg * d.nstrip;
        base += n;
        if (owner) owner->insert(owner->end(), (size_t)n, (int32_t)tab.size());
        tab.push_back(d);
    }
    return base;
}

// Launch sequence of a batched solve: depth of each launch and its buffers.
struct Launch {
    int T;
    int src_sel, dst_sel;
};

std::vector<Launch> batch_schedule(int iters, int T) {
    std::vector<int> depths;
    split_run(iters, T, depths);
    const int L = (int)depths.size();
    std::vector<Launch> out;
    for (int l = 0; l < L; ++l) {
        const int dst = ((L - 1 - l) % 2 == 0) ? 1 : 2;  // the last launch writes out (A)
        const int src = l == 0 ? 0 : out.back().dst_sel;
        out.push_back({depths[l], src, dst});
    }
    return out;
}

// Enqueues (does not capture) a batched solve with explicit (C, T, R).
// dtab[T'] / owner[T'] hold device copies of the work tables for each depth
// used.
int enqueue_batched(const std::vector<Launch>& sched, const std::map<int, ImageDesc*>& dtab,
                    const std::map<int, int32_t*>& owner, const std::map<int, int64_t>& items,
                    int C, int R, int mode, const float* lam, float dt, hipStream_t st) {
    for (size_t l = 0; l < sched.size(); ++l) {
        const Launch& L = sched[l];
        LaunchArgs a{lam, dt, L.src_sel, L.dst_sel, R};
        const hipError_t e = launch_stream_batched(C, L.T, mode, dtab.at(L.T), owner.at(L.T),
                                                   items.at(L.T), a, st);
        if (e != hipSuccess) return hip_fail(e, "launch of the batched kernel");
    }
    return WMC_OK;
}

// Device-side work tables of one batched plan.
struct BatchTables {
    std::map<int, ImageDesc*> dtab;  // per launch depth
    std::map<int, int32_t*> owner;   // image of each work item, per launch depth
    std::map<int, int64_t> items;
};

// Uploads the work tables of depth T into `t` (memory owned by `e`).
int upload_tables(PlanEntry& e, BatchTables& t, const std::vector<BatchImg>& imgs, int C, int T,
                  int R) {
    std::vector<ImageDesc> tab;
    std::vector<int32_t> own;
    const int64_t n = build_table(imgs, C, T, R, tab, &own);
    void* p = nullptr;
    int rc = device_alloc(e, sizeof(ImageDesc) * tab.size(), &p);
    if (rc) return rc;
    WMC_HIP(hipMemcpy(p, tab.data(), sizeof(ImageDesc) * tab.size(), hipMemcpyHostToDevice),
            "hipMemcpy (work table)");
    void* q = nullptr;
    rc = device_alloc(e, sizeof(int32_t) * std::max<size_t>(1, own.size()), &q);
    if (rc) return rc;
    if (!own.empty())
        WMC_HIP(hipMemcpy(q, own.data(), sizeof(int32_t) * own.size(), hipMemcpyHostToDevice),
                "hipMemcpy (item owners)");
    t.dtab[T] = static_cast<ImageDesc*>(p);
    t.owner[T] = static_cast<int32_t*>(q);
    t.items[T] = n;
    return WMC_OK;
}

// Full batched solve with a fixed tuning.
int batched_run(const std::vector<BatchImg>& imgs, const float* lam, int iters, float dt,
                int mode, int C, int T, int R, bool use_graph, int dev, hipStream_t st) {
    const std::vector<Launch> sched = batch_schedule(iters, T);
    std::string key = "batched|";
    key_add(key, C);
    key_add(key, T);
    key_add(key, R);
    key_add(key, mode);
    key_add(key, iters);
    key_add(key, dt);
    key_add(key, lam);
    key_add(key, dev);
    for (const BatchImg& b : imgs) key_add(key, b);
    auto prepare = [&](PlanEntry& e) -> int {
        auto t = std::make_shared<BatchTables>();
        for (const Launch& L : sched) {
            if (t->dtab.count(L.T)) continue;
            const int rc = upload_tables(e, *t, imgs, C, L.T, R);
            if (rc) return rc;
        }
        e.data = t;
        return WMC_OK;
    };
    auto enqueue = [&](hipStream_t s, PlanEntry& e) -> int {
        const BatchTables& t = *static_cast<const BatchTables*>(e.data.get());
        return enqueue_batched(sched, t.dtab, t.owner, t.items, C, R, mode, lam, dt, s);
    };
    return run_plan(key, dev, st, use_graph, prepare, enqueue);
}

// ---------------------------------------------------------------------------
// single plane-set solve: schedule with checkpoints
// ---------------------------------------------------------------------------
struct SLaunch {
    int T;
    const float* src;
    float* dst;
    float* traj[3];  // checkpoints reached after sweeps 1..T-1 of this launch (or null)
    float* traj_in;  // checkpoint 0 (the solve's U^0), stored by the first launch
};

// Launch sequence of a single plane-set solve.  Checkpoint states that fall
// inside a fused launch are stored by the trajectory variant when it exists
// for T (2..kTrajMaxT); otherwise launches end at every checkpoint.
std::vector<SLaunch> solve_schedule(int iters, int T, int ckpt_every, const float* src0,
                                    float* u_out, float* ws, float* ckpt, int64_t set_stride) {
    std::vector<int> depth;
    std::vector<int> end_t;
    int t = 0;
    const bool traj = ckpt && ckpt_every > 0 && T >= 2 && T <= kTrajMaxT;
    while (t < iters) {
        int stop = iters;
        if (ckpt && ckpt_every > 0 && !traj)
            stop = std::min(iters, (t / ckpt_every + 1) * ckpt_every);
        std::vector<int> parts;
        split_run(stop - t, T, parts);
        for (int d : parts) {
            t += d;
            depth.push_back(d);
            end_t.push_back(t);
        }
    }
    const int L = (int)depth.size();
    std::vector<SLaunch> out(L);
    for (int l = L - 1; l >= 0; --l) {
        float* dst;
        if (l == L - 1) dst = u_out;
        else if (ckpt && end_t[l] % ckpt_every == 0)
            dst = ckpt + (int64_t)(end_t[l] / ckpt_every) * set_stride;
        else
            dst = (out[l + 1].dst == u_out) ? ws : u_out;
        out[l].dst = dst;
        out[l].T = depth[l];
        for (int k = 0; k < 3; ++k) out[l].traj[k] = nullptr;
        // a trajectory launch stores its input rows as it reads them, so the
        // first one writes checkpoint 0 without a copy of its own
        out[l].traj_in = (traj && l == 0 && depth[l] >= 2) ? ckpt : nullptr;
        if (traj) {
            const int t0 = end_t[l] - depth[l];
            for (int k = 1; k < depth[l]; ++k)
                if ((t0 + k) % ckpt_every == 0)
                    out[l].traj[k - 1] = ckpt + (int64_t)((t0 + k) / ckpt_every) * set_stride;
        }
    }
    for (int l = 0; l < L; ++l) out[l].src = l == 0 ? src0 : out[l - 1].dst;
    return out;
}

int enqueue_single(const wmc_shape& s, const float* src, const float* f, float* dst,
                   const float* lam, float dt, int C, int T, int R, hipStream_t st,
                   float* const* traj = nullptr, float* traj_in = nullptr) {
    const int mode = f ? kModeData : kModeFlow;
    const bool vec = vec_cols({src, f, dst}, s.ld, s.n > 1 ? s.ps : 0) >= C;
    ImageDesc d{};
    d.src0 = src;
    d.f = f;
    d.bufA = dst;
    d.bufB = dst;
    d.ld = s.ld;
    d.ps = s.ps;
    d.H = (int32_t)s.h;
    d.W = (int32_t)s.w;
    d.channels = (int32_t)s.n;
    d.lam_index = 0;
    d.lam_stride = 1;
    d.nstrip = strip_count((int)s.w, C, T);
    d.nseg = seg_count((int)s.h, R);
    d.vec = vec ? 1 : 0;
    LaunchArgs a{lam, dt, 0, 1, R};
    // the input state: stored by the launch itself when its vector-only
    // build runs, else copied first
    if (traj_in && !(T >= 2 && vector_only(d, C))) {
        const hipError_t e = launch_copy_planes(src, traj_in, s.n, s.h, s.w, s.ld, s.ps, st);
        if (e != hipSuccess) return hip_fail(e, "checkpoint copy");
        traj_in = nullptr;
    }
    a.traj_in = traj_in;
    bool any = a.traj_in != nullptr;
    for (int k = 0; traj && k < 3; ++k) {
        a.traj[k] = k < T - 1 ? traj[k] : nullptr;
        any = any || a.traj[k];
    }
    const hipError_t e = any ? launch_stream_traj(C, T, mode, d, a, st)
                             : launch_stream_single(C, T, mode, false, d, a, st);
    if (e != hipSuccess) return hip_fail(e, "launch of the streaming kernel");
    return WMC_OK;
}

// One launch of `sweeps` fused l1 primal-dual sweeps (Sec. 5.3).
int enqueue_l1(const wmc_shape& s, const float* src, const float* dsrc, const float* f,
               float* dst, float* ddst, const float* lam, float alpha, float dt, int C, int T,
               int R, hipStream_t st) {
    const bool vec = vec_cols({src, f, dst}, s.ld, s.n > 1 ? s.ps : 0) >= C;
    ImageDesc d{};
    d.src0 = src;
    d.f = f;
    d.bufA = dst;
    d.bufB = dst;
    d.dsrc0 = dsrc;
    d.dA = ddst;
    d.dB = ddst;
    d.ld = s.ld;
    d.ps = s.ps;
    d.H = (int32_t)s.h;
    d.W = (int32_t)s.w;
    d.channels = (int32_t)s.n;
    d.lam_index = 0;
    d.lam_stride = 1;
    d.nstrip = strip_count((int)s.w, C, T);
    d.nseg = seg_count((int)s.h, R);
    d.vec = vec ? 1 : 0;
    LaunchArgs a{lam, dt, 0, 1, R, alpha};
    const hipError_t e = launch_stream_single(C, T, kModeL1, false, d, a, st);
    if (e != hipSuccess) return hip_fail(e, "launch of the l1 streaming kernel");
    return WMC_OK;
}

// ---------------------------------------------------------------------------
// autotuner
// ---------------------------------------------------------------------------
// Times `run(C, T, R, stream)` (one launch of T sweeps) for every candidate and
// returns the fastest per sweep.  Synchronises st.
template <class Run, class Rows>
int tune_search(Run&& run, Rows&& rows, hipStream_t st, Tuned* best_out) {
    hipEvent_t e0, e1;
    WMC_HIP(hipEventCreate(&e0), "hipEventCreate");
    WMC_HIP(hipEventCreate(&e1), "hipEventCreate");
    struct Cand {
        double per_sweep;
        Tuned t;
    };
    std::vector<Cand> cands;
    Tuned best_t{2, 4, 64};
    int rc = WMC_OK;
    // best of `reps` timings of `launches` back-to-back launches, per sweep
    auto time_of = [&](const Tuned& t, int launches, int reps, double* per_sweep) -> int {
        int r = run(t.C, t.T, t.R, st);  // warm-up
        if (r) return r;
        float ms_best = 1e30f;
        for (int rep = 0; rep < reps; ++rep) {
            WMC_HIP(hipEventRecord(e0, st), "hipEventRecord");
            for (int l = 0; l < launches; ++l) {
                r = run(t.C, t.T, t.R, st);
                if (r) return r;
            }
            WMC_HIP(hipEventRecord(e1, st), "hipEventRecord");
            WMC_HIP(hipEventSynchronize(e1), "hipEventSynchronize");
            float ms = 0.0f;
            WMC_HIP(hipEventElapsedTime(&ms, e0, e1), "hipEventElapsedTime");
            ms_best = std::min(ms_best, ms);
        }
        *per_sweep = ms_best / ((double)t.T * launches);
        return WMC_OK;
    };
    // best of `reps` replays of one graph of `launches` launches, per sweep:
    // the solve replays its launch sequence as a graph, so the final stage
    // times the candidates the same way.  The warm-up launch on st creates
    // whatever the candidate's plan needs, so that the capture records
    // kernel launches only.
    hipStream_t cs = nullptr;
    auto time_graph = [&](const Tuned& t, int launches, int reps, double* per_sweep) -> int {
        int r = run(t.C, t.T, t.R, st);  // warm-up
        if (r) return r;
        if (!cs) WMC_HIP(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking), "hipStreamCreateWithFlags");
        hipGraph_t g = nullptr;
        hipGraphExec_t ex = nullptr;
        WMC_HIP(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal), "hipStreamBeginCapture");
        for (int l = 0; l < launches && r == WMC_OK; ++l) r = run(t.C, t.T, t.R, cs);
        const hipError_t ce = hipStreamEndCapture(cs, &g);
        if (r == WMC_OK && ce != hipSuccess) r = hip_fail(ce, "hipStreamEndCapture");
        if (r == WMC_OK) {
            const hipError_t ie = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
            if (ie != hipSuccess) r = hip_fail(ie, "hipGraphInstantiate");
        }
        float ms_best = 1e30f;
        for (int rep = -1; rep < reps && r == WMC_OK; ++rep) {  // rep -1: warm-up replay
            hipError_t e = hipEventRecord(e0, st);
            if (e == hipSuccess) e = hipGraphLaunch(ex, st);
            if (e == hipSuccess) e = hipEventRecord(e1, st);
            if (e == hipSuccess) e = hipEventSynchronize(e1);
            float ms = 0.0f;
            if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
            if (e != hipSuccess) r = hip_fail(e, "timing a graph replay");
            else if (rep >= 0) ms_best = std::min(ms_best, ms);
        }
        if (ex) (void)hipGraphExecDestroy(ex);
        if (g) (void)hipGraphDestroy(g);
        if (r) return r;
        *per_sweep = ms_best / ((double)t.T * launches);
        return WMC_OK;
    };
    // launches of T sweeps covering at least `sweeps` sweeps
    auto launches_for = [](int T, int sweeps) { return std::max(1, (sweeps + T - 1) / T); };
    const bool verbose = std::getenv("WMC_TUNE_VERBOSE") != nullptr;  // stage timings to stderr
    // Two timed stages.  A fresh device first runs about 40 sweeps of one
    // shape so that its clocks have risen before anything is timed.  Every candidate
    // is then timed on single launches (best of three), and the six fastest
    // again as graph replays of at least 64 sweeps (best of five), which
    // decide: runs of 32 sweeps, best of three, measured noisier than either
    // and dropped the fastest shape from the final comparison on some
    // devices.
    {
        const Tuned w{2, 4, rows(2, 4).empty() ? 16 : rows(2, 4)[0]};
        for (int l = 0; l < 10 && rc == WMC_OK; ++l) rc = run(w.C, w.T, w.R, st);
        if (rc == WMC_OK) {
            const hipError_t e = hipStreamSynchronize(st);
            if (e != hipSuccess) rc = hip_fail(e, "hipStreamSynchronize");
        }
        if (rc) goto done;
    }
    for (int C : {1, 2, 4})
        for (int T : {1, 2, 3, 4, 6, 8})
            for (int R : rows(C, T)) {
                double ps = 0.0;
                rc = time_of(Tuned{C, T, R}, 1, 3, &ps);
                if (rc) goto done;
                cands.push_back({ps, Tuned{C, T, R}});
            }
    std::sort(cands.begin(), cands.end(),
              [](const Cand& x, const Cand& y) { return x.per_sweep < y.per_sweep; });
    if (verbose)
        for (const Cand& c : cands)
            std::fprintf(stderr, "wmc tune 1: C=%d T=%d R=%d %.4f us/sweep\n", c.t.C, c.t.T, c.t.R,
                         c.per_sweep * 1e3);
    if (cands.size() > 6) cands.resize(6);
    {
        double best = 1e30;
        for (const Cand& c : cands) {
            double ps = 0.0;
            rc = time_graph(c.t, launches_for(c.t.T, 64), 5, &ps);
            if (rc) goto done;
            if (verbose)
                std::fprintf(stderr, "wmc tune 2: C=%d T=%d R=%d %.4f us/sweep\n", c.t.C, c.t.T,
                             c.t.R, ps * 1e3);
            if (ps < best) {
                best = ps;
                best_t = c.t;
            }
        }
    }
done:
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (cs) (void)hipStreamDestroy(cs);
    if (rc) return rc;
    *best_out = best_t;
    return WMC_OK;
}

enum class TuneMode { Off, Cached, Force, Auto };

TuneMode tune_mode() {
    const char* v = std::getenv("WMC_TUNE");
    if (!v) return TuneMode::Auto;
    if (!std::strcmp(v, "off")) return TuneMode::Off;
    if (!std::strcmp(v, "cached")) return TuneMode::Cached;
    if (!std::strcmp(v, "force")) return TuneMode::Force;
    return TuneMode::Auto;
}

std::string arch_name(int dev) {
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return "unknown";
    std::string a = prop.gcnArchName;
    const size_t c = a.find(':');
    return c == std::string::npos ? a : a.substr(0, c);
}

// Looks up / searches a tuning.  `search` fills *t; `deflt` is the fallback.
template <class Search>
int get_tuning(const std::string& key, Tuned deflt, Search&& search, Tuned* t) {
    const TuneMode m = tune_mode();
    if (m == TuneMode::Off) {
        *t = deflt;
        return WMC_OK;
    }
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        load_tune_file();
        auto it = g_tune.find(key);
        if (m != TuneMode::Force && it != g_tune.end()) {
            *t = it->second;
            return WMC_OK;
        }
    }
    if (m == TuneMode::Cached) {
        *t = deflt;
        return WMC_OK;
    }
    Tuned found = deflt;
    int rc = search(&found);
    if (rc) return rc;
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune[key] = found;
    save_tune_file();
    *t = found;
    return WMC_OK;
}

std::string single_tune_key(int dev, const wmc_shape& s, int mode) {
    std::ostringstream k;
    // exact shape: the best row count depends on how the work items fill
    // the device's wave slots
    k << arch_name(dev) << "|single2|" << (mode == kModeData ? "data" : "flow") << "|h" << s.h
      << "|w" << s.w << "|n" << s.n;
    return k.str();
}

// alt (or null): a second writable plane set; the candidates then ping-pong
// between alt and ws as the solve does (U never the same buffer as f, each
// launch reading what the previous one wrote), instead of reading src.
int tune_single(int dev, const wmc_shape& s, const float* src, const float* f, const float* lam,
                float dt, float* ws, hipStream_t st, Tuned* t, float* alt = nullptr) {
    const int mode = f ? kModeData : kModeFlow;
    const int C0 = std::min(2, vec_cols({src, f, ws, alt}, s.ld, s.n > 1 ? s.ps : 0));
    const Tuned deflt{C0, 3, default_rows(s.n, s.h, s.w, C0, 3, dev, mode)};
    auto search = [&](Tuned* out) {
        int flip = 0;
        auto run = [&](int C, int T, int R, hipStream_t ss) {
            if (alt) {
                float* a = (flip & 1) ? ws : alt;
                float* b = (flip & 1) ? alt : ws;
                ++flip;
                return enqueue_single(s, a, f, b, lam, dt, C, T, R, ss);
            }
            return enqueue_single(s, src, f, ws, lam, dt, C, T, R, ss);
        };
        auto rows = [&](int C, int T) { return candidate_rows(s.n, s.h, s.w, C, T, dev, mode); };
        return tune_search(run, rows, st, out);
    };
    return get_tuning(single_tune_key(dev, s, mode), deflt, search, t);
}

// The tuning tune_single would return, without searching: the cached entry of
// this shape, else the default (no device work, no allocation).
Tuned cached_single_tuning(int dev, const wmc_shape& s, const float* src, const float* f,
                           const float* ws) {
    const int mode = f ? kModeData : kModeFlow;
    const int C0 = std::min(2, vec_cols({src, f, ws}, s.ld, s.n > 1 ? s.ps : 0));
    Tuned t{C0, 3, default_rows(s.n, s.h, s.w, C0, 3, dev, mode)};
    if (tune_mode() == TuneMode::Off) return t;
    std::lock_guard<std::mutex> lk(g_tune_mu);
    load_tune_file();
    auto it = g_tune.find(single_tune_key(dev, s, mode));
    if (it != g_tune.end()) t = it->second;
    return t;
}

std::string batch_tune_key(int dev, const std::vector<BatchImg>& imgs, int mode) {
    int64_t px = 0;
    std::vector<int64_t> ws;
    for (const BatchImg& b : imgs) {
        px += b.h * b.w * b.channels;
        ws.push_back(b.w);
    }
    std::sort(ws.begin(), ws.end());
    std::ostringstream k;
    k << arch_name(dev) << "|batch2|" << (mode == kModeData ? "data" : "flow") << "|px" << ilog2_ceil(px)
      << "|wmed" << ilog2_ceil(ws[ws.size() / 2]) << "|imgs" << ilog2_ceil((int64_t)imgs.size());
    return k.str();
}

int tune_batch(int dev, const std::vector<BatchImg>& imgs, const float* lam, float dt, int mode,
               hipStream_t st, Tuned* t) {
    int64_t hmax = 1;
    for (const BatchImg& b : imgs) hmax = std::max(hmax, b.h);
    const Tuned deflt{2, 4, 32};
    auto search = [&](Tuned* out) {
        // one launch of T sweeps reading the inputs and writing the workspace
        auto run = [&](int C, int T, int R, hipStream_t ss) {
            std::vector<Launch> one{{T, 0, 2}};
            std::string key = "tune|";
            key_add(key, C);
            key_add(key, T);
            key_add(key, R);
            key_add(key, mode);
            key_add(key, dev);
            for (const BatchImg& b : imgs) key_add(key, b);
            auto prepare = [&](PlanEntry& e) -> int {
                auto tb = std::make_shared<BatchTables>();
                const int rc = upload_tables(e, *tb, imgs, C, T, R);
                if (rc) return rc;
                e.data = tb;
                return WMC_OK;
            };
            auto enqueue = [&](hipStream_t s2, PlanEntry& e) -> int {
                const BatchTables& tb = *static_cast<const BatchTables*>(e.data.get());
                return enqueue_batched(one, tb.dtab, tb.owner, tb.items, C, R, mode, lam, dt, s2);
            };
            return run_plan(key, dev, ss, false, prepare, enqueue);
        };
        // plain row counts, and near 16, 32 and 64 the one whose item count
        // best fills whole rounds of the device's resident waves (one wave
        // per item, as in the single-image launch)
        auto rows = [&](int C, int T) {
            std::vector<int> out;
            auto add = [&](int R) {
                if (R < 2 * T && R < hmax) return;
                if (R > 2 * hmax && R != 8) return;
                if (std::find(out.begin(), out.end(), R) == out.end()) out.push_back(R);
            };
            for (int R : {8, 16, 32, 64, 128}) add(R);
            int per_cu = stream_blocks_per_cu(C, T, mode);
            const int64_t slots = (int64_t)num_cu(dev) * std::max(1, per_cu) * 4;
            std::vector<int64_t> strips;
            for (const BatchImg& b : imgs) strips.push_back((int64_t)b.channels * strip_count((int)b.w, C, T));
            for (int R0 : {16, 32, 64}) {
                int bestR = 0;
                double best = 1e30;
                for (int R = std::max(2 * T, R0 * 3 / 4); R <= R0 * 5 / 4; ++R) {
                    int64_t items = 0;
                    for (size_t i = 0; i < imgs.size(); ++i)
                        items += strips[i] * seg_count((int)imgs[i].h, R);
                    const double rounds = (double)items / (double)slots;
                    const double loss = std::ceil(rounds) / rounds;
                    if (loss <= best) {
                        best = loss;
                        bestR = R;
                    }
                }
                if (bestR) add(bestR);
            }
            return out;
        };
        return tune_search(run, rows, st, out);
    };
    return get_tuning(batch_tune_key(dev, imgs, mode), deflt, search, t);
}

int resolve_tuning(const wmc_tuning* tune, Tuned auto_t, Tuned* t, bool* graph) {
    *t = auto_t;
    *graph = true;
    if (!tune) return WMC_OK;
    if (tune->cols) {
        if (tune->cols != 1 && tune->cols != 2 && tune->cols != 4)
            return fail(WMC_EINVAL, "tuning: cols must be 1, 2 or 4");
        t->C = tune->cols;
    }
    if (tune->tsteps) {
        if (!valid_T(tune->tsteps)) return fail(WMC_EINVAL, "tuning: tsteps must be 1, 2, 3, 4, 6 or 8");
        t->T = tune->tsteps;
    }
    if (tune->seg_rows) {
        if (tune->seg_rows < 1) return fail(WMC_EINVAL, "tuning: seg_rows must be >= 1");
        t->R = tune->seg_rows;
    }
    *graph = tune->use_graph != 0;
    return WMC_OK;
}

bool tuning_complete(const wmc_tuning* tune) {
    return tune && tune->cols && tune->tsteps && tune->seg_rows;
}

}  // namespace

// ===========================================================================
// C ABI
// ===========================================================================
extern "C" {

const char* wmc_last_error(void) { return g_err.c_str(); }

size_t wmc_solve_workspace(wmc_shape s) {
    if (check_shape(s)) return 0;
    return (size_t)set_stride_elems(s) * sizeof(float);
}

int64_t wmc_set_stride(wmc_shape s) {
    if (check_shape(s)) return 0;
    return set_stride_elems(s);
}

int64_t wmc_num_checkpoints(int iters, int ckpt_every) {
    if (iters <= 0 || ckpt_every <= 0) return 0;
    return (iters + ckpt_every - 1) / ckpt_every;
}

int wmc_compute(const float* u, float* hw, wmc_shape s, void* stream) {
    g_err.clear();
    int rc = check_shape(s);
    if (rc) return rc;
    if (!u || !hw) return fail(WMC_EINVAL, "wmc_compute: null pointer");
    const int64_t ext = extent_elems(s);
    if (overlaps(range_of(u, ext, 4), range_of(hw, ext, 4)))
        return fail(WMC_EINVAL, "wmc_compute: output overlaps input");
    int dev;
    rc = check_device(&dev);
    if (rc) return rc;
    const int C = std::min(2, vec_cols({u, hw}, s.ld, s.n > 1 ? s.ps : 0));
    const int R = default_rows(s.n, s.h, s.w, C, 1, dev, kModeCompute);
    ImageDesc d{};
    d.src0 = u;
    d.bufA = hw;
    d.bufB = hw;
    d.ld = s.ld;
    d.ps = s.ps;
    d.H = (int32_t)s.h;
    d.W = (int32_t)s.w;
    d.channels = (int32_t)s.n;
    d.lam_stride = 1;
    d.nstrip = strip_count((int)s.w, C, 1);
    d.nseg = seg_count((int)s.h, R);
    d.vec = 1;
    LaunchArgs a{nullptr, 0.0f, 0, 1, R};
    const hipError_t e = launch_stream_single(C, 1, kModeCompute, false, d, a, as_stream(stream));
    if (e != hipSuccess) return hip_fail(e, "wmc_compute launch");
    return WMC_OK;
}

int wmc_step(const float* u, const float* f, float* u_out, const float* lam, float dt,
             uint8_t* argmin_out, wmc_shape s, void* stream) {
    g_err.clear();
    int rc = check_shape(s);
    if (rc) return rc;
    if (!u || !u_out) return fail(WMC_EINVAL, "wmc_step: null u or u_out");
    if (f && !lam) return fail(WMC_EINVAL, "wmc_step: lam is required with a data term");
    if (!std::isfinite(dt)) return fail(WMC_EINVAL, "wmc_step: dt must be finite");
    const int64_t ext = extent_elems(s);
    const Range ro = range_of(u_out, ext, 4);
    if (overlaps(ro, range_of(u, ext, 4)) || overlaps(ro, range_of(f, ext, 4)) ||
        overlaps(ro, range_of(argmin_out, ext, 1)))
        return fail(WMC_EINVAL, "wmc_step: u_out overlaps an input (updates are synchronous)");
    if (argmin_out && (overlaps(range_of(argmin_out, ext, 1), range_of(u, ext, 4)) ||
                       overlaps(range_of(argmin_out, ext, 1), range_of(f, ext, 4))))
        return fail(WMC_EINVAL, "wmc_step: argmin_out overlaps an input");
    int dev;
    rc = check_device(&dev);
    if (rc) return rc;
    const int mode = f ? kModeData : kModeFlow;
    const int C = std::min(2, vec_cols({u, f, u_out}, s.ld, s.n > 1 ? s.ps : 0));
    const int R = default_rows(s.n, s.h, s.w, C, 1, dev, mode);
    ImageDesc d{};
    d.src0 = u;
    d.f = f;
    d.bufA = u_out;
    d.bufB = u_out;
    d.amap = argmin_out;
    d.ld = s.ld;
    d.ps = s.ps;
    d.H = (int32_t)s.h;
    d.W = (int32_t)s.w;
    d.channels = (int32_t)s.n;
    d.lam_stride = 1;
    d.nstrip = strip_count((int)s.w, C, 1);
    d.nseg = seg_count((int)s.h, R);
    d.vec = 1;
    LaunchArgs a{lam, dt, 0, 1, R};
    const hipError_t e =
        launch_stream_single(C, 1, mode, argmin_out != nullptr, d, a, as_stream(stream));
    if (e != hipSuccess) return hip_fail(e, "wmc_step launch");
    return WMC_OK;
}

int wmc_solve(const float* f, const float* u0, float* u_out, const float* lam, int iters,
              float dt, float* ckpt, int ckpt_every, const wmc_tuning* tune, void* ws,
              size_t ws_bytes, wmc_shape s, void* stream) {
    return wmc::solve_impl(f, u0, u_out, lam, iters, dt, ckpt, ckpt_every, tune, ws, ws_bytes, s,
                           stream, false);
}

}  // extern "C"

int wmc::report_error(int code, const std::string& msg) { return fail(code, msg); }

// wmc_solve's body.  With `noalloc` (the static-scratch entry point) it takes
// no checkpoints, runs no tuning search (a complete `tune`, else the cached
// tuning of this shape, else the default), captures no graph and reports a
// workspace that is too small as WMC_EINVAL: the scratch has a fixed size.
int wmc::solve_impl(const float* f, const float* u0, float* u_out, const float* lam, int iters,
                    float dt, float* ckpt, int ckpt_every, const wmc_tuning* tune, void* ws,
                    size_t ws_bytes, wmc_shape s, void* stream, bool noalloc) {
    g_err.clear();
    if (noalloc && ckpt) return fail(WMC_EINVAL, "wmc_solve_noalloc: no checkpoints");
    int rc = check_shape(s);
    if (rc) return rc;
    if (!u_out) return fail(WMC_EINVAL, "wmc_solve: null u_out");
    if (!f && !u0) return fail(WMC_EINVAL, "wmc_solve: the curvature flow (f == NULL) needs u0");
    if (f && !lam) return fail(WMC_EINVAL, "wmc_solve: lam is required with a data term");
    if (iters < 0) return fail(WMC_EINVAL, "wmc_solve: iters must be >= 0");
    if (!std::isfinite(dt)) return fail(WMC_EINVAL, "wmc_solve: dt must be finite");
    if (ckpt && ckpt_every < 1) return fail(WMC_EINVAL, "wmc_solve: ckpt_every must be >= 1");
    const int64_t ext = extent_elems(s);
    const int64_t stride = set_stride_elems(s);
    const size_t need = wmc_solve_workspace(s);
    if (noalloc && iters >= 2 && need > ws_bytes)
        return fail(WMC_EINVAL, "wmc_solve_noalloc: one plane set (" + std::to_string(need) +
                                    " bytes) exceeds the static scratch (" +
                                    std::to_string(ws_bytes) + " bytes)");
    if (iters >= 2 && (!ws || ws_bytes < need))
        return fail(WMC_ENOMEM, "wmc_solve: workspace smaller than wmc_solve_workspace()");
    const float* src0 = u0 ? u0 : f;
    const int64_t nck = ckpt ? wmc_num_checkpoints(iters, ckpt_every) : 0;
    const Range ro = range_of(u_out, ext, 4), rs = range_of(src0, ext, 4), rf = range_of(f, ext, 4);
    const Range rw = range_of(iters >= 2 ? ws : nullptr, ext, 4);
    const Range rc_ = range_of(nck ? ckpt : nullptr, (nck - 1) * stride + ext, 4);
    if (overlaps(ro, rs) || overlaps(ro, rf) || overlaps(ro, rw) || overlaps(ro, rc_))
        return fail(WMC_EINVAL, "wmc_solve: u_out overlaps an input, ckpt or ws");
    if (overlaps(rw, rs) || overlaps(rw, rf) || overlaps(rw, rc_) || overlaps(rc_, rs) ||
        overlaps(rc_, rf))
        return fail(WMC_EINVAL, "wmc_solve: ws / ckpt overlap the inputs or each other");
    int dev;
    rc = check_device(&dev);
    if (rc) return rc;
    hipStream_t st = as_stream(stream);
    if (iters == 0) {
        const hipError_t e = launch_copy_planes(src0, u_out, s.n, s.h, s.w, s.ld, s.ps, st);
        return e == hipSuccess ? WMC_OK : hip_fail(e, "copy");
    }
    const int mode = f ? kModeData : kModeFlow;
    Tuned t{};
    bool graph = true;
    if (tuning_complete(tune)) {
        rc = resolve_tuning(tune, Tuned{2, 4, 64}, &t, &graph);
    } else if (noalloc) {
        rc = resolve_tuning(tune, cached_single_tuning(dev, s, src0, f, static_cast<float*>(ws)),
                            &t, &graph);
    } else {
        Tuned auto_t{};
        // with a workspace the candidates ping-pong between u_out and ws
        // (contents irrelevant to the timing) rather than reading f, so that,
        // as in the solve, U and f are different planes
        rc = tune_single(dev, s, iters >= 2 ? u_out : src0, f, lam, dt,
                         iters >= 2 ? static_cast<float*>(ws) : u_out, st,
                         &auto_t, iters >= 2 ? u_out : nullptr);
        if (rc) return rc;
        rc = resolve_tuning(tune, auto_t, &t, &graph);
    }
    if (rc) return rc;
    // checkpoints closer together than T would cut the fused launches short:
    // use the deepest launch that stores states inside itself instead
    if (nck && ckpt_every < t.T && t.T > kTrajMaxT) {
        t.T = kTrajMaxT;
        t.R = default_rows(s.n, s.h, s.w, t.C, t.T, dev, mode, true);
    } else if (nck && t.T >= 2 && t.T <= kTrajMaxT && !tuning_complete(tune) &&
               stream_traj_blocks_per_cu(t.C, t.T, mode, likely_vector_only(s.w, t.C, t.T)) !=
                   stream_single_blocks_per_cu(t.C, t.T, mode, false,
                                               likely_vector_only(s.w, t.C, t.T))) {
        // the trajectory variant holds fewer waves: fill its rounds instead
        t.R = default_rows(s.n, s.h, s.w, t.C, t.T, dev, mode, true);
    }
    const std::vector<SLaunch> sched =
        solve_schedule(iters, t.T, ckpt ? ckpt_every : 0, src0, u_out, static_cast<float*>(ws),
                       nck ? ckpt : nullptr, stride);
    auto enqueue = [&](hipStream_t ss, PlanEntry&) -> int {
        if (nck && !(sched.size() && sched[0].traj_in)) {
            const hipError_t e = launch_copy_planes(src0, ckpt, s.n, s.h, s.w, s.ld, s.ps, ss);
            if (e != hipSuccess) return hip_fail(e, "checkpoint copy");
        }
        for (const SLaunch& L : sched) {
            const int r = enqueue_single(s, L.src, f, L.dst, lam, dt, t.C, L.T, t.R, ss, L.traj,
                                         L.traj_in);
            if (r) return r;
        }
        return WMC_OK;
    };
    if (!graph || noalloc) {
        PlanEntry direct;
        return enqueue(st, direct);
    }
    std::string key = "solve|";
    key_add(key, s);
    key_add(key, f);
    key_add(key, u0);
    key_add(key, u_out);
    key_add(key, lam);
    key_add(key, iters);
    key_add(key, dt);
    key_add(key, ckpt);
    key_add(key, ckpt_every);
    key_add(key, ws);
    key_add(key, t);
    key_add(key, dev);
    auto prepare = [](PlanEntry&) { return WMC_OK; };
    return run_plan(key, dev, st, true, prepare, enqueue);
}

extern "C" {

size_t wmc_l1_workspace(wmc_shape s) {
    if (check_shape(s)) return 0;
    return 2 * (size_t)set_stride_elems(s) * sizeof(float);
}

int wmc_solve_l1(const float* f, const float* u0, const float* d0, float* u_out, float* d_out,
                 const float* lam, float alpha, int iters, float dt, const wmc_tuning* tune,
                 void* ws, size_t ws_bytes, wmc_shape s, void* stream) {
    g_err.clear();
    int rc = check_shape(s);
    if (rc) return rc;
    if (!f || !lam || !u_out || !d_out)
        return fail(WMC_EINVAL, "wmc_solve_l1: f, lam, u_out and d_out are required");
    if (!(alpha > 0.0f) || !std::isfinite(alpha)) return fail(WMC_EINVAL, "wmc_solve_l1: alpha must be > 0");
    if (iters < 0) return fail(WMC_EINVAL, "wmc_solve_l1: iters must be >= 0");
    if (!std::isfinite(dt)) return fail(WMC_EINVAL, "wmc_solve_l1: dt must be finite");
    const int64_t ext = extent_elems(s);
    const int64_t set = set_stride_elems(s);
    if (iters >= 2 && (!ws || ws_bytes < wmc_l1_workspace(s)))
        return fail(WMC_ENOMEM, "wmc_solve_l1: workspace smaller than wmc_l1_workspace()");
    const float* src0 = u0 ? u0 : f;
    float* wsU = static_cast<float*>(ws);
    float* wsD = ws ? static_cast<float*>(ws) + set : nullptr;
    const Range ro = range_of(u_out, ext, 4), rd = range_of(d_out, ext, 4);
    const Range rw = range_of(iters >= 2 ? ws : nullptr, 2 * set, 4);
    for (const Range& in : {range_of(f, ext, 4), range_of(u0, ext, 4), range_of(d0, ext, 4)})
        if (overlaps(ro, in) || overlaps(rd, in) || overlaps(rw, in))
            return fail(WMC_EINVAL, "wmc_solve_l1: an output or ws overlaps an input");
    if (overlaps(ro, rd) || overlaps(ro, rw) || overlaps(rd, rw))
        return fail(WMC_EINVAL, "wmc_solve_l1: outputs overlap each other or ws");
    int dev;
    rc = check_device(&dev);
    if (rc) return rc;
    hipStream_t st = as_stream(stream);
    if (iters == 0) {
        hipError_t e = launch_copy_planes(src0, u_out, s.n, s.h, s.w, s.ld, s.ps, st);
        if (e == hipSuccess) {
            if (d0) e = launch_copy_planes(d0, d_out, s.n, s.h, s.w, s.ld, s.ps, st);
            else e = launch_fill_f32(d_out, ext, 0.0f, st);
        }
        return e == hipSuccess ? WMC_OK : hip_fail(e, "copy");
    }
    Tuned t{};
    bool graph = true;
    if (tuning_complete(tune)) {
        rc = resolve_tuning(tune, Tuned{2, 3, 16}, &t, &graph);
    } else {
        const Tuned deflt{std::min(2, vec_cols({src0, f, u_out}, s.ld, s.n > 1 ? s.ps : 0)), 3,
                          default_rows(s.n, s.h, s.w, 2, 3, dev, kModeL1)};
        std::ostringstream k;
        k << arch_name(dev) << "|single2|l1|h" << s.h << "|w" << s.w << "|n" << s.n;
        auto search = [&](Tuned* out) {
            float* scratchU = iters >= 2 ? wsU : u_out;
            float* scratchD = iters >= 2 ? wsD : d_out;
            // time launches shaped like the solve's: U and f different
            // planes, and a dual plane read (every launch after the first
            // reads one).  With a workspace, u_out and d_out serve as those
            // planes (their contents do not matter for the timing; the
            // solve overwrites them)
            const float* usrc = iters >= 2 ? u_out : src0;
            const float* dsrc = iters >= 2 ? d_out : d0;
            auto run = [&](int C, int T, int R, hipStream_t ss) {
                return enqueue_l1(s, usrc, dsrc, f, scratchU, scratchD, lam, alpha, dt, C, T, R, ss);
            };
            auto rows = [&](int C, int T) {
                return candidate_rows(s.n, s.h, s.w, C, T, dev, kModeL1);
            };
            return tune_search(run, rows, st, out);
        };
        Tuned auto_t{};
        rc = get_tuning(k.str(), deflt, search, &auto_t);
        if (rc) return rc;
        rc = resolve_tuning(tune, auto_t, &t, &graph);
    }
    if (rc) return rc;
    // launch depths and the (U, d) buffer pair each launch writes: the last
    // writes the outputs, consecutive launches alternate with the workspace
    std::vector<int> depth;
    split_run(iters, t.T, depth);
    const int L = (int)depth.size();
    std::vector<int> to_out(L);
    for (int l = L - 1; l >= 0; --l) to_out[l] = (l == L - 1) ? 1 : !to_out[l + 1];
    auto enqueue = [&](hipStream_t ss, PlanEntry&) -> int {
        const float* su = src0;
        const float* sd = d0;
        for (int l = 0; l < L; ++l) {
            float* du = to_out[l] ? u_out : wsU;
            float* dd = to_out[l] ? d_out : wsD;
            const int r = enqueue_l1(s, su, sd, f, du, dd, lam, alpha, dt, t.C, depth[l], t.R, ss);
            if (r) return r;
            su = du;
            sd = dd;
        }
        return WMC_OK;
    };
    if (!graph) {
        PlanEntry scratch;
        return enqueue(st, scratch);
    }
    std::string key = "l1|";
    key_add(key, s);
    key_add(key, f);
    key_add(key, u0);
    key_add(key, d0);
    key_add(key, u_out);
    key_add(key, d_out);
    key_add(key, lam);
    key_add(key, alpha);
    key_add(key, iters);
    key_add(key, dt);
    key_add(key, ws);
    key_add(key, t);
    key_add(key, dev);
    auto prepare = [](PlanEntry&) { return WMC_OK; };
    return run_plan(key, dev, st, true, prepare, enqueue);
}

int wmc_solve_tuning(const float* f, const float* u0, const float* lam, float dt, void* ws,
                     size_t ws_bytes, wmc_shape s, wmc_tuning* out, void* stream) {
    g_err.clear();
    int rc = check_shape(s);
    if (rc) return rc;
    if (!out) return fail(WMC_EINVAL, "wmc_solve_tuning: null out");
    if (!f && !u0) return fail(WMC_EINVAL, "wmc_solve_tuning: the curvature flow needs u0");
    if (f && !lam) return fail(WMC_EINVAL, "wmc_solve_tuning: lam is required with a data term");
    if (!ws || ws_bytes < wmc_solve_workspace(s))
        return fail(WMC_ENOMEM, "wmc_solve_tuning: workspace smaller than wmc_solve_workspace()");
    const int64_t ext = extent_elems(s);
    // with room for two plane sets (the second at the next 256-byte offset)
    // the candidates ping-pong between them, as the solve does; with one
    // they read U from u0 (or f)
    const size_t set_bytes = (size_t)set_stride_elems(s) * sizeof(float);
    const size_t alt_off = (set_bytes + 255) / 256 * 256;
    float* alt = ws_bytes >= alt_off + set_bytes
                     ? reinterpret_cast<float*>(static_cast<char*>(ws) + alt_off)
                     : nullptr;
    const Range rw = range_of(ws, alt ? (int64_t)((alt_off + set_bytes) / 4) : ext, 4);
    if (overlaps(rw, range_of(f, ext, 4)) || overlaps(rw, range_of(u0, ext, 4)))
        return fail(WMC_EINVAL, "wmc_solve_tuning: ws overlaps an input");
    int dev;
    rc = check_device(&dev);
    if (rc) return rc;
    Tuned t{};
    rc = tune_single(dev, s, u0 ? u0 : f, f, lam, dt, static_cast<float*>(ws), as_stream(stream), &t,
                     alt);
    if (rc) return rc;
    out->cols = t.C;
    out->tsteps = t.T;
    out->seg_rows = t.R;
    out->use_graph = 1;
    return WMC_OK;
}

size_t wmc_batched_workspace(const wmc_image* imgs, int n_imgs) {
    if (!imgs || n_imgs <= 0) return 0;
    size_t total = 0;
    for (int i = 0; i < n_imgs; ++i) {
        const wmc_image& m = imgs[i];
        if (m.channels < 1 || m.h < 1 || m.w < 1 || m.ld < m.w) return 0;
        const int64_t ext = (int64_t)(m.channels - 1) * m.ps + (m.h - 1) * m.ld + m.w;
        total += (size_t)((ext + 63) / 64 * 64) * sizeof(float);
    }
    return total;
}

int wmc_solve_batched(const wmc_image* imgs, int n_imgs, const float* lam, int iters, float dt,
                      const wmc_tuning* tune, void* ws, size_t ws_bytes, void* stream) {
    g_err.clear();
    if (!imgs || n_imgs < 1) return fail(WMC_EINVAL, "wmc_solve_batched: no images");
    if (iters < 0) return fail(WMC_EINVAL, "wmc_solve_batched: iters must be >= 0");
    if (!std::isfinite(dt)) return fail(WMC_EINVAL, "wmc_solve_batched: dt must be finite");
    const bool data = imgs[0].f != nullptr;
    std::vector<BatchImg> b(n_imgs);
    std::vector<Range> outs(n_imgs), ins;
    size_t off = 0;
    for (int i = 0; i < n_imgs; ++i) {
        const wmc_image& m = imgs[i];
        wmc_shape s{m.channels, m.h, m.w, m.ld, m.ps};
        int rc = check_shape(s);
        if (rc) return fail(rc, "wmc_solve_batched: image " + std::to_string(i) + ": " + g_err);
        if (!m.out) return fail(WMC_EINVAL, "wmc_solve_batched: null out");
        if ((m.f != nullptr) != data)
            return fail(WMC_EINVAL, "wmc_solve_batched: all images must have a data term or none");
        if (!m.f && !m.u0) return fail(WMC_EINVAL, "wmc_solve_batched: flow images need u0");
        if (data && m.lam_index < 0) return fail(WMC_EINVAL, "wmc_solve_batched: lam_index < 0");
        const int64_t ext = extent_elems(s);
        outs[i] = range_of(m.out, ext, 4);
        ins.push_back(range_of(m.u0, ext, 4));
        ins.push_back(range_of(m.f, ext, 4));
        b[i] = BatchImg{m.u0 ? m.u0 : m.f, m.f, m.out,
                        static_cast<float*>(ws) ? reinterpret_cast<float*>(static_cast<char*>(ws) + off)
                                                : nullptr,
                        m.h, m.w, m.ld, m.ps, m.channels, m.lam_index, 0};
        off += (size_t)((ext + 63) / 64 * 64) * sizeof(float);
    }
    if (data && !lam) return fail(WMC_EINVAL, "wmc_solve_batched: lam is required with a data term");
    if (iters >= 2 && (!ws || ws_bytes < off))
        return fail(WMC_ENOMEM, "wmc_solve_batched: workspace smaller than wmc_batched_workspace()");
    const Range rw = range_of(iters >= 2 ? ws : nullptr, (int64_t)off, 1);
    for (int i = 0; i < n_imgs; ++i) {
        if (overlaps(outs[i], rw)) return fail(WMC_EINVAL, "wmc_solve_batched: out overlaps ws");
        for (const Range& r : ins)
            if (overlaps(outs[i], r)) return fail(WMC_EINVAL, "wmc_solve_batched: out overlaps an input");
        for (int j = i + 1; j < n_imgs; ++j)
            if (overlaps(outs[i], outs[j])) return fail(WMC_EINVAL, "wmc_solve_batched: outputs overlap");
    }
    for (const Range& r : ins)
        if (overlaps(rw, r)) return fail(WMC_EINVAL, "wmc_solve_batched: ws overlaps an input");
    int dev;
    int rc = check_device(&dev);
    if (rc) return rc;
    hipStream_t st = as_stream(stream);
    if (iters == 0) {
        for (int i = 0; i < n_imgs; ++i) {
            const hipError_t e =
                launch_copy_planes(b[i].src, b[i].out, b[i].channels, b[i].h, b[i].w, b[i].ld, b[i].ps, st);
            if (e != hipSuccess) return hip_fail(e, "copy");
        }
        return WMC_OK;
    }
    const int mode = data ? kModeData : kModeFlow;
    Tuned t{};
    bool graph = true;
    if (tuning_complete(tune)) {
        rc = resolve_tuning(tune, Tuned{2, 4, 32}, &t, &graph);
    } else {
        Tuned auto_t{};
        rc = tune_batch(dev, b, lam, dt, mode, st, &auto_t);
        if (rc) return rc;
        rc = resolve_tuning(tune, auto_t, &t, &graph);
    }
    if (rc) return rc;
    return batched_run(b, lam, iters, dt, mode, t.C, t.T, t.R, graph, dev, st);
}

int wmc_autotune(const wmc_image* imgs, int n_imgs, int iters, wmc_tuning* out, void* ws,
                 size_t ws_bytes, void* stream) {
    g_err.clear();
    if (!imgs || n_imgs < 1 || !out) return fail(WMC_EINVAL, "wmc_autotune: bad arguments");
    (void)iters;
    const bool data = imgs[0].f != nullptr;
    std::vector<BatchImg> b(n_imgs);
    size_t off = 0;
    for (int i = 0; i < n_imgs; ++i) {
        const wmc_image& m = imgs[i];
        wmc_shape s{m.channels, m.h, m.w, m.ld, m.ps};
        int rc = check_shape(s);
        if (rc) return rc;
        if ((m.f != nullptr) != data || (!m.f && !m.u0) || !m.out)
            return fail(WMC_EINVAL, "wmc_autotune: inconsistent image descriptors");
        const int64_t ext = extent_elems(s);
        b[i] = BatchImg{m.u0 ? m.u0 : m.f, m.f, m.out,
                        reinterpret_cast<float*>(static_cast<char*>(ws) + off), m.h, m.w, m.ld, m.ps,
                        m.channels, m.lam_index, 0};
        off += (size_t)((ext + 63) / 64 * 64) * sizeof(float);
    }
    if (!ws || ws_bytes < off) return fail(WMC_ENOMEM, "wmc_autotune: workspace too small");
    int dev;
    int rc = check_device(&dev);
    if (rc) return rc;
    // lambda values only steer the arithmetic, not the timing: use a device zero
    float* zl = nullptr;
    WMC_HIP(hipMalloc(&zl, 256 * sizeof(float)), "hipMalloc");
    hipStream_t st = as_stream(stream);
    rc = WMC_OK;
    if (launch_fill_f32(zl, 256, 1.0f, st) != hipSuccess) rc = fail(WMC_EHIP, "fill");
    Tuned t{};
    if (!rc) {
        for (BatchImg& x : b) x.lam_index = 0;
        rc = tune_batch(dev, b, zl, 0.0f, data ? kModeData : kModeFlow, st, &t);
    }
    (void)hipStreamSynchronize(st);
    (void)hipFree(zl);
    if (rc) return rc;
    out->cols = t.C;
    out->tsteps = t.T;
    out->seg_rows = t.R;
    out->use_graph = 1;
    return WMC_OK;
}

// dL/dlam partial sums are kept for up to this many steps before they are
// reduced (at least one checkpoint segment, up to 64 steps: one float per
// work item and step): the reductions add the steps in descending order
// either way.
int lam_slots(int iters, int c) { return std::max(c, std::min(64, std::max(iters, 1))); }

// Largest adjoint work-item count over the lane widths (the lambda partial
// buffer is sized for it).
int64_t adj_items_max(const wmc_shape& s) {
    int64_t items = 0;
    for (int C : {1, 2, 4}) items = std::max(items, adj_items(s.n, s.h, s.w, C));
    return items;
}

size_t wmc_backward_workspace(wmc_shape s, int iters, int ckpt_every) {
    if (check_shape(s) || iters < 0 || ckpt_every < 1) return 0;
    const size_t set = (size_t)set_stride_elems(s) * sizeof(float);
    const int c = std::min(ckpt_every, std::max(iters, 1));
    const size_t states = (size_t)std::max(c - 1, 0) * set;
    const size_t grads = 2 * set;
    // dL/dlam partial sums: one per work item and step of a segment, sized for
    // the column width with the most work items
    const int64_t items = adj_items_max(s);
    const size_t part = (size_t)lam_slots(iters, c) * (size_t)items * sizeof(float);
    const size_t sums = (size_t)s.n * lam_slots(iters, c) * sizeof(float);  // per-slot lambda sums
    return states + grads + (part + 255) / 256 * 256 + sums;
}

int wmc_backward(const float* f, const float* u0, const float* lam, int iters, float dt,
                 const float* ckpt, int ckpt_every, const float* g_out, float* g_f, float* g_u0,
                 float* g_lam, void* ws, size_t ws_bytes, wmc_shape s, void* stream) {
    g_err.clear();
    int rc = check_shape(s);
    if (rc) return rc;
    if (!f && !u0) return fail(WMC_EINVAL, "wmc_backward: the curvature flow needs u0");
    if (f && !lam) return fail(WMC_EINVAL, "wmc_backward: lam is required with a data term");
    if (iters < 0 || ckpt_every < 1) return fail(WMC_EINVAL, "wmc_backward: bad iters / ckpt_every");
    if (iters > 0 && !ckpt) return fail(WMC_EINVAL, "wmc_backward: checkpoints are required");
    if (!g_out) return fail(WMC_EINVAL, "wmc_backward: null g_out");
    if (!std::isfinite(dt)) return fail(WMC_EINVAL, "wmc_backward: dt must be finite");
    if (s.ld > INT32_MAX) return fail(WMC_EINVAL, "wmc_backward: ld must be < 2^31");
    const size_t need = wmc_backward_workspace(s, iters, ckpt_every);
    if (!ws || ws_bytes < need) return fail(WMC_ENOMEM, "wmc_backward: workspace too small");
    const int64_t ext = extent_elems(s);
    const Range rw = range_of(ws, (int64_t)need, 1);
    for (const void* p : {(const void*)g_f, (const void*)g_u0})
        if (p && (overlaps(range_of(p, ext, 4), rw) || overlaps(range_of(p, ext, 4), range_of(g_out, ext, 4))))
            return fail(WMC_EINVAL, "wmc_backward: outputs overlap the workspace or g_out");
    if (g_f && g_u0 && overlaps(range_of(g_f, ext, 4), range_of(g_u0, ext, 4)))
        return fail(WMC_EINVAL, "wmc_backward: g_f and g_u0 overlap");
    int dev;
    rc = check_device(&dev);
    if (rc) return rc;
    hipStream_t st = as_stream(stream);
    const int64_t set = set_stride_elems(s);
    char* w = static_cast<char*>(ws);
    const int c = std::min(ckpt_every, std::max(iters, 1));
    float* states = reinterpret_cast<float*>(w);
    w += (size_t)std::max(c - 1, 0) * set * sizeof(float);
    float* gA = reinterpret_cast<float*>(w);
    w += set * sizeof(float);
    float* gB = reinterpret_cast<float*>(w);
    w += set * sizeof(float);
    float* part = reinterpret_cast<float*>(w);
    float* lam_sums = reinterpret_cast<float*>(
        w + ((size_t)lam_slots(iters, c) * (size_t)adj_items_max(s) * sizeof(float) + 255) / 256 * 256);
    const bool data = f != nullptr;
    // recompute launches: plain single sweeps, paired columns when aligned
    const int C1 = std::min(2, vec_cols({ckpt, states, f, u0}, s.ld, s.n > 1 ? s.ps : 0));
    const int mode1 = data ? kModeData : kModeFlow;
    int R1[kTrajMaxT + 1] = {0};
    for (int T = 1; T <= kTrajMaxT; ++T) R1[T] = default_rows(s.n, s.h, s.w, C1, T, dev, mode1, T > 1);
    const int G = lam_slots(iters, c);
    // adjoint launches (WMC_ADJ_COLS=2|4 selects wider lanes)
    const char* env_cols = std::getenv("WMC_ADJ_COLS");
    int CA = 1;
    if (env_cols && (std::atoi(env_cols) == 2 || std::atoi(env_cols) == 4)) CA = std::atoi(env_cols);
    const bool vecA = vec_cols({ckpt, states, f, gA, gB, g_f}, s.ld, s.n > 1 ? s.ps : 0) >= CA;
    AdjArgs a{};
    a.f = f;
    a.g_f = data ? g_f : nullptr;
    a.part = (data && g_lam) ? part : nullptr;
    a.lam = lam;
    a.dt = dt;
    a.n = s.n;
    a.h = s.h;
    a.w = s.w;
    a.ld = s.ld;
    a.ps = s.ps;
    a.C = CA;
    a.R = adj_rows(s.n, s.h, s.w, CA);
    // WMC_ADJ_ROWS=R: rows per adjoint work item, at least the default (the
    // workspace holds the lambda partials of the default item count)
    if (const char* env_rows = std::getenv("WMC_ADJ_ROWS")) {
        const int r = std::atoi(env_rows);
        if (r > a.R && r <= 4096) a.R = r;
    }
    a.nstrip = adj_strip_count((int)s.w, CA);
    a.nseg = seg_count((int)s.h, a.R);
    a.vec = vecA ? 1 : 0;
    const int64_t items = (int64_t)s.n * a.nstrip * a.nseg;
    hipError_t e;
    // dL/dlam: the first reduction of the partial sums starts from zero;
    // only without one (flow mode, no step) is it cleared here
    bool lam_first = true;
    if (g_lam && !(a.part && iters >= 1)) {
        e = launch_fill_f32(g_lam, s.n, 0.0f, st);
        if (e != hipSuccess) return hip_fail(e, "fill");
    }
    // dL/df: the first adjoint step writes it without reading it (every
    // pixel is owned by one work item); with no step it starts at zero
    if (data && g_f && iters == 0) {
        e = launch_fill_f32(g_f, (s.n - 1) * s.ps + (s.h - 1) * s.ld + s.w, 0.0f, st);
        if (e != hipSuccess) return hip_fail(e, "fill");
    }
    a.gf_first = 1;
    // the first adjoint step reads g_out itself; the steps then alternate
    // between gA and gB, and the last one writes g_u0 when it is wanted
    const float* gcur = g_out;
    float* gbuf[2] = {gA, gB};
    int gnext = 0;
    int left = iters;
    const int nseg = (int)wmc_num_checkpoints(iters, ckpt_every);
    int used = 0;  // dL/dlam slots holding steps not yet reduced (slot G-1 first)
    for (int sg = nseg - 1; sg >= 0; --sg) {
        const int t0 = sg * ckpt_every;
        const int t1 = std::min(t0 + ckpt_every, iters);
        std::vector<const float*> st_ptr(t1 - t0);
        st_ptr[0] = ckpt + (int64_t)sg * set;
        // recompute the segment's states: fused launches of up to kTrajMaxT
        // sweeps that store every state (bitwise the same as single sweeps)
        for (int j = 0; j < t1 - t0 - 1;) {
            const int T = std::min(kTrajMaxT, t1 - t0 - 1 - j);
            float* traj[3] = {nullptr, nullptr, nullptr};
            for (int k = 1; k < T; ++k) traj[k - 1] = states + (int64_t)(j + k - 1) * set;
            float* dst = states + (int64_t)(j + T - 1) * set;
            rc = enqueue_single(s, st_ptr[j], f, dst, lam, dt, C1, T, R1[T], st, traj);
            if (rc) return rc;
            for (int k = 1; k <= T; ++k) st_ptr[j + k] = states + (int64_t)(j + k - 1) * set;
            j += T;
        }
        for (int t = t1 - 1; t >= t0; --t) {
            float* dst = (left == 1 && g_u0) ? g_u0 : gbuf[gnext];
            a.u = st_ptr[t - t0];
            a.g = gcur;
            a.g_prev = dst;
            a.slot = G - 1 - used;
            // the last step adds dL/dU^0 into dL/df itself when U^0 = f
            a.gf_fold = (left == 1 && data && g_f && !u0) ? 1 : 0;
            e = launch_adjoint_step(a, st);
            if (e != hipSuccess) return hip_fail(e, "adjoint launch");
            a.gf_first = 0;
            if (dst == gbuf[gnext]) gnext ^= 1;
            gcur = dst;
            --left;
            if (a.part && ++used == G) {
                e = launch_lambda_reduce(part, G, items, items / s.n, s.n, lam_first, g_lam,
                                         lam_sums, st);
                if (e != hipSuccess) return hip_fail(e, "lambda reduction");
                lam_first = false;
                used = 0;
            }
        }
    }
    if (a.part && used > 0) {
        e = launch_lambda_reduce(part + (int64_t)(G - used) * items, used, items, items / s.n, s.n,
                                 lam_first, g_lam, lam_sums, st);
        if (e != hipSuccess) return hip_fail(e, "lambda reduction");
    }
    if (g_u0 && iters == 0) {
        e = launch_copy_planes(g_out, g_u0, s.n, s.h, s.w, s.ld, s.ps, st);
        if (e != hipSuccess) return hip_fail(e, "copy");
    }
    if (data && g_f && !u0 && iters == 0) {
        e = launch_add_planes(gcur, g_f, s.n, s.h, s.w, s.ld, s.ps, st);
        if (e != hipSuccess) return hip_fail(e, "accumulate");
    }
    return WMC_OK;
}

size_t wmc_layer_workspace(wmc_shape s, int K) {
    if (check_shape(s) || K < 1 || K > 16) return 0;
    return (size_t)layer_part_floats(s.n, s.h, s.w, K) * sizeof(float);
}

int wmc_layer_forward(const float* u, const float* w, int K, float* out, uint8_t* sel,
                      wmc_shape s, void* stream) {
    g_err.clear();
    int rc = check_shape(s);
    if (rc) return rc;
    if (!u || !w || !out) return fail(WMC_EINVAL, "wmc_layer_forward: null pointer");
    if (K < 1 || K > 16) return fail(WMC_EINVAL, "wmc_layer_forward: K must be in [1, 16]");
    const int64_t ext = extent_elems(s);
    const Range ro = range_of(out, ext, 4), ru = range_of(u, ext, 4), rs = range_of(sel, ext, 1);
    if (overlaps(ro, ru) || overlaps(rs, ru) || overlaps(rs, ro) ||
        overlaps(range_of(w, 9 * K, 4), ro) || overlaps(range_of(w, 9 * K, 4), rs))
        return fail(WMC_EINVAL, "wmc_layer_forward: buffers overlap");
    int dev;
    rc = check_device(&dev);
    if (rc) return rc;
    const hipError_t e = launch_layer_forward(u, w, K, out, sel, s.n, s.h, s.w, s.ld, s.ps,
                                              as_stream(stream));
    return e == hipSuccess ? WMC_OK : hip_fail(e, "wmc_layer_forward launch");
}

int wmc_layer_backward(const float* u, const float* w, int K, const uint8_t* sel,
                       const float* g_out, float* g_u, float* g_w, void* ws, size_t ws_bytes,
                       wmc_shape s, void* stream) {
    g_err.clear();
    int rc = check_shape(s);
    if (rc) return rc;
    if (!u || !w || !sel || !g_out) return fail(WMC_EINVAL, "wmc_layer_backward: null pointer");
    if (K < 1 || K > 16) return fail(WMC_EINVAL, "wmc_layer_backward: K must be in [1, 16]");
    if (!g_u && !g_w) return WMC_OK;
    const size_t need = wmc_layer_workspace(s, K);
    if (g_w && (!ws || ws_bytes < need))
        return fail(WMC_ENOMEM, "wmc_layer_backward: workspace smaller than wmc_layer_workspace()");
    const int64_t ext = extent_elems(s);
    const Range rgu = range_of(g_u, ext, 4), rgw = range_of(g_w, 9 * K, 4);
    const Range rws = range_of(g_w ? ws : nullptr, (int64_t)need, 1);
    for (const Range& r : {range_of(u, ext, 4), range_of(g_out, ext, 4), range_of(sel, ext, 1),
                           range_of(w, 9 * K, 4)})
        if (overlaps(r, rgu) || overlaps(r, rgw) || overlaps(r, rws))
            return fail(WMC_EINVAL, "wmc_layer_backward: outputs overlap inputs");
    if (overlaps(rgu, rgw) || overlaps(rgu, rws) || overlaps(rgw, rws))
        return fail(WMC_EINVAL, "wmc_layer_backward: outputs overlap each other or the workspace");
    int dev;
    rc = check_device(&dev);
    if (rc) return rc;
    const hipError_t e = launch_layer_backward(u, w, K, sel, g_out, g_u, static_cast<float*>(ws),
                                               g_w, s.n, s.h, s.w, s.ld, s.ps, as_stream(stream));
    return e == hipSuccess ? WMC_OK : hip_fail(e, "wmc_layer_backward launch");
}

size_t wmc_workspace_bytes(int op, wmc_shape s, int iters, int ckpt_every) {
    switch (op) {
        case WMC_OP_SOLVE:
        case WMC_OP_FD_FLOW: return wmc_solve_workspace(s);
        case WMC_OP_SOLVE_L1: return wmc_l1_workspace(s);
        case WMC_OP_BACKWARD: return wmc_backward_workspace(s, iters, ckpt_every);
        case WMC_OP_LAYER_BACKWARD: return wmc_layer_workspace(s, iters);
        default: return 0;
    }
}

// ---- 3-D volumes -------------------------------------------------------------
namespace {

int64_t extent3(const wmc_shape3& s) {
    return (s.n - 1) * s.vs + (s.d - 1) * s.ss + (s.h - 1) * s.ld + s.w;
}

int check_shape3(const wmc_shape3& s) {
    if (s.n < 1 || s.d < 1 || s.h < 1 || s.w < 1)
        return fail(WMC_EINVAL, "shape3: n, d, h and w must be >= 1");
    if (s.d >= kMaxSide || s.h >= kMaxSide || s.w >= kMaxSide)
        return fail(WMC_EINVAL, "shape3: d, h and w must be < 2^30");
    if (s.n > 65535) return fail(WMC_EINVAL, "shape3: at most 65535 volumes per call");
    if (s.ld < s.w) return fail(WMC_EINVAL, "shape3: ld must be >= w");
    if (s.d > 1 && s.ss < (s.h - 1) * s.ld + s.w)
        return fail(WMC_EINVAL, "shape3: ss must be >= (h-1)*ld + w when d > 1");
    if (s.n > 1 && s.vs < (s.d - 1) * s.ss + (s.h - 1) * s.ld + s.w)
        return fail(WMC_EINVAL, "shape3: vs must be >= (d-1)*ss + (h-1)*ld + w when n > 1");
    if (s.ss < 0 || s.vs < 0) return fail(WMC_EINVAL, "shape3: strides must be >= 0");
    if (s.n * s.h * ((s.w + 63) / 64) > (int64_t)1 << 31)
        return fail(WMC_EINVAL, "shape3: too many rows for one launch");
    return WMC_OK;
}

int64_t set_stride3(const wmc_shape3& s) {
    const int64_t e = extent3(s), nv = s.n * s.vs;
    return nv >= e ? nv : e;
}

}  // namespace

int wmc3_compute(const float* u, float* hw, wmc_shape3 s, void* stream) {
    g_err.clear();
    int rc = check_shape3(s);
    if (rc) return rc;
    if (!u || !hw) return fail(WMC_EINVAL, "wmc3_compute: null pointer");
    const int64_t ext = extent3(s);
    if (overlaps(range_of(u, ext, 4), range_of(hw, ext, 4)))
        return fail(WMC_EINVAL, "wmc3_compute: output overlaps input");
    int dev;
    rc = check_device(&dev);
    if (rc) return rc;
    const hipError_t e = launch_stream3d(u, nullptr, hw, nullptr, 0.0f, kModeCompute, s.n, s.d, s.h,
                                         s.w, s.ld, s.ss, s.vs, as_stream(stream));
    return e == hipSuccess ? WMC_OK : hip_fail(e, "wmc3_compute launch");
}

int wmc3_step(const float* u, const float* f, float* u_out, const float* lam, float dt,
              uint8_t* argmin_out, wmc_shape3 s, void* stream) {
    g_err.clear();
    int rc = check_shape3(s);
    if (rc) return rc;
    if (!u || !u_out) return fail(WMC_EINVAL, "wmc3_step: null pointer");
    if (f && !lam) return fail(WMC_EINVAL, "wmc3_step: lam is required with a data term");
    if (!std::isfinite(dt)) return fail(WMC_EINVAL, "wmc3_step: dt must be finite");
    const int64_t ext = extent3(s);
    const Range ro = range_of(u_out, ext, 4), ra = range_of(argmin_out, ext, 1);
    if (overlaps(ro, range_of(u, ext, 4)) || overlaps(ro, range_of(f, ext, 4)) || overlaps(ro, ra))
        return fail(WMC_EINVAL, "wmc3_step: u_out overlaps an input (updates are synchronous)");
    if (overlaps(ra, range_of(u, ext, 4)) || overlaps(ra, range_of(f, ext, 4)))
        return fail(WMC_EINVAL, "wmc3_step: argmin_out overlaps an input");
    int dev;
    rc = check_device(&dev);
    if (rc) return rc;
    const hipError_t e = launch_stream3d(u, f, u_out, lam, dt, f ? kModeData : kModeFlow, s.n, s.d,
                                         s.h, s.w, s.ld, s.ss, s.vs, as_stream(stream), argmin_out);
    return e == hipSuccess ? WMC_OK : hip_fail(e, "wmc3_step launch");
}

size_t wmc3_solve_workspace(wmc_shape3 s) {
    if (check_shape3(s)) return 0;
    return (size_t)set_stride3(s) * sizeof(float);
}

int64_t wmc3_set_stride(wmc_shape3 s) {
    if (check_shape3(s)) return 0;
    return set_stride3(s);
}

namespace {

// Copies every volume of src to dst (layout s).
hipError_t copy_volumes(const float* src, float* dst, const wmc_shape3& s, hipStream_t st) {
    for (int64_t v = 0; v < s.n; ++v) {
        const hipError_t e = launch_copy_planes(src + v * s.vs, dst + v * s.vs, s.d, s.h, s.w, s.ld,
                                                s.ss, st);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// Output buffer of each of `iters` single-sweep launches: u_out for the
// last, the checkpoint slot for a state that is one, otherwise ws or u_out
// alternately so that no launch writes the buffer it reads.
std::vector<float*> sweep_targets3(int iters, float* u_out, float* ws, float* ckpt, int ckpt_every,
                                   int64_t set) {
    std::vector<float*> dst(iters);
    for (int t = iters - 1; t >= 0; --t) {
        if (t == iters - 1) dst[t] = u_out;
        else if (ckpt && (t + 1) % ckpt_every == 0) dst[t] = ckpt + (int64_t)((t + 1) / ckpt_every) * set;
        else dst[t] = (dst[t + 1] == u_out) ? ws : u_out;
    }
    return dst;
}

}  // namespace

int wmc3_solve(const float* f, const float* u0, float* u_out, const float* lam, int iters,
               float dt, float* ckpt, int ckpt_every, void* ws, size_t ws_bytes, wmc_shape3 s,
               void* stream) {
    g_err.clear();
    int rc = check_shape3(s);
    if (rc) return rc;
    if (!u_out) return fail(WMC_EINVAL, "wmc3_solve: null u_out");
    if (!f && !u0) return fail(WMC_EINVAL, "wmc3_solve: the flow (f == NULL) needs u0");
    if (f && !lam) return fail(WMC_EINVAL, "wmc3_solve: lam is required with a data term");
    if (iters < 0 || !std::isfinite(dt)) return fail(WMC_EINVAL, "wmc3_solve: bad iters or dt");
    if (ckpt && ckpt_every < 1) return fail(WMC_EINVAL, "wmc3_solve: ckpt_every must be >= 1");
    const int64_t ext = extent3(s), set = set_stride3(s);
    if (iters >= 2 && (!ws || ws_bytes < wmc3_solve_workspace(s)))
        return fail(WMC_ENOMEM, "wmc3_solve: workspace smaller than wmc3_solve_workspace()");
    const float* src0 = u0 ? u0 : f;
    const int64_t nck = ckpt ? wmc_num_checkpoints(iters, ckpt_every) : 0;
    const Range ro = range_of(u_out, ext, 4), rw = range_of(iters >= 2 ? ws : nullptr, ext, 4);
    const Range rc_ = range_of(ckpt, nck > 0 ? (nck - 1) * set + ext : 0, 4);
    for (const Range& r : {range_of(src0, ext, 4), range_of(f, ext, 4)})
        if (overlaps(ro, r) || overlaps(rw, r) || overlaps(rc_, r))
            return fail(WMC_EINVAL, "wmc3_solve: buffers overlap");
    if (overlaps(ro, rw) || overlaps(rc_, ro) || overlaps(rc_, rw))
        return fail(WMC_EINVAL, "wmc3_solve: u_out, ws and ckpt must not overlap");
    int dev;
    rc = check_device(&dev);
    if (rc) return rc;
    hipStream_t st = as_stream(stream);
    if (nck > 0) {
        const hipError_t e = copy_volumes(src0, ckpt, s, st);  // checkpoint 0 = U^0
        if (e != hipSuccess) return hip_fail(e, "checkpoint copy");
    }
    if (iters == 0) {
        const hipError_t e = copy_volumes(src0, u_out, s, st);
        return e == hipSuccess ? WMC_OK : hip_fail(e, "copy");
    }
    const std::vector<float*> dst =
        sweep_targets3(iters, u_out, static_cast<float*>(ws), nck > 0 ? ckpt : nullptr, ckpt_every, set);
    const float* src = src0;
    for (int t = 0; t < iters; ++t) {
        const hipError_t e = launch_stream3d(src, f, dst[t], lam, dt, f ? kModeData : kModeFlow, s.n,
                                             s.d, s.h, s.w, s.ld, s.ss, s.vs, st);
        if (e != hipSuccess) return hip_fail(e, "wmc3_solve launch");
        src = dst[t];
    }
    return WMC_OK;
}

size_t wmc3_backward_workspace(wmc_shape3 s, int iters, int ckpt_every) {
    if (check_shape3(s) || iters < 0 || ckpt_every < 1) return 0;
    const size_t set = (size_t)set_stride3(s) * sizeof(float);
    const int c = std::min(ckpt_every, std::max(iters, 1));
    const size_t states = (size_t)std::max(c - 1, 0) * set;
    const size_t grads = 2 * set;
    const size_t sel = ((size_t)set_stride3(s) + 255) / 256 * 256;  // one byte per voxel
    const int G = lam_slots(iters, c);
    const size_t part = ((size_t)G * (size_t)adjsel3_items(s.n, s.d, s.h, s.w) * sizeof(float) + 255) /
                        256 * 256;
    const size_t sums = (size_t)s.n * G * sizeof(float);
    return states + grads + sel + part + sums;
}

int wmc3_backward(const float* f, const float* u0, const float* lam, int iters, float dt,
                  const float* ckpt, int ckpt_every, const float* g_out, float* g_f, float* g_u0,
                  float* g_lam, void* ws, size_t ws_bytes, wmc_shape3 s, void* stream) {
    g_err.clear();
    int rc = check_shape3(s);
    if (rc) return rc;
    if (!f && !u0) return fail(WMC_EINVAL, "wmc3_backward: the flow needs u0");
    if (f && !lam) return fail(WMC_EINVAL, "wmc3_backward: lam is required with a data term");
    if (iters < 0 || ckpt_every < 1) return fail(WMC_EINVAL, "wmc3_backward: bad iters / ckpt_every");
    if (iters > 0 && !ckpt) return fail(WMC_EINVAL, "wmc3_backward: checkpoints are required");
    if (!g_out) return fail(WMC_EINVAL, "wmc3_backward: null g_out");
    if (!std::isfinite(dt)) return fail(WMC_EINVAL, "wmc3_backward: dt must be finite");
    const size_t need = wmc3_backward_workspace(s, iters, ckpt_every);
    if (!ws || ws_bytes < need) return fail(WMC_ENOMEM, "wmc3_backward: workspace too small");
    const int64_t ext = extent3(s), set = set_stride3(s);
    const Range rw = range_of(ws, (int64_t)need, 1), rg = range_of(g_out, ext, 4);
    for (const void* p : {(const void*)g_f, (const void*)g_u0})
        if (p && (overlaps(range_of(p, ext, 4), rw) || overlaps(range_of(p, ext, 4), rg)))
            return fail(WMC_EINVAL, "wmc3_backward: outputs overlap the workspace or g_out");
    if (g_f && g_u0 && overlaps(range_of(g_f, ext, 4), range_of(g_u0, ext, 4)))
        return fail(WMC_EINVAL, "wmc3_backward: g_f and g_u0 overlap");
    int dev;
    rc = check_device(&dev);
    if (rc) return rc;
    hipStream_t st = as_stream(stream);
    const bool data = f != nullptr;
    const int c = std::min(ckpt_every, std::max(iters, 1));
    char* w = static_cast<char*>(ws);
    float* states = reinterpret_cast<float*>(w);
    w += (size_t)std::max(c - 1, 0) * set * sizeof(float);
    float* gbuf[2] = {reinterpret_cast<float*>(w), reinterpret_cast<float*>(w) + set};
    w += 2 * set * sizeof(float);
    uint8_t* sel = reinterpret_cast<uint8_t*>(w);
    w += ((size_t)set + 255) / 256 * 256;
    const int G = lam_slots(iters, c);
    const int64_t items = adjsel3_items(s.n, s.d, s.h, s.w);
    float* part = reinterpret_cast<float*>(w);
    w += ((size_t)G * (size_t)items * sizeof(float) + 255) / 256 * 256;
    float* lam_sums = reinterpret_cast<float*>(w);
    float* apart = (data && g_lam) ? part : nullptr;
    hipError_t e;
    bool lam_first = true;
    if (g_lam && !(apart && iters >= 1)) {
        e = launch_fill_f32(g_lam, s.n, 0.0f, st);
        if (e != hipSuccess) return hip_fail(e, "fill");
    }
    if (iters == 0) {
        if (g_u0) {
            e = copy_volumes(g_out, g_u0, s, st);
            if (e != hipSuccess) return hip_fail(e, "copy");
        }
        if (data && g_f) {
            // dL/df = dL/dU^0 when U^0 = f, else zero
            if (!u0) e = copy_volumes(g_out, g_f, s, st);
            else
                for (int64_t v = 0; v < s.n && e == hipSuccess; ++v)
                    for (int64_t z = 0; z < s.d && e == hipSuccess; ++z)
                        e = launch_fill_f32(g_f + v * s.vs + z * s.ss, (s.h - 1) * s.ld + s.w, 0.0f, st);
            if (e != hipSuccess) return hip_fail(e, "copy");
        }
        return WMC_OK;
    }
    const float* gcur = g_out;
    int gnext = 0;
    int left = iters;
    int used = 0;
    bool gf_first = true;
    const int nseg = (int)wmc_num_checkpoints(iters, ckpt_every);
    for (int sg = nseg - 1; sg >= 0; --sg) {
        const int t0 = sg * ckpt_every;
        const int t1 = std::min(t0 + ckpt_every, iters);
        std::vector<const float*> ust(t1 - t0);
        ust[0] = ckpt + (int64_t)sg * set;
        // recompute the segment's states, one sweep per launch (bitwise those of the solve)
        for (int j = 1; j < t1 - t0; ++j) {
            float* dst = states + (int64_t)(j - 1) * set;
            e = launch_stream3d(ust[j - 1], f, dst, lam, dt, data ? kModeData : kModeFlow, s.n, s.d,
                                s.h, s.w, s.ld, s.ss, s.vs, st);
            if (e != hipSuccess) return hip_fail(e, "recompute launch");
            ust[j] = dst;
        }
        for (int t = t1 - 1; t >= t0; --t) {
            float* dst = (left == 1 && g_u0) ? g_u0 : gbuf[gnext];
            e = launch_adjsel3d(ust[t - t0], f, gcur, data ? g_f : nullptr, sel, apart, G - 1 - used,
                                gf_first, lam, dt, s.n, s.d, s.h, s.w, s.ld, s.ss, s.vs, st);
            if (e != hipSuccess) return hip_fail(e, "adjoint selection launch");
            gf_first = false;
            // the last step also adds dL/dU^0 into dL/df when U^0 = f
            float* fold = (left == 1 && data && g_f && !u0) ? g_f : nullptr;
            e = launch_adjgather3d(gcur, sel, dst, fold, lam, dt, data, s.n, s.d, s.h, s.w, s.ld, s.ss,
                                   s.vs, st);
            if (e != hipSuccess) return hip_fail(e, "adjoint gather launch");
            if (dst == gbuf[gnext]) gnext ^= 1;
            gcur = dst;
            --left;
            if (apart && ++used == G) {
                e = launch_lambda_reduce(part, G, items, items / s.n, s.n, lam_first, g_lam, lam_sums, st);
                if (e != hipSuccess) return hip_fail(e, "lambda reduction");
                lam_first = false;
                used = 0;
            }
        }
    }
    if (apart && used > 0) {
        e = launch_lambda_reduce(part + (int64_t)(G - used) * items, used, items, items / s.n, s.n,
                                 lam_first, g_lam, lam_sums, st);
        if (e != hipSuccess) return hip_fail(e, "lambda reduction");
    }
    return WMC_OK;
}

int wmc_fd_compute(const float* u, float* hw, float eps, wmc_shape s, void* stream) {
    g_err.clear();
    int rc = check_shape(s);
    if (rc) return rc;
    if (!u || !hw) return fail(WMC_EINVAL, "wmc_fd_compute: null pointer");
    if (!(eps >= 0.0f) || !std::isfinite(eps)) return fail(WMC_EINVAL, "wmc_fd_compute: eps must be >= 0");
    const int64_t ext = extent_elems(s);
    if (overlaps(range_of(u, ext, 4), range_of(hw, ext, 4)))
        return fail(WMC_EINVAL, "wmc_fd_compute: output overlaps input");
    int dev;
    rc = check_device(&dev);
    if (rc) return rc;
    const hipError_t e = launch_fd(u, hw, s.n, s.h, s.w, s.ld, s.ps, 0.0f, eps, false, as_stream(stream));
    return e == hipSuccess ? WMC_OK : hip_fail(e, "wmc_fd_compute launch");
}

int wmc_fd_flow(const float* u0, float* u_out, int iters, float dt, float eps, void* ws,
                size_t ws_bytes, wmc_shape s, void* stream) {
    g_err.clear();
    int rc = check_shape(s);
    if (rc) return rc;
    if (!u0 || !u_out) return fail(WMC_EINVAL, "wmc_fd_flow: null pointer");
    if (iters < 0 || !std::isfinite(dt) || !(eps >= 0.0f) || !std::isfinite(eps))
        return fail(WMC_EINVAL, "wmc_fd_flow: bad iters, dt or eps");
    const int64_t ext = extent_elems(s);
    if (iters >= 2 && (!ws || ws_bytes < wmc_solve_workspace(s)))
        return fail(WMC_ENOMEM, "wmc_fd_flow: workspace smaller than wmc_solve_workspace()");
    const Range ro = range_of(u_out, ext, 4), ri = range_of(u0, ext, 4);
    const Range rw = range_of(iters >= 2 ? ws : nullptr, ext, 4);
    if (overlaps(ro, ri) || overlaps(ro, rw) || overlaps(rw, ri))
        return fail(WMC_EINVAL, "wmc_fd_flow: buffers overlap");
    int dev;
    rc = check_device(&dev);
    if (rc) return rc;
    hipStream_t st = as_stream(stream);
    if (iters == 0) {
        const hipError_t e = launch_copy_planes(u0, u_out, s.n, s.h, s.w, s.ld, s.ps, st);
        return e == hipSuccess ? WMC_OK : hip_fail(e, "copy");
    }
    const float* src = u0;
    for (int t = 0; t < iters; ++t) {
        // the last step writes u_out, the ones before alternate with ws
        float* dst = ((iters - 1 - t) % 2 == 0) ? u_out : static_cast<float*>(ws);
        const hipError_t e = launch_fd(src, dst, s.n, s.h, s.w, s.ld, s.ps, dt, eps, true, st);
        if (e != hipSuccess) return hip_fail(e, "wmc_fd_flow launch");
        src = dst;
    }
    return WMC_OK;
}

int wmc_bw_probe(int op, const float* a, const float* b, float* o, int64_t n, int flags,
                 void* stream) {
    g_err.clear();
    if (op != WMC_PROBE_COPY && op != WMC_PROBE_ADD) return fail(WMC_EINVAL, "wmc_bw_probe: op");
    if (flags & ~WMC_PROBE_NONTEMPORAL) return fail(WMC_EINVAL, "wmc_bw_probe: unknown flags");
    if (n <= 0 || n % 4) return fail(WMC_EINVAL, "wmc_bw_probe: n must be a positive multiple of 4");
    if (!a || !o || (op == WMC_PROBE_ADD && !b)) return fail(WMC_EINVAL, "wmc_bw_probe: null pointer");
    for (const void* p : {static_cast<const void*>(a), static_cast<const void*>(b),
                          static_cast<const void*>(o)})
        if (reinterpret_cast<uintptr_t>(p) % 16)
            return fail(WMC_EINVAL, "wmc_bw_probe: pointers must be 16-byte aligned");
    const Range ro = range_of(o, n, 4);
    if (overlaps(ro, range_of(a, n, 4)) || (op == WMC_PROBE_ADD && overlaps(ro, range_of(b, n, 4))))
        return fail(WMC_EINVAL, "wmc_bw_probe: o overlaps an input");
    int rc = check_device(nullptr);
    if (rc) return rc;
    const hipError_t e = launch_bw_probe(op == WMC_PROBE_ADD, (flags & WMC_PROBE_NONTEMPORAL) != 0,
                                         a, b, o, n, as_stream(stream));
    return e == hipSuccess ? WMC_OK : hip_fail(e, "wmc_bw_probe launch");
}

int wmc_selftest(void) {
    g_err.clear();
    int dev;
    int rc = check_device(&dev);
    if (rc) return rc;
    int* d = nullptr;
    WMC_HIP(hipMalloc(&d, 4 * sizeof(int)), "hipMalloc");
    int h[4] = {0, 0, 0, 0};
    hipError_t e = launch_selftest(d, nullptr);
    if (e == hipSuccess) e = hipMemcpy(h, d, sizeof h, hipMemcpyDeviceToHost);
    (void)hipFree(d);
    if (e != hipSuccess) return hip_fail(e, "selftest");
    for (int i = 0; i < 4; ++i)
        if (h[i] != 1) return fail(WMC_EHIP, "selftest: DPP wave shifts do not move data as assumed");
    return WMC_OK;
}

void wmc_release(void) {
    {
        std::lock_guard<std::mutex> lk(g_plan_mu);
        g_plans.clear();
        for (auto& kv : g_capture_stream) (void)hipStreamDestroy(kv.second);
        g_capture_stream.clear();
    }
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune.clear();
    g_tune_loaded = false;
}

}  // extern "C"
