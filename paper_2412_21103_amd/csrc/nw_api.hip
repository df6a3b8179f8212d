// C-ABI entry points of libnw: argument checks on the host, workspace sizing
// and dispatch to the kernels.  No GPU work is queued unless every check
// passes.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <initializer_list>
#include <mutex>
#include <utility>
#include <vector>

#include "nw_internal.h"

namespace nw {

Consts dirs_consts(const nw_scoring& sc) {
    return Consts{4 * (sc.match - 2 * sc.gap) + 2, 4 * (sc.mismatch - 2 * sc.gap) + 2, sc.gap};
}
Consts score_consts(const nw_scoring& sc) {
    return Consts{sc.match - 2 * sc.gap, sc.mismatch - 2 * sc.gap, sc.gap};
}

// ---- device-fault words and the wait limit ----

namespace {
constexpr int kMaxFaultDevices = 64;
struct FaultWords {
    std::once_flag once;
    uint32_t* host = nullptr;  // pinned, one word per device
    uint32_t* dev = nullptr;   // the same memory as the kernels address it
};
FaultWords& fault_words() {
    static FaultWords f;
    return f;
}
std::atomic<int32_t> g_spin_limit{kDefaultSpinLimit};
std::atomic<int64_t> g_walk_limit{kDefaultWalkLimit};

// One pinned host allocation per process, made on first use.
void init_fault_words() {
    FaultWords& F = fault_words();
    std::call_once(F.once, [&] {
        void* h = nullptr;
        if (hipHostMalloc(&h, kMaxFaultDevices * sizeof(uint32_t), hipHostMallocMapped) != hipSuccess) return;
        std::memset(h, 0, kMaxFaultDevices * sizeof(uint32_t));
        void* d = nullptr;
        if (hipHostGetDevicePointer(&d, h, 0) != hipSuccess) d = h;
        F.host = (uint32_t*)h;
        F.dev = (uint32_t*)d;
    });
}
}  // namespace

int take_fault(int device) {
    FaultWords& F = fault_words();
    if (!F.host || device < 0 || device >= kMaxFaultDevices) return 0;
    volatile uint32_t* w = F.host + device;
    if (*w == 0) return 0;
    *w = 0;
    return 1;
}

int device_info(DeviceInfo* out, bool may_allocate) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return NW_EDEVICE;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return NW_EDEVICE;
    out->device = dev;
    out->cus = prop.multiProcessorCount;
    out->supported = std::strncmp(prop.gcnArchName, "gfx950", 6) == 0;
    if (may_allocate) init_fault_words();
    FaultWords& F = fault_words();
    out->fault = (F.dev && dev < kMaxFaultDevices) ? F.dev + dev : nullptr;
    out->spin_limit = g_spin_limit.load();
    out->walk_limit = g_walk_limit.load();
    if (!out->supported) return NW_ENOTSUP;
    // a fault reported by earlier work on this device surfaces here, once
    return take_fault(dev) ? NW_EDEVICE : NW_OK;
}

// Host checks shared by all entry points.
static int check_scoring(const nw_scoring& sc, bool dirs) {
    const int64_t big = 1 << 20;
    if (std::llabs(sc.match) > big || std::llabs(sc.mismatch) > big || std::llabs(sc.gap) > big)
        return NW_ERANGE;
    // terms beyond a signed byte run the byte-comparing sweep (needs_wide),
    // which holds them in 23 bits
    const Consts K = dirs ? dirs_consts(sc) : score_consts(sc);
    if (std::llabs(K.kdm) >= kWideTermLimit || std::llabs(K.kdx) >= kWideTermLimit) return NW_ERANGE;
    return NW_OK;
}

static int check_lengths(int64_t m, int64_t n, const nw_scoring& sc) {
    if (m < 0 || n < 0) return NW_EINVAL;
    if (m > INT32_MAX / 4 || n > INT32_MAX / 4) return NW_ERANGE;
    const int64_t c = std::max(std::llabs(sc.match), std::llabs(sc.mismatch)) + std::llabs(sc.gap);
    if (c * (m + n) >= (int64_t(1) << 27)) return NW_ERANGE;
    return NW_OK;
}

// ---- optional kernel timing ----

namespace {
struct ProfState {
    bool on = false;
    std::vector<hipEvent_t> pool;  // events, reused across sessions
    size_t used = 0;
    std::vector<std::pair<const char*, int>> marks;  // (name, index of start event)
};
ProfState& prof() {
    static ProfState s;
    return s;
}
hipEvent_t prof_event() {
    ProfState& P = prof();
    if (P.used == P.pool.size()) {
        hipEvent_t e = nullptr;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        P.pool.push_back(e);
    }
    return P.pool[P.used++];
}
}  // namespace

ProfScope::ProfScope(const char* n, hipStream_t s) : name(n), st(s), slot(-1) {
    ProfState& P = prof();
    if (!P.on) return;
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(st, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) return;
    hipEvent_t e = prof_event();
    if (!e) return;
    slot = (int)P.used - 1;
    (void)hipEventRecord(e, st);
}

ProfScope::~ProfScope() {
    if (slot < 0) return;
    ProfState& P = prof();
    hipEvent_t e = prof_event();
    if (!e) return;
    (void)hipEventRecord(e, st);
    P.marks.emplace_back(name, slot);
}

// ---- NW_GRAPH: captured launch sequences keyed by the call's arguments ----

namespace {
constexpr size_t kMaxGraphs = 256;
struct GraphEntry {
    std::vector<uint64_t> key;
    hipGraphExec_t exec;
};
struct GraphCache {
    std::mutex mu;
    std::vector<GraphEntry> entries;
};
GraphCache& graphs() {
    static GraphCache c;
    return c;
}
}  // namespace

std::vector<uint64_t> graph_key(std::initializer_list<uint64_t> words) { return std::vector<uint64_t>(words); }

// Run `launch` (which queues this call's kernels on st) directly, or through
// a cached graph when `use` is set.
template <class F>
int with_graph(bool use, std::vector<uint64_t> key, hipStream_t st, F&& launch) {
    if (!use) return launch();
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(st, &cs) != hipSuccess) return NW_EDEVICE;
    if (cs != hipStreamCaptureStatusNone) return launch();  // recorded into the caller's graph
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return NW_EDEVICE;
    key.push_back((uint64_t)(uintptr_t)st);
    key.push_back((uint64_t)dev);
    GraphCache& C = graphs();
    std::lock_guard<std::mutex> lock(C.mu);
    for (const GraphEntry& e : C.entries)
        if (e.key == key) return hipGraphLaunch(e.exec, st) == hipSuccess ? NW_OK : NW_EDEVICE;
    if (C.entries.size() >= kMaxGraphs) return launch();
    if (hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal) != hipSuccess) return NW_EDEVICE;
    const int r = launch();
    hipGraph_t graph = nullptr;
    const hipError_t e = hipStreamEndCapture(st, &graph);
    if (r != NW_OK || e != hipSuccess || !graph) {
        if (graph) (void)hipGraphDestroy(graph);
        return r != NW_OK ? r : NW_EDEVICE;
    }
    hipGraphExec_t exec = nullptr;
    const hipError_t ie = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (ie != hipSuccess) return NW_EDEVICE;
    C.entries.push_back(GraphEntry{std::move(key), exec});
    return hipGraphLaunch(exec, st) == hipSuccess ? NW_OK : NW_EDEVICE;
}

void release_graphs() {
    GraphCache& C = graphs();
    std::lock_guard<std::mutex> lock(C.mu);
    for (GraphEntry& e : C.entries) (void)hipGraphExecDestroy(e.exec);
    C.entries.clear();
}

static uint64_t w(const void* p) { return (uint64_t)(uintptr_t)p; }
static uint64_t w(int64_t v) { return (uint64_t)v; }
static uint64_t wsc(const nw_scoring& sc) {
    return ((uint64_t)(uint32_t)sc.match << 32) ^ ((uint64_t)(uint32_t)sc.mismatch << 16) ^ (uint32_t)sc.gap;
}

// ---- nw_align without a workspace argument and without allocation ----
//
// The workspace of nw_align_noalloc is this file-scope array: one copy per
// device, allocated when the library's code object is loaded on that device
// and held until the process ends.  Host code never passes the array's name
// to a kernel (on the host it is a stand-in, not a device address): the
// device address comes from hipGetSymbolAddress, once per device, and only
// that address is used.
static __device__ __align__(256) uint8_t scratch[NW_SCRATCH_BYTES];

struct ScratchAddrs {
    std::mutex mu;
    void* ptr[kMaxFaultDevices] = {};
};
static ScratchAddrs& scratch_addrs() {
    static ScratchAddrs s;
    return s;
}

// Device address of this device's scratch array (resolved on first use, with
// the device current), or nullptr if it cannot be resolved.
static void* scratch_on(int device) {
    if (device < 0 || device >= kMaxFaultDevices) return nullptr;
    ScratchAddrs& S = scratch_addrs();
    std::lock_guard<std::mutex> lock(S.mu);
    if (!S.ptr[device]) {
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return nullptr;
        S.ptr[device] = p;
    }
    return S.ptr[device];
}

}  // namespace nw

using namespace nw;

extern "C" {

const char* nw_strerror(int status) {
    switch (status) {
        case NW_OK: return "success";
        case NW_EINVAL: return "invalid argument (null pointer, negative length or count, bad flag)";
        case NW_ERANGE: return "lengths or scoring constants exceed the overflow guard";
        case NW_ENOSPC: return "path capacity or workspace too small (or the pair exceeds nw_align_noalloc's scratch)";
        case NW_EDEVICE: return "HIP error while queueing work, or a device fault reported by earlier work";
        case NW_ENOTSUP: return "current device is not a gfx950 GPU";
        default: return "unknown status";
    }
}

int nw_version(void) { return 200; }

int nw_init(void) {
    DeviceInfo di;
    const int st = device_info(&di);
    if (st == NW_ENOTSUP) return st;
    if (!fault_words().host) return NW_EDEVICE;
    if (!scratch_on(di.device)) return NW_EDEVICE;
    return st;
}

int nw_sync(void* stream) {
    if (hipStreamSynchronize((hipStream_t)stream) != hipSuccess) return NW_EDEVICE;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return NW_EDEVICE;
    return take_fault(dev) ? NW_EDEVICE : NW_OK;
}

int nw_set_wait_limit(int32_t polls) {
    if (polls < 0) return NW_EINVAL;
    g_spin_limit.store(polls == 0 ? kDefaultSpinLimit : polls);
    return NW_OK;
}

int nw_set_walk_limit(int64_t moves) {
    if (moves < 0) return NW_EINVAL;
    g_walk_limit.store(moves == 0 ? kDefaultWalkLimit : moves);
    return NW_OK;
}

int nw_sweep_costs(int32_t* costs, int32_t* tuned) {
    if (!costs) return NW_EINVAL;
    DeviceInfo di;
    const int st = device_info(&di);
    if (st) return st;
    step_costs(di.device, true, costs);
    step_costs(di.device, false, costs + 3);
    if (tuned) *tuned = tuned_costs(di.device) ? 1 : 0;
    return NW_OK;
}

int nw_set_sweep_costs(const int32_t* costs) {
    if (!costs) return NW_EINVAL;
    for (int c = 0; c < 6; ++c)
        if (costs[c] < 1 || costs[c] > (1 << 20)) return NW_EINVAL;
    DeviceInfo di;
    const int st = device_info(&di);
    if (st) return st;
    set_step_costs(di.device, costs, costs + 3);
    return NW_OK;
}

void nw_release_caches(void) {
    release_graphs();
    reset_step_costs();
}

int nw_profile_begin(void) {
    ProfState& P = prof();
    P.on = true;
    P.used = 0;
    P.marks.clear();
    return NW_OK;
}

int nw_profile_end(nw_kernel_time* out, int32_t cap, int32_t* count) {
    ProfState& P = prof();
    P.on = false;
    if (!count || (cap > 0 && !out)) return NW_EINVAL;
    std::vector<nw_kernel_time> acc;
    for (auto& mk : P.marks) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, P.pool[mk.second], P.pool[mk.second + 1]) != hipSuccess)
            return NW_EDEVICE;
        size_t i = 0;
        while (i < acc.size() && std::strcmp(acc[i].name, mk.first) != 0) ++i;
        if (i == acc.size()) acc.push_back(nw_kernel_time{mk.first, 0, 0.0});
        acc[i].launches += 1;
        acc[i].total_ms += ms;
    }
    *count = (int32_t)acc.size();
    for (int32_t i = 0; i < cap && i < (int32_t)acc.size(); ++i) out[i] = acc[i];
    P.marks.clear();
    P.used = 0;
    return NW_OK;
}

// ---------------------------------------------------------------- one pair

static const size_t kDescBytes = 1024;  // one-pair descriptor at the front of ws

static bool use_coop(int64_t m, int64_t n) { return m >= 1 && n >= kCoopMinCols; }

static size_t single_workspace_bytes(int64_t m, int64_t n, bool dirs, const DeviceInfo& di) {
    if (use_coop(m, n)) return coop_workspace_bytes(m, n, dirs);
    const int32_t ml = (int32_t)std::max<int64_t>(std::max(m, n), 1);
    return kDescBytes + batch_workspace_bytes(1, ml, dirs, di);
}

int nw_align_workspace_size(int64_t m, int64_t n, uint32_t flags, size_t* bytes) {
    if (!bytes || (flags & ~NW_SCORE_ONLY)) return NW_EINVAL;
    if (m < 0 || n < 0) return NW_EINVAL;
    if (m > INT32_MAX / 4 || n > INT32_MAX / 4) return NW_ERANGE;
    DeviceInfo di;
    int st = device_info(&di);
    if (st) return st;
    *bytes = single_workspace_bytes(m, n, !(flags & NW_SCORE_ONLY), di);
    return NW_OK;
}

__global__ void k_single_desc(int64_t* d64, int32_t* d32, int64_t b_off, int32_t m, int32_t n) {
    if (threadIdx.x == 0) {
        d64[0] = 0;       // a_off
        d64[1] = b_off;   // b_off
        d64[2] = 0;       // path_off
        d32[0] = m;       // a_len
        d32[1] = n;       // b_len
    }
}

// Argument checks of nw_align and nw_align_noalloc (all before any work).
static int check_align_args(const uint8_t* a, int64_t m, const uint8_t* b, int64_t n, const nw_scoring& sc,
                            uint32_t flags, const int32_t* score, const uint8_t* path, int64_t path_cap,
                            const int64_t* path_len) {
    if (flags & ~NW_SCORE_ONLY) return NW_EINVAL;
    const bool dirs = !(flags & NW_SCORE_ONLY);
    int st = check_lengths(m, n, sc);
    if (st) return st;
    if ((m > 0 && !a) || (n > 0 && !b) || !score) return NW_EINVAL;
    if (dirs && (!path_len || (m + n > 0 && !path))) return NW_EINVAL;
    if (dirs && path_cap < m + n) return NW_ENOSPC;
    return check_scoring(sc, dirs);
}

// The single-pair path on a workspace of ws_bytes >= single_workspace_bytes:
// the cooperative multi-wave engine from 512 columns, else the batch engine on
// a one-pair descriptor written into the workspace.
static int align_on(const uint8_t* a, int64_t m, const uint8_t* b, int64_t n, const nw_scoring& sc, bool dirs,
                    int32_t* score, uint8_t* path, int64_t* path_len, void* ws, size_t ws_bytes,
                    hipStream_t s, const DeviceInfo& di) {
    if (use_coop(m, n)) return launch_coop(a, m, b, n, sc, dirs, score, path, path_len, ws, ws_bytes, s, di);
    const int32_t ml = (int32_t)std::max<int64_t>(std::max(m, n), 1);

    uint8_t* base = (uint8_t*)ws;
    int64_t* d64 = (int64_t*)base;
    int32_t* d32 = (int32_t*)(base + 64);
    const uint8_t* pa = (m > 0) ? a : b;
    const uint8_t* pb = (n > 0) ? b : pa;
    if (!pa) {  // both empty: any valid device pointer works as a pool base
        pa = pb = (const uint8_t*)ws;
    }
    const int64_t b_off = (int64_t)((intptr_t)pb - (intptr_t)pa);
    hipLaunchKernelGGL(k_single_desc, dim3(1), dim3(64), 0, s, d64, d32, b_off, (int32_t)m, (int32_t)n);

    BatchJob J{};
    J.allpairs = false;
    J.njobs = 1;
    J.pool = pa;
    J.a_off = d64;
    J.b_off = d64 + 1;
    J.a_len = d32;
    J.b_len = d32 + 1;
    J.max_len = ml;
    J.sc = sc;
    J.dirs = dirs;
    J.scores = score;
    J.paths = path;
    J.path_off = d64 + 2;
    J.path_len = nullptr;
    J.path_len64 = dirs ? path_len : nullptr;
    return launch_batch(J, base + kDescBytes, ws_bytes - kDescBytes, s, di);
}

int nw_align(const uint8_t* a, int64_t m, const uint8_t* b, int64_t n, nw_scoring sc,
             uint32_t flags, int32_t* score, uint8_t* path, int64_t path_cap,
             int64_t* path_len, void* ws, size_t ws_bytes, void* stream) {
    int st = check_align_args(a, m, b, n, sc, flags, score, path, path_cap, path_len);
    if (st) return st;
    if (!ws) return NW_EINVAL;
    const bool dirs = !(flags & NW_SCORE_ONLY);
    DeviceInfo di;
    if ((st = device_info(&di))) return st;
    if (ws_bytes < single_workspace_bytes(m, n, dirs, di)) return NW_ENOSPC;
    return align_on(a, m, b, n, sc, dirs, score, path, path_len, ws, ws_bytes, (hipStream_t)stream, di);
}

int nw_align_noalloc(const uint8_t* a, int64_t m, const uint8_t* b, int64_t n, nw_scoring sc,
                     uint32_t flags, int32_t* score, uint8_t* path, int64_t path_cap,
                     int64_t* path_len, void* stream) {
    int st = check_align_args(a, m, b, n, sc, flags, score, path, path_cap, path_len);
    if (st) return st;
    const bool dirs = !(flags & NW_SCORE_ONLY);
    DeviceInfo di;
    if ((st = device_info(&di, false))) return st;
    if (single_workspace_bytes(m, n, dirs, di) > NW_SCRATCH_BYTES) return NW_ENOSPC;
    void* ws = scratch_on(di.device);
    if (!ws) return NW_EDEVICE;
    return align_on(a, m, b, n, sc, dirs, score, path, path_len, ws, NW_SCRATCH_BYTES, (hipStream_t)stream, di);
}

int nw_align_noalloc_fits(int64_t m, int64_t n, uint32_t flags) {
    if (flags & ~NW_SCORE_ONLY) return NW_EINVAL;
    if (m < 0 || n < 0) return NW_EINVAL;
    if (m > INT32_MAX / 4 || n > INT32_MAX / 4) return NW_ERANGE;
    DeviceInfo di;
    int st = device_info(&di, false);
    if (st) return st;
    return single_workspace_bytes(m, n, !(flags & NW_SCORE_ONLY), di) <= NW_SCRATCH_BYTES ? NW_OK : NW_ENOSPC;
}

// ------------------------------------------------------------------ batch

int nw_align_batch_workspace_size(int32_t npairs, int32_t max_len, uint32_t flags, size_t* bytes) {
    if (!bytes || npairs < 0 || max_len < 0 || (flags & ~(NW_SCORE_ONLY | NW_GRAPH))) return NW_EINVAL;
    DeviceInfo di;
    int st = device_info(&di);
    if (st) return st;
    *bytes = batch_workspace_bytes(npairs, std::max(max_len, 1), !(flags & NW_SCORE_ONLY), di);
    return NW_OK;
}

int nw_align_batch(int32_t npairs, const uint8_t* pool, const int64_t* a_off,
                   const int32_t* a_len, const int64_t* b_off, const int32_t* b_len,
                   int32_t max_len, nw_scoring sc, uint32_t flags, int32_t* scores,
                   uint8_t* paths, const int64_t* path_off, int32_t* path_len, void* ws,
                   size_t ws_bytes, void* stream) {
    if (npairs < 0 || max_len < 0 || (flags & ~(NW_SCORE_ONLY | NW_GRAPH))) return NW_EINVAL;
    if ((flags & NW_GRAPH) && !stream) return NW_EINVAL;
    const bool dirs = !(flags & NW_SCORE_ONLY);
    int st = check_lengths(max_len, max_len, sc);
    if (st) return st;
    if ((st = check_scoring(sc, dirs))) return st;
    if (npairs == 0) return NW_OK;
    if (!pool || !a_off || !a_len || !b_off || !b_len || !scores || !ws) return NW_EINVAL;
    if (dirs && (!paths || !path_off || !path_len)) return NW_EINVAL;
    DeviceInfo di;
    if ((st = device_info(&di))) return st;
    BatchJob J{};
    J.allpairs = false;
    J.njobs = npairs;
    J.pool = pool;
    J.a_off = a_off;
    J.a_len = a_len;
    J.b_off = b_off;
    J.b_len = b_len;
    J.max_len = std::max(max_len, 1);
    J.sc = sc;
    J.dirs = dirs;
    J.scores = scores;
    J.paths = paths;
    J.path_off = path_off;
    J.path_len = dirs ? path_len : nullptr;
    hipStream_t s = (hipStream_t)stream;
    return with_graph((flags & NW_GRAPH) != 0,
                      graph_key({1, w((int64_t)npairs), w(pool), w(a_off), w(a_len), w(b_off), w(b_len),
                                 w((int64_t)max_len), wsc(sc), w((int64_t)flags), w(scores), w(paths),
                                 w(path_off), w(path_len), w(ws), w((int64_t)ws_bytes)}),
                      s, [&] { return launch_batch(J, ws, ws_bytes, s, di); });
}

// -------------------------------------------------------------- autotuner

int nw_autotune(int32_t npairs, const uint8_t* pool, const int64_t* a_off, const int32_t* a_len,
                const int64_t* b_off, const int32_t* b_len, int32_t max_len, int32_t* scores, uint8_t* paths,
                const int64_t* path_off, int32_t* path_len, void* ws, size_t ws_bytes, int32_t* costs,
                void* stream) {
    if (npairs < 1 || max_len < 1) return NW_EINVAL;
    const nw_scoring sc{1, -1, -1};
    int st = check_lengths(max_len, max_len, sc);
    if (st) return st;
    if (!pool || !a_off || !a_len || !b_off || !b_len || !scores || !paths || !path_off || !path_len || !ws)
        return NW_EINVAL;
    DeviceInfo di;
    if ((st = device_info(&di))) return st;
    if (ws_bytes < batch_workspace_bytes(1, max_len, true, di)) return NW_ENOSPC;
    hipStream_t s = (hipStream_t)stream;
    std::vector<int32_t> ml(npairs), nl(npairs);
    if (hipMemcpyAsync(ml.data(), a_len, (size_t)npairs * 4, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipMemcpyAsync(nl.data(), b_len, (size_t)npairs * 4, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return NW_EDEVICE;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return NW_EDEVICE;
    int32_t table[2][3];
    int rc = NW_OK;
    for (int dirs = 1; dirs >= 0 && rc == NW_OK; --dirs) {
        double per_unit[3];
        for (int c = 0; c < 3 && rc == NW_OK; ++c) {
            const int C = 2 << c;
            const int64_t cols = 64 * C;
            double units = 0;  // sum over pairs of strips x (rows + ramp)
            for (int32_t k = 0; k < npairs; ++k)
                if (ml[k] > 0 && nl[k] > 0 && ml[k] <= max_len && nl[k] <= max_len)
                    units += (double)((nl[k] + cols - 1) / cols) * (double)(ml[k] + 64);
            BatchJob J{};
            J.njobs = npairs;
            J.pool = pool;
            J.a_off = a_off;
            J.a_len = a_len;
            J.b_off = b_off;
            J.b_len = b_len;
            J.max_len = max_len;
            J.sc = sc;
            J.dirs = dirs != 0;
            J.scores = scores;
            J.paths = paths;
            J.path_off = path_off;
            J.path_len = dirs ? path_len : nullptr;
            J.force_cols = C;
            float best = 1e30f;
            for (int rep = 0; rep < 3 && rc == NW_OK; ++rep) {
                if (hipEventRecord(e0, s) != hipSuccess) rc = NW_EDEVICE;
                if (rc == NW_OK) rc = launch_batch(J, ws, ws_bytes, s, di);
                float ms = 0.f;
                if (rc == NW_OK && (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                                    hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
                    rc = NW_EDEVICE;
                if (rep > 0) best = std::min(best, ms);  // the first run warms up
            }
            per_unit[c] = units > 0 ? (double)best / units : 1.0;
        }
        for (int c = 0; c < 3; ++c) {
            const double rel = (c == 2) ? 1.0 : per_unit[c] / per_unit[2];
            table[dirs][c] = (int32_t)std::lround(std::max(1.0, std::min(1e5, 1000.0 * rel)));
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc != NW_OK) return rc;
    set_step_costs(di.device, table[1], table[0]);
    if (costs)
        for (int c = 0; c < 3; ++c) {
            costs[c] = table[1][c];
            costs[3 + c] = table[0][c];
        }
    return NW_OK;
}

// ---------------------------------------------------------- certified band

// the flags the banded and learned calls accept
constexpr uint32_t kBandFlags = NW_SCORE_ONLY | NW_GRAPH | NW_BAND_DOUBLING | NW_BAND_ONE_LAUNCH;

int nw_align_batch_banded_workspace_size(int32_t npairs, int32_t max_len, uint32_t flags,
                                         size_t* bytes) {
    if (!bytes || npairs < 0 || max_len < 0 || (flags & ~kBandFlags))
        return NW_EINVAL;
    DeviceInfo di;
    int st = device_info(&di);
    if (st) return st;
    *bytes = batch_workspace_bytes(npairs, std::max(max_len, 1), !(flags & NW_SCORE_ONLY), di);
    return NW_OK;
}

static int run_banded(int32_t npairs, const uint8_t* pool, const int64_t* a_off, const int32_t* a_len,
                      const int64_t* b_off, const int32_t* b_len, int32_t max_len, nw_scoring sc,
                      uint32_t flags, const int32_t* w_init, int32_t w_default, float fallback_frac,
                      int32_t* scores, uint8_t* paths, const int64_t* path_off, int32_t* path_len,
                      int32_t* w_used, uint8_t* status, int64_t* cells, int64_t* cells_so, void* ws,
                      size_t ws_bytes,
                      hipStream_t stream, const DeviceInfo& di) {
    BatchJob J{};
    const bool dirs = !(flags & NW_SCORE_ONLY);
    J.allpairs = false;
    J.njobs = npairs;
    J.pool = pool;
    J.a_off = a_off;
    J.a_len = a_len;
    J.b_off = b_off;
    J.b_len = b_len;
    J.max_len = std::max(max_len, 1);
    J.sc = sc;
    J.dirs = dirs;
    J.scores = scores;
    J.paths = paths;
    J.path_off = path_off;
    J.path_len = dirs ? path_len : nullptr;
    J.banded = true;
    J.band_doubling = (flags & NW_BAND_DOUBLING) != 0;
    J.band_one_launch = (flags & NW_BAND_ONE_LAUNCH) != 0;
    J.w_init = w_init;
    J.w_default = w_default;
    J.frac_1024 = (int32_t)(fallback_frac * 1024.f);
    J.w_used = w_used;
    J.status = status;
    J.cells = cells;
    J.cells_so = cells_so;
    return launch_batch(J, ws, ws_bytes, stream, di);
}

// Host checks shared by the banded and learned entry points.
static int check_banded(int32_t npairs, const uint8_t* pool, const int64_t* a_off, const int32_t* a_len,
                        const int64_t* b_off, const int32_t* b_len, int32_t max_len, nw_scoring sc,
                        uint32_t flags, float fallback_frac, const int32_t* scores, const uint8_t* paths,
                        const int64_t* path_off, const int32_t* path_len, const void* ws,
                        bool ws_stream_ok) {
    if (npairs < 0 || max_len < 0 || (flags & ~kBandFlags)) return NW_EINVAL;
    if ((flags & NW_GRAPH) && !ws_stream_ok) return NW_EINVAL;
    if (!(fallback_frac > 0.f) || fallback_frac > 64.f) return NW_EINVAL;
    const bool dirs = !(flags & NW_SCORE_ONLY);
    int st = check_lengths(max_len, max_len, sc);
    if (st) return st;
    if ((st = check_scoring(sc, dirs))) return st;
    if (npairs == 0) return NW_OK;
    if (!pool || !a_off || !a_len || !b_off || !b_len || !scores || !ws) return NW_EINVAL;
    if (dirs && (!paths || !path_off || !path_len)) return NW_EINVAL;
    return NW_OK;
}

int nw_align_batch_banded(int32_t npairs, const uint8_t* pool, const int64_t* a_off,
                          const int32_t* a_len, const int64_t* b_off, const int32_t* b_len,
                          int32_t max_len, nw_scoring sc, uint32_t flags, const int32_t* w_init,
                          int32_t w_default, float fallback_frac, int32_t* scores, uint8_t* paths,
                          const int64_t* path_off, int32_t* path_len, int32_t* w_used,
                          uint8_t* status, int64_t* cells, int64_t* cells_so, void* ws, size_t ws_bytes,
                          void* stream) {
    if (w_default < 0) return NW_EINVAL;
    int st = check_banded(npairs, pool, a_off, a_len, b_off, b_len, max_len, sc, flags, fallback_frac,
                          scores, paths, path_off, path_len, ws, stream != nullptr);
    if (st || npairs == 0) return st;
    DeviceInfo di;
    if ((st = device_info(&di))) return st;
    hipStream_t s = (hipStream_t)stream;
    return with_graph((flags & NW_GRAPH) != 0,
                      graph_key({2, w((int64_t)npairs), w(pool), w(a_off), w(a_len), w(b_off), w(b_len),
                                 w((int64_t)max_len), wsc(sc), w((int64_t)flags), w(w_init), w((int64_t)w_default),
                                 w((int64_t)(fallback_frac * 1048576.f)), w(scores), w(paths), w(path_off),
                                 w(path_len), w(w_used), w(status), w(cells), w(cells_so), w(ws),
                                 w((int64_t)ws_bytes)}),
                      s, [&] {
                          return run_banded(npairs, pool, a_off, a_len, b_off, b_len, max_len, sc, flags, w_init,
                                            w_default, fallback_frac, scores, paths, path_off, path_len, w_used,
                                            status, cells, cells_so, ws, ws_bytes, s, di);
                      });
}

// ------------------------------------------------------------- band model

static bool mlp_ok(const nw_mlp* mlp, bool training) {
    return mlp && mlp->params && mlp->params_bf16 && (!training || (mlp->adam_m && mlp->adam_v)) &&
           mlp->step >= 0;
}

int nw_mlp_sync(const nw_mlp* mlp, void* stream) {
    if (!mlp_ok(mlp, false)) return NW_EINVAL;
    DeviceInfo di;
    int st = device_info(&di);
    if (st) return st;
    return launch_quantize(mlp->params, mlp->params_bf16, (hipStream_t)stream);
}

int nw_mlp_features(int32_t npairs, const uint8_t* pool, const int64_t* a_off, const int32_t* a_len,
                    const int64_t* b_off, const int32_t* b_len, float* x, void* stream) {
    if (npairs < 0) return NW_EINVAL;
    if (npairs == 0) return NW_OK;
    if (!pool || !a_off || !a_len || !b_off || !b_len || !x) return NW_EINVAL;
    DeviceInfo di;
    int st = device_info(&di);
    if (st) return st;
    return launch_features(npairs, pool, a_off, a_len, b_off, b_len, x, (hipStream_t)stream);
}

int nw_mlp_forward(const nw_mlp* mlp, int32_t rows, const float* x, float* yhat, void* stream) {
    if (rows < 0 || !mlp_ok(mlp, false)) return NW_EINVAL;
    if (rows == 0) return NW_OK;
    if (!x || !yhat) return NW_EINVAL;
    DeviceInfo di;
    int st = device_info(&di);
    if (st) return st;
    return launch_mlp_forward(rows, x, mlp->params, mlp->params_bf16, yhat, (hipStream_t)stream, di);
}

int nw_mlp_widths(int32_t npairs, const float* yhat, const int32_t* a_len, const int32_t* b_len,
                  float margin, int32_t* w, void* stream) {
    if (npairs < 0 || !(margin >= 0.f) || margin > 1e6f) return NW_EINVAL;
    if (npairs == 0) return NW_OK;
    if (!yhat || !a_len || !b_len || !w) return NW_EINVAL;
    DeviceInfo di;
    int st = device_info(&di);
    if (st) return st;
    return launch_widths(npairs, yhat, a_len, b_len, margin, w, (hipStream_t)stream);
}

int nw_band_labels(int32_t npairs, const int32_t* scores, const int32_t* a_len, const int32_t* b_len,
                   nw_scoring sc, int32_t* w_cert, float* target, void* stream) {
    if (npairs < 0) return NW_EINVAL;
    int st = check_scoring(sc, false);
    if (st) return st;
    const int32_t cd = std::max(sc.match, sc.mismatch);
    if (!(2 * (int64_t)sc.gap < cd)) return NW_EINVAL;
    if (npairs == 0) return NW_OK;
    if (!scores || !a_len || !b_len || (!w_cert && !target)) return NW_EINVAL;
    DeviceInfo di;
    if ((st = device_info(&di))) return st;
    return launch_band_labels(npairs, scores, a_len, b_len, cd, sc.gap, w_cert, target, (hipStream_t)stream);
}

int nw_path_labels(int32_t npairs, const uint8_t* paths, const int64_t* path_off, const int32_t* path_len,
                   const int32_t* a_len, const int32_t* b_len, int32_t* w_path, float* target, void* stream) {
    if (npairs < 0) return NW_EINVAL;
    if (npairs == 0) return NW_OK;
    if (!paths || !path_off || !path_len || !a_len || !b_len || (!w_path && !target)) return NW_EINVAL;
    DeviceInfo di;
    int st = device_info(&di);
    if (st) return st;
    return launch_path_labels(npairs, paths, path_off, path_len, a_len, b_len, w_path, target,
                              (hipStream_t)stream);
}

int nw_mlp_train_workspace_size(int32_t batch, size_t* bytes) {
    if (!bytes || batch < 1) return NW_EINVAL;
    *bytes = mlp_train_workspace_bytes(batch);
    return NW_OK;
}

static int check_train(const nw_mlp* mlp, int32_t batch, const float* x, const float* target, float tau,
                       float lr, const void* ws, size_t ws_bytes) {
    if (!mlp_ok(mlp, lr > 0.f) || batch < 1 || !x || !target || !ws) return NW_EINVAL;
    if (!(tau > 0.f && tau < 1.f) || !(lr >= 0.f)) return NW_EINVAL;
    if (ws_bytes < mlp_train_workspace_bytes(batch)) return NW_ENOSPC;
    return NW_OK;
}

int nw_mlp_train_step(nw_mlp* mlp, int32_t batch, const float* x, const float* target, const int32_t* rows,
                      float tau, float lr, float* loss, float* grad, void* ws, size_t ws_bytes,
                      void* stream) {
    int st = check_train(mlp, batch, x, target, tau, lr, ws, ws_bytes);
    if (st) return st;
    DeviceInfo di;
    if ((st = device_info(&di))) return st;
    return launch_mlp_train_step(mlp, batch, x, target, rows, tau, lr, loss, grad, ws, (hipStream_t)stream,
                                 di);
}

int nw_mlp_train_epoch(nw_mlp* mlp, int32_t n, const float* x, const float* target, const int32_t* order,
                       int32_t batch, float tau, float lr, float* losses, void* ws, size_t ws_bytes,
                       void* stream) {
    if (n < 0 || !order || !(lr > 0.f)) return NW_EINVAL;
    int st = check_train(mlp, batch, x, target, tau, lr, ws, ws_bytes);
    if (st) return st;
    DeviceInfo di;
    if ((st = device_info(&di))) return st;
    for (int32_t b = 0, i0 = 0; i0 < n; ++b, i0 += batch) {
        const int32_t rows = std::min(batch, n - i0);
        st = launch_mlp_train_step(mlp, rows, x, target, order + i0, tau, lr, losses ? losses + b : nullptr,
                                   nullptr, ws, (hipStream_t)stream, di);
        if (st) return st;
    }
    return NW_OK;
}

// Learned-band workspace: the banded engine's, then x, yhat and w.
static size_t learned_extra_bytes(int32_t npairs) {
    const size_t n = (size_t)std::max(npairs, 1);
    return align_up(n * NW_MLP_INPUTS * sizeof(float), 256) + align_up(n * sizeof(float), 256) +
           align_up(n * sizeof(int32_t), 256);
}

int nw_align_batch_learned_workspace_size(int32_t npairs, int32_t max_len, uint32_t flags, size_t* bytes) {
    if (!bytes || npairs < 0 || max_len < 0 || (flags & ~kBandFlags))
        return NW_EINVAL;
    DeviceInfo di;
    int st = device_info(&di);
    if (st) return st;
    *bytes = align_up(batch_workspace_bytes(npairs, std::max(max_len, 1), !(flags & NW_SCORE_ONLY), di),
                      256) +
             learned_extra_bytes(npairs);
    return NW_OK;
}

int nw_align_batch_learned(int32_t npairs, const uint8_t* pool, const int64_t* a_off, const int32_t* a_len,
                           const int64_t* b_off, const int32_t* b_len, int32_t max_len, nw_scoring sc,
                           uint32_t flags, const nw_mlp* mlp, float margin, float fallback_frac,
                           int32_t* scores, uint8_t* paths, const int64_t* path_off, int32_t* path_len,
                           int32_t* w_used, uint8_t* status, int64_t* cells, int64_t* cells_so, void* ws,
                           size_t ws_bytes, void* stream) {
    if (!mlp_ok(mlp, false) || !(margin >= 0.f) || margin > 1e6f) return NW_EINVAL;
    int st = check_banded(npairs, pool, a_off, a_len, b_off, b_len, max_len, sc, flags, fallback_frac, scores,
                          paths, path_off, path_len, ws, stream != nullptr);
    if (st || npairs == 0) return st;
    DeviceInfo di;
    if ((st = device_info(&di))) return st;
    const size_t band_bytes =
        align_up(batch_workspace_bytes(npairs, std::max(max_len, 1), !(flags & NW_SCORE_ONLY), di), 256);
    if (ws_bytes < band_bytes + learned_extra_bytes(npairs)) return NW_ENOSPC;
    char* base = (char*)ws + band_bytes;
    float* x = (float*)base;
    float* yhat = (float*)(base + align_up((size_t)npairs * NW_MLP_INPUTS * sizeof(float), 256));
    int32_t* wv = (int32_t*)((char*)yhat + align_up((size_t)npairs * sizeof(float), 256));
    hipStream_t s = (hipStream_t)stream;
    return with_graph(
        (flags & NW_GRAPH) != 0,
        graph_key({3, w((int64_t)npairs), w(pool), w(a_off), w(a_len), w(b_off), w(b_len), w((int64_t)max_len),
                   wsc(sc), w((int64_t)flags), w(mlp->params), w(mlp->params_bf16),
                   w((int64_t)(margin * 1048576.f)), w((int64_t)(fallback_frac * 1048576.f)), w(scores), w(paths),
                   w(path_off), w(path_len), w(w_used), w(status), w(cells), w(cells_so), w(ws),
                   w((int64_t)ws_bytes)}),
        s, [&] {
            int r;
            if ((r = launch_features(npairs, pool, a_off, a_len, b_off, b_len, x, s))) return r;
            if ((r = launch_mlp_forward(npairs, x, mlp->params, mlp->params_bf16, yhat, s, di))) return r;
            if ((r = launch_widths(npairs, yhat, a_len, b_len, margin, wv, s))) return r;
            return run_banded(npairs, pool, a_off, a_len, b_off, b_len, max_len, sc, flags, wv, 0, fallback_frac,
                              scores, paths, path_off, path_len, w_used, status, cells, cells_so, ws, band_bytes,
                              s, di);
        });
}

// -------------------------------------------------------------- all pairs

int nw_allpairs_workspace_size(int32_t nseq, int32_t max_len, size_t* bytes) {
    if (!bytes || nseq < 0 || max_len < 0) return NW_EINVAL;
    if ((int64_t)nseq * (nseq + 1) / 2 > INT32_MAX) return NW_ERANGE;
    DeviceInfo di;
    int st = device_info(&di);
    if (st) return st;
    *bytes = batch_workspace_bytes((int32_t)((int64_t)nseq * (nseq + 1) / 2), std::max(max_len, 1),
                                   false, di);
    return NW_OK;
}

int nw_allpairs_scores(int32_t nseq, const uint8_t* pool, const int64_t* off, const int32_t* len,
                       int32_t max_len, nw_scoring sc, int32_t* out, void* ws, size_t ws_bytes,
                       void* stream) {
    if (nseq < 0 || max_len < 0) return NW_EINVAL;
    if ((int64_t)nseq * (nseq + 1) / 2 > INT32_MAX) return NW_ERANGE;
    int st = check_lengths(max_len, max_len, sc);
    if (st) return st;
    if ((st = check_scoring(sc, false))) return st;
    if (nseq == 0) return NW_OK;
    if (!pool || !off || !len || !out || !ws) return NW_EINVAL;
    DeviceInfo di;
    if ((st = device_info(&di))) return st;
    BatchJob J{};
    J.allpairs = true;
    J.njobs = (int32_t)((int64_t)nseq * (nseq + 1) / 2);
    J.nseq = nseq;
    J.pool = pool;
    J.a_off = off;
    J.a_len = len;
    J.b_off = off;
    J.b_len = len;
    J.max_len = std::max(max_len, 1);
    J.sc = sc;
    J.dirs = false;
    J.matrix = out;
    return launch_batch(J, ws, ws_bytes, (hipStream_t)stream, di);
}

// -------------------------------------------------------------- center star

int nw_center_star_workspace_size(int32_t nseq, int32_t max_len, size_t* bytes) {
    if (!bytes || nseq < 0 || max_len < 0) return NW_EINVAL;
    if ((int64_t)nseq * std::max(max_len, 1) >= INT32_MAX) return NW_ERANGE;
    DeviceInfo di;
    int st = device_info(&di);
    if (st) return st;
    *bytes = center_star_workspace_bytes(nseq, std::max(max_len, 1), di);
    return NW_OK;
}

int nw_center_star(int32_t nseq, const uint8_t* pool, const int64_t* off, const int32_t* len, int32_t max_len,
                   nw_scoring sc, const int32_t* scores, uint8_t gap_byte, int32_t* center, uint8_t* msa,
                   int64_t width_cap, int64_t* width, void* ws, size_t ws_bytes, void* stream) {
    if (nseq < 0 || max_len < 0 || width_cap < 0) return NW_EINVAL;
    if ((int64_t)nseq * std::max(max_len, 1) >= INT32_MAX) return NW_ERANGE;
    int st = check_lengths(max_len, max_len, sc);
    if (st) return st;
    if ((st = check_scoring(sc, true))) return st;
    if (nseq == 0) return NW_OK;
    if (!pool || !off || !len || !scores || !center || !width || !ws || (width_cap > 0 && !msa)) return NW_EINVAL;
    DeviceInfo di;
    if ((st = device_info(&di))) return st;
    return launch_center_star(nseq, pool, off, len, std::max(max_len, 1), sc, scores, gap_byte, center, msa,
                              width_cap, width, ws, ws_bytes, (hipStream_t)stream, di);
}

int nw_cooptimal_workspace_size(int32_t npairs, int32_t max_len, int32_t k, size_t* bytes) {
    if (!bytes || npairs < 0 || max_len < 0 || k < 0) return NW_EINVAL;
    DeviceInfo di;
    int st = device_info(&di);
    if (st) return st;
    *bytes = cooptimal_workspace_bytes(npairs, std::max(max_len, 1), k, di);
    return NW_OK;
}

int nw_cooptimal(int32_t npairs, const uint8_t* pool, const int64_t* a_off, const int32_t* a_len,
                 const int64_t* b_off, const int32_t* b_len, int32_t max_len, nw_scoring sc, int32_t* scores,
                 uint64_t* counts, uint8_t* saturated, int32_t k, uint8_t* paths, const int64_t* path_off,
                 int32_t* path_len, int32_t* n_paths, void* ws, size_t ws_bytes, void* stream) {
    if (npairs < 0 || max_len < 0 || k < 0) return NW_EINVAL;
    if ((int64_t)npairs * k > INT32_MAX) return NW_ERANGE;
    int st = check_lengths(max_len, max_len, sc);
    if (st) return st;
    if ((st = check_scoring(sc, false))) return st;
    if (npairs == 0) return NW_OK;
    if (!pool || !a_off || !a_len || !b_off || !b_len || !scores || !counts || !saturated || !ws) return NW_EINVAL;
    if (k > 0 && (!paths || !path_off || !path_len || !n_paths)) return NW_EINVAL;
    DeviceInfo di;
    if ((st = device_info(&di))) return st;
    return launch_cooptimal(npairs, pool, a_off, a_len, b_off, b_len, std::max(max_len, 1), sc, scores, counts,
                            saturated, k, paths, path_off, path_len, n_paths, ws, ws_bytes, (hipStream_t)stream, di);
}

}  // extern "C"
