// One long pair on the whole GPU: cooperative column strips.
//
// The n columns are cut into strips of 64*C columns.  A block holds four
// waves (one per SIMD) and sweeps four consecutive strips; blocks take strip
// groups from an atomic ticket counter, so a wave only ever waits for the
// strip to its left, whose owner took an earlier ticket and is therefore
// already running or done: the schedule cannot deadlock, and the grid never
// needs more blocks than fit on the device.  A strip's right boundary column
// goes to the next strip through 64-bit {value, epoch} slots (TaggedIO), so
// the fill runs as one anti-diagonal front across all strips, each strip a
// fixed lag behind its left neighbour.
//
// The traceback then walks the stored direction words from (m, n) with one
// wave (walk_back), and writes the path in forward order.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>

#include "nw_internal.h"
#include "nw_strip.h"

namespace nw {

constexpr int kCoopWaves = 4;
constexpr int kCoopThreads = kWave * kCoopWaves;
// Dynamic LDS request that leaves room for only one block per CU, so the
// blocks spread over all CUs instead of doubling up.
constexpr size_t kCoopDynLds = 96 * 1024;

struct CoopArgs {
    const uint8_t* a;
    const uint8_t* b;
    int m, n;
    int kdm, kdx, gap, vinit;
    int nstrips, ngroups, G;
    uint32_t* dirs;
    uint64_t* bnd;
    int64_t bnd_stride;
    int32_t* ticket;
    int32_t* err;
    uint32_t epoch;
    int32_t* score;
};

template <int C, bool DIRS>
__global__ __launch_bounds__(kCoopThreads) void k_coop(CoopArgs A) {
    extern __shared__ uint32_t dyn[];
    __shared__ int ticket_s;
    const int wave = threadIdx.x >> 6;
    uint32_t* lds = dyn + wave * StripShape<C>::kLdsWords;
    constexpr int kCols = kWave * C;
    for (;;) {
        if (threadIdx.x == 0) ticket_s = atomicAdd(A.ticket, 1);
        __syncthreads();
        const int k = uniform(ticket_s);
        __syncthreads();
        if (k >= A.ngroups) break;
        const int s = k * kCoopWaves + wave;
        if (s < A.nstrips) {
            const int j0 = s * kCols;
            const int ksel = (A.n - 1 - j0) % C;
            const TaggedIO io{s == 0 ? nullptr : A.bnd + (int64_t)(s - 1) * A.bnd_stride,
                              s == A.nstrips - 1 ? nullptr : A.bnd + (int64_t)s * A.bnd_stride,
                              A.m,
                              A.vinit,
                              A.epoch,
                              A.err};
            const int32_t v = sweep_strip<C, DIRS>(A.a, A.m, A.b, A.n, j0, A.kdm, A.kdx, A.vinit, io,
                                                   DIRS ? A.dirs + (size_t)s * A.G * kWave * C : nullptr,
                                                   lds, ksel);
            if (s == A.nstrips - 1) {
                const int lsel = (A.n - 1 - j0) / C;
                const int32_t vv = __builtin_amdgcn_readlane(v, lsel);
                A.score[0] = (DIRS ? ((vv - 1) >> 2) : vv) + A.gap * (A.m + A.n);
            }
        }
    }
}

struct WalkArgs {
    const uint32_t* dirs;
    int m, n, G;
    uint8_t* rev;
    uint8_t* path;
    int64_t* path_len;
    int32_t* score;
    const int32_t* err;
};

// Traceback of the cooperative fill (also reports a boundary-wait failure of
// the fill as score INT32_MIN and path length -3).
template <int C>
__global__ __launch_bounds__(kWave) void k_walk(WalkArgs W) {
    __shared__ uint32_t lds[kWave * C];
    const int lane = lane_id();
    if (__hip_atomic_load(W.err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) {
        W.score[0] = INT32_MIN;
        if (W.path_len) W.path_len[0] = -3;
        return;
    }
    if (!W.dirs) return;
    const int64_t len = walk_back<C>(W.dirs, W.m, W.n, W.G, lds, W.rev);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
    if (len < 0) {
        W.path_len[0] = -2;
        return;
    }
    for (int64_t x = lane; x < len; x += kWave) W.path[x] = W.rev[len - 1 - x];
    W.path_len[0] = len;
}

__global__ void k_zero_small(int32_t* p, int n) {
    int i = threadIdx.x;
    if (i < n) p[i] = 0;
}

// ---- host side ----

constexpr int kCoopC = 1;

struct CoopLayout {
    int nstrips, ngroups, G;
    int64_t bnd_stride;
    size_t off_bnd, off_dirs, off_rev, total;
};

static CoopLayout coop_layout(int64_t m, int64_t n, bool dirs) {
    CoopLayout L{};
    const int64_t cols = (int64_t)kWave * kCoopC;
    L.nstrips = (int)((n + cols - 1) / cols);
    L.ngroups = (L.nstrips + kCoopWaves - 1) / kCoopWaves;
    L.G = groups_for_rows((int)m);
    L.bnd_stride = (int64_t)align_up((size_t)(m + 1), 32);
    size_t off = 256;
    L.off_bnd = off;
    off = align_up(off + (size_t)std::max(L.nstrips - 1, 0) * L.bnd_stride * 8, 256);
    L.off_dirs = off;
    if (dirs) off = align_up(off + (size_t)L.nstrips * L.G * kWave * kCoopC * 4, 256);
    L.off_rev = off;
    if (dirs) off = align_up(off + (size_t)(m + n + 16), 256);
    L.total = off;
    return L;
}

size_t coop_workspace_bytes(int64_t m, int64_t n, bool dirs) { return coop_layout(m, n, dirs).total; }

static uint32_t next_epoch() {
    static std::atomic<uint32_t> counter{
        (uint32_t)std::chrono::steady_clock::now().time_since_epoch().count()};
    return (counter.fetch_add(1) << 1) | 1u;  // never 0, the value of fresh memory
}

template <bool DIRS>
static hipError_t launch_coop_kernel(const CoopArgs& A, int grid, hipStream_t st) {
    static bool configured = false;
    if (!configured) {
        hipError_t e = hipFuncSetAttribute((const void*)k_coop<kCoopC, DIRS>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)kCoopDynLds);
        if (e != hipSuccess) return e;
        configured = true;
    }
    {
        ProfScope ps(DIRS ? "nw_fill_coop" : "nw_fill_coop_score", st);
        hipLaunchKernelGGL((k_coop<kCoopC, DIRS>), dim3(grid), dim3(kCoopThreads), kCoopDynLds, st, A);
    }
    return hipGetLastError();
}

int launch_coop(const uint8_t* a, int64_t m, const uint8_t* b, int64_t n, const nw_scoring& sc,
                bool dirs, int32_t* score, uint8_t* path, int64_t* path_len, void* ws,
                size_t ws_bytes, hipStream_t st, const DeviceInfo& di) {
    const CoopLayout L = coop_layout(m, n, dirs);
    if (ws_bytes < L.total) return NW_ENOSPC;
    uint8_t* base = (uint8_t*)ws;
    const Consts K = dirs ? dirs_consts(sc) : score_consts(sc);
    CoopArgs A{};
    A.a = a;
    A.b = b;
    A.m = (int)m;
    A.n = (int)n;
    A.kdm = K.kdm;
    A.kdx = K.kdx;
    A.gap = sc.gap;
    A.vinit = dirs ? 1 : 0;
    A.nstrips = L.nstrips;
    A.ngroups = L.ngroups;
    A.G = L.G;
    A.dirs = dirs ? (uint32_t*)(base + L.off_dirs) : nullptr;
    A.bnd = (uint64_t*)(base + L.off_bnd);
    A.bnd_stride = L.bnd_stride;
    A.ticket = (int32_t*)base;
    A.err = (int32_t*)(base + 64);
    A.epoch = next_epoch();
    A.score = score;
    hipLaunchKernelGGL(k_zero_small, dim3(1), dim3(64), 0, st, (int32_t*)base, 64);
    const int grid = std::max(1, std::min(L.ngroups, di.cus));
    hipError_t e = dirs ? launch_coop_kernel<true>(A, grid, st) : launch_coop_kernel<false>(A, grid, st);
    if (e != hipSuccess) return NW_EDEVICE;
    {
        WalkArgs W{};
        W.dirs = A.dirs;
        W.m = (int)m;
        W.n = (int)n;
        W.G = L.G;
        W.rev = base + L.off_rev;
        W.path = path;
        W.path_len = path_len;
        W.score = score;
        W.err = A.err;
        ProfScope ps("nw_walk_single", st);
        hipLaunchKernelGGL(k_walk<kCoopC>, dim3(1), dim3(kWave), 0, st, W);
    }
    return hipGetLastError() == hipSuccess ? NW_OK : NW_EDEVICE;
}

}  // namespace nw
