// Persistent batch engine: many independent pairs (or the all-pairs matrix)
// in one launch, one wave per pair.
//
// Jobs are ordered largest-first (by m*n, bucketed by log2) so the long pairs
// start early and the tail is short.  Each wave owns a private slot of
// workspace (boundary column, direction words, reversed path) and pulls jobs
// from an atomic counter until none are left; every wave reaches the exit.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "nw_internal.h"
#include "nw_strip.h"

namespace nw {

constexpr int kWavesPerBlock = 4;
constexpr int kBlockThreads = kWave * kWavesPerBlock;
constexpr int kBlocksPerCu = 2;
constexpr int kBuckets = 64;

struct KArgs {
    int32_t njobs, nseq;
    const uint8_t* pool;
    const int64_t* a_off;
    const int32_t* a_len;
    const int64_t* b_off;
    const int32_t* b_len;
    int32_t max_len;
    int32_t kdm, kdx, gap;
    int32_t* scores;
    uint8_t* paths;
    const int64_t* path_off;
    int32_t* path_len;
    int64_t* path_len64;
    int32_t* matrix;
    // workspace
    int32_t* queue;
    int32_t* hist;
    int32_t* cursor;
    int32_t* order;
    int32_t* bnd;
    int64_t bnd_stride;
    uint32_t* dirs;
    int64_t dirs_stride;
    uint8_t* rev;
    int64_t rev_stride;
};

struct Pair {
    const uint8_t* a;
    const uint8_t* b;
    int m, n;
    int row, col;  // all-pairs: matrix indices
};

// i <= j enumeration of an nseq x nseq upper triangle, row-major.
__device__ __forceinline__ void unrank_upper(int64_t q, int nseq, int* pi, int* pj) {
    const double N = (double)nseq;
    double disc = (2.0 * N + 1.0) * (2.0 * N + 1.0) - 8.0 * (double)q;
    int i = (int)(((2.0 * N + 1.0) - sqrt(disc > 0 ? disc : 0.0)) * 0.5);
    if (i < 0) i = 0;
    if (i > nseq - 1) i = nseq - 1;
    auto start = [&](int r) { return (int64_t)r * nseq - (int64_t)r * (r - 1) / 2; };
    while (i > 0 && start(i) > q) --i;
    while (i + 1 < nseq && start(i + 1) <= q) ++i;
    *pi = i;
    *pj = i + (int)(q - start(i));
}

template <bool ALLPAIRS>
__device__ __forceinline__ Pair get_pair(const KArgs& A, int job) {
    Pair p;
    if constexpr (ALLPAIRS) {
        int i, j;
        unrank_upper(job, A.nseq, &i, &j);
        p.row = i;
        p.col = j;
        p.a = A.pool + A.a_off[i];
        p.m = A.a_len[i];
        p.b = A.pool + A.a_off[j];
        p.n = A.a_len[j];
    } else {
        p.row = job;
        p.col = 0;
        p.a = A.pool + A.a_off[job];
        p.m = A.a_len[job];
        p.b = A.pool + A.b_off[job];
        p.n = A.b_len[job];
    }
    return p;
}

// ---- planning kernels: zero the counters, bucket jobs by cost, scatter ----

__global__ void k_zero(int32_t* p, int n) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0;
}

__device__ __forceinline__ int cost_bucket(int64_t cost) {
    // 0..63, larger cost -> larger bucket
    return cost <= 0 ? 0 : 63 - __clzll((unsigned long long)cost);
}

template <bool ALLPAIRS>
__global__ void k_hist(KArgs A) {
    int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= A.njobs) return;
    Pair p = get_pair<ALLPAIRS>(A, q);
    atomicAdd(&A.hist[cost_bucket((int64_t)p.m * p.n)], 1);
}

__global__ void k_scan(int32_t* hist, int32_t* cursor) {
    if (threadIdx.x == 0) {
        int32_t run = 0;
        for (int b = kBuckets - 1; b >= 0; --b) {
            cursor[b] = run;
            run += hist[b];
        }
    }
}

template <bool ALLPAIRS>
__global__ void k_scatter(KArgs A) {
    int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= A.njobs) return;
    Pair p = get_pair<ALLPAIRS>(A, q);
    int pos = atomicAdd(&A.cursor[cost_bucket((int64_t)p.m * p.n)], 1);
    A.order[pos] = q;
}

// ---- the persistent engine ----

__device__ __forceinline__ void fence_wave_memory() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

template <int C, bool DIRS, bool ALLPAIRS>
__global__ __launch_bounds__(kBlockThreads) void k_batch(KArgs A) {
    __shared__ uint32_t smem[kWavesPerBlock][StripShape<C>::kLdsWords];
    const int wave = threadIdx.x >> 6;
    const int lane = lane_id();
    uint32_t* lds = smem[wave];
    const int64_t slot = (int64_t)blockIdx.x * kWavesPerBlock + wave;
    int32_t* bnd = A.bnd + slot * A.bnd_stride;
    uint32_t* dirs = DIRS ? A.dirs + slot * A.dirs_stride : nullptr;
    uint8_t* rev = DIRS ? A.rev + slot * A.rev_stride : nullptr;
    const int32_t vinit = DIRS ? 1 : 0;
    constexpr int kCols = kWave * C;

    // The job loop keeps every lane active on every path: the queue ticket
    // comes from an atomic that all lanes execute (lane 0 adds 1, the others
    // 0, so lane 0 reads the ticket), and every lane stores the same outputs.
    // A lane-0-only branch near the back edge lets the compiler split the loop
    // per lane, after which readfirstlane no longer reads lane 0.
    for (;;) {
        const int p = uniform(atomicAdd(A.queue, lane == 0 ? 1 : 0));
        if (p >= A.njobs) break;
        const int job = uniform(A.order[p]);
        const Pair P = get_pair<ALLPAIRS>(A, job);
        const int m = uniform(P.m), n = uniform(P.n);

        int32_t score;
        bool ok = (m <= A.max_len && n <= A.max_len && m >= 0 && n >= 0);
        int64_t plen = 0;
        if (!ok) {
            score = INT32_MIN;
            plen = -1;
        } else if (m == 0 || n == 0) {
            score = A.gap * (m + n);
            if constexpr (DIRS && !ALLPAIRS) {
                uint8_t* out = A.paths + A.path_off[job];
                const uint8_t mv = (m == 0) ? 3 : 2;
                for (int x = lane; x < m + n; x += kWave) out[x] = mv;
                plen = m + n;
            }
        } else {
            const int nstrips = (n + kCols - 1) / kCols;
            const int G = groups_for_rows(m);
            int32_t vlast = 0;
            for (int s = 0; s < nstrips; ++s) {
                const int j0 = s * kCols;
                const int ksel = (n - 1 - j0) % C;
                const PlainIO io{s == 0 ? nullptr : bnd, s == nstrips - 1 ? nullptr : bnd, m, vinit};
                vlast = sweep_strip<C, DIRS>(P.a, m, P.b, n, j0, A.kdm, A.kdx, vinit, io,
                                             DIRS ? dirs + (size_t)s * G * kWave * C : nullptr,
                                             lds, ksel);
                fence_wave_memory();
            }
            const int lastj0 = (nstrips - 1) * kCols;
            const int lsel = (n - 1 - lastj0) / C;
            const int32_t v = __builtin_amdgcn_readlane(vlast, lsel);
            score = (DIRS ? ((v - 1) >> 2) : v) + A.gap * (m + n);
            if constexpr (DIRS && !ALLPAIRS) {
                int64_t len = walk_back<C>(dirs, m, n, G, lds, rev);
                fence_wave_memory();
                if (len < 0) {
                    plen = -2;
                } else {
                    uint8_t* out = A.paths + A.path_off[job];
                    for (int64_t x = lane; x < len; x += kWave) out[x] = rev[len - 1 - x];
                    plen = len;
                }
            }
        }
        if constexpr (ALLPAIRS) {
            A.matrix[(int64_t)P.row * A.nseq + P.col] = score;
            A.matrix[(int64_t)P.col * A.nseq + P.row] = score;
        } else {
            A.scores[job] = score;
            if (A.path_len) A.path_len[job] = (int32_t)plen;
            if (A.path_len64) A.path_len64[job] = plen;
        }
    }
}

// ---- host side ----

static int choose_cols(int32_t max_len) {
    if (max_len > 768) return 8;
    if (max_len > 256) return 4;
    return 2;
}

struct Layout {
    int C;
    int64_t nslots, grid;
    size_t off_order, off_bnd, off_dirs, off_rev, total;
    int64_t bnd_stride, dirs_stride, rev_stride;
};

static Layout layout_for(int32_t njobs, int32_t max_len, bool dirs, const DeviceInfo& di) {
    Layout L{};
    L.C = choose_cols(max_len);
    const int64_t cols = (int64_t)kWave * L.C;
    const int64_t want = ((int64_t)njobs + kWavesPerBlock - 1) / kWavesPerBlock;
    const int64_t cap = (int64_t)di.cus * kBlocksPerCu;
    L.grid = std::max<int64_t>(1, std::min(want, cap));
    L.nslots = L.grid * kWavesPerBlock;
    const int64_t ml = std::max<int32_t>(max_len, 1);
    L.bnd_stride = (int64_t)align_up((size_t)(ml + 2), 64);
    const int64_t groups = groups_for_rows((int)ml);
    const int64_t nstrips = (ml + cols - 1) / cols;
    L.dirs_stride = dirs ? (int64_t)align_up((size_t)(nstrips * groups * kWave * L.C), 64) : 0;
    L.rev_stride = dirs ? (int64_t)align_up((size_t)(2 * ml + 4), 256) : 0;
    size_t off = 1024;  // header: queue, hist[64], cursor[64]
    L.off_order = off;
    off = align_up(off + (size_t)std::max(njobs, 1) * 4, 256);
    L.off_bnd = off;
    off = align_up(off + (size_t)L.nslots * L.bnd_stride * 4, 256);
    L.off_dirs = off;
    off = align_up(off + (size_t)L.nslots * L.dirs_stride * 4, 256);
    L.off_rev = off;
    off = align_up(off + (size_t)L.nslots * L.rev_stride, 256);
    L.total = off;
    return L;
}

size_t batch_workspace_bytes(int32_t njobs, int32_t max_len, bool dirs, const DeviceInfo& di) {
    return layout_for(njobs, max_len, dirs, di).total;
}

template <int C, bool DIRS, bool ALLPAIRS>
static void launch_engine(const KArgs& A, int64_t grid, hipStream_t st) {
    ProfScope ps(ALLPAIRS ? "nw_allpairs" : (DIRS ? "nw_batch" : "nw_batch_score"), st);
    hipLaunchKernelGGL((k_batch<C, DIRS, ALLPAIRS>), dim3((unsigned)grid), dim3(kBlockThreads), 0, st, A);
}

template <bool ALLPAIRS>
static void launch_c(int C, bool dirs, const KArgs& A, int64_t grid, hipStream_t st) {
    if (dirs) {
        if (C == 8) launch_engine<8, true, ALLPAIRS>(A, grid, st);
        else if (C == 4) launch_engine<4, true, ALLPAIRS>(A, grid, st);
        else launch_engine<2, true, ALLPAIRS>(A, grid, st);
    } else {
        if (C == 8) launch_engine<8, false, ALLPAIRS>(A, grid, st);
        else if (C == 4) launch_engine<4, false, ALLPAIRS>(A, grid, st);
        else launch_engine<2, false, ALLPAIRS>(A, grid, st);
    }
}

int launch_batch(const BatchJob& job, void* ws, size_t ws_bytes, hipStream_t st, const DeviceInfo& di) {
    const Layout L = layout_for(job.njobs, job.max_len, job.dirs, di);
    if (ws_bytes < L.total) return NW_ENOSPC;
    if (job.njobs == 0) return NW_OK;
    uint8_t* base = (uint8_t*)ws;
    const Consts K = job.dirs ? dirs_consts(job.sc) : score_consts(job.sc);
    KArgs A{};
    A.njobs = job.njobs;
    A.nseq = job.nseq;
    A.pool = job.pool;
    A.a_off = job.a_off;
    A.a_len = job.a_len;
    A.b_off = job.b_off;
    A.b_len = job.b_len;
    A.max_len = job.max_len;
    A.kdm = K.kdm;
    A.kdx = K.kdx;
    A.gap = job.sc.gap;
    A.scores = job.scores;
    A.paths = job.paths;
    A.path_off = job.path_off;
    A.path_len = job.path_len;
    A.path_len64 = job.path_len64;
    A.matrix = job.matrix;
    A.queue = (int32_t*)base;
    A.hist = (int32_t*)(base + 64 * 4);
    A.cursor = (int32_t*)(base + 128 * 4);
    A.order = (int32_t*)(base + L.off_order);
    A.bnd = (int32_t*)(base + L.off_bnd);
    A.bnd_stride = L.bnd_stride;
    A.dirs = (uint32_t*)(base + L.off_dirs);
    A.dirs_stride = L.dirs_stride;
    A.rev = base + L.off_rev;
    A.rev_stride = L.rev_stride;

    const unsigned pb = (unsigned)((job.njobs + 255) / 256);
    hipLaunchKernelGGL(k_zero, dim3(1), dim3(256), 0, st, (int32_t*)base, 256);
    if (job.allpairs) {
        hipLaunchKernelGGL(k_hist<true>, dim3(pb), dim3(256), 0, st, A);
        hipLaunchKernelGGL(k_scan, dim3(1), dim3(64), 0, st, A.hist, A.cursor);
        hipLaunchKernelGGL(k_scatter<true>, dim3(pb), dim3(256), 0, st, A);
        launch_c<true>(L.C, job.dirs, A, L.grid, st);
    } else {
        hipLaunchKernelGGL(k_hist<false>, dim3(pb), dim3(256), 0, st, A);
        hipLaunchKernelGGL(k_scan, dim3(1), dim3(64), 0, st, A.hist, A.cursor);
        hipLaunchKernelGGL(k_scatter<false>, dim3(pb), dim3(256), 0, st, A);
        launch_c<false>(L.C, job.dirs, A, L.grid, st);
    }
    return hipGetLastError() == hipSuccess ? NW_OK : NW_EDEVICE;
}

}  // namespace nw
