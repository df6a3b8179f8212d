// Persistent batch engine: many independent pairs (or the all-pairs matrix)
// in one launch, one wave per pair.
//
// Jobs are ordered largest-first (by m*n, eight buckets per octave) so the
// long pairs start early and the tail is short.  Each wave owns a private
// slot of workspace (boundary column, direction words, reversed path) and
// pulls jobs from an atomic counter until none are left; every wave reaches
// the exit.  A banded call with paths first runs every pair's score-only
// first pass in a launch of its own (k_probe), then orders the pairs again by
// the cost of their remaining passes.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>

#include "nw_internal.h"
#include "nw_strip.h"

namespace nw {

constexpr int kWavesPerBlock = 4;
constexpr int kBlockThreads = kWave * kWavesPerBlock;
// Resident blocks of four waves per CU (= waves per SIMD).  Score-only sweeps
// fit in 128 VGPRs and run 4 per SIMD, which hides their LDS and boundary
// latencies (all-pairs 83 -> 67 ms); sweeps with directions keep 2: more would
// stretch each pair's wave, and the largest pairs already set the makespan.
constexpr int blocks_per_cu(bool dirs) { return dirs ? 2 : 4; }
constexpr int kBuckets = 512;  // cost buckets per alphabet class

struct KArgs {
    int32_t njobs, nseq;
    // certified band (nw_align_batch_banded)
    const int32_t* w_init;  // per pair initial half-width, or null
    int32_t w_default;
    int32_t frac_1024;      // fall back to the full grid once the band is this fraction of m (x1024)
    int32_t prio_jobs;      // the first prio_jobs jobs of the order run at raised wave priority
    int32_t cd;             // max(match, mismatch)
    int32_t band_ok;        // the certificate applies (2 gap < cd)
    int32_t band_doubling;  // widen a failed band by doubling (else to its certified width)
    int32_t* w_used;
    uint8_t* status;
    int64_t* cells;
    int64_t* cells_so;      // of those, the cells of score-only passes
    const uint8_t* pool;
    const int64_t* a_off;
    const int32_t* a_len;
    const int64_t* b_off;
    const int32_t* b_len;
    int32_t max_len;
    int32_t kdm, kdx, gap;
    int32_t kdm_w, kdx_w;   // the W-domain (score-only) terms, for score-only passes of a sweep with directions
    // per-step cost of a sweep with C = 2, 4, 8 columns per lane (relative
    // units); the engine picks, per pair and pass, the width whose strips x
    // (rows + ramp) x step cost is smallest
    int32_t step_cost[3];     // per step of the 2-, 4-, 8-column sweeps (this launch's mode)
    int32_t step_cost_so[3];  // the same without directions (the score-only passes of a banded launch)
    int32_t* scores;
    uint8_t* paths;
    const int64_t* path_off;
    int32_t* path_len;
    int64_t* path_len64;
    int32_t* matrix;
    // workspace
    int32_t* queue;   // next position of the four-symbol part of the order
    int32_t* queue2;  // next position of the wide part
    int32_t* n_narrow;  // positions 0 .. n_narrow-1 hold pairs of at most four distinct bytes
    int32_t* hist;
    int32_t* cursor;
    int32_t* order;
    uint32_t* masks;  // byte-presence masks, eight words per sequence (pairs: a of job k at 2k, b at 2k+1)
    int32_t* bnd;
    int64_t bnd_stride;
    uint32_t* dirs;
    int64_t dirs_stride;
    uint8_t* rev;
    int64_t rev_stride;
    uint32_t* fault;  // host-visible device-fault word (may be null)
    // A banded launch with paths whose score-only first passes ran before it,
    // in their own launch (k_probe, phase 1): per job, that pass's score and
    // cells; phase 2 is the launch that continues from them.
    int32_t* probe_score;
    int64_t* probe_cells;
    int32_t probe_phase;
    int32_t force_wide;  // every pair compares bytes (constants beyond a signed byte)
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

// ---- the certified band's schedule of widths ----

struct BandPlan {
    int w0;       // the first pass's half-width
    int mn;       // min(m, n)
    int64_t dlt;  // |n - m|
};

// The first width: the pair's proposal (or the launch default).  The
// fallback test uses the narrowest sweep's band height: full grid once
// 128 + |D| + 2w >= frac * m.  A first width beyond that is first tried at
// the widest band below it, so only a failed band sends a pair to the full
// grid.
__device__ __forceinline__ BandPlan band_plan(const KArgs& A, int job, int m, int n) {
    BandPlan b;
    b.w0 = max(0, A.w_init ? A.w_init[job] : A.w_default);
    b.mn = min(m, n);
    b.dlt = n > m ? n - m : m - n;
    const int64_t fb_num = (int64_t)A.frac_1024 * m - 1024 * (2 * kWave + b.dlt) - 1;
    const int64_t w_fb = fb_num >= 0 ? fb_num / 2048 : -1;
    if (b.w0 < b.mn && w_fb >= 0 && b.w0 > w_fb) b.w0 = (int)w_fb;
    return b;
}

// Whether pass number `passes` (0 = the first) at half-width w takes the
// full grid.  A pass after a failed one is certain to certify (unless
// doubling), so it takes the full grid only once the band covers every row
// of a strip; a first pass, which may fail, already does so at fallback_frac
// of the rows.
__device__ __forceinline__ bool band_full(const KArgs& A, int m, const BandPlan& b, int w, int passes) {
    const int64_t lim = (passes > 0 && !A.band_doubling) ? 1024 : A.frac_1024;
    return !A.band_ok || w >= b.mn || (int64_t)(2 * kWave + b.dlt + 2 * (int64_t)w) * 1024 >= lim * m;
}

// The best score a path that leaves band(w) can reach (U_out).
__device__ __forceinline__ int64_t band_u_out(const KArgs& A, const BandPlan& b, int w) {
    return (int64_t)A.cd * (b.mn - w - 1) + (int64_t)A.gap * (b.dlt + 2 * (int64_t)w + 2);
}

// The width a failed band's score certifies.  The failed score S_R <=
// U_out(w).  U_out falls by cd - 2 gap per unit of w, so the smallest w'
// with S_R > U_out(w') is num / (cd - 2 gap) + 1 > w.  The next region
// contains this one (it is wider, and its sweep width is no narrower, so its
// strips' row ranges cover these), so its score is at least S_R and the next
// pass certifies.
__device__ __forceinline__ int band_widen(const KArgs& A, const BandPlan& b, int w, int32_t score) {
    const int64_t num = (int64_t)A.cd * (b.mn - 1) + (int64_t)A.gap * (b.dlt + 2) - score;
    const int64_t den = (int64_t)A.cd - 2 * (int64_t)A.gap;
    return (int)min((int64_t)b.mn, max((int64_t)w + 1, num / den + 1));
}

// Cost of job q in a banded launch that continues from its probe (phase
// 2): the cells of the passes still to come, those with directions counted
// twice.  A first pass that certified is swept again with directions; one
// that failed widens to the width its score certifies, with directions in
// band(1.5 w0 + 16); a first pass on the full grid stays there.
__device__ __forceinline__ int64_t band_job_cost(const KArgs& A, int q, int m, int n) {
    const int64_t mn64 = (int64_t)m * n;
    if (m <= 0 || n <= 0 || m > A.max_len || n > A.max_len) return mn64;
    const BandPlan bp = band_plan(A, q, m, n);
    if (band_full(A, m, bp, bp.w0, 0)) return 2 * mn64;
    auto area = [&](int w) { return (int64_t)n * min((int64_t)m, (int64_t)kWave * 8 + bp.dlt + 2 * (int64_t)w); };
    const int32_t s = A.probe_score[q];
    if ((int64_t)s > band_u_out(A, bp, bp.w0)) return 2 * area(bp.w0);
    const int w1 = band_widen(A, bp, bp.w0, s);
    if (band_full(A, m, bp, w1, 1)) return 2 * mn64;
    return area(w1) + area(min(w1, bp.w0 + bp.w0 / 2 + 16));
}

// ---- planning kernels: zero the counters, bucket jobs by cost, scatter ----

// Byte-presence mask of every sequence (seq_mask), one wave per sequence.
// Sequence q is a pair's a (q even) or b (q odd), or, for all-pairs, the q-th
// sequence.
template <bool ALLPAIRS>
__global__ __launch_bounds__(256) void k_alpha(KArgs A, int32_t nseq) {
    __shared__ uint32_t bits[4][8];
    const int wave = threadIdx.x >> 6;
    const int q = blockIdx.x * 4 + wave;
    if (q >= nseq) return;
    const int64_t off = ALLPAIRS ? A.a_off[q] : ((q & 1) ? A.b_off[q >> 1] : A.a_off[q >> 1]);
    const int32_t len = ALLPAIRS ? A.a_len[q] : ((q & 1) ? A.b_len[q >> 1] : A.a_len[q >> 1]);
    seq_mask(A.pool + off, max(len, 0), A.masks + (int64_t)q * 8, bits[wave]);
}

__global__ void k_zero(int32_t* p, int n) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0;
}

// 0..511, larger cost -> larger bucket: eight buckets per octave (by the three
// bits below the leading one), so the queue runs within 1/8 octave of
// largest-first
__device__ __forceinline__ int cost_bucket(int64_t cost) {
    if (cost < 8) return cost <= 0 ? 0 : (int)cost;
    const int e = 63 - __clzll((unsigned long long)cost);
    return 8 * e + (int)((cost >> (e - 3)) & 7);
}

// Mask indices of job q's two sequences.
template <bool ALLPAIRS>
__device__ __forceinline__ void mask_index(const Pair& p, int q, int64_t* qa, int64_t* qb) {
    *qa = ALLPAIRS ? p.row : 2 * (int64_t)q;
    *qb = ALLPAIRS ? p.col : 2 * (int64_t)q + 1;
}

// Bucket of job q: its cost bucket, plus kBuckets if the pair needs the
// byte-comparing sweep (code_shift < 0).
template <bool ALLPAIRS>
__device__ __forceinline__ int job_bucket(const KArgs& A, int q) {
    Pair p = get_pair<ALLPAIRS>(A, q);
    bool wide = A.force_wide != 0;
    if (!wide && p.m > 0 && p.n > 0) {
        int64_t qa, qb;
        mask_index<ALLPAIRS>(p, q, &qa, &qb);
        wide = code_shift(A.masks + qa * 8, A.masks + qb * 8) < 0;
    }
    int64_t cost = (int64_t)p.m * p.n;
    if constexpr (!ALLPAIRS) {
        if (A.probe_phase == 2) cost = band_job_cost(A, q, p.m, p.n);
    }
    return cost_bucket(cost) + (wide ? kBuckets : 0);
}

// All-pairs jobs fall into few buckets, so their atomics on the global
// counters collide: there each block counts its jobs per bucket in LDS first
// and adds one count per occupied bucket (130,816 jobs: 268 us per kernel
// with one global atomic per job).  Pairs keep one atomic per job: the
// scatter below then leaves them in the order the batch was measured in
// (placing them by block ran the 4096-pair batch's kernel 5% slower).
// Blocks of 256 threads.
constexpr int kBucketsAll = 2 * kBuckets;

template <bool ALLPAIRS>
__global__ __launch_bounds__(256) void k_hist(KArgs A) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if constexpr (!ALLPAIRS) {
        if (q < A.njobs) atomicAdd(&A.hist[job_bucket<false>(A, q)], 1);
    } else {
        __shared__ int32_t cnt[kBucketsAll];
        for (int i = threadIdx.x; i < kBucketsAll; i += blockDim.x) cnt[i] = 0;
        __syncthreads();
        if (q < A.njobs) atomicAdd(&cnt[job_bucket<true>(A, q)], 1);
        __syncthreads();
        for (int i = threadIdx.x; i < kBucketsAll; i += blockDim.x)
            if (cnt[i] != 0) atomicAdd(&A.hist[i], cnt[i]);
    }
}

// Start of every bucket in the order: the four-symbol pairs first, largest
// cost first, then the wide pairs, largest first; n_narrow is where the wide
// part begins.  One wave: lane l takes ranks 16l .. 16l+15 (rank r < 512 is
// four-symbol bucket 511 - r, rank r >= 512 wide bucket 1535 - r).
__global__ __launch_bounds__(64) void k_scan(int32_t* hist, int32_t* cursor, int32_t* n_narrow) {
    constexpr int kPer = 2 * kBuckets / kWave;
    const int lane = lane_id();
    auto bucket = [](int r) { return r < kBuckets ? kBuckets - 1 - r : 3 * kBuckets - 1 - r; };
    int32_t h[kPer];
    int32_t sum = 0;
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
        h[k] = hist[bucket(kPer * lane + k)];
        sum += h[k];
    }
    int32_t incl = sum;
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        const int32_t y = __shfl_up(incl, d);
        if (lane >= d) incl += y;
    }
    int32_t run = incl - sum;
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
        cursor[bucket(kPer * lane + k)] = run;
        run += h[k];
    }
    // the four-symbol part ends after lane 31 (rank 511)
    const int32_t narrow = __shfl(incl, kWave / 2 - 1);
    if (lane == 0) *n_narrow = narrow;
}

// All-pairs: each block takes one range of positions per occupied bucket
// from the global cursor, then places its jobs in it by their rank within the
// block (the order inside a bucket is arbitrary either way).
template <bool ALLPAIRS>
__global__ __launch_bounds__(256) void k_scatter(KArgs A) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if constexpr (!ALLPAIRS) {
        if (q < A.njobs) A.order[atomicAdd(&A.cursor[job_bucket<false>(A, q)], 1)] = q;
    } else {
        __shared__ int32_t cnt[kBucketsAll];
        __shared__ int32_t base[kBucketsAll];
        for (int i = threadIdx.x; i < kBucketsAll; i += blockDim.x) cnt[i] = 0;
        __syncthreads();
        const int bkt = (q < A.njobs) ? job_bucket<true>(A, q) : 0;
        const int rank = (q < A.njobs) ? atomicAdd(&cnt[bkt], 1) : 0;
        __syncthreads();
        for (int i = threadIdx.x; i < kBucketsAll; i += blockDim.x)
            if (cnt[i] != 0) base[i] = atomicAdd(&A.cursor[i], cnt[i]);
        __syncthreads();
        if (q < A.njobs) A.order[base[bkt] + rank] = q;
    }
}

// ---- the persistent engine ----

__device__ __forceinline__ void fence_wave_memory() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

constexpr int32_t kNegV = -(1 << 30) + 1;  // -infinity in the V domain (ends in tag 1)
constexpr int32_t kNegW = -(1 << 29);      // -infinity in the W domain

// Fill one pair over the region {rows r0(s)+1 .. re(s)} of every strip s:
// the whole grid when `full`, else the staircase of strips that covers
// band(w) = { min(0,D) - w <= j - i <= max(0,D) + w }, D = n - m.  Cells
// outside the region are -infinity; the first row and column keep their
// values.  Returns V (or W) at (m, n); *G_out gets the direction groups per
// strip and *cells the number of cells swept.
template <int C, bool DIRS, bool WIDE>
__device__ __forceinline__ int32_t fill_pair(const KArgs& A, const uint8_t* pa, const uint8_t* pb,
                                             int m, int n, uint32_t shift, bool full, int w, int32_t* bnd,
                                             int32_t* spare, uint32_t* dirs, uint32_t* lds, int* G_out,
                                             int64_t* cells) {
    constexpr int kCols = kWave * C;
    const int32_t vinit = DIRS ? 1 : 0;
    const int32_t vneg = DIRS ? kNegV : kNegW;
    const int lo_d = min(0, n - m), hi_d = max(0, n - m);
    const int nstrips = (n + kCols - 1) / kCols;
    const int height = full ? m : min(m, kCols + hi_d - lo_d + 2 * w);
    const int G = groups_for_rows(height);
    *G_out = G;
    int32_t vlast = 0;
    int prev_lo = 1, prev_hi = m;  // previous strip's rows
    int64_t swept = 0;
    for (int s = 0; s < nstrips; ++s) {
        const int j0 = s * kCols;
        const int rs = full ? 1 : max(1, j0 + 1 - hi_d - w);
        const int re = full ? m : min(m, j0 + kCols - lo_d + w);
        const int r0 = rs - 1, rows = re - rs + 1;
        const int ksel = (n - 1 - j0) % C;
        PlainIO io{s == 0 ? nullptr : bnd, s == nstrips - 1 ? nullptr : bnd, spare, rows, vinit};
        io.r0 = r0;
        io.in_hi = (s == 0) ? m : prev_hi;
        io.beyond = full ? 0 : vneg;
        const int32_t vtop = (r0 == 0) ? vinit : vneg;
        int32_t dg0 = vinit;
        if (s > 0 && r0 > 0) dg0 = (r0 >= prev_lo && r0 <= prev_hi) ? bnd[r0] : vneg;
        vlast = sweep_strip<C, DIRS, WIDE>(pa + r0, rows, pb, n, j0, DIRS ? A.kdm : A.kdm_w, DIRS ? A.kdx : A.kdx_w,
                                           shift, vtop, dg0, io,
                                     DIRS ? dirs + (size_t)s * G * kWave * C : nullptr, lds, ksel);
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
        prev_lo = rs;
        prev_hi = re;
        swept += (int64_t)rows * min(kCols, n - j0);
    }
    *cells += swept;
    const int lsel = (n - 1 - (nstrips - 1) * kCols) / C;
    return __builtin_amdgcn_readlane(vlast, lsel);
}

// Boundary IO of a strip swept in row ranges of both domains (fill_mixed):
// the boundary column stays in the W domain; a range swept with directions
// converts what it reads (V = 4W + 1, -infinity kept at kNegV without
// overflow) and what it writes (W = V >> 2).
struct MixIO : PlainIO {
    bool vdom = false;
    __device__ __forceinline__ int32_t value(Slot x, int r) const {
        if (r > m) return beyond;
        if (!bin) return vinit;
        if (r0 + r > in_hi) return beyond;
        return vdom ? max(4 * max(x, kNegW) + 1, kNegV) : x;
    }
    __device__ __forceinline__ void store(int r, int32_t v, bool want) const {
        int32_t* dst = (want && bout != nullptr) ? bout + r0 + r : spare;
        *dst = vdom ? (v >> 2) : v;
    }
};

// One pass over band(w) (or the full grid) that records directions only in
// the rows band(w2) covers in each strip, w2 <= w.  Each strip is swept in up
// to three row ranges -- score-only above band(w2)'s rows, with directions
// inside them, score-only below -- and the lanes carry their values from one
// range to the next (converted between the W and V domains).  The scores are
// those of band(w); the directions are band(w)'s at the cells of band(w2)'s
// staircase, stored with band(w2)'s layout (*G_out groups per strip), so a
// walk that stays in those rows follows band(w)'s traceback.  Returns W at
// (m, n); *cells_so gets the cells swept without directions.
template <int C, bool WIDE>
__device__ __forceinline__ int32_t fill_pair_mixed(const KArgs& A, const uint8_t* pa, const uint8_t* pb, int m,
                                                   int n, uint32_t shift, bool full, int w, int w2, int32_t* bnd,
                                                   int32_t* spare, uint32_t* dirs, uint32_t* lds, int* G_out,
                                                   int64_t* cells, int64_t* cells_so) {
    constexpr int kCols = kWave * C;
    const int lo_d = min(0, n - m), hi_d = max(0, n - m);
    const int nstrips = (n + kCols - 1) / kCols;
    const int G2 = groups_for_rows(min(m, kCols + hi_d - lo_d + 2 * w2));
    *G_out = G2;
    int32_t last = 0;
    bool last_v = false;
    int prev_lo = 1, prev_hi = m;
    int64_t swept = 0, swept_so = 0;
    for (int s = 0; s < nstrips; ++s) {
        const int j0 = s * kCols;
        const int cols = min(kCols, n - j0);
        const int rs = full ? 1 : max(1, j0 + 1 - hi_d - w);
        const int re = full ? m : min(m, j0 + kCols - lo_d + w);
        const int rd0 = max(rs, j0 + 1 - hi_d - w2);   // rows with directions: rd0 .. rd1
        const int rd1 = min(re, j0 + kCols - lo_d + w2);
        const int ksel = (n - 1 - j0) % C;
        // ranges: [rs, rd0-1] score-only, [rd0, rd1] with directions, [rd1+1, re] score-only
        const int ra[3] = {rs, rd0, rd1 + 1};
        const int rb[3] = {rd0 - 1, rd1, re};
        // the previous strip's last column one row above each range (W), read
        // before the ranges of this strip overwrite the boundary
        int32_t dgw[3];
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            const int r0 = ra[q] - 1;
            dgw[q] = 0;
            if (s > 0 && r0 > 0) dgw[q] = (r0 >= prev_lo && r0 <= prev_hi) ? bnd[r0] : kNegW;
        }
        // lanes start from the row above the strip's region: the grid's first
        // row, or -infinity
        int32_t st[C];
#pragma unroll
        for (int k = 0; k < C; ++k) st[k] = (rs == 1) ? 0 : kNegW;
        bool st_v = false;  // domain of st
        // the three ranges, each with its own sweep
        auto range = [&](const int q) {
            const int rows = rb[q] - ra[q] + 1;
            if (rows <= 0) return;
            const bool vd = (q == 1);
            if (vd != st_v) {
#pragma unroll
                for (int k = 0; k < C; ++k) st[k] = vd ? max(4 * max(st[k], kNegW) + 1, kNegV) : (st[k] >> 2);
                st_v = vd;
            }
            const int r0 = ra[q] - 1;
            MixIO io;
            io.bin = s == 0 ? nullptr : bnd;
            io.bout = s == nstrips - 1 ? nullptr : bnd;
            io.spare = spare;
            io.m = rows;
            io.vinit = vd ? 1 : 0;
            io.r0 = r0;
            io.in_hi = (s == 0) ? m : prev_hi;
            io.beyond = full ? 0 : (vd ? kNegV : kNegW);
            io.vdom = vd;
            const int32_t dg0 = vd ? max(4 * max(dgw[q], kNegW) + 1, kNegV) : dgw[q];
            if (vd) {
                last = sweep_strip<C, true, WIDE, MixIO, true>(pa + r0, rows, pb, n, j0, A.kdm, A.kdx, shift, 0, dg0,
                                                               io, dirs + (size_t)s * G2 * kWave * C, lds, ksel, st);
            } else {
                last = sweep_strip<C, false, WIDE, MixIO, true>(pa + r0, rows, pb, n, j0, A.kdm_w, A.kdx_w, shift, 0,
                                                                dg0, io, nullptr, lds, ksel, st);
                swept_so += (int64_t)rows * cols;
            }
            last_v = vd;
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
        };
        range(0);
        range(1);
        range(2);
        prev_lo = rs;
        prev_hi = re;
        swept += (int64_t)(re - rs + 1) * cols;
    }
    *cells += swept;
    *cells_so += swept_so;
    const int lsel = (n - 1 - (nstrips - 1) * kCols) / C;
    const int32_t v = __builtin_amdgcn_readlane(last, lsel);
    return last_v ? (v >> 2) : v;
}

template <bool WIDE>
__device__ __forceinline__ int32_t fill_mixed(int C, const KArgs& A, const uint8_t* pa, const uint8_t* pb, int m,
                                              int n, uint32_t shift, bool full, int w, int w2, int32_t* bnd,
                                              int32_t* spare, uint32_t* dirs, uint32_t* lds, int* G, int64_t* cells,
                                              int64_t* cells_so) {
    if (C == 8)
        return fill_pair_mixed<8, WIDE>(A, pa, pb, m, n, shift, full, w, w2, bnd, spare, dirs, lds, G, cells, cells_so);
    if (C == 4)
        return fill_pair_mixed<4, WIDE>(A, pa, pb, m, n, shift, full, w, w2, bnd, spare, dirs, lds, G, cells, cells_so);
    return fill_pair_mixed<2, WIDE>(A, pa, pb, m, n, shift, full, w, w2, bnd, spare, dirs, lds, G, cells, cells_so);
}

// Band height (rows per strip) of band(w) for a C-column sweep.
__device__ __forceinline__ int band_height(int C, int m, int n, int w) {
    const int dlt = n > m ? n - m : m - n;
    return (int)min((int64_t)m, (int64_t)kWave * C + dlt + 2 * (int64_t)w);
}

// Sweep width for one pass (the full grid, or band(w)): the C in {2, 4, 8},
// at least c_min, with the least modelled time, strips x (rows per strip +
// ramp) x step cost.  w_dirs: -2 a pass in the launch's own mode, -1 a
// score-only pass, >= 0 a pass with directions only in band(w_dirs)'s rows
// (three row ranges per strip, so two more ramps).
__device__ __forceinline__ int pick_cols(const KArgs& A, int m, int n, bool full, int w, int c_min = 2,
                                         int w_dirs = -2) {
    int best = 8;
    int64_t best_cost = INT64_MAX;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const int C = 2 << c;
        if (C < c_min) continue;
        const int64_t strips = (n + kWave * C - 1) / (kWave * C);
        const int height = full ? m : band_height(C, m, n, w);
        int64_t per_strip;
        if (w_dirs >= 0) {
            const int hd = min(height, band_height(C, m, n, w_dirs));
            per_strip = (int64_t)(hd + kWave) * A.step_cost[c] + (int64_t)(height - hd + 2 * kWave) * A.step_cost_so[c];
        } else {
            per_strip = (int64_t)(height + kWave) * (w_dirs == -1 ? A.step_cost_so[c] : A.step_cost[c]);
        }
        const int64_t cost = strips * per_strip;
        if (cost < best_cost) {
            best_cost = cost;
            best = C;
        }
    }
    return best;
}

// One pass with sweep width C; WIDE: the byte-comparing sweep (pairs with
// more than four distinct bytes).
template <bool DIRS, bool WIDE>
__device__ __forceinline__ int32_t fill_any(int C, const KArgs& A, const uint8_t* pa, const uint8_t* pb, int m,
                                            int n, uint32_t shift, bool full, int w, int32_t* bnd, int32_t* spare,
                                            uint32_t* dirs, uint32_t* lds, int* G, int64_t* cells) {
    if (C == 8) return fill_pair<8, DIRS, WIDE>(A, pa, pb, m, n, shift, full, w, bnd, spare, dirs, lds, G, cells);
    if (C == 4) return fill_pair<4, DIRS, WIDE>(A, pa, pb, m, n, shift, full, w, bnd, spare, dirs, lds, G, cells);
    return fill_pair<2, DIRS, WIDE>(A, pa, pb, m, n, shift, full, w, bnd, spare, dirs, lds, G, cells);
}

__device__ __forceinline__ int64_t walk_checked(int C, const uint32_t* dirs, int m, int n, int G, uint8_t* rev,
                                                int band_hi, int span_lo) {
    if (C == 8) return walk_back<8, true>(dirs, m, n, G, nullptr, rev, band_hi, span_lo);
    if (C == 4) return walk_back<4, true>(dirs, m, n, G, nullptr, rev, band_hi, span_lo);
    return walk_back<2, true>(dirs, m, n, G, nullptr, rev, band_hi, span_lo);
}

__device__ __forceinline__ int64_t walk_any(int C, const uint32_t* dirs, int m, int n, int G, uint32_t* lds,
                                            uint8_t* rev, int band_hi) {
    if (C == 8) return walk_back<8>(dirs, m, n, G, lds, rev, band_hi);
    if (C == 4) return walk_back<4>(dirs, m, n, G, lds, rev, band_hi);
    return walk_back<2>(dirs, m, n, G, lds, rev, band_hi);
}

// WIDE: this launch serves the wide part of the order (pairs with more than
// four distinct bytes) with the byte-comparing sweep; otherwise the
// four-symbol part with the one-hot lookup.
template <bool DIRS, bool ALLPAIRS, bool BANDED, bool WIDE>
__global__ __launch_bounds__(kBlockThreads, blocks_per_cu(DIRS)) void k_batch(KArgs A) {
    __shared__ uint32_t smem[kWavesPerBlock][StripShape<8>::kLdsWords];
    const int wave = threadIdx.x >> 6;
    const int lane = lane_id();
    uint32_t* lds = smem[wave];
    const int64_t slot = (int64_t)blockIdx.x * kWavesPerBlock + wave;
    int32_t* bnd = A.bnd + slot * A.bnd_stride;
    int32_t* spare = bnd + A.bnd_stride - 1;  // past every grid row (stride >= max_len + 2)
    uint32_t* dirs = DIRS ? A.dirs + slot * A.dirs_stride : nullptr;
    uint8_t* rev = DIRS ? A.rev + slot * A.rev_stride : nullptr;

    // The job loop keeps every lane active on every path: the queue ticket
    // comes from an atomic that all lanes execute (lane 0 adds 1, the others
    // 0, so lane 0 reads the ticket), and every lane stores the same outputs.
    // A lane-0-only branch near the back edge lets the compiler split the loop
    // per lane, after which readfirstlane no longer reads lane 0.
    const int part_lo = WIDE ? uniform(*A.n_narrow) : 0;
    const int part_hi = WIDE ? A.njobs : uniform(*A.n_narrow);
    // an empty part (usually the wide one) exits before touching the queue:
    // every wave's atomic on the one counter cost 19 us on the 4096-pair batch
    if (part_lo >= part_hi) return;
    for (;;) {
        const int p = part_lo + uniform(atomicAdd(WIDE ? A.queue2 : A.queue, lane == 0 ? 1 : 0));
        if (p >= part_hi) break;
        // the largest jobs (the front of the order) set the makespan: their
        // waves win the issue arbitration against the SIMD's other waves
        if ((p - part_lo) < A.prio_jobs) __builtin_amdgcn_s_setprio(2);
        else __builtin_amdgcn_s_setprio(0);
        const int job = uniform(A.order[p]);
        const Pair P = get_pair<ALLPAIRS>(A, job);
        const int m = uniform(P.m), n = uniform(P.n);

        int32_t score;
        bool ok = (m <= A.max_len && n <= A.max_len && m >= 0 && n >= 0);
        // the pair's code field (the wide part of the order compares bytes)
        uint32_t shift = 0;
        if (!WIDE && ok && m > 0 && n > 0) {
            int64_t qa, qb;
            mask_index<ALLPAIRS>(P, job, &qa, &qb);
            shift = (uint32_t)max(0, uniform(code_shift(A.masks + qa * 8, A.masks + qb * 8)));
        }
        int64_t plen = 0;
        // banded outputs for pairs that never reach the band loop: no band,
        // no cells (an empty pair counts as solved on the full grid)
        int32_t w_out = -1;
        uint32_t st_out = ok ? (0x40u | (A.band_ok ? 0u : 0x80u)) : 0u;
        int64_t cells_out = 0, cells_so_out = 0;
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
            int G = 0;
            int64_t cells = 0;
            bool full = true;
            int w = 0;
            int C = 8;
            int w_dirs = -1;  // >= 0: the last pass recorded directions only in band(w_dirs)
            int passes = 0;
            if constexpr (BANDED) {
                // certified band: sweep band(w); if the region's score does not
                // beat the best score any path leaving band(w) can reach, widen the
                // band to the width that this score itself certifies, or take the
                // full grid once the band is so wide that it is cheaper
                const BandPlan bp = band_plan(A, job, m, n);
                w = bp.w0;
                int c_min = 2;
                // With widening, a first pass that does not certify serves only to
                // find the region's score, so it runs score-only (no direction
                // words); one that does certify is swept again, same band, with
                // directions.  Doubled passes all record directions.
                bool probe = DIRS && !A.band_doubling;
                bool certified_first = false;
                int mixed_next = -1;  // after a failed first pass: record directions only in its band
                for (;;) {
                    full = band_full(A, m, bp, w, passes);
                    const bool score_only = probe && !full;
                    // the path most likely lies near the failed first pass's
                    // band: directions in band(1.5 w0 + 16), scores elsewhere
                    const int wd_next = (DIRS && mixed_next >= 0) ? min(w, mixed_next + mixed_next / 2 + 16) : -2;
                    C = uniform(pick_cols(A, m, n, full, w, c_min, score_only ? -1 : wd_next));
                    int32_t v;
                    w_dirs = -1;
                    if (DIRS && mixed_next >= 0) {
                        w_dirs = wd_next;
                        mixed_next = -1;
                        v = fill_mixed<WIDE>(C, A, P.a, P.b, m, n, shift, full, w, w_dirs, bnd, spare, dirs, lds, &G,
                                             &cells, &cells_so_out);
                        score = v + A.gap * (m + n);
                    } else if (score_only && A.probe_phase == 2) {
                        // this pass ran in the probe launch (k_probe)
                        score = A.probe_score[job];
                        cells += A.probe_cells[job];
                        cells_so_out += A.probe_cells[job];
                    } else if (score_only) {
                        const int64_t before = cells;
                        v = fill_any<false, WIDE>(C, A, P.a, P.b, m, n, shift, false, w, bnd, spare, nullptr, lds, &G,
                                                  &cells);
                        cells_so_out += cells - before;
                        score = v + A.gap * (m + n);
                    } else {
                        v = fill_any<DIRS, WIDE>(C, A, P.a, P.b, m, n, shift, full, w, bnd, spare, dirs, lds, &G,
                                                 &cells);
                        score = (DIRS ? ((v - 1) >> 2) : v) + A.gap * (m + n);
                    }
                    ++passes;
                    probe = false;
                    if (full) break;
                    if ((int64_t)score > band_u_out(A, bp, w)) {
                        if (passes == 1) certified_first = true;
                        if (!score_only) break;
                        c_min = C;  // the same band again, with directions
                        continue;
                    }
                    if (A.band_doubling) {
                        w = max(1, 2 * w);
                        continue;
                    }
                    if (score_only) mixed_next = w;
                    w_dirs = -1;
                    w = band_widen(A, bp, w, score);
                    c_min = C;
                }
                w_out = full ? -1 : w;
                const int extra = min(passes - 1, 31);
                st_out = (uint32_t)((certified_first ? 1 : 0) | (extra << 1) | (full ? 0x40 : 0) |
                                    (A.band_ok ? 0 : 0x80));
                cells_out = cells;
            } else {
                C = uniform(pick_cols(A, m, n, true, 0));
                const int32_t v =
                    fill_any<DIRS, WIDE>(C, A, P.a, P.b, m, n, shift, true, 0, bnd, spare, dirs, lds, &G, &cells);
                score = (DIRS ? ((v - 1) >> 2) : v) + A.gap * (m + n);
            }
            if constexpr (DIRS && !ALLPAIRS) {
                const int band_hi = full ? (1 << 30) : max(0, n - m) + w;
                int64_t len;
                if (BANDED && w_dirs >= 0) {
                    // directions exist only in band(w_dirs)'s rows: a walk that
                    // would leave them stops, and band(w) is swept again with
                    // directions everywhere
                    len = walk_checked(C, dirs, m, n, G, rev, max(0, n - m) + w_dirs, w_dirs - min(0, n - m));
                    while (len == -3) {
                        // the walk left them: the same pass again with directions in
                        // a band four times as wide, or everywhere once that covers
                        // band(w)
                        fence_wave_memory();
                        ++passes;
                        st_out = (st_out & ~0x3Eu) | ((uint32_t)min(passes - 1, 31) << 1);
                        w_dirs = 4 * w_dirs + 64;
                        if (w_dirs >= w) {
                            fill_any<DIRS, WIDE>(C, A, P.a, P.b, m, n, shift, full, w, bnd, spare, dirs, lds, &G,
                                                 &cells);
                            cells_out = cells;
                            len = walk_any(C, dirs, m, n, G, lds, rev, band_hi);
                            break;
                        }
                        fill_mixed<WIDE>(C, A, P.a, P.b, m, n, shift, full, w, w_dirs, bnd, spare, dirs, lds, &G,
                                         &cells, &cells_so_out);
                        cells_out = cells;
                        len = walk_checked(C, dirs, m, n, G, rev, max(0, n - m) + w_dirs, w_dirs - min(0, n - m));
                    }
                } else {
                    len = walk_any(C, dirs, m, n, G, lds, rev, band_hi);
                }
                fence_wave_memory();
                if (len < 0) {
                    plen = -2;  // a corrupt direction tag: only a device fault can cause it
                    if (lane == 0) report_fault(A.fault);
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
            if constexpr (BANDED) {
                if (A.w_used) A.w_used[job] = w_out;
                if (A.status) A.status[job] = (uint8_t)st_out;
                if (A.cells) A.cells[job] = cells_out;
                if (A.cells_so) A.cells_so[job] = cells_so_out;
            }
        }
    }
}

// The score-only first passes of a banded launch with paths, on their own:
// each pair whose first pass is score-only (widening, not the full grid)
// sweeps band(w0) without directions and leaves the region's score and the
// cells swept in probe_score / probe_cells, which the launch with paths
// (phase 2) takes in place of that pass.  Same order, sweep width and result
// as that pass in k_batch; run at the score-only occupancy, 4 waves per SIMD
// instead of 2.  Each wave's boundary slot lies in the direction-word area,
// which this launch does not otherwise use (the host checks it fits).
template <bool WIDE>
__global__ __launch_bounds__(kBlockThreads, blocks_per_cu(false)) void k_probe(KArgs A) {
    __shared__ uint32_t smem[kWavesPerBlock][StripShape<8>::kLdsWords];
    const int wave = threadIdx.x >> 6;
    const int lane = lane_id();
    uint32_t* lds = smem[wave];
    const int64_t slot = (int64_t)blockIdx.x * kWavesPerBlock + wave;
    int32_t* bnd = A.bnd + slot * A.bnd_stride;
    int32_t* spare = bnd + A.bnd_stride - 1;
    // every lane runs every path of the job loop (as in k_batch)
    const int part_lo = WIDE ? uniform(*A.n_narrow) : 0;
    const int part_hi = WIDE ? A.njobs : uniform(*A.n_narrow);
    if (part_lo >= part_hi) return;
    for (;;) {
        const int p = part_lo + uniform(atomicAdd(WIDE ? A.queue2 : A.queue, lane == 0 ? 1 : 0));
        if (p >= part_hi) break;
        if ((p - part_lo) < A.prio_jobs) __builtin_amdgcn_s_setprio(2);
        else __builtin_amdgcn_s_setprio(0);
        const int job = uniform(A.order[p]);
        const Pair P = get_pair<false>(A, job);
        const int m = uniform(P.m), n = uniform(P.n);
        if (m > A.max_len || n > A.max_len || m <= 0 || n <= 0) continue;
        const BandPlan bp = band_plan(A, job, m, n);
        if (band_full(A, m, bp, bp.w0, 0)) continue;
        uint32_t shift = 0;
        if (!WIDE) {
            int64_t qa, qb;
            mask_index<false>(P, job, &qa, &qb);
            shift = (uint32_t)max(0, uniform(code_shift(A.masks + qa * 8, A.masks + qb * 8)));
        }
        const int C = uniform(pick_cols(A, m, n, false, bp.w0, 2, -1));
        int G = 0;
        int64_t cells = 0;
        const int32_t v =
            fill_any<false, WIDE>(C, A, P.a, P.b, m, n, shift, false, bp.w0, bnd, spare, nullptr, lds, &G, &cells);
        A.probe_score[job] = v + A.gap * (m + n);
        A.probe_cells[job] = cells;
    }
}

// ---- host side ----

// Relative per-step cost of the 2-, 4- and 8-column sweeps.  Defaults:
// instructions per step of the compiled loops (16-step groups, stores and
// refills included).  nw_autotune replaces them, per device, with measured
// times (tuning_table).
constexpr int32_t kStepCostDirs[3] = {16, 27, 48};
constexpr int32_t kStepCostScore[3] = {12, 18, 31};
constexpr int kMaxDevices = 64;

namespace {
struct Tuning {
    std::mutex mu;
    bool tuned[kMaxDevices] = {};
    int32_t cost[kMaxDevices][2][3] = {};  // [device][dirs][width]
};
Tuning& tuning() {
    static Tuning t;
    return t;
}
}  // namespace

bool tuned_costs(int device) {
    Tuning& T = tuning();
    std::lock_guard<std::mutex> lock(T.mu);
    return device >= 0 && device < kMaxDevices && T.tuned[device];
}

void step_costs(int device, bool dirs, int32_t out[3]) {
    Tuning& T = tuning();
    std::lock_guard<std::mutex> lock(T.mu);
    const bool have = device >= 0 && device < kMaxDevices && T.tuned[device];
    for (int c = 0; c < 3; ++c)
        out[c] = have ? T.cost[device][dirs][c] : (dirs ? kStepCostDirs[c] : kStepCostScore[c]);
}

void set_step_costs(int device, const int32_t dirs[3], const int32_t score[3]) {
    if (device < 0 || device >= kMaxDevices) return;
    Tuning& T = tuning();
    std::lock_guard<std::mutex> lock(T.mu);
    for (int c = 0; c < 3; ++c) {
        T.cost[device][1][c] = dirs[c];
        T.cost[device][0][c] = score[c];
    }
    T.tuned[device] = true;
}

void reset_step_costs() {
    Tuning& T = tuning();
    std::lock_guard<std::mutex> lock(T.mu);
    for (bool& t : T.tuned) t = false;
}

// Cost weight that keeps a width from ever being picked (products stay far
// below 2^63 for every admissible length).
constexpr int32_t kExcluded = 1 << 20;
constexpr int kMaxCols = 8;  // slots are sized for the widest sweep, which bounds the others

struct Layout {
    int64_t nslots, grid;
    size_t off_order, off_masks, off_probe_score, off_probe_cells, off_bnd, off_dirs, off_rev, total;
    int64_t bnd_stride, dirs_stride, rev_stride;
};

// A persistent wave needs a private slot that holds the directions of the
// largest pair's full grid (0.25 B per cell).  The workspace-size query asks
// for one slot per resident wave, up to kSlotBudget of the device's HBM;
// a launch uses as many slots as the workspace it is given holds (at least
// one block's worth), so a smaller workspace only costs parallelism.  The
// budget is sized for a 288 GB part: pairs of 20,000 bases need 100 MB per
// slot, and all 2048 resident waves of the sweeps with directions then take
// 205 GB (measured on the 8192-pair learned-band workload: 1328 waves within
// 128 GiB, 208 -> 188 ms full DP and 64 -> 56.5 ms learned band with 2048).
constexpr size_t kSlotBudget = size_t(240) << 30;
// queue (0), queue2 (4), n_narrow (8), hist[1024] (1024), cursor[1024] (5120)
constexpr size_t kHeaderBytes = 9216;

static Layout layout_for(int32_t njobs, int32_t max_len, bool dirs, const DeviceInfo& di,
                         size_t ws_limit = SIZE_MAX) {
    Layout L{};
    const int64_t cols = (int64_t)kWave * kMaxCols;
    const int64_t ml = std::max<int32_t>(max_len, 1);
    L.bnd_stride = (int64_t)align_up((size_t)(ml + 2), 64);
    const int64_t groups = groups_for_rows((int)ml);
    const int64_t nstrips = (ml + cols - 1) / cols;
    L.dirs_stride = dirs ? (int64_t)align_up((size_t)(nstrips * groups * cols), 64) : 0;
    L.rev_stride = dirs ? (int64_t)align_up((size_t)(2 * ml + 4), 256) : 0;
    // bytes per block of slots (the three per-slot arrays are padded per array)
    const size_t per_block = (size_t)kWavesPerBlock * ((size_t)L.bnd_stride * 4 + (size_t)L.dirs_stride * 4 +
                                                       (size_t)L.rev_stride);
    // masks: eight words for each of the 2 njobs sequences (pairs), which also
    // covers the nseq <= njobs sequences of all-pairs
    const size_t mask_bytes = align_up((size_t)std::max(njobs, 1) * 2 * 32, 256);
    // the probe launch's records: a score (4 B) and a cell count (8 B) per job
    const size_t probe_bytes =
        align_up((size_t)std::max(njobs, 1) * 4, 256) + align_up((size_t)std::max(njobs, 1) * 8, 256);
    const size_t fixed =
        align_up(kHeaderBytes + (size_t)std::max(njobs, 1) * 4, 256) + mask_bytes + probe_bytes + 3 * 256;
    const int64_t want = ((int64_t)njobs + kWavesPerBlock - 1) / kWavesPerBlock;
    int64_t grid = std::min<int64_t>(std::max<int64_t>(want, 1), (int64_t)di.cus * blocks_per_cu(dirs));
    const size_t budget = std::min(ws_limit, fixed + std::max(kSlotBudget, per_block));
    if (budget < fixed + per_block) {
        L.total = fixed + per_block;  // too small: the caller gets NW_ENOSPC
        L.grid = 0;
        return L;
    }
    grid = std::max<int64_t>(1, std::min<int64_t>(grid, (int64_t)((budget - fixed) / per_block)));
    L.grid = grid;
    L.nslots = L.grid * kWavesPerBlock;
    size_t off = kHeaderBytes;
    L.off_order = off;
    off = align_up(off + (size_t)std::max(njobs, 1) * 4, 256);
    L.off_masks = off;
    off += mask_bytes;
    L.off_probe_score = off;
    off += align_up((size_t)std::max(njobs, 1) * 4, 256);
    L.off_probe_cells = off;
    off += align_up((size_t)std::max(njobs, 1) * 8, 256);
    L.off_bnd = off;
    off = align_up(off + (size_t)L.nslots * L.bnd_stride * 4, 256);
    L.off_dirs = off;
    off = align_up(off + (size_t)L.nslots * L.dirs_stride * 4, 256);
    L.off_rev = off;
    off = align_up(off + (size_t)L.nslots * L.rev_stride, 256);
    // report the size the slot count was derived from, so that a workspace of
    // exactly this size yields the same grid again
    L.total = std::max(off, fixed + (size_t)L.grid * per_block);
    return L;
}

size_t batch_workspace_bytes(int32_t njobs, int32_t max_len, bool dirs, const DeviceInfo& di) {
    return layout_for(njobs, max_len, dirs, di).total;
}

// The four-symbol part, then the wide part (a launch that finds the wide
// part empty exits at once).
template <bool DIRS, bool ALLPAIRS, bool BANDED>
static void launch_engine(const KArgs& A, int64_t grid, hipStream_t st) {
    {
        ProfScope ps(BANDED ? (DIRS ? "nw_batch_banded" : "nw_batch_banded_score")
                            : (ALLPAIRS ? "nw_allpairs" : (DIRS ? "nw_batch" : "nw_batch_score")),
                     st);
        hipLaunchKernelGGL((k_batch<DIRS, ALLPAIRS, BANDED, false>), dim3((unsigned)grid), dim3(kBlockThreads), 0,
                           st, A);
    }
    ProfScope ps("nw_batch_wide", st);
    hipLaunchKernelGGL((k_batch<DIRS, ALLPAIRS, BANDED, true>), dim3((unsigned)grid), dim3(kBlockThreads), 0, st,
                       A);
}

// The score-only first passes of a banded launch with paths (k_probe), then
// the order again for the launch with paths, which continues from the
// records (*A becomes phase 2).  The probe waves' boundary slots go in the
// direction-word area, as many as fit.
static void launch_probe(KArgs& A, const Layout& L, const DeviceInfo& di, int32_t njobs, hipStream_t st) {
    const size_t per_block = (size_t)kWavesPerBlock * (size_t)L.bnd_stride * 4;
    const int64_t want = ((int64_t)njobs + kWavesPerBlock - 1) / kWavesPerBlock;
    const int64_t room = (int64_t)((L.off_rev - L.off_dirs) / per_block);
    const int64_t grid = std::min<int64_t>(std::min<int64_t>(want, (int64_t)di.cus * blocks_per_cu(false)), room);
    if (grid < 1) return;  // no room: k_batch sweeps the first passes itself
    A.probe_phase = 2;
    KArgs P = A;
    P.probe_phase = 1;
    P.bnd = (int32_t*)A.dirs;
    P.prio_jobs = (int32_t)std::min<int64_t>(njobs, grid * kWavesPerBlock);
    {
        ProfScope ps("nw_batch_banded_probe", st);
        hipLaunchKernelGGL(k_probe<false>, dim3((unsigned)grid), dim3(kBlockThreads), 0, st, P);
    }
    {
        ProfScope ps("nw_batch_wide", st);
        hipLaunchKernelGGL(k_probe<true>, dim3((unsigned)grid), dim3(kBlockThreads), 0, st, P);
    }
    // a new largest-first order by the cost of what is left of each job
    constexpr int kHeaderInts = (int)(kHeaderBytes / 4);
    const unsigned pb = (unsigned)((njobs + 255) / 256);
    hipLaunchKernelGGL(k_zero, dim3((kHeaderInts + 255) / 256), dim3(256), 0, st, A.queue, kHeaderInts);
    hipLaunchKernelGGL(k_hist<false>, dim3(pb), dim3(256), 0, st, A);
    hipLaunchKernelGGL(k_scan, dim3(1), dim3(64), 0, st, A.hist, A.cursor, A.n_narrow);
    hipLaunchKernelGGL(k_scatter<false>, dim3(pb), dim3(256), 0, st, A);
}

int launch_batch(const BatchJob& job, void* ws, size_t ws_bytes, hipStream_t st, const DeviceInfo& di) {
    const Layout L = layout_for(job.njobs, job.max_len, job.dirs, di, ws_bytes);
    if (L.grid == 0 || ws_bytes < L.total) return NW_ENOSPC;
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
    const Consts KW = score_consts(job.sc);
    A.kdm_w = KW.kdm;
    A.kdx_w = KW.kdx;
    A.gap = job.sc.gap;
    step_costs(di.device, job.dirs, A.step_cost);
    step_costs(di.device, false, A.step_cost_so);
    if (job.force_cols) {
        for (int c = 0; c < 3; ++c) {
            A.step_cost[c] = ((2 << c) == job.force_cols) ? 1 : kExcluded;
            A.step_cost_so[c] = A.step_cost[c];
        }
    }
    A.scores = job.scores;
    A.paths = job.paths;
    A.path_off = job.path_off;
    A.path_len = job.path_len;
    A.path_len64 = job.path_len64;
    A.matrix = job.matrix;
    A.w_init = job.w_init;
    A.w_default = job.w_default;
    A.frac_1024 = job.frac_1024;
    // the first round of jobs (one per wave) runs at raised priority: once a
    // wave moves on to a later, smaller job, the SIMD's arbitration favours
    // the wave still on its large first job, which shortens the tail
    // (measured: 4096-pair batch 1.70 -> 1.56 ms, full DP of the 8192-pair
    // workload 190 -> 174 ms, a quarter or half of the waves less)
    A.prio_jobs = (int32_t)std::min<int64_t>(job.njobs, L.grid * kWavesPerBlock);
    A.cd = std::max(job.sc.match, job.sc.mismatch);
    A.band_ok = 2 * job.sc.gap < A.cd ? 1 : 0;
    A.band_doubling = job.band_doubling ? 1 : 0;
    A.w_used = job.w_used;
    A.status = job.status;
    A.cells = job.cells;
    A.cells_so = job.cells_so;
    A.force_wide = needs_wide(K) ? 1 : 0;
    A.probe_phase = 0;
    A.probe_score = (int32_t*)(base + L.off_probe_score);
    A.probe_cells = (int64_t*)(base + L.off_probe_cells);
    A.queue = (int32_t*)base;
    A.queue2 = (int32_t*)(base + 4);
    A.n_narrow = (int32_t*)(base + 8);
    A.hist = (int32_t*)(base + 1024);
    A.cursor = (int32_t*)(base + 5120);
    A.order = (int32_t*)(base + L.off_order);
    A.masks = (uint32_t*)(base + L.off_masks);
    A.bnd = (int32_t*)(base + L.off_bnd);
    A.bnd_stride = L.bnd_stride;
    A.dirs = (uint32_t*)(base + L.off_dirs);
    A.dirs_stride = L.dirs_stride;
    A.rev = base + L.off_rev;
    A.rev_stride = L.rev_stride;
    A.fault = di.fault;

    const unsigned pb = (unsigned)((job.njobs + 255) / 256);
    constexpr int kHeaderInts = (int)(kHeaderBytes / 4);
    hipLaunchKernelGGL(k_zero, dim3((kHeaderInts + 255) / 256), dim3(256), 0, st, (int32_t*)base, kHeaderInts);
    const int32_t nseq = job.allpairs ? job.nseq : 2 * job.njobs;
    if (job.allpairs) hipLaunchKernelGGL(k_alpha<true>, dim3((nseq + 3) / 4), dim3(256), 0, st, A, nseq);
    else hipLaunchKernelGGL(k_alpha<false>, dim3((nseq + 3) / 4), dim3(256), 0, st, A, nseq);
    if (job.allpairs) {
        hipLaunchKernelGGL(k_hist<true>, dim3(pb), dim3(256), 0, st, A);
        hipLaunchKernelGGL(k_scan, dim3(1), dim3(64), 0, st, A.hist, A.cursor, A.n_narrow);
        hipLaunchKernelGGL(k_scatter<true>, dim3(pb), dim3(256), 0, st, A);
        launch_engine<false, true, false>(A, L.grid, st);
    } else {
        hipLaunchKernelGGL(k_hist<false>, dim3(pb), dim3(256), 0, st, A);
        hipLaunchKernelGGL(k_scan, dim3(1), dim3(64), 0, st, A.hist, A.cursor, A.n_narrow);
        hipLaunchKernelGGL(k_scatter<false>, dim3(pb), dim3(256), 0, st, A);
        if (job.banded) {
            if (job.dirs && !job.band_doubling && !job.band_one_launch) launch_probe(A, L, di, job.njobs, st);
            if (job.dirs) launch_engine<true, false, true>(A, L.grid, st);
            else launch_engine<false, false, true>(A, L.grid, st);
        } else {
            if (job.dirs) launch_engine<true, false, false>(A, L.grid, st);
            else launch_engine<false, false, false>(A, L.grid, st);
        }
    }
    return hipGetLastError() == hipSuccess ? NW_OK : NW_EDEVICE;
}

}  // namespace nw
