// Co-optimal alignments (Sec. 2.4 keeps every path that reaches the optimal
// score): per pair, the number N of optimal paths, kept modulo 2^64 with a
// flag for N >= 2^64, and optionally the first k of those paths in the order
// a depth-first search from (m,n) meets them when it tries the diagonal, then
// the vertical, then the horizontal move at every cell (the first one is the
// single tie-broken path of nw_align_batch).
//
// Fill.  One wave per pair from a persistent largest-first queue.  Lane l
// holds columns j0+2l+1 and j0+2l+2 of a 128-column strip and sweeps the rows
// on a skewed front (lane l is at row t+1-l at step t).  Per cell it keeps
//     W = H - gap*(i+j)   (Eq. 1 becomes W = max(Wd + s - 2gap, Wu, Wl)),
// and the count as three 32-bit words: the number of optimal paths modulo
// 2^64 and a flag word, 1 once the number reaches 2^64.  A cell's count is
// the sum of the counts of the neighbours whose candidate equals the maximum,
// added with carries chained into the flag word, which is then clamped to 1
// (so the low words stay exact modulo 2^64).  The left neighbour's values
// come by DPP from lane l-1; lane 0 takes the previous strip's last column,
// which lane 63 wrote to a per-wave buffer one row per step.  Every 64 steps
// the wave stages in LDS the next 64 rows of that column and the row words
// (substitution bytes) of the 128 rows around its front, and each step reads
// them one step ahead.  With k > 0 the three tie bits of every cell are
// packed 8 per step into a 32-bit word per lane every 4 steps.
//
// Enumeration.  The same wave then walks: path 0 takes the first optimal move
// at every cell from (m,n); each later path goes back to the deepest cell of
// the previous one that still has an untried optimal move, takes the next
// one, and again the first moves from there.  Every cell reached this way
// has an optimal move (or is the origin), so no walk dead-ends.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <type_traits>

#include "nw_common.h"
#include "nw_internal.h"

namespace nw {

namespace {

constexpr int kCoCols = 2;                       // columns per lane
constexpr int kCoStrip = kWave * kCoCols;        // columns per strip
constexpr int kCoWaves = 4;                      // waves per block
#ifndef NW_COOPT_BLOCKS_PER_CU
#define NW_COOPT_BLOCKS_PER_CU 4
#endif
constexpr int kCoBlocksPerCu = NW_COOPT_BLOCKS_PER_CU;
// Listing paths keeps one wave per pair (no teams), so its largest pairs set
// the time and fewer waves per SIMD serve them better; its slots (tie bits
// for a whole pair) are also large.
constexpr int kCoPathBlocksPerCu = 2;
constexpr int co_blocks_per_cu(bool paths) { return paths ? kCoPathBlocksPerCu : kCoBlocksPerCu; }
#ifndef NW_COOPT_TEAM_BUCKET
#define NW_COOPT_TEAM_BUCKET (8 * 16)  // cost bucket of 2^16 cells
#endif
constexpr int kCoBuckets = 512;                  // 8 cost buckets per octave
constexpr size_t kCoHeader = 8192;               // hist[512], cursor[512], next_job, next_team, n_team (ints)
constexpr int kCoHeaderInts = 2 * kCoBuckets + 3;
constexpr int kTeamRing = 8;                     // boundary columns in flight per team
constexpr int kMoveD = 1, kMoveU = 2, kMoveL = 3;

struct CoArgs {
    int32_t npairs;
    const uint8_t* pool;
    const int64_t* a_off;
    const int32_t* a_len;
    const int64_t* b_off;
    const int32_t* b_len;
    int32_t max_len;
    int32_t kdm, kdx;  // s - 2*gap for a match and a mismatch
    int32_t gap;
    int32_t* scores;
    uint64_t* counts;
    uint8_t* saturated;
    int32_t k;
    uint8_t* paths;
    const int64_t* path_off;
    int32_t* path_len;
    int32_t* n_paths;
    int32_t* hist;
    int32_t* cursor;
    int32_t* next_job;   // solo queue: positions n_team .. npairs-1 of order
    int32_t* next_team;  // team queue: positions 0 .. n_team-1
    int32_t* n_team;
    int32_t team_bucket;  // pairs in this cost bucket or above go to teams
    int32_t* order;
    uint8_t* slots;
    int64_t slot_bytes;
    int64_t off_tie;   // within a slot
    int64_t off_walk;  // within a slot
    int32_t spin;      // polls before a team wait gives up
    int32_t prio_jobs; // the first prio_jobs single-wave jobs run at raised wave priority
    uint32_t* fault;   // host-visible device-fault word (may be null)
    uint32_t* masks;   // byte-presence masks: a of pair p at 16p, b at 16p+8
    int32_t force_wide;  // every pair compares bytes (constants beyond a signed byte)
};

__device__ __forceinline__ int cost_bucket(int64_t cost) {
    if (cost < 8) return (int)max<int64_t>(cost, 0);
    const int e = 63 - __builtin_clzll((unsigned long long)cost);
    return 8 * e + (int)((cost >> (e - 3)) & 7);
}

// Byte-presence masks of every pair's two sequences (seq_mask), one wave each.
__global__ __launch_bounds__(256) void k_co_alpha(CoArgs A) {
    __shared__ uint32_t bits[4][8];
    const int wave = threadIdx.x >> 6;
    const int q = blockIdx.x * 4 + wave;
    if (q >= 2 * A.npairs) return;
    const int p = q >> 1;
    const int64_t off = (q & 1) ? A.b_off[p] : A.a_off[p];
    const int32_t len = (q & 1) ? A.b_len[p] : A.a_len[p];
    seq_mask(A.pool + off, max(len, 0), A.masks + (int64_t)q * 8, bits[wave]);
}

// The pair's code field (code_shift), or -1 to compare bytes.
__device__ __forceinline__ int pair_shift(const CoArgs& A, int p) {
    if (A.force_wide) return -1;
    return uniform(code_shift(A.masks + (int64_t)p * 16, A.masks + (int64_t)p * 16 + 8));
}

__device__ __forceinline__ bool pair_ok(const CoArgs& A, int p) {
    const int32_t m = A.a_len[p], n = A.b_len[p];
    return m >= 0 && n >= 0 && m <= A.max_len && n <= A.max_len;
}

__global__ void k_co_zero(int32_t* p, int32_t n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0;
}

__global__ void k_co_hist(CoArgs A) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= A.npairs) return;
    const int b = pair_ok(A, p) ? cost_bucket((int64_t)A.a_len[p] * A.b_len[p]) : 0;
    atomicAdd(&A.hist[b], 1);
}

// One block of kCoBuckets threads: cursor[b] = number of pairs in buckets
// above b (largest first).
__global__ __launch_bounds__(kCoBuckets) void k_co_scan(CoArgs A) {
    __shared__ int32_t s[kCoBuckets];
    const int t = threadIdx.x;
    s[t] = A.hist[kCoBuckets - 1 - t];  // reversed: bucket 511 first
    __syncthreads();
    for (int d = 1; d < kCoBuckets; d <<= 1) {
        const int32_t y = t >= d ? s[t - d] : 0;
        __syncthreads();
        s[t] += y;
        __syncthreads();
    }
    const int b = kCoBuckets - 1 - t;
    A.cursor[b] = s[t] - A.hist[b];
    // the team queue: every pair in a bucket at or above team_bucket, which
    // the largest-first order puts first
    if (b == A.team_bucket - 1) *A.n_team = s[t] - A.hist[b];
}

__global__ void k_co_scatter(CoArgs A) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= A.npairs) return;
    const int b = pair_ok(A, p) ? cost_bucket((int64_t)A.a_len[p] * A.b_len[p]) : 0;
    A.order[atomicAdd(&A.cursor[b], 1)] = p;
}

// A count: the number of optimal paths modulo 2^64 (lo, hi) and a third
// word that is 1 once the number reaches 2^64 and 0 before (the flag).
struct Count {
    uint32_t lo, hi, ex;
};

__device__ __forceinline__ Count pick(bool e, const Count& c) {
    return Count{e ? c.lo : 0u, e ? c.hi : 0u, e ? c.ex : 0u};
}

// a + b on three words with the carries chained (v_add_co / v_addc_co)
__device__ __forceinline__ Count add3w(const Count& a, const Count& b) {
    unsigned c1, c2, c3;
    Count r;
    r.lo = __builtin_addc(a.lo, b.lo, 0u, &c1);
    r.hi = __builtin_addc(a.hi, b.hi, c1, &c2);
    r.ex = __builtin_addc(a.ex, b.ex, c2, &c3);
    return r;
}

// One cell: the maximum of the three candidates, and the sum of the counts
// of those equal to it (the flag word clamped to 1, so the low words stay
// the count modulo 2^64).  Returns the tie bits (1 diagonal, 2 vertical,
// 4 horizontal).
__device__ __forceinline__ uint32_t cell(int32_t cd, int32_t wu, int32_t wl, const Count& nd, const Count& nu,
                                         const Count& nl, int32_t& w, Count& n) {
    const int32_t h = imax3(cd, wu, wl);
    const bool eD = cd == h, eU = wu == h, eL = wl == h;
    n = add3w(add3w(pick(eD, nd), pick(eU, nu)), pick(eL, nl));
    asm("v_min_u32 %0, %1, 1" : "=v"(n.ex) : "v"(n.ex));
    w = h;
    return (eD ? 1u : 0u) | (eU ? 2u : 0u) | (eL ? 4u : 0u);
}

// A boundary cell handed from one strip to the next: W, N (low, high), F.
struct BCell {
    int32_t w;
    uint32_t nl, nh, f;
};

// Per-wave LDS: the row words of the 128 rows around the front (rows T-63 ..
// T+64 for the block of 64 steps starting at T) and the previous strip's
// column for rows T+1 .. T+64.
struct WaveLds {
    uint32_t rw[2 * kWave];
    BCell col[kWave];
};

// Everything a wave hands to itself through global memory (the strip
// boundary, the tie words, the walk's state) is read back by the same wave,
// on the same CU: a workgroup-scope fence (its stores complete) and loads
// that bypass L1 suffice; no L2 writeback is needed.
__device__ __forceinline__ void fence_wave_mem() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

__device__ __forceinline__ BCell load_bcell(const BCell* p) {
    const int32_t* q = (const int32_t*)p;
    return BCell{load_coherent(q), (uint32_t)load_coherent(q + 1), (uint32_t)load_coherent(q + 2),
                 (uint32_t)load_coherent(q + 3)};
}

// Tie bits of cell (i,j), 1 <= i <= m, 1 <= j <= n, from the packed words of
// the fill (strip s, group g of 4 steps, lane l).
__device__ __forceinline__ uint32_t tie_bits(const uint32_t* tie, int64_t groups, int32_t i, int32_t j) {
    const int32_t c = j - 1;
    const int32_t s = c / kCoStrip, w = c % kCoStrip, l = w >> 1, kk = w & 1;
    const int32_t t = i - 1 + l;
    const uint32_t word = load_coherent_u32(tie + ((int64_t)s * groups + (t >> 2)) * kWave + l);
    return (word >> (8 * (t & 3) + 4 * kk)) & 7u;
}

// Team hand-off between the waves of a block: a strip publishes, in LDS, how
// many rows of its last column it has written to global memory, tagged with
// the strip (tag = (strip+1) << 32 | rows).
struct Hand {
    int64_t* prog_in;   // the previous strip's counter (nullptr: solo wave)
    int64_t* prog_out;  // this strip's counter (nullptr: nobody reads it)
    int32_t* err;       // set when a wait gives up (LDS, shared by the team)
    int32_t spin;       // polls before a wait gives up
};

// Wait until the counter reaches `need` (every wait ends: producers never
// wait on their consumers; the limit only guards against a fault).  Once any
// wait of the team has given up (err set), every wait returns at once, so a
// failed pair drains in a few polls per strip block instead of a full limit
// each.
__device__ __forceinline__ void wait_rows(const int64_t* prog, int64_t need, int32_t* err, int32_t spin) {
    for (int32_t it = 0;; ++it) {
        const int64_t v = __hip_atomic_load(prog, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        const int64_t vu = ((int64_t)uniform((int32_t)(v >> 32)) << 32) | (uint32_t)uniform((int32_t)v);
        if (vu >= need) break;
        if (uniform(__hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP)) != 0) break;
        if (it >= spin) {
            __hip_atomic_store(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            break;
        }
        __builtin_amdgcn_s_sleep(2);
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

__device__ __forceinline__ void publish_rows(int64_t* prog, int s, int32_t rows) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");  // the column's stores are done
    __hip_atomic_store(prog, ((int64_t)(s + 1) << 32) | (uint32_t)rows, __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_WORKGROUP);
}

// One strip s of a pair (m, n >= 1): reads the previous strip's column from
// `bin` (s > 0) and writes its own last column to `bout` (if not the last
// strip).  The lane that holds column n leaves its row-m values in w_end and
// n_end (last strip only).
// WIDE compares bytes (wide_word row words); otherwise bytes are codes
// (x >> shift) & 3 looked up through the one-hot dot product.
template <bool ENUM, bool WIDE>
__device__ void fill_strip(const CoArgs& A, WaveLds& S, const uint8_t* a, const uint8_t* b, int32_t m, int32_t n,
                           uint32_t shift, int s, int nstrips, const BCell* bin, BCell* bout, const Hand& H,
                           uint32_t* tie, int32_t& w_end, Count& n_end) {
    const int lane = lane_id();
    const int32_t steps = m + kWave - 1;
    const int64_t groups = ((int64_t)steps + 3) / 4;
    const int j0 = s * kCoStrip;
    const int32_t c0 = j0 + 2 * lane + 1, c1 = c0 + 1;
    const uint32_t x0 = c0 <= n ? (uint32_t)b[c0 - 1] : 0u, x1 = c1 <= n ? (uint32_t)b[c1 - 1] : 0u;
    const uint32_t oh0 = WIDE ? x0 : 1u << (8 * sym_code(x0, shift));
    const uint32_t oh1 = WIDE ? x1 : 1u << (8 * sym_code(x1, shift));
    // lanes past column n stay at row 0; rows run 1..m for the others
    const uint32_t rows = c0 <= n ? (uint32_t)m : 0u;
    const bool hand = lane == kWave - 1 && s + 1 < nstrips;
    // row 0: W = 0 and one path everywhere
    int32_t w0 = 0, w1 = 0;
    Count n0{1u, 0u, 0u}, n1{1u, 0u, 0u};
    int32_t dw = 0;  // diagonal input of column 0: the last step's left input
    Count dn{1u, 0u, 0u};
    uint32_t tw = 0;
    fence_wave_mem();
    for (int32_t T = 0; T < steps; T += kWave) {
        {
            const int32_t r = T + 1 + lane;
            if (s > 0 && H.prog_in) wait_rows(H.prog_in, ((int64_t)s << 32) | (uint32_t)min(T + kWave, m), H.err, H.spin);
            const uint32_t older = T == 0 ? 0u : S.rw[kWave + lane];
            const uint32_t word = r > m ? 0u : WIDE ? wide_word(true, a[r - 1], A.kdx)
                                                    : row_word(sym_code(a[r - 1], shift), A.kdm, A.kdx);
            BCell c{0, 1u, 0u, 0u};
            if (s > 0 && r <= m) c = load_bcell(bin + r);
            __builtin_amdgcn_wave_barrier();
            S.rw[lane] = older;
            S.rw[kWave + lane] = word;
            S.col[lane] = c;
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        }
        const int32_t cnt = min(kWave, steps - T);
        // this step's row word and boundary cell, read one step ahead
        int32_t rw_next = (int32_t)S.rw[kWave - lane];
        BCell in_next = S.col[0];
        // one step: lane l at row T+u+1-l.  CHECK keeps lanes outside
        // rows 1..m (and past column n) where they are; the blocks whose
        // steps all lie in 63..m-1 have every lane inside and skip it.
        auto step = [&](auto check, int32_t u) {
            constexpr bool CHECK = decltype(check)::value;
            const int32_t t = T + u;
            const uint32_t rm1 = (uint32_t)(t - lane);  // row - 1
            const int32_t rw = rw_next;
            const BCell in = in_next;
            const int32_t un = min(u + 1, kWave - 1);
            rw_next = (int32_t)S.rw[kWave + un - lane];
            in_next = S.col[un];
            const int32_t lw = dpp_from_left(in.w, w1);
            const Count ln{(uint32_t)dpp_from_left((int32_t)in.nl, (int32_t)n1.lo),
                           (uint32_t)dpp_from_left((int32_t)in.nh, (int32_t)n1.hi),
                           (uint32_t)dpp_from_left((int32_t)in.f, (int32_t)n1.ex)};
            uint32_t bits = 0;
            if (!CHECK || rm1 < rows) {
                int32_t nw0, nw1;
                Count nn0, nn1;
                // bytes compared: the row's byte against the column's (oh0/oh1)
                const uint32_t rbyte = (uint32_t)rw & 0x1FFu;
                const int32_t rmis = rw >> 9;
                const int32_t cd0 = WIDE ? dw + (rbyte == oh0 ? A.kdm : rmis)
                                         : __builtin_amdgcn_sdot4(rw, (int32_t)oh0, dw, false);
                const uint32_t b0 = cell(cd0, w0, lw, dn, n0, ln, nw0, nn0);
                const int32_t cd1 = WIDE ? w0 + (rbyte == oh1 ? A.kdm : rmis)
                                         : __builtin_amdgcn_sdot4(rw, (int32_t)oh1, w0, false);
                const uint32_t b1 = cell(cd1, w1, nw0, n0, n1, nn0, nw1, nn1);
                w0 = nw0;
                n0 = nn0;
                w1 = nw1;
                n1 = nn1;
                bits = b0 | (b1 << 4);
                // lane 63 hands its second column to the next strip
                if (hand) bout[rm1 + 1] = BCell{w1, n1.lo, n1.hi, n1.ex};
            }
            dw = lw;
            dn = ln;
            if (ENUM) {
                tw = (tw >> 8) | (bits << 24);
                if ((t & 3) == 3 || t == steps - 1) {
                    const uint32_t sh = (uint32_t)(8 * (3 - (t & 3)));
                    tie[((int64_t)s * groups + (t >> 2)) * kWave + lane] = tw >> sh;
                }
            }
        };
        int32_t u = 0;
        if (T >= kWave - 1 && T + cnt <= m && j0 + kCoStrip <= n) {
            const std::false_type all_in{};
            for (; u + 1 < cnt; u += 2) {
                step(all_in, u);
                step(all_in, u + 1);
            }
            if (u < cnt) step(all_in, u);
        } else {
            const std::true_type edge{};
            for (; u + 1 < cnt; u += 2) {
                step(edge, u);
                step(edge, u + 1);
            }
            if (u < cnt) step(edge, u);
        }
        // lane 63 wrote row r at step r + 62
        if (H.prog_out) publish_rows(H.prog_out, s, min(m, max(0, T + cnt - 1 - (kWave - 2))));
    }
    if (s + 1 == nstrips) {
        // lanes stop at row m, so the lane holding column n has H(m,n)
        if (c0 == n) {
            w_end = w0;
            n_end = n0;
        } else if (c1 == n) {
            w_end = w1;
            n_end = n1;
        }
    }
    fence_wave_mem();
}

// The fill of one pair (m, n >= 1) by one wave: strips in order, the
// boundary column alternating between the two buffers of the wave's slot.
template <bool ENUM, bool WIDE>
__device__ void fill_pair(const CoArgs& A, uint8_t* slot, WaveLds& S, int p, int32_t m, int32_t n, uint32_t shift,
                          int32_t& w_end, Count& n_end) {
    const uint8_t* a = A.pool + A.a_off[p];
    const uint8_t* b = A.pool + A.b_off[p];
    BCell* bnd = (BCell*)slot;  // two buffers of max_len+1 rows
    const int64_t bstride = (int64_t)A.max_len + 1;
    uint32_t* tie = (uint32_t*)(slot + A.off_tie);
    const int nstrips = (n + kCoStrip - 1) / kCoStrip;
    const Hand solo{nullptr, nullptr, nullptr, 0};
    for (int s = 0; s < nstrips; ++s)
        fill_strip<ENUM, WIDE>(A, S, a, b, m, n, shift, s, nstrips, bnd + (s & 1) * bstride,
                               bnd + ((s & 1) ^ 1) * bstride, solo, tie, w_end, n_end);
}

// Scalar walk state: moves, remaining options and the cell before each move.
struct Walk {
    uint8_t* mv;
    uint8_t* alt;
    int32_t* ci;
    int32_t* cj;
};

__device__ __forceinline__ uint32_t options(const uint32_t* tie, int64_t groups, int32_t i, int32_t j) {
    if (i == 0) return 4u;
    if (j == 0) return 2u;
    return tie_bits(tie, groups, i, j);
}

// From cell (i,j) at depth d, always the first optimal move, to the origin.
// All lanes run it with the same values and store the same bytes (no
// lane-only branch inside the loop).  Returns the depth.
__device__ int32_t descend(const uint32_t* tie, int64_t groups, const Walk& W, int32_t i, int32_t j, int32_t d) {
    while (i > 0 || j > 0) {
        const uint32_t o = uniform((int32_t)options(tie, groups, i, j));
        const uint32_t bit = o & (0u - o);  // lowest set bit: D, then U, then L
        const int mv = bit == 1u ? kMoveD : (bit == 2u ? kMoveU : kMoveL);
        W.mv[d] = (uint8_t)mv;
        W.alt[d] = (uint8_t)(o & ~bit);
        W.ci[d] = i;
        W.cj[d] = j;
        if (mv != kMoveL) --i;
        if (mv != kMoveU) --j;
        ++d;
    }
    return d;
}

__device__ void emit_path(const CoArgs& A, const Walk& W, int p, int r, int32_t m, int32_t n, int32_t len) {
    fence_wave_mem();
    uint8_t* out = A.paths + A.path_off[p] + (int64_t)r * (m + n);
    for (int32_t x = lane_id(); x < len; x += kWave)
        out[x] = (uint8_t)__hip_atomic_load(W.mv + (len - 1 - x), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    A.path_len[(int64_t)p * A.k + r] = len;  // every lane, same value
}

// The job loop keeps every lane active on every path: the queue ticket comes
// from an atomic that all lanes execute (lane 0 adds 1, the others 0), and
// every lane stores the same outputs.  A lane-only branch near a back edge
// would let the compiler split the loop per lane, and readfirstlane would
// then stop reading lane 0.
template <bool ENUM>
__global__ __launch_bounds__(kWave * kCoWaves, co_blocks_per_cu(ENUM)) void k_count(CoArgs A) {
    __shared__ WaveLds lds[kCoWaves];
    const int lane = lane_id();
    const int wv = threadIdx.x / kWave;
    const int64_t wave = (int64_t)blockIdx.x * kCoWaves + wv;
    uint8_t* slot = A.slots + wave * A.slot_bytes;
    if (!ENUM) {
        // Teams: the four waves of the block share the largest pairs, wave w
        // taking strips w, w+4, ...  Strip s writes its last column to ring
        // buffer s % 8 (the two buffers of each of the block's four slots) and
        // publishes its progress in prog[s % 8]; strip s+8 reuses the buffer
        // only after strip s+4 has finished, which needs strip s+1 finished.
        __shared__ int64_t prog[kTeamRing];
        __shared__ int32_t team_job, team_err;
        const int64_t bstride = (int64_t)A.max_len + 1;
        uint8_t* block_slots = A.slots + (int64_t)blockIdx.x * kCoWaves * A.slot_bytes;
        auto ring = [&](int c) { return (BCell*)(block_slots + (int64_t)(c >> 1) * A.slot_bytes) + (c & 1) * bstride; };
        const int n_team = uniform(__hip_atomic_load(A.n_team, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
        for (;;) {
            __syncthreads();
            if (wv == 0) {
                const int j = uniform(atomicAdd(A.next_team, lane == 0 ? 1 : 0));
                team_job = j;
                prog[lane & (kTeamRing - 1)] = 0;
                team_err = 0;
            }
            __syncthreads();
            const int job = uniform(team_job);
            if (job >= n_team) break;
            const int p = uniform(A.order[job]);
            const int32_t m = uniform(A.a_len[p]), n = uniform(A.b_len[p]);
            const int nstrips = (n + kCoStrip - 1) / kCoStrip;
            const uint8_t* a = A.pool + A.a_off[p];
            const uint8_t* b = A.pool + A.b_off[p];
            const int sh = (m > 0 && n > 0) ? pair_shift(A, p) : 0;
            int32_t w_end = 0;
            Count n_end{1u, 0u, 0u};
            for (int s = wv; s < nstrips; s += kCoWaves) {
                const Hand H{s > 0 ? &prog[(s - 1) % kTeamRing] : nullptr,
                             s + 1 < nstrips ? &prog[s % kTeamRing] : nullptr, &team_err, A.spin};
                if (sh < 0)
                    fill_strip<false, true>(A, lds[wv], a, b, m, n, 0u, s, nstrips,
                                            s > 0 ? ring((s - 1) % kTeamRing) : nullptr, ring(s % kTeamRing), H,
                                            nullptr, w_end, n_end);
                else
                    fill_strip<false, false>(A, lds[wv], a, b, m, n, (uint32_t)sh, s, nstrips,
                                             s > 0 ? ring((s - 1) % kTeamRing) : nullptr, ring(s % kTeamRing), H,
                                             nullptr, w_end, n_end);
            }
            __syncthreads();
            if (wv == (nstrips - 1) % kCoWaves) {
                const int src = ((n - 1) % kCoStrip) / kCoCols;
                w_end = __shfl(w_end, src);
                n_end = Count{(uint32_t)__shfl((int32_t)n_end.lo, src), (uint32_t)__shfl((int32_t)n_end.hi, src),
                              (uint32_t)__shfl((int32_t)n_end.ex, src)};
                const bool bad = uniform(team_err) != 0;
                if (bad && lane == 0) report_fault(A.fault);
                // every lane of the wave, the same values
                A.scores[p] = bad ? INT32_MIN : w_end + A.gap * (m + n);
                A.counts[p] = bad ? 0 : (((uint64_t)n_end.hi << 32) | n_end.lo);
                A.saturated[p] = bad ? 0 : (uint8_t)n_end.ex;
            }
        }
    }
    const int first = ENUM ? 0 : uniform(__hip_atomic_load(A.n_team, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
    for (;;) {
        const int job = first + uniform(atomicAdd(A.next_job, lane == 0 ? 1 : 0));
        if (job >= A.npairs) break;
        // the first round (the largest single-wave jobs) wins the SIMD's issue
        // arbitration against waves already on later, smaller jobs
        if (job - first < A.prio_jobs) __builtin_amdgcn_s_setprio(2);
        else __builtin_amdgcn_s_setprio(0);
        const int p = uniform(A.order[job]);
        const int32_t m = uniform(A.a_len[p]), n = uniform(A.b_len[p]);
        const bool ok = m >= 0 && n >= 0 && m <= A.max_len && n <= A.max_len;
        int32_t score = INT32_MIN;
        uint64_t count = 0;
        uint32_t flag = 0;
        int32_t got = 0;
        if (ok) {
            int32_t w_end = 0;
            Count n_end{1u, 0u, 0u};
            if (m > 0 && n > 0) {
                const int sh = pair_shift(A, p);
                if (sh < 0) fill_pair<ENUM, true>(A, slot, lds[wv], p, m, n, 0u, w_end, n_end);
                else fill_pair<ENUM, false>(A, slot, lds[wv], p, m, n, (uint32_t)sh, w_end, n_end);
                // the lane that holds column n at row m has the result
                const int src = ((n - 1) % kCoStrip) / kCoCols;
                w_end = __shfl(w_end, src);
                n_end = Count{(uint32_t)__shfl((int32_t)n_end.lo, src), (uint32_t)__shfl((int32_t)n_end.hi, src),
                              (uint32_t)__shfl((int32_t)n_end.ex, src)};
            }
            score = w_end + A.gap * (m + n);
            count = ((uint64_t)n_end.hi << 32) | n_end.lo;
            flag = n_end.ex;
            if (ENUM && A.k > 0) {
                const int64_t groups = ((int64_t)m + kWave - 1 + 3) / 4;
                const uint32_t* tie = (const uint32_t*)(slot + A.off_tie);
                const int32_t L = m + n + 1;
                Walk W{slot + A.off_walk, slot + A.off_walk + L, nullptr, nullptr};
                W.ci = (int32_t*)(slot + A.off_walk + ((2 * (int64_t)L + 15) & ~(int64_t)15));
                W.cj = W.ci + L;
                fence_wave_mem();
                int32_t d = descend(tie, groups, W, m, n, 0);
                emit_path(A, W, p, 0, m, n, d);
                got = 1;
                while (got < A.k) {
                    fence_wave_mem();
                    // deepest position with an untried move, 64 positions at a time
                    int32_t q = -1;
                    for (int32_t hi = d - 1; hi >= 0 && q < 0; hi -= kWave) {
                        const int32_t x = hi - lane;
                        const bool has = x >= 0 && __hip_atomic_load(W.alt + x, __ATOMIC_RELAXED,
                                                                     __HIP_MEMORY_SCOPE_AGENT) != 0;
                        const uint64_t ball = __ballot(has);
                        if (ball) q = hi - (int32_t)__builtin_ctzll(ball);
                    }
                    if (q < 0) break;
                    const int32_t i = uniform(__hip_atomic_load(W.ci + q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
                    const int32_t j = uniform(__hip_atomic_load(W.cj + q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
                    const uint32_t o = (uint32_t)uniform(
                        (int32_t)__hip_atomic_load(W.alt + q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
                    const uint32_t bit = o & (0u - o);
                    const int mv = bit == 1u ? kMoveD : (bit == 2u ? kMoveU : kMoveL);
                    fence_wave_mem();  // every lane has read alt[q] before any lane rewrites it
                    W.mv[q] = (uint8_t)mv;
                    W.alt[q] = (uint8_t)(o & ~bit);
                    d = descend(tie, groups, W, i - (mv != kMoveL ? 1 : 0), j - (mv != kMoveU ? 1 : 0), q + 1);
                    emit_path(A, W, p, got, m, n, d);
                    ++got;
                }
            }
        }
        // every lane, the same values
        A.scores[p] = score;
        A.counts[p] = count;
        A.saturated[p] = (uint8_t)flag;
        if (ENUM) A.n_paths[p] = got;
    }
}

struct CoLayout {
    int64_t slot_bytes, off_tie, off_walk;
    size_t off_order, off_masks, off_slots;
    int64_t full_slots;
};

CoLayout co_layout(int32_t npairs, int32_t max_len, int32_t k, const DeviceInfo& di) {
    CoLayout L{};
    const int64_t ml = std::max(max_len, 1);
    int64_t off = (int64_t)align_up((size_t)(2 * (ml + 1)) * sizeof(BCell), 256);  // boundary: 2 buffers
    L.off_tie = off;
    if (k > 0) {
        const int64_t strips = (ml + kCoStrip - 1) / kCoStrip;
        const int64_t groups = (ml + kWave - 1 + 3) / 4;
        off += (int64_t)align_up((size_t)(strips * groups * kWave * 4), 256);
        L.off_walk = off;
        const int64_t Lw = 2 * ml + 1;
        off += (int64_t)align_up(align_up(2 * (size_t)Lw, 16) + 8 * (size_t)Lw, 256);
    } else {
        L.off_walk = off;
    }
    L.slot_bytes = off;
    L.off_order = kCoHeader;
    L.off_masks = align_up(kCoHeader + (size_t)std::max(npairs, 1) * 4, 256);
    L.off_slots = align_up(L.off_masks + (size_t)std::max(npairs, 1) * 64, 256);
    const int64_t resident = (int64_t)di.cus * co_blocks_per_cu(k > 0) * kCoWaves;
    const int64_t needed = ((int64_t)std::max(npairs, 1) + kCoWaves - 1) / kCoWaves * kCoWaves;
    L.full_slots = std::min(resident, needed);
    return L;
}

}  // namespace

size_t cooptimal_workspace_bytes(int32_t npairs, int32_t max_len, int32_t k, const DeviceInfo& di) {
    const CoLayout L = co_layout(npairs, max_len, k, di);
    return L.off_slots + (size_t)L.full_slots * (size_t)L.slot_bytes;
}

int launch_cooptimal(int32_t npairs, const uint8_t* pool, const int64_t* a_off, const int32_t* a_len,
                     const int64_t* b_off, const int32_t* b_len, int32_t max_len, const nw_scoring& sc,
                     int32_t* scores, uint64_t* counts, uint8_t* saturated, int32_t k, uint8_t* paths,
                     const int64_t* path_off, int32_t* path_len, int32_t* n_paths, void* ws, size_t ws_bytes,
                     hipStream_t st, const DeviceInfo& di) {
    const CoLayout L = co_layout(npairs, max_len, k, di);
    if (ws_bytes < L.off_slots + (size_t)kCoWaves * (size_t)L.slot_bytes) return NW_ENOSPC;
    int64_t slots = std::min<int64_t>(L.full_slots, (int64_t)((ws_bytes - L.off_slots) / (size_t)L.slot_bytes));
    slots = slots / kCoWaves * kCoWaves;
    uint8_t* base = (uint8_t*)ws;
    const Consts K = score_consts(sc);
    CoArgs A{};
    A.npairs = npairs;
    A.pool = pool;
    A.a_off = a_off;
    A.a_len = a_len;
    A.b_off = b_off;
    A.b_len = b_len;
    A.max_len = std::max(max_len, 1);
    A.kdm = K.kdm;
    A.kdx = K.kdx;
    A.gap = sc.gap;
    A.scores = scores;
    A.counts = counts;
    A.saturated = saturated;
    A.k = k;
    A.paths = paths;
    A.path_off = path_off;
    A.path_len = path_len;
    A.n_paths = n_paths;
    A.hist = (int32_t*)base;
    A.cursor = A.hist + kCoBuckets;
    A.next_job = A.cursor + kCoBuckets;
    A.next_team = A.next_job + 1;
    A.n_team = A.next_job + 2;
    // pairs of 2^16 cells or more are filled by teams (counts only)
    A.team_bucket = k > 0 ? kCoBuckets : NW_COOPT_TEAM_BUCKET;
    A.order = (int32_t*)(base + L.off_order);
    A.masks = (uint32_t*)(base + L.off_masks);
    A.force_wide = needs_wide(K) ? 1 : 0;
    A.slots = base + L.off_slots;
    A.slot_bytes = L.slot_bytes;
    A.off_tie = L.off_tie;
    A.off_walk = L.off_walk;
    A.spin = di.spin_limit;
    A.fault = di.fault;
    A.prio_jobs = (int32_t)std::min<int64_t>(npairs, slots);
    const unsigned pg = (unsigned)((npairs + 255) / 256);
    hipLaunchKernelGGL(k_co_zero, dim3((kCoHeaderInts + 255) / 256), dim3(256), 0, st, A.hist, kCoHeaderInts);
    hipLaunchKernelGGL(k_co_alpha, dim3((unsigned)((2 * (int64_t)npairs + 3) / 4)), dim3(256), 0, st, A);
    hipLaunchKernelGGL(k_co_hist, dim3(pg), dim3(256), 0, st, A);
    hipLaunchKernelGGL(k_co_scan, dim3(1), dim3(kCoBuckets), 0, st, A);
    hipLaunchKernelGGL(k_co_scatter, dim3(pg), dim3(256), 0, st, A);
    {
        ProfScope ps(k > 0 ? "nw_cooptimal_paths" : "nw_cooptimal", st);
        const dim3 grid((unsigned)(slots / kCoWaves));
        if (k > 0)
            hipLaunchKernelGGL(k_count<true>, grid, dim3(kWave * kCoWaves), 0, st, A);
        else
            hipLaunchKernelGGL(k_count<false>, grid, dim3(kWave * kCoWaves), 0, st, A);
    }
    return hipGetLastError() == hipSuccess ? NW_OK : NW_EDEVICE;
}

}  // namespace nw
