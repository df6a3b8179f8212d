// One long pair on the whole GPU: cooperative column strips.
//
// The n columns are cut into strips of 64*C columns.  A block holds four
// waves (one per SIMD) and sweeps four consecutive strips; blocks take strip
// groups from an atomic ticket counter, so a wave only ever waits for the
// strip to its left, whose owner took an earlier ticket and is therefore
// already running or done: the schedule cannot deadlock, and the grid never
// needs more blocks than fit on the device.  A strip's right boundary column
// goes to the next strip through a ring in LDS when both strips belong to
// one block and through 64-bit {value, epoch} slots in HBM otherwise
// (CoopIO), so the fill runs as one anti-diagonal front across all strips,
// each strip a fixed lag behind its left neighbour.
//
// Traceback.  Paths of up to a few thousand moves are walked back by one wave
// (k_tb_walk).  For longer ones one serial walk from (m, n) would take one dependent lookup per
// move (about 130k moves for a 65,536-base pair), so every strip first walks
// its own part of the path in parallel (k_tb_spec), starting from a guessed
// entry row: the row near the diagonal where the strip's right boundary
// column (left behind by the fill) scores best.  The strip notes, for each of
// its columns, the rows its walk visited and the move index at which it
// entered the column.  Then every strip at once (k_tb_merge) takes as its true
// entry the exit row of the next strip's speculative walk: if that cell lies
// on its own walk, the rest of the strip is that walk's suffix (walks from the
// same cell are identical), otherwise the strip walks from the entry until it
// meets its speculative walk.  If every strip meets it, each segment's offset
// follows from a prefix sum (k_tb_fix) and a last pass (k_tb_emit) writes
// every strip's segment, reversed, at its offset.  If one leaves its strip
// without meeting it (parallel co-optimal paths that never touch, common for
// unrelated sequences), the entries are not known at once and k_tb_fix walks
// the whole path with one wave as k_tb_walk does.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>

#include "nw_internal.h"
#include "nw_strip.h"

namespace nw {

constexpr int kCoopWaves = 4;  // waves per block of the traceback kernels
constexpr int kCoopThreads = kWave * kCoopWaves;
// Waves per block of the fill: consecutive strips, handing their boundary
// column over through LDS rings inside the block and HBM slots between blocks.
// Two (the 512 strips of a 65,536-column pair on all 256 CUs) measured
// slower: half the hops then cross blocks (fill 4.57 against 4.23 ms).
constexpr int kFillWaves = 4;
constexpr int kFillThreads = kWave * kFillWaves;
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
    const uint32_t* epoch;  // this call's slot tag, written by k_prep
    int32_t spin;           // polls before a boundary wait gives up
    int32_t* score;
    uint32_t* fault;        // host-visible device-fault word (may be null)
    const uint32_t* masks;  // byte-presence masks of a and b (eight words each), written by k_coop_alpha
    int32_t force_wide;     // compare bytes whatever the masks say (constants beyond a signed byte)
};

// Dynamic LDS of a block: the waves' row tables, then one boundary ring per
// wave (the ring wave w reads, written by wave w-1), a spare slot, and the
// rings' consumed-row counters.
template <int C>
struct CoopLds {
    static constexpr int kTableWords = kFillWaves * StripShape<C>::kLdsWords;
    static constexpr int kTableWordsAligned = (kTableWords + 1) & ~1;
    static constexpr int kRingWords = 2 * kRing;
    static constexpr int kSpareWord = kTableWordsAligned + kFillWaves * kRingWords;
    static constexpr int kCountWord = kSpareWord + 2;
    static constexpr int kWords = kCountWord + kFillWaves;
};

template <int C, bool DIRS, int IN, int OUT>
__device__ __forceinline__ int32_t coop_sweep(const CoopArgs& A, uint32_t epoch, uint32_t shift, bool wide, int s,
                                              int wave, uint32_t* lds, uint32_t* dyn, int j0, int ksel) {
    lds_u64* rings = (lds_u64*)(dyn + CoopLds<C>::kTableWordsAligned);
    lds_i32* consumed = (lds_i32*)(dyn + CoopLds<C>::kCountWord);
    uint64_t* col = A.bnd + (int64_t)s * A.bnd_stride;
    const CoopIO<IN, OUT, DIRS> io{s > 0 ? col - A.bnd_stride : nullptr,
                                   col,
                                   col + A.bnd_stride - 1,
                                   rings + wave * kRing,
                                   rings + ((wave + 1) % kFillWaves) * kRing,
                                   (lds_u64*)(dyn + CoopLds<C>::kSpareWord),
                                   consumed + wave,
                                   consumed + (wave + 1) % kFillWaves,
                                   A.m,
                                   A.vinit,
                                   epoch,
                                   A.err,
                                   A.spin};
    uint32_t* dirs = DIRS ? A.dirs + (size_t)s * A.G * kWave * C : nullptr;
    if (wide)
        return sweep_strip<C, DIRS, true>(A.a, A.m, A.b, A.n, j0, A.kdm, A.kdx, shift, A.vinit, A.vinit, io, dirs, lds,
                                          ksel);
    return sweep_strip<C, DIRS, false>(A.a, A.m, A.b, A.n, j0, A.kdm, A.kdx, shift, A.vinit, A.vinit, io, dirs, lds,
                                       ksel);
}

template <int C, bool DIRS>
__global__ __launch_bounds__(kFillThreads) void k_coop(CoopArgs A) {
    extern __shared__ uint32_t dyn[];
    __shared__ int ticket_s;
    const int wave = threadIdx.x >> 6;
    uint32_t* lds = dyn + wave * StripShape<C>::kLdsWords;
    constexpr int kCols = kWave * C;
    // the slot tag of this call (k_prep advances it per launch, so replays of
    // a captured graph never accept a previous replay's slots)
    const uint32_t epoch = (uint32_t)uniform((int32_t)__hip_atomic_load(A.epoch, __ATOMIC_RELAXED,
                                                                          __HIP_MEMORY_SCOPE_AGENT));
    // the pair's code field, or compared bytes
    const int shift_or = uniform(code_shift(A.masks, A.masks + 8));
    const bool wide = A.force_wide != 0 || shift_or < 0;
    const uint32_t shift = (uint32_t)max(shift_or, 0);
    for (;;) {
        if (threadIdx.x == 0) ticket_s = atomicAdd(A.ticket, 1);
        __syncthreads();
        const int k = uniform(ticket_s);
        // every wave is done with the previous group's rings: clear them and
        // their counters (row tags start at 1, so a zero slot is never ready)
        for (int q = CoopLds<C>::kTableWordsAligned + threadIdx.x; q < CoopLds<C>::kWords; q += kFillThreads)
            ((__attribute__((address_space(3))) uint32_t*)dyn)[q] = 0;
        __syncthreads();
        if (k >= A.ngroups) break;
        const int s = k * kFillWaves + wave;
        if (s < A.nstrips) {
            const int j0 = s * kCols;
            const int ksel = (A.n - 1 - j0) % C;
            const bool last = (s == A.nstrips - 1);
            int32_t v;
            // input: none (first strip), the block's previous wave (LDS), or the
            // previous block's last wave (HBM); output likewise
            if (s == 0) {
                v = last ? coop_sweep<C, DIRS, kIoNone, kIoNone>(A, epoch, shift, wide, s, wave, lds, dyn, j0, ksel)
                         : coop_sweep<C, DIRS, kIoNone, kIoLds>(A, epoch, shift, wide, s, wave, lds, dyn, j0, ksel);
            } else if (wave == 0) {
                v = last ? coop_sweep<C, DIRS, kIoGlobal, kIoNone>(A, epoch, shift, wide, s, wave, lds, dyn, j0, ksel)
                         : coop_sweep<C, DIRS, kIoGlobal, kIoLds>(A, epoch, shift, wide, s, wave, lds, dyn, j0, ksel);
            } else if (wave < kFillWaves - 1) {
                v = last ? coop_sweep<C, DIRS, kIoLds, kIoNone>(A, epoch, shift, wide, s, wave, lds, dyn, j0, ksel)
                         : coop_sweep<C, DIRS, kIoLds, kIoLds>(A, epoch, shift, wide, s, wave, lds, dyn, j0, ksel);
            } else {
                v = last ? coop_sweep<C, DIRS, kIoLds, kIoNone>(A, epoch, shift, wide, s, wave, lds, dyn, j0, ksel)
                         : coop_sweep<C, DIRS, kIoLds, kIoGlobal>(A, epoch, shift, wide, s, wave, lds, dyn, j0, ksel);
            }
            if (last) {
                const int lsel = (A.n - 1 - j0) / C;
                const int32_t vv = __builtin_amdgcn_readlane(v, lsel);
                A.score[0] = (DIRS ? ((vv - 1) >> 2) : vv) + A.gap * (A.m + A.n);
            }
        }
    }
}

// Score-only calls: report a boundary-wait failure of the fill as INT32_MIN
// and in the device-fault word.
__global__ void k_check_fill(const int32_t* err, int32_t* score, uint32_t* fault) {
    if (threadIdx.x == 0 && __hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) {
        score[0] = INT32_MIN;
        report_fault(fault);
    }
}

// ---- parallel traceback over strips ----

constexpr int kInfoHead = 8;  // len, start_row, exit_row, lo/hi of the entry column, pad
constexpr int kGuessSpan = 4096;  // rows searched on each side of the diagonal for an entry guess

struct TbArgs {
    const uint32_t* dirs;
    int m, n, G, nstrips;
    const uint64_t* bnd;  // right boundary column of every strip but the last
    int64_t bnd_stride;
    int32_t key_gap;      // 4 * gap: V + key_gap * i orders a column's rows like H
    uint8_t* seg;        // per strip: speculative moves, backward order
    uint8_t* rw;         // per strip: re-walk moves, backward order
    int64_t seg_stride;
    int32_t* info;       // per strip: kInfoHead ints, then lo[], hi[], idx[] per column
    int64_t info_stride;
    int32_t* fix;        // per strip: rw_len, seg_from, total_len, offset
    int32_t* summary;    // [0] tail (vertical moves at column 0), [1] path length, [2] error, [4] a re-walk
                         // left its strip, [5] a corrupt tag in k_tb_merge, [6] k_tb_fix wrote the path
    const int32_t* err;  // fill failure flag
    uint8_t* path;
    int64_t* path_len;
    int32_t* score;
    int64_t cap;         // path capacity, m + n
    uint32_t* fault;     // host-visible device-fault word (may be null)
};

template <int C>
__global__ __launch_bounds__(kCoopThreads) void k_tb_spec(TbArgs T) {
    constexpr int kCols = kWave * C;
    __shared__ uint32_t win_lds[kCoopWaves][kWave * C];
    __shared__ int32_t col_lds[kCoopWaves][3][kCols];
    const int wave = threadIdx.x >> 6;
    const int lane = lane_id();
    const int s = blockIdx.x * kCoopWaves + wave;
    if (s >= T.nstrips) return;
    if (__hip_atomic_load(T.err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) return;
    const int j_lo = s * kCols + 1;
    const int j_hi = min((s + 1) * kCols, T.n);
    int i = T.m, j = T.n;
    if (s < T.nstrips - 1) {
        // Entry guess: the row where the strip's right boundary column scores
        // best, searched within kGuessSpan rows of the proportional diagonal.
        const int64_t c = ((int64_t)j_hi * T.m + T.n / 2) / T.n;
        const int r0 = (int)max<int64_t>(1, c - kGuessSpan), r1 = (int)min<int64_t>(T.m, c + kGuessSpan);
        const uint64_t* col = T.bnd + (int64_t)s * T.bnd_stride;
        int32_t best_key = INT32_MIN, best_row = r0;
        for (int r = r0 + lane; r <= r1; r += kWave) {
            const int32_t key = (int32_t)(uint32_t)col[r] + T.key_gap * r;
            if (key > best_key) {
                best_key = key;
                best_row = r;
            }
        }
#pragma unroll
        for (int d = 1; d < kWave; d <<= 1) {
            const int32_t ok = __shfl_xor(best_key, d);
            const int32_t orow = __shfl_xor(best_row, d);
            if (ok > best_key || (ok == best_key && orow < best_row)) {
                best_key = ok;
                best_row = orow;
            }
        }
        i = uniform(best_row);
        j = j_hi;
    }
    const int start_row = i;
    int32_t* lo = col_lds[wave][0];
    int32_t* hi = col_lds[wave][1];
    int32_t* idx = col_lds[wave][2];
    for (int c = lane; c < kCols; c += kWave) {
        lo[c] = -1;
        hi[c] = -1;
        idx[c] = -1;
    }
    __builtin_amdgcn_wave_barrier();
    DirWindow<C> win(T.dirs, T.G, win_lds[wave]);
    uint8_t* out = T.seg + (int64_t)s * T.seg_stride;
    int q = 0, cur = -1;
    bool bad = false;
    while (j >= j_lo) {
        const int c = j - j_lo;
        if (c != cur) {
            hi[c] = i;
            idx[c] = q;
            cur = c;
        }
        lo[c] = i;
        int mv = 3;
        if (i > 0) {
            const int tag = win.tag(i, j);
            if (tag == 0) {
                bad = true;
                break;
            }
            mv = 4 - tag;
        }
        out[q++] = (uint8_t)mv;
        if (mv == 1) {
            --i;
            --j;
        } else if (mv == 2) {
            --i;
        } else {
            --j;
        }
    }
    __builtin_amdgcn_wave_barrier();
    int32_t* rec = T.info + (int64_t)s * T.info_stride;
    const int cR = j_hi - j_lo;
    if (lane == 0) {
        rec[0] = q;
        rec[1] = start_row;
        rec[2] = i;
        rec[3] = lo[cR];
        rec[4] = hi[cR];
        rec[5] = bad ? 1 : 0;
    }
    for (int c = lane; c < kCols; c += kWave) {
        rec[kInfoHead + c] = lo[c];
        rec[kInfoHead + kCols + c] = hi[c];
        rec[kInfoHead + 2 * kCols + c] = idx[c];
    }
}

// Re-walk strip s from its true entry row e (at the strip's last column)
// until the walk meets the strip's speculative walk, recorded per column as
// the row range lo..hi it visited and the move index at which it entered the
// column, or leaves the strip.  The re-walk's moves go to the strip's rw
// buffer.  Returns whether it met the speculative walk; sets rw_len, seg_from
// (how many speculative moves the merged walk skips), exit_row (if it did not
// meet), and error (a corrupt tag).
template <int C>
__device__ bool rewalk(const TbArgs& T, int s, int e, int32_t (*col)[kWave * C], DirWindow<C>& win, int& rw_len,
                       int& seg_from, int& exit_row, int& error) {
    constexpr int kCols = kWave * C;
    const int lane = lane_id();
    const int j_lo = s * kCols + 1;
    const int32_t* rec = T.info + (int64_t)s * T.info_stride + kInfoHead;
    for (int c = lane; c < kCols; c += kWave) {
        col[0][c] = rec[c];
        col[1][c] = rec[kCols + c];
        col[2][c] = rec[2 * kCols + c];
    }
    __builtin_amdgcn_wave_barrier();
    uint8_t* out = T.rw + (int64_t)s * T.seg_stride;
    int i = e, j = min((s + 1) * kCols, T.n);
    bool merged = false;
    rw_len = 0;
    while (j >= j_lo) {
        const int c = j - j_lo;
        const int clo = col[0][c], chi = col[1][c];
        if (chi >= 0 && clo <= i && i <= chi) {
            seg_from = col[2][c] + (chi - i);
            merged = true;
            break;
        }
        int mv = 3;
        if (i > 0) {
            const int tag = win.tag(i, j);
            if (tag == 0) {
                error = 1;
                break;
            }
            mv = 4 - tag;
        }
        out[rw_len++] = (uint8_t)mv;
        if (mv == 1) {
            --i;
            --j;
        } else if (mv == 2) {
            --i;
        } else {
            --j;
        }
    }
    exit_row = i;
    __builtin_amdgcn_wave_barrier();
    return merged;
}

// All strips at once, one wave each.  If every re-walk meets its strip's
// speculative walk, the true path leaves each strip where that walk leaves
// it, so the entry row of strip s is the speculative exit row of strip s + 1
// and no strip has to wait for another.  A re-walk that leaves its strip
// without meeting the walk breaks that assumption: the flag it raises makes
// k_tb_fix walk the whole path with one wave instead.
template <int C>
__global__ __launch_bounds__(kCoopThreads) void k_tb_merge(TbArgs T) {
    constexpr int kCols = kWave * C;
    __shared__ uint32_t win_lds[kCoopWaves][kWave * C];
    __shared__ int32_t col_lds[kCoopWaves][3][kCols];
    const int wave = threadIdx.x >> 6;
    const int s = blockIdx.x * kCoopWaves + wave;
    if (s >= T.nstrips) return;
    if (__hip_atomic_load(T.err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) return;
    const int32_t* rec = T.info + (int64_t)s * T.info_stride;
    const int len = rec[0], start = rec[1], loR = rec[3], hiR = rec[4];
    int error = rec[5];
    const int e = (s == T.nstrips - 1) ? T.m : T.info[(int64_t)(s + 1) * T.info_stride + 2];
    int rw_len = 0, seg_from = 0, exit_row = 0;
    if (s == T.nstrips - 1) {
        seg_from = 0;
    } else if (hiR >= 0 && loR <= e && e <= hiR) {
        seg_from = start - e;
    } else {
        DirWindow<C> win(T.dirs, T.G, win_lds[wave]);
        if (!rewalk<C>(T, s, e, col_lds[wave], win, rw_len, seg_from, exit_row, error))
            __hip_atomic_store(T.summary + 4, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    if (error) __hip_atomic_store(T.summary + 5, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (lane_id() == 0) {
        int32_t* f = T.fix + 4 * (int64_t)s;
        f[0] = rw_len;
        f[1] = seg_from;
        f[2] = rw_len + (len - seg_from);
    }
}

// One wave walks the whole path back from (m, n) on the stored directions
// (walk_back: scalar state, a register window, diagonal runs in one step)
// into the walk-move buffer, then writes it out in forward order.  Returns
// the number of moves, or -1 for a corrupt tag.
template <int C>
__device__ int64_t walk_whole(const TbArgs& T) {
    const int64_t len = walk_back<C>(T.dirs, T.m, T.n, T.G, nullptr, T.seg);
    if (len < 0 || len > T.cap) return -1;
    // the moves were written by other lanes of this wave
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    for (int64_t x = lane_id(); x < len; x += kWave) T.path[x] = T.seg[len - 1 - x];
    return len;
}

// Paths of up to a few thousand moves: the one-wave walk is shorter than the
// per-strip walks, their merge and their placement together.
template <int C>
__global__ __launch_bounds__(kWave) void k_tb_walk(TbArgs T) {
    int64_t len = -3;  // fill failure
    if (__hip_atomic_load(T.err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0) len = walk_whole<C>(T);
    if (lane_id() == 0) {
        if (len < 0) {
            T.score[0] = INT32_MIN;
            T.path_len[0] = len == -3 ? -3 : -2;
            report_fault(T.fault);
        } else {
            T.path_len[0] = len;
        }
    }
}

// Offsets of every strip's segment.  When some re-walk left its strip without
// meeting the speculative walk, the strips' entries are not known at once;
// one wave then walks the whole path back instead (as k_tb_walk) and writes
// it out itself.
template <int C>
__global__ __launch_bounds__(kWave) void k_tb_fix(TbArgs T) {
    const int lane = lane_id();
    if (__hip_atomic_load(T.err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) {
        if (lane == 0) T.summary[2] = 3;
        return;
    }
    if (__hip_atomic_load(T.summary + 4, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) {
        const int64_t len = walk_whole<C>(T);
        if (lane == 0) {
            T.summary[2] = len < 0 ? 1 : 0;
            T.summary[6] = 1;  // the path is out
            if (len >= 0) T.path_len[0] = len;
        }
        return;
    }
    // k_tb_merge has placed every strip: the path reaches column 0 where
    // strip 0's speculative walk does
    int error = __hip_atomic_load(T.summary + 5, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const int e = T.info[2];
    // e is the row at which the path reaches column 0: that many vertical
    // moves come first in forward order, then strips 0, 1, ... in turn
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
    int64_t off = e;
    for (int b = 0; b < T.nstrips; b += kWave) {
        const int sq = b + lane;
        const int32_t tl = (sq < T.nstrips) ? T.fix[4 * (int64_t)sq + 2] : 0;
        // inclusive prefix sum across the wave
        int32_t x = tl;
#pragma unroll
        for (int d = 1; d < kWave; d <<= 1) {
            const int32_t y = __shfl_up(x, d);
            if (lane >= d) x += y;
        }
        if (sq < T.nstrips) T.fix[4 * (int64_t)sq + 3] = (int32_t)(off + x - tl);
        off += __builtin_amdgcn_readlane(x, kWave - 1);
    }
    if (off > T.cap || off < 0) error = 1;  // never expected: a consistent path has <= m + n moves
    if (lane == 0) {
        T.summary[0] = 0;
        T.summary[1] = (int32_t)off;
        T.summary[2] = error;
        T.summary[3] = e;
    }
}

template <int C>
__global__ __launch_bounds__(kCoopThreads) void k_tb_emit(TbArgs T) {
    const int wave = threadIdx.x >> 6;
    const int lane = lane_id();
    const int s = blockIdx.x * kCoopWaves + wave;
    if (T.summary[2] != 0) {
        if (s == 0 && lane == 0) {
            T.score[0] = INT32_MIN;
            T.path_len[0] = T.summary[2] == 3 ? -3 : -2;
            report_fault(T.fault);
        }
        return;
    }
    if (T.summary[6] != 0) return;  // k_tb_fix walked and wrote the whole path
    if (s == 0) {
        const int tail = T.summary[3];
        for (int x = lane; x < tail; x += kWave) T.path[x] = 2;
        if (lane == 0) T.path_len[0] = T.summary[1];
    }
    if (s >= T.nstrips) return;
    const int32_t* f = T.fix + 4 * (int64_t)s;
    const int rw_len = f[0], seg_from = f[1], L = f[2], o = f[3];
    const uint8_t* rw = T.rw + (int64_t)s * T.seg_stride;
    const uint8_t* sg = T.seg + (int64_t)s * T.seg_stride + seg_from - rw_len;
    for (int x = lane; x < L; x += kWave) {
        const int y = L - 1 - x;
        if ((int64_t)o + x < T.cap) T.path[o + x] = (y < rw_len) ? rw[y] : sg[y];
    }
}

// Workspace header words of the cooperative engine (the masks take words
// 64..79).
constexpr int kHdrTicket = 0, kHdrErr = 16, kHdrSummary = 32, kHdrEpoch = 48, kHdrMasks = 64;
constexpr size_t kCoopHeaderBytes = 512;

// Byte-presence masks of a and b (zeroed by k_prep): every wave takes a
// chunk of kAlphaChunk bytes of a, or of b, and ORs its chunk_mask in.
constexpr int64_t kAlphaChunk = 8192;
__global__ __launch_bounds__(256) void k_coop_alpha(const uint8_t* a, int64_t m, const uint8_t* b, int64_t n,
                                                    uint32_t* masks) {
    __shared__ uint32_t bits[4][8];
    const int wave = threadIdx.x >> 6;
    const int64_t w = (int64_t)blockIdx.x * 4 + wave;
    const int64_t ca = (m + kAlphaChunk - 1) / kAlphaChunk;
    const bool on_a = w < ca;
    const int64_t start = (on_a ? w : w - ca) * kAlphaChunk;
    const int64_t len = on_a ? m : n;
    if (start >= len) return;
    const uint32_t mk = chunk_mask((on_a ? a : b) + start, min(kAlphaChunk, len - start), bits[wave]);
    const int lane = lane_id();
    if (lane < 8 && mk != 0) atomicOr(masks + (on_a ? 0 : 8) + lane, mk);
}

// The slot tag of the latest cooperative fill on this device.  A boundary
// slot is taken as ready once it carries the reading call's tag, so no two
// launches whose slots can meet in memory may share one: workspaces are
// reused, and a fresh one can hold any earlier call's slots.  Tags therefore
// only move forward on a device (modulo 2^32, ordered by signed difference):
// each launch takes the later of the host's value for the call and the
// previous tag, plus two.  Eager calls bring a new host value each; replays
// of a captured graph bring the same host value again, and the device word
// moves them on.
__device__ uint32_t g_coop_tag;

// Before each fill: clear the ticket, the failure flag, the traceback summary
// and the byte masks, and take the call's slot tag.
__global__ void k_prep(int32_t* hdr, uint32_t host_epoch) {
    const int i = threadIdx.x;
    if (i < kHdrEpoch || (i >= kHdrMasks && i < kHdrMasks + 16)) hdr[i] = 0;
    if (i == 0) {
        uint32_t prev = __hip_atomic_load(&g_coop_tag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        uint32_t tag;
        for (;;) {
            const uint32_t base = ((int32_t)(host_epoch - prev) > 0) ? host_epoch : prev;
            tag = (base + 2u) | 1u;  // odd: never the 0 of fresh memory
            if (__hip_atomic_compare_exchange_strong(&g_coop_tag, &prev, tag, __ATOMIC_RELAXED,
                                                     __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
                break;
        }
        hdr[kHdrEpoch] = (int32_t)tag;
    }
}

// ---- host side ----

constexpr int kCoopC = 2;  // 128-column strips: half the hops of 64-column ones at a 1.3x step cost
static_assert(CoopLds<kCoopC>::kWords * 4 <= kCoopDynLds, "cooperative fill LDS");

struct CoopLayout {
    int nstrips, ngroups, G;
    int64_t bnd_stride, seg_stride, info_stride;
    size_t off_bnd, off_dirs, off_info, off_fix, off_seg, off_rw, total;
};

// Workspace: [ticket, err, summary | boundary slots | directions |
// per-strip walk records | per-strip fix-up records | walk moves | re-walk moves]
static CoopLayout coop_layout(int64_t m, int64_t n, bool dirs) {
    CoopLayout L{};
    const int64_t cols = (int64_t)kWave * kCoopC;
    L.nstrips = (int)((n + cols - 1) / cols);
    L.ngroups = (L.nstrips + kFillWaves - 1) / kFillWaves;
    L.G = groups_for_rows((int)m);
    L.bnd_stride = (int64_t)align_up((size_t)(m + 2), 32);  // rows 0..m and a spare slot
    L.seg_stride = (int64_t)align_up((size_t)(m + cols + 16), 64);
    L.info_stride = kInfoHead + 3 * cols;
    const size_t ns = (size_t)L.nstrips;
    size_t off = kCoopHeaderBytes;
    L.off_bnd = off;
    off = align_up(off + (size_t)L.nstrips * L.bnd_stride * 8, 256);  // one column per strip
    L.off_dirs = off;
    if (dirs) {
        off = align_up(off + ns * L.G * kWave * kCoopC * 4, 256);
        L.off_info = off;
        off = align_up(off + ns * L.info_stride * 4, 256);
        L.off_fix = off;
        off = align_up(off + ns * 16, 256);
        L.off_seg = off;
        off = align_up(off + ns * L.seg_stride, 256);
        L.off_rw = off;
        off = align_up(off + ns * L.seg_stride, 256);
    }
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
        hipLaunchKernelGGL((k_coop<kCoopC, DIRS>), dim3(grid), dim3(kFillThreads), kCoopDynLds, st, A);
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
    int32_t* hdr = (int32_t*)base;
    A.ticket = hdr + kHdrTicket;
    A.err = hdr + kHdrErr;
    A.epoch = (const uint32_t*)(hdr + kHdrEpoch);
    A.spin = di.spin_limit;
    A.score = score;
    A.fault = di.fault;
    A.masks = (const uint32_t*)(hdr + kHdrMasks);
    A.force_wide = needs_wide(K) ? 1 : 0;
    hipLaunchKernelGGL(k_prep, dim3(1), dim3(128), 0, st, hdr, next_epoch());
    {
        const int64_t chunks = (m + kAlphaChunk - 1) / kAlphaChunk + (n + kAlphaChunk - 1) / kAlphaChunk;
        hipLaunchKernelGGL(k_coop_alpha, dim3((unsigned)std::max<int64_t>(1, (chunks + 3) / 4)), dim3(256), 0, st, a,
                           m, b, n, (uint32_t*)(hdr + kHdrMasks));
    }
    const int grid = std::max(1, std::min(L.ngroups, di.cus));
    hipError_t e = dirs ? launch_coop_kernel<true>(A, grid, st) : launch_coop_kernel<false>(A, grid, st);
    if (e != hipSuccess) return NW_EDEVICE;
    if (!dirs) {
        hipLaunchKernelGGL(k_check_fill, dim3(1), dim3(64), 0, st, A.err, score, di.fault);
    } else {
        TbArgs T{};
        T.dirs = A.dirs;
        T.m = (int)m;
        T.n = (int)n;
        T.G = L.G;
        T.nstrips = L.nstrips;
        T.bnd = A.bnd;
        T.bnd_stride = A.bnd_stride;
        T.key_gap = 4 * sc.gap;
        T.seg = base + L.off_seg;
        T.rw = base + L.off_rw;
        T.seg_stride = L.seg_stride;
        T.info = (int32_t*)(base + L.off_info);
        T.info_stride = L.info_stride;
        T.fix = (int32_t*)(base + L.off_fix);
        T.summary = hdr + kHdrSummary;
        T.err = A.err;
        T.fault = di.fault;
        T.path = path;
        T.path_len = path_len;
        T.score = score;
        T.cap = m + n;
        const unsigned blocks = (unsigned)((L.nstrips + kCoopWaves - 1) / kCoopWaves);
        if (m + n <= di.walk_limit) {
            ProfScope ps("nw_tb_walk", st);
            hipLaunchKernelGGL(k_tb_walk<kCoopC>, dim3(1), dim3(kWave), 0, st, T);
            return hipGetLastError() == hipSuccess ? NW_OK : NW_EDEVICE;
        }
        {
            ProfScope ps("nw_tb_spec", st);
            hipLaunchKernelGGL(k_tb_spec<kCoopC>, dim3(blocks), dim3(kCoopThreads), 0, st, T);
        }
        {
            ProfScope ps("nw_tb_merge", st);
            hipLaunchKernelGGL(k_tb_merge<kCoopC>, dim3(blocks), dim3(kCoopThreads), 0, st, T);
        }
        {
            ProfScope ps("nw_tb_fix", st);
            hipLaunchKernelGGL(k_tb_fix<kCoopC>, dim3(1), dim3(kWave), 0, st, T);
        }
        {
            ProfScope ps("nw_tb_emit", st);
            hipLaunchKernelGGL(k_tb_emit<kCoopC>, dim3(blocks), dim3(kCoopThreads), 0, st, T);
        }
    }
    return hipGetLastError() == hipSuccess ? NW_OK : NW_EDEVICE;
}

}  // namespace nw
