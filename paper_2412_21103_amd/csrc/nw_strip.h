// Column-strip wavefront engine and windowed traceback (one wave each).
//
// A strip is 64*C consecutive columns of one pair.  Lane l owns columns
// j0 + C*l + k (k = 0..C-1) and at step t works on row i = t - l + 1, so the
// wave sweeps the strip top to bottom along a skewed anti-diagonal front: the
// cell's vertical and diagonal inputs are the lane's own registers from the
// previous step, the horizontal input of column k > 0 is the value just
// produced for column k-1, and the horizontal input of column 0 is the
// previous step's last-column value of lane l-1, moved across lanes with one
// DPP wave shift.  Lane 0 takes that value from a queue register R: R is
// shifted left one lane per step, so lane 0 consumes the next row's
// left-boundary value while lane 63 appends its own last-column value, which
// is the strip's right boundary for the next strip.  Every 16 steps lanes
// 48..63 (the last 16 outputs) are written out and lanes 0..15 are refilled
// with the next 16 inputs; whatever sits in lanes 16..47 reaches lane 0 only
// after the next refill has overwritten it, so inputs are needed just one
// group (16 rows) ahead.
//
// Boundary columns travel through an IO policy: PlainIO for a wave that
// sweeps all strips of a pair itself, TaggedIO when neighbouring strips run
// on different waves (see the cooperative kernel).
//
// The substitution term comes from a per-row table in LDS: for row i the word
// holds four signed bytes, byte y = term(a_i == y).  Lane (l, k) reads byte
// b_j of the row it is on with one ds_read_i8.  Rows outside 1..m hold -128,
// which freezes the lanes that are above or below the matrix (see
// nw_common.h), so the sweep needs no per-lane predicates.
//
// Directions: each lane shifts the 2-bit tag of every cell of column k into a
// 32-bit accumulator; after 16 steps lane l stores its C words contiguously,
// giving the layout  dirs[strip][group g][lane l][column k]  (one word per
// 16 consecutive steps of one column).  Step t of lane l is row t - l + 1, so
// cell (i, j) lives in word (g = (i-1+l) / 16) at bits 2*((i-1+l) % 16).
#pragma once

#include "nw_common.h"

namespace nw {

constexpr int kWinRows = 192;   // rows per table window
constexpr int kWinGroups = 8;   // 16-step groups served by one window

template <int C>
struct StripShape {
    static constexpr int kCols = kWave * C;
    // LDS words per wave: two table windows, or the traceback window
    static constexpr int kLdsWords = (2 * kWinRows > 64 * C) ? 2 * kWinRows : 64 * C;
};

// Lane 63 finishes row m at step m + 62, and its value enters the queue at the
// start of step m + 63, which must lie in a group that the loop runs (the
// group's end flushes it).  So the sweep runs floor((m + 63) / 16) + 1 groups.
__host__ __device__ __forceinline__ int groups_for_rows(int m) { return (m + 79) >> 4; }
__host__ __device__ __forceinline__ int steps_for_rows(int m) { return groups_for_rows(m) << 4; }

// Fill one table window: word p <-> row wlo + p.
__device__ __forceinline__ void write_window(uint32_t* win, const uint8_t* a, int m, int wlo,
                                             int kdm, int kdx, int lane) {
#pragma unroll
    for (int e = 0; e < kWinRows / kWave; ++e) {
        int p = lane + kWave * e;
        int r = wlo + p;
        uint32_t w = kSentinelWord;
        if (r >= 1 && r <= m) w = row_word(a[r - 1], kdm, kdx);
        win[p] = w;
    }
}

// Boundary IO for a wave that owns every strip of its pair: the previous
// strip's right column sits in the wave's own scratch (bin, indexed by grid
// row), the next strip's goes to the same buffer (bout; reads of a row happen
// before its overwrite).  The sweep may cover only grid rows r0+1 .. r0+m
// (a band); its rows are numbered locally from 1.  Inputs for grid rows above
// in_hi, or beyond the sweep, lie outside the previous strip's region and
// read `beyond`, a value that never wins (0, or the -infinity sentinel of a
// band).  A missing bin means the grid's first column (vinit).
struct PlainIO {
    const int32_t* bin;
    int32_t* bout;
    int m;
    int32_t vinit;
    int r0 = 0;
    int in_hi = 1 << 30;
    int32_t beyond = 0;
    using Slot = int32_t;
    __device__ __forceinline__ Slot load(int r, bool want) const {
        return (want && bin && r <= m && r0 + r <= in_hi) ? bin[r0 + r] : 0;
    }
    __device__ __forceinline__ int32_t value(Slot x, int r) const {
        if (r > m) return beyond;
        if (!bin) return vinit;
        return (r0 + r <= in_hi) ? x : beyond;
    }
    __device__ __forceinline__ bool ready(Slot, int, bool) const { return true; }
    __device__ __forceinline__ void store(int r, int32_t v, bool want) const {
        if (bout && want) bout[r0 + r] = v;
    }
    __device__ __forceinline__ void fail() const {}
    __device__ __forceinline__ bool failed() const { return false; }
};

// Boundary IO between strips swept by different waves, possibly on different
// CUs or XCDs.  Each row slot is 64 bits, {value, epoch}, written with one
// device-coherent atomic store; the reader polls the slot until it carries the
// current call's epoch, so no separate flag (and no cache write-back) is
// needed.  Polling gives up after a bounded number of rounds and raises *err.
struct TaggedIO {
    const uint64_t* bin;
    uint64_t* bout;
    int m;
    int32_t vinit;
    uint32_t epoch;
    int32_t* err;
    bool in_local;   // the left neighbour runs on the same CU (same block)
    bool out_local;  // the right neighbour runs on the same CU
    using Slot = uint64_t;
    // Waves of one block share the CU's L1, so block-local neighbours use
    // workgroup-scope accesses (plain, L1-coherent); other neighbours may sit
    // on another XCD and use device-scope (sc1) accesses.
    __device__ __forceinline__ Slot load(int r, bool want) const {
        if (!(want && bin && r <= m)) return 0;
        return in_local ? __hip_atomic_load(bin + r, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP)
                        : __hip_atomic_load(bin + r, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    __device__ __forceinline__ int32_t value(Slot x, int r) const {
        return r > m ? 0 : (bin ? (int32_t)(uint32_t)x : vinit);
    }
    __device__ __forceinline__ bool ready(Slot x, int r, bool want) const {
        return !(want && bin && r <= m) || (uint32_t)(x >> 32) == epoch;
    }
    __device__ __forceinline__ void store(int r, int32_t v, bool want) const {
        if (!(bout && want)) return;
        const uint64_t x = ((uint64_t)epoch << 32) | (uint32_t)v;
        if (out_local) __hip_atomic_store(bout + r, x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        else __hip_atomic_store(bout + r, x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    __device__ __forceinline__ void fail() const {
        __hip_atomic_store(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    __device__ __forceinline__ bool failed() const {
        return __hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0;
    }
};

constexpr int kSpinLimit = 1 << 16;  // polling rounds before a boundary wait gives up

// Load slot r (for the lanes with `want`) until every such lane sees a ready
// slot.  The loop condition is wave-uniform.
template <class IO>
__device__ __forceinline__ typename IO::Slot wait_slot(const IO& io, int r, bool want) {
    typename IO::Slot x = io.load(r, want);
    for (int spin = 0; spin < kSpinLimit; ++spin) {
        if (__builtin_amdgcn_ballot_w64(!io.ready(x, r, want)) == 0) return x;
        if (io.failed()) return x;  // another wait already gave up: drain quickly
        __builtin_amdgcn_s_sleep(2);
        x = io.load(r, want);
    }
    io.fail();
    return x;
}

// Sweep one strip.  Returns, per lane, V (or W) of its column `ksel` after
// the last row (the frozen final value).
// `a` points at the sweep's first row and `m` counts its rows (a band sweeps
// grid rows r0+1 .. r0+m with a = seq + r0).  Every lane starts from `vtop`,
// the row above the sweep (the grid's first row, or -infinity inside a band),
// except that lane 0's first diagonal input is `dg0`, the previous strip's
// last column one row above the sweep.
template <int C, bool DIRS, class IO>
__device__ __forceinline__ int32_t sweep_strip(const uint8_t* __restrict__ a, int m,
                                               const uint8_t* __restrict__ b, int n, int j0, int kdm,
                                               int kdx, int32_t vtop, int32_t dg0, const IO& io,
                                               uint32_t* __restrict__ dirs, uint32_t* lds, int ksel) {
    const int lane = lane_id();
    const bool lane0 = (lane == 0);
    int32_t V[C];
    uint32_t acc[C];
    uint32_t bcode[C];
#pragma unroll
    for (int k = 0; k < C; ++k) {
        V[k] = vtop;
        acc[k] = 0;
        int j = j0 + C * lane + k;
        bcode[k] = (j < n) ? (uint32_t)(b[j] & 3) : 0u;
    }
    int32_t Dg = lane0 ? dg0 : vtop;
    int32_t R = io.value(wait_slot(io, lane + 1, lane < 16), lane + 1);
    // boundary values for the refill of lanes 0..15 at the end of group 0
    int rin = 16 + 1 + lane;
    typename IO::Slot Rin = io.load(rin, lane < 16);

    const int NG = groups_for_rows(m);
    // window 0 covers groups [0, 8): rows [-63, 129)
    int g0 = 0;
    int cur = 0;
    write_window(lds, a, m, -63, kdm, kdx, lane);
    // prefetch the next window's symbols
    uint8_t pf[kWinRows / kWave];
#pragma unroll
    for (int e = 0; e < kWinRows / kWave; ++e) {
        int r = 16 * kWinGroups - 63 + lane + kWave * e;
        pf[e] = (r >= 1 && r <= m) ? a[r - 1] : (uint8_t)0xFF;
    }

    const int8_t* lds8 = reinterpret_cast<const int8_t*>(lds);
    for (int g = 0; g < NG; ++g) {
        int gg = g - g0;
        if (gg == kWinGroups) {
            // switch windows: materialise the prefetched rows, then prefetch the next
            cur ^= 1;
            g0 += kWinGroups;
            gg = 0;
            uint32_t* win = lds + cur * kWinRows;
#pragma unroll
            for (int e = 0; e < kWinRows / kWave; ++e) {
                int p = lane + kWave * e;
                win[p] = (pf[e] == 0xFF) ? kSentinelWord : row_word(pf[e], kdm, kdx);
            }
#pragma unroll
            for (int e = 0; e < kWinRows / kWave; ++e) {
                int r = 16 * (g0 + kWinGroups) - 63 + lane + kWave * e;
                pf[e] = (r >= 1 && r <= m) ? a[r - 1] : (uint8_t)0xFF;
            }
        }
        // byte address of (row of step 16g, this lane, column k) in the window;
        // the mask shows the compiler the address is non-negative so the
        // per-step offsets 4u fold into the ds_read immediate
        const uint32_t base = (uint32_t)(cur * kWinRows * 4 + 4 * (64 - lane) + 64 * gg);
        uint32_t addr[C];
#pragma unroll
        for (int k = 0; k < C; ++k) addr[k] = (base + bcode[k]) & 0x7FFFu;


        // Narrow strips have too little work per step to hide the LDS latency
        // behind other waves, so their whole group of table reads is issued up
        // front; wide strips read one step at a time.
        constexpr bool kHoist = (C <= 2);
        int32_t kdh[kHoist ? 16 : 1][C];
        if constexpr (kHoist) {
#pragma unroll
            for (int u = 0; u < 16; ++u)
#pragma unroll
                for (int k = 0; k < C; ++k) kdh[u][k] = (int32_t)lds8[addr[k] + 4 * u];
        }

#pragma unroll
        for (int u = 0; u < 16; ++u) {
            const int32_t Lr = shift_in_from_left(R, V[C - 1], lane0);
            int32_t left = Lr;
            int32_t diag = Dg;
            int32_t tail = 0;  // the last column's previous value (+1 in the V domain)
#pragma unroll
            for (int k = 0; k < C; ++k) {
                int32_t kd;
                if constexpr (kHoist) kd = kdh[u][k];
                else kd = (int32_t)lds8[addr[k] + 4 * u];
                const int32_t up = V[k];
                const int32_t cD = diag + kd;
                int32_t v;
                if constexpr (DIRS) {
                    const int32_t cU = up + 1;
                    const int32_t r = imax3(cD, cU, left);
                    acc[k] = shift_in_tag((uint32_t)r, acc[k]);
                    v = clear_tag(r);
                    if (k == C - 1) tail = cU;
                } else {
                    v = imax3(cD, up, left);
                    if (k == C - 1) tail = up;
                }
                diag = up;
                V[k] = v;
                left = v;
            }
            // lane 63 appends its last column's value of the previous step; in the
            // V domain that value is taken as cU = V + 1, whose register is free
            // now, and the 1 comes off when the group's outputs are stored
            R = dpp_from_right(tail, R);
            Dg = Lr;
        }
        __builtin_amdgcn_sched_barrier(0);  // keep the refill's wait after the steps
        // Group end.  Take this group's refill, then issue the next group's
        // boundary load before this group's stores: vector-memory operations
        // retire in order, so a load queued behind a device-coherent store
        // would make the next refill wait for that store's round trip.
        if (__builtin_amdgcn_ballot_w64(!io.ready(Rin, rin, lane < 16)) != 0)
            Rin = wait_slot(io, rin, lane < 16);
        const int32_t refill = io.value(Rin, rin);
        rin += 16;
        Rin = io.load(rin, lane < 16);
        __builtin_amdgcn_sched_barrier(0);
        if constexpr (DIRS) {
            uint32_t* dst = dirs + ((size_t)g * kWave + lane) * C;
#pragma unroll
            for (int k = 0; k < C; ++k) dst[k] = acc[k];
        }
        {
            const int r = 16 * g + lane - 111;
            io.store(r, DIRS ? R - 1 : R, lane >= 48 && r >= 1 && r <= m);
        }
        R = (lane < 16) ? refill : R;
    }
    int32_t out = V[0];
#pragma unroll
    for (int k = 1; k < C; ++k)
        if (k == ksel) out = V[k];
    return out;
}

// Cached access to the stored direction words of one pair: a window of
// 4 groups x 16 lanes x C words in LDS, anchored at the top-right (latest
// group, highest lane) of the last miss, which suits walks that move to
// lower steps and lower lanes.  Every lane of the wave calls tag() with the
// same cell and gets the same (wave-uniform) answer.
//
// For a band, strip s swept grid rows r0(s)+1 .. with r0(s) =
// max(0, s*64*C - band_hi) and every strip has G groups of storage.
template <int C>
struct DirWindow {
    const uint32_t* dirs;
    int G;
    uint32_t* lds;  // >= 64*C words
    int band_hi;
    int sw, gw, lw;
    __device__ __forceinline__ DirWindow(const uint32_t* d, int groups, uint32_t* l, int bhi = 1 << 30)
        : dirs(d), G(groups), lds(l), band_hi(bhi), sw(-1), gw(0), lw(0) {}
    // 2-bit tag of interior cell (i, j), 1 <= i, 1 <= j (3 diagonal, 2 vertical,
    // 1 horizontal; 0 means corrupt data)
    __device__ __forceinline__ int tag(int i, int j) {
        constexpr int kCols = kWave * C;
        const int col0 = j - 1;
        const int s = col0 / kCols;
        const int w = col0 - s * kCols;
        const int l = w / C;
        const int k = w - l * C;
        const int r0 = max(0, s * kCols - band_hi);
        const int t = i - r0 - 1 + l;
        const int g = t >> 4;
        if (s != sw || g > gw || g < gw - 3 || l > lw || l < lw - 15) {
            sw = s;
            gw = g;
            lw = l;
            const int lane = lane_id();
            const int gq = gw - 3 + (lane >> 4);
            const int lq = lw - 15 + (lane & 15);
            if (gq >= 0 && lq >= 0) {
                const uint32_t* src = dirs + (((size_t)sw * G + gq) * kWave + lq) * C;
#pragma unroll
                for (int kk = 0; kk < C; ++kk) lds[lane * C + kk] = src[kk];
            }
            __builtin_amdgcn_wave_barrier();
        }
        const int slot = ((g - gw + 3) << 4) + (l - lw + 15);
        const uint32_t word = (uint32_t)uniform((int32_t)lds[slot * C + k]);
        return (int)((word >> (2 * (t & 15))) & 3u);
    }
};

// Walk the stored directions of one pair from (m, n) back to (0, 0), one wave,
// through a small LDS window of 4 groups x 16 lanes x C words anchored at the
// current cell.  rev[q] gets the q-th move counted from the end.  Returns the
// number of moves, or -1 if a stored tag is invalid.
template <int C>
__device__ __forceinline__ int64_t walk_back(const uint32_t* __restrict__ dirs, int m, int n,
                                             int groups_per_strip, uint32_t* lds,
                                             uint8_t* __restrict__ rev, int band_hi = 1 << 30) {
    const int lane = lane_id();
    int i = m, j = n;
    int64_t q = 0;
    DirWindow<C> win(dirs, groups_per_strip, lds, band_hi);
    while (i > 0 && j > 0) {
        const int tag = win.tag(i, j);
        if (tag == 0) return -1;
        const int mv = 4 - tag;
        rev[q] = (uint8_t)mv;  // every lane stores the same byte
        ++q;
        if (mv == 1) {
            --i;
            --j;
        } else if (mv == 2) {
            --i;
        } else {
            --j;
        }
    }
    // first column: vertical moves; first row: horizontal moves
    for (int x = lane; x < i; x += kWave) rev[q + x] = 2;
    q += i;
    for (int x = lane; x < j; x += kWave) rev[q + x] = 3;
    q += j;
    return q;
}

}  // namespace nw
