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
// is the strip's right boundary for the next strip.  The sweep runs in groups
// of kGroup = 32 steps: at a group's end lanes 32..63 (the last 32 outputs)
// are written out and lanes 0..31 are refilled with the next 32 inputs, so
// inputs are needed just one group ahead.  Group-end bookkeeping (refill,
// output, table upkeep, stores) is paid once per 32 steps.
//
// Boundary columns travel through an IO policy: PlainIO for a wave that
// sweeps all strips of a pair itself, CoopIO when neighbouring strips run on
// different waves (see the cooperative kernel).
//
// The substitution term comes from a per-row table in LDS (a circular buffer,
// see kTabRows): for row i the word holds four signed bytes, byte y =
// term(a_i == y).  Lane (l, k) reads byte
// b_j of the row it is on with one ds_read_i8.  Rows outside 1..m hold -128,
// which freezes the lanes that are above or below the matrix (see
// nw_common.h), so the sweep needs no per-lane predicates.
//
// Directions: each lane shifts the 2-bit tag of every cell of column k into a
// 32-bit accumulator, one per 16 steps (two per group); lane l stores its C
// words of each half contiguously, giving the layout
//   dirs[strip][16-step group g][lane l][column k]
// (one word per 16 consecutive steps of one column).  Step t of lane l is
// row t - l + 1, so cell (i, j) lives in word (g = (i-1+l) / 16) at bits
// 2*((i-1+l) % 16).
#pragma once

#include "nw_common.h"

namespace nw {

constexpr int kGroup = 32;  // steps per group

// Row table: a circular LDS buffer of kTabRows row words (row i at index
// i & (kTabRows - 1)) followed by a copy of its first kGroup words, so the
// kGroup rows one lane reads in a group are always contiguous and the
// per-step offsets fold into the ds_read immediates.  Rows outside 1..m hold
// the sentinel word.  Word kTabSpare takes the writes of lanes with nothing
// to write.
constexpr int kTabRows = 256;
constexpr int kTabSpare = kTabRows + kGroup;
constexpr int kTabWords = kTabSpare + 1;

template <int C>
struct StripShape {
    static constexpr int kCols = kWave * C;
    // LDS words per wave: the row table, or the traceback window
    static constexpr int kLdsWords = (kTabWords > 64 * C) ? kTabWords : 64 * C;
};

// Lane 63 finishes row m at step m + 62, and its value enters the queue in
// step m + 63, which must lie in a group that the loop runs (the group's end
// flushes it).  So the sweep runs floor((m + 63) / 32) + 1 groups, and stores
// twice as many 16-step direction words per column.
__host__ __device__ __forceinline__ int sweep_groups(int m) { return (m + 95) >> 5; }
__host__ __device__ __forceinline__ int groups_for_rows(int m) { return 2 * sweep_groups(m); }  // 16-step units

// Group-end memory traffic is issued by every lane without a branch: lanes
// with nothing to load or store use a spare slot.  Vector memory operations
// of a wave retire in order and stores count in the same counter as loads,
// so with a branch around a store the compiler cannot tell how many
// operations follow a load and waits for all of them (vmcnt(0)); branch-free
// issue lets it wait for exactly the load a refill needs, and the previous
// group's stores stay in flight behind the steps.

// Boundary IO for a wave that owns every strip of its pair: the previous
// strip's right column sits in the wave's own scratch (bin, indexed by grid
// row), the next strip's goes to the same buffer (bout; reads of a row happen
// before its overwrite).  The sweep may cover only grid rows r0+1 .. r0+m
// (a band); its rows are numbered locally from 1.  Inputs for grid rows above
// in_hi, or beyond the sweep, lie outside the previous strip's region and
// read `beyond`, a value that never wins (0, or the -infinity sentinel of a
// band).  A missing bin means the grid's first column (vinit).  `spare` is a
// scratch slot nobody reads.
struct PlainIO {
    const int32_t* bin;
    int32_t* bout;
    int32_t* spare;
    int m;
    int32_t vinit;
    int r0 = 0;
    int in_hi = 1 << 30;
    int32_t beyond = 0;
    using Slot = int32_t;
    static constexpr int kPrefetch = 2;  // groups a refill is loaded ahead (0: read at the group end)
    __device__ __forceinline__ Slot load(int r, bool want) const {
        const bool ok = want && bin != nullptr && r <= m && r0 + r <= in_hi;
        const int32_t* src = ok ? bin + r0 + r : spare;
        return *src;
    }
    __device__ __forceinline__ int32_t value(Slot x, int r) const {
        if (r > m) return beyond;
        if (!bin) return vinit;
        return (r0 + r <= in_hi) ? x : beyond;
    }
    __device__ __forceinline__ bool ready(Slot, int, bool) const { return true; }
    __device__ __forceinline__ void store(int r, int32_t v, bool want) const {
        int32_t* dst = (want && bout != nullptr) ? bout + r0 + r : spare;
        *dst = v;
    }
    __device__ __forceinline__ void fail() const {}
    __device__ __forceinline__ bool failed() const { return false; }
    __device__ __forceinline__ int spin_limit() const { return 1; }
    __device__ __forceinline__ int room_probe() const { return 0; }
    __device__ __forceinline__ void wait_room(int, int&) const {}
    __device__ __forceinline__ void mark_consumed(int) const {}
};

typedef __attribute__((address_space(3))) uint64_t lds_u64;
typedef __attribute__((address_space(3))) int32_t lds_i32;

constexpr int kRing = 1024;  // rows per LDS boundary ring

// Boundary IO of the cooperative fill, typed by where the strip's input and
// output column live (so each wave's code waits only on the counter its
// input uses):
//   kIoNone   - no neighbour (first strip: the grid's first column; last
//               strip: no output);
//   kIoLds    - the neighbour is another wave of the same block: a ring of
//               kRing 64-bit {value, row} slots in LDS.  The reader polls until
//               the slot carries the row it wants and publishes the last row it
//               has read after each refill; the writer overwrites a slot only
//               once the row kRing below has been read;
//   kIoGlobal - the neighbour is in another block, possibly on another XCD:
//               64-bit {value, epoch} slots in HBM written with device-scope
//               stores; the reader polls until a slot carries the call's epoch.
// With KEEP, ring output is also stored plainly to the global column, which
// the traceback reads after the fill.
enum { kIoNone = 0, kIoLds = 1, kIoGlobal = 2 };

template <int IN, int OUT, bool KEEP>
struct CoopIO {
    const uint64_t* bin;  // global input column (kIoGlobal)
    uint64_t* bout;       // global output column (kIoGlobal, or KEEP)
    uint64_t* gspare;     // global slot nobody reads
    lds_u64* lin;         // LDS input ring (kIoLds)
    lds_u64* lout;        // LDS output ring (kIoLds)
    lds_u64* lspare;      // LDS slot nobody reads
    lds_i32* cin;         // last row read from the input ring (published here)
    lds_i32* cout;        // last row the output ring's reader has read
    int m;
    int32_t vinit;
    uint32_t epoch;
    int32_t* err;
    int32_t spin;  // polls before a wait gives up (the watchdog)
    using Slot = uint64_t;
    // a global refill is loaded one group (32 steps, about one L2 round trip)
    // ahead; a deeper prefetch would only add lag to the hop
    static constexpr int kPrefetch = (IN == kIoGlobal) ? 1 : 0;
    __device__ __forceinline__ Slot load(int r, bool want) const {
        const bool ok = want && r <= m;
        if constexpr (IN == kIoLds) {
            lds_u64* p = ok ? lin + (r & (kRing - 1)) : lspare;
            return *(volatile lds_u64*)p;
        } else if constexpr (IN == kIoGlobal) {
            const uint64_t* p = ok ? bin + r : gspare;
            return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        } else {
            return 0;
        }
    }
    __device__ __forceinline__ int32_t value(Slot x, int r) const {
        if (r > m) return 0;
        return IN == kIoNone ? vinit : (int32_t)(uint32_t)x;
    }
    __device__ __forceinline__ bool ready(Slot x, int r, bool want) const {
        if constexpr (IN == kIoNone) return true;
        const uint32_t tag = (IN == kIoLds) ? (uint32_t)r : epoch;
        return !(want && r <= m) || (uint32_t)(x >> 32) == tag;
    }
    __device__ __forceinline__ void store(int r, int32_t v, bool want) const {
        if constexpr (OUT == kIoLds) {
            lds_u64* p = want ? lout + (r & (kRing - 1)) : lspare;
            *(volatile lds_u64*)p = ((uint64_t)(uint32_t)r << 32) | (uint32_t)v;
            if constexpr (KEEP) {
                uint64_t* q = want ? bout + r : gspare;
                *q = ((uint64_t)epoch << 32) | (uint32_t)v;
            }
        } else if constexpr (OUT == kIoGlobal) {
            uint64_t* q = want ? bout + r : gspare;
            __hip_atomic_store(q, ((uint64_t)epoch << 32) | (uint32_t)v, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
        }
    }
    __device__ __forceinline__ void fail() const {
        __hip_atomic_store(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    __device__ __forceinline__ bool failed() const {
        return __hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0;
    }
    __device__ __forceinline__ int spin_limit() const { return spin; }
    // The output ring's reader progress, read one group before it is needed.
    __device__ __forceinline__ int room_probe() const {
        if constexpr (OUT == kIoLds) return *(volatile lds_i32*)cout;
        else return 0;
    }
    // Before rows up to r_hi go out: the ring slots they take must be free.
    // `probe` is a possibly stale (hence lower) reading of the reader's progress.
    __device__ __forceinline__ void wait_room(int r_hi, int& probe) const {
        if constexpr (OUT == kIoLds) {
            const int need = r_hi - kRing;
            probe = uniform(probe);
            if (__builtin_expect(probe >= need, 1)) return;
            for (int it = 0; probe < need; ++it) {
                if (it >= spin) {
                    fail();
                    return;
                }
                if ((it & 31) == 31 && failed()) return;
                __builtin_amdgcn_s_sleep(1);
                probe = uniform(*(volatile lds_i32*)cout);
            }
        }
    }
    // After a refill: every row up to r_hi has been read from the input ring.
    __device__ __forceinline__ void mark_consumed(int r_hi) const {
        if constexpr (IN == kIoLds) *(volatile lds_i32*)cin = r_hi;
    }
};

// Load slot r (for the lanes with `want`) until every such lane sees a ready
// slot.  The loop condition is wave-uniform.  The shared failure flag is a
// device-scope load (a round trip to L2), so it is checked only every 32 polls:
// after one wait has given up, every later wait of the call returns within 32
// polls.
template <class IO>
__device__ __forceinline__ typename IO::Slot wait_slot(const IO& io, int r, bool want) {
    typename IO::Slot x = io.load(r, want);
    const int limit = io.spin_limit();
    for (int spin = 0; spin < limit; ++spin) {
        if (__builtin_amdgcn_ballot_w64(!io.ready(x, r, want)) == 0) return x;
        if ((spin & 31) == 31 && io.failed()) return x;  // a wait gave up: drain quickly
        __builtin_amdgcn_s_sleep(1);
        x = io.load(r, want);
    }
    io.fail();
    return x;
}

// Row word of grid row r of the sweep (r in 1..m), from its byte x: the
// substitution terms of x's code (sym_code with the pair's field offset), or,
// when bytes are compared, the byte and its mismatch term (wide_word).
template <bool WIDE>
__device__ __forceinline__ uint32_t table_word(int r, int m, uint32_t x, int kdm, int kdx, uint32_t shift) {
    const bool valid = (r >= 1 && r <= m);
    if constexpr (WIDE) {
        return wide_word(valid, x, kdx);
    } else {
        // the word is computed for every lane and then selected: written as
        // one conditional expression it became a branch inside the sweep loop
        // in some builds, and the kernel's registers then spilled
        const uint32_t w = row_word(sym_code(x, shift), kdm, kdx);
        return valid ? w : kSentinelWord;
    }
}

// Write row r's word to the table (index r & 255, and its mirror copy when the
// index is below kGroup), or, for lanes with `skip`, to the spare word.
__device__ __forceinline__ void table_put(uint32_t* tab, int r, uint32_t w, bool skip) {
    const int i = r & (kTabRows - 1);
    tab[skip ? kTabSpare : i] = w;
    tab[skip ? kTabSpare : (i < kGroup ? kTabRows + i : i)] = w;
}

// Sweep one strip.  Returns, per lane, V (or W) of its column `ksel` after
// the last row (the frozen final value).  Bytes are compared through their
// codes (sym_code with the pair's field offset `shift`), or directly (WIDE).
// `a` points at the sweep's first row and `m` counts its rows (a band sweeps
// grid rows r0+1 .. r0+m with a = seq + r0).  Every lane starts from `vtop`,
// the row above the sweep (the grid's first row, or -infinity inside a band),
// except that lane 0's first diagonal input is `dg0`, the previous strip's
// last column one row above the sweep.  With STATE the lanes start instead
// from their columns' values in the row above, vst[0..C), and leave their
// values after the last row there: a strip can be swept in consecutive row
// ranges, each with or without directions (the lanes above a range's first
// row keep their values, as above the grid, because rows are monotone).
template <int C, bool DIRS, bool WIDE, class IO, bool STATE = false>
__device__ __forceinline__ int32_t sweep_strip(const uint8_t* __restrict__ a, int m,
                                               const uint8_t* __restrict__ b, int n, int j0, int kdm,
                                               int kdx, uint32_t shift, int32_t vtop, int32_t dg0, const IO& io,
                                               uint32_t* __restrict__ dirs, uint32_t* lds, int ksel,
                                               int32_t* vst = nullptr) {
    const int lane = lane_id();
    const bool lane0 = (lane == 0);
    int32_t V[C];
    uint32_t acc0[C], acc1[C];  // direction words of the group's two halves
    uint32_t bcode[C];
#pragma unroll
    for (int k = 0; k < C; ++k) {
        if constexpr (STATE) V[k] = vst[k];
        else V[k] = vtop;
        acc0[k] = 0;
        acc1[k] = 0;
        int j = j0 + C * lane + k;
        const uint32_t x = (j < n) ? (uint32_t)b[j] : 0u;
        bcode[k] = WIDE ? x : sym_code(x, shift);
    }
    uint32_t onehot[C];  // 1 in byte (code of b[j]) of column j: selects that row-word byte in v_dot4
#pragma unroll
    for (int k = 0; k < C; ++k) onehot[k] = 1u << (8 * (bcode[k] & 3u));
    int32_t Dg = lane0 ? dg0 : vtop;

    // Row table: rows -63 .. 64 serve groups 0 and 1; each group end writes the
    // rows of the group after next, from base codes loaded two groups earlier.
    for (int p = lane; p < 128; p += kWave) {
        const int r = p - 63;
        table_put(lds, r, table_word<WIDE>(r, m, (r >= 1 && r <= m) ? a[r - 1] : 0u, kdm, kdx, shift), false);
    }
    const int mc = max(m, 1);
    uint32_t pfa = a[min(max(65 + lane, 1), mc) - 1];  // rows 65..96: written at the end of group 0
    uint32_t pfb = a[min(max(97 + lane, 1), mc) - 1];  // rows 97..128: end of group 1
    __builtin_amdgcn_wave_barrier();

    int32_t R = io.value(wait_slot(io, lane + 1, lane < kGroup), lane + 1);
    // Refill of lanes 0..31 at the end of group g: rows 32g + 33 + lane.  The
    // group loop runs in pairs so that even groups keep their prefetched
    // refill and table bytes in one set of registers and odd groups in
    // another, each reloaded in place two groups ahead: a loop-carried copy of
    // a register with a load in flight would make the compiler wait for it.
    int rin = kGroup + 1 + lane;
    typename IO::Slot RinA = 0, RinB = 0;
    if constexpr (IO::kPrefetch >= 1) RinA = io.load(rin, lane < kGroup);
    if constexpr (IO::kPrefetch == 2) RinB = io.load(rin + kGroup, lane < kGroup);
    int probe = io.room_probe();

    const int NG = sweep_groups(m);

    // 16 steps starting at step 32g + 16h, tags into acc[]
    auto half = [&](const int g, const int h, uint32_t (&acc)[C]) {
        // word index of the row of the half's first step for this lane; the
        // per-step offsets u fold into the ds_read immediate
        const uint32_t base = (uint32_t)((kGroup * g + 16 * h - lane + 1) & (kTabRows - 1));

        // Narrow strips have too little work per step to hide the LDS latency
        // behind other waves, so the half's table reads are issued up front;
        // wide strips read one step at a time.  Each step reads one row word
        // (the four substitution terms of the row's base); v_dot4 with the
        // column's one-hot b-code picks its term and adds the diagonal.
        constexpr bool kHoist = (C <= 2);
        uint32_t rwh[kHoist ? 16 : 1];
        if constexpr (kHoist) {
#pragma unroll
            for (int u = 0; u < 16; ++u) rwh[u] = lds[base + u];
        }

#pragma unroll
        for (int u = 0; u < 16; ++u) {
            const int32_t Lr = shift_in_from_left(R, V[C - 1], lane0);
            int32_t left = Lr;
            int32_t diag = Dg;
            int32_t tail = 0;  // the last column's previous value (+1 in the V domain)
            uint32_t rw;
            if constexpr (kHoist) rw = rwh[u];
            else rw = lds[base + u];
            // wide alphabets: the row's byte and its mismatch term
            const uint32_t rbyte = rw & 0x1FFu;
            const int32_t rmis = (int32_t)rw >> 9;
#pragma unroll
            for (int k = 0; k < C; ++k) {
                const int32_t up = V[k];
                int32_t cD;
                if constexpr (WIDE) cD = diag + ((rbyte == bcode[k]) ? kdm : rmis);
                else cD = __builtin_amdgcn_sdot4((int)rw, (int)onehot[k], diag, false);
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
    };

    auto store_dirs = [&](uint32_t* dst, const uint32_t (&acc)[C]) {
        // a lane's C words are contiguous (and 4C-byte aligned): store them with
        // the widest stores that fit
        if constexpr (C % 4 == 0) {
#pragma unroll
            for (int k = 0; k < C; k += 4)
                *reinterpret_cast<uint4*>(dst + k) = make_uint4(acc[k], acc[k + 1], acc[k + 2], acc[k + 3]);
        } else if constexpr (C == 2) {
            *reinterpret_cast<uint2*>(dst) = make_uint2(acc[0], acc[1]);
        } else {
#pragma unroll
            for (int k = 0; k < C; ++k) dst[k] = acc[k];
        }
    };

    // Rin: this group's refill; Rnext: the next group's (the other parity's
    // register, loaded here when the prefetch is one group deep)
    auto group = [&](const int g, typename IO::Slot& Rin, typename IO::Slot& Rnext, uint32_t& pf) {
        half(g, 0, acc0);
        half(g, 1, acc1);
        __builtin_amdgcn_sched_barrier(0);  // keep the refill's wait after the steps
        // Group end: issue a fresh refill read, do the stores (all branch-free),
        // then take the refill and issue the loads of later groups.  The
        // outputs go out before the wait for input, so a wave that waits
        // holds up nobody downstream.
        if constexpr (IO::kPrefetch == 0) Rin = io.load(rin, lane < kGroup);
        {
            const int r = kGroup * g + 2 * kGroup + 1 + lane;  // table rows of group g + 2
            table_put(lds, r, table_word<WIDE>(r, m, pf, kdm, kdx, shift), lane >= kGroup);
            pf = a[min(max(r + 2 * kGroup, 1), mc) - 1];  // rows of group g + 4, written at the end of g + 2
        }
        if constexpr (DIRS) {
            store_dirs(dirs + ((size_t)(2 * g) * kWave + lane) * C, acc0);
            store_dirs(dirs + ((size_t)(2 * g + 1) * kWave + lane) * C, acc1);
        }
        {
            // lanes 32..63 hold the group's outputs: rows 32g - 63 .. 32g - 32
            const int r = kGroup * g + lane - 95;
            io.wait_room(kGroup * g - 32, probe);
            io.store(r, DIRS ? R - 1 : R, lane >= kGroup && r >= 1 && r <= m);
            probe = io.room_probe();
        }
        __builtin_amdgcn_sched_barrier(0);
        if (__builtin_expect(__builtin_amdgcn_ballot_w64(!io.ready(Rin, rin, lane < kGroup)) != 0, 0))
            Rin = wait_slot(io, rin, lane < kGroup);
        const int32_t refill = io.value(Rin, rin);
        // rin is per lane (rin + lane); the refill ends at lane 31's row
        io.mark_consumed(uniform(rin) + kGroup - 1);
        if constexpr (IO::kPrefetch == 1) Rnext = io.load(rin + kGroup, lane < kGroup);
        if constexpr (IO::kPrefetch == 2) Rin = io.load(rin + 2 * kGroup, lane < kGroup);
        rin += kGroup;
        R = (lane < kGroup) ? refill : R;
    };
    int g = 0;
    for (; g + 1 < NG; g += 2) {
        group(g, RinA, RinB, pfa);
        group(g + 1, RinB, RinA, pfb);
    }
    if (g < NG) group(g, RinA, RinB, pfa);
    if constexpr (STATE) {
#pragma unroll
        for (int k = 0; k < C; ++k) vst[k] = V[k];
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

// Walk the stored directions of one pair from (m, n) back to (0, 0), one wave.
// The walk is one dependent chain of lookups, so it runs on wave-uniform
// scalar state.  Optimal paths are mostly diagonal, so the 64 lanes read the
// tags of the next 64 diagonal cells at once and the walk takes a whole run of
// diagonal moves in one step; every other move costs a few scalar operations
// and one v_readlane:
//  - the cell's strip s, lane l, column k and step t = i - r0(s) - 1 + l are
//    kept up to date move by move, without divisions (tags 2 and 3 step up a
//    row, tags 1 and 3 step left a column);
//  - the direction words come from a window of 4 groups x 16 lanes x C words
//    anchored at (group gw, lane lw) as its top-right corner and held flat in
//    C VGPRs: word x = ((g-gw+3)*16 + l-lw+15)*C + k sits in lane x % 64 of
//    register x / 64.  A move reads it from a copy of the current register,
//    which changes only when x crosses a 64-word boundary.  The walk only
//    moves up and left, so it leaves the window through its lowest group, its
//    leftmost lane or into the previous strip; then the window is reloaded
//    around the current cell;
//  - moves collect one per lane in a VGPR and go out 64 bytes at a time.
// The lane index is computed here, not shared with the fill: values derived
// from it would otherwise be hoisted to the kernel's start and held in VGPRs
// across the sweeps.  rev[q] gets the q-th move counted from the end.
// Returns the number of moves, or -1 if a stored tag is invalid.
//
// For a band, strip s swept grid rows r0(s)+1 .. with r0(s) =
// max(0, s*64*C - band_hi) and every strip has G groups of storage.
// CHECKED: the directions cover only rows r0(s)+1 .. min(m, (s+1)*64*C +
// span_lo) of each strip; a walk that would leave them returns -3 before it
// reads outside (the caller then records directions over a wider region).
template <int C, bool CHECKED = false>
__device__ __forceinline__ int64_t walk_back(const uint32_t* __restrict__ dirs, int m, int n,
                                             int groups_per_strip, uint32_t* /*lds*/,
                                             uint8_t* __restrict__ rev, int band_hi = 1 << 30,
                                             int span_lo = 1 << 30) {
    constexpr int kCols = kWave * C;
    constexpr int kLogC = (C == 8) ? 3 : (C == 4) ? 2 : (C == 2) ? 1 : 0;
    int lane;
    asm volatile("v_mbcnt_lo_u32_b32 %0, -1, 0\n\tv_mbcnt_hi_u32_b32 %0, -1, %0" : "=v"(lane));
    const int G = groups_per_strip;
    int i = m, j = n;
    int64_t q = 0;
    uint32_t win[C];
#pragma unroll
    for (int r = 0; r < C; ++r) win[r] = 0;
    uint32_t buf = 0;
    // the lookahead tree: lane 1 + d after move d + 1 (1 L, 2 U, 3 D), lane
    // 4 + 3*d0 + d1 after two, lane 13 + 9*d0 + 3*d1 + d2 after three (digits
    // d = tag - 1); la, lb: rows and columns the lane's moves take
    int lvl = 4, la = 0, lb = 0;
    {
        int dg[3] = {-1, -1, -1};
        if (lane == 0) {
            lvl = 0;
        } else if (lane < 4) {
            lvl = 1;
            dg[0] = lane - 1;
        } else if (lane < 13) {
            lvl = 2;
            dg[0] = (lane - 4) / 3;
            dg[1] = (lane - 4) % 3;
        } else if (lane < 40) {
            lvl = 3;
            dg[0] = (lane - 13) / 9;
            dg[1] = ((lane - 13) / 3) % 3;
            dg[2] = (lane - 13) % 3;
        }
#pragma unroll
        for (int e = 0; e < 3; ++e) {
            if (dg[e] >= 0) {
                la += (dg[e] + 1) >> 1;
                lb += (dg[e] + 1) & 1;
            }
        }
    }
    while (i > 0 && j > 0) {
        const int col0 = j - 1;
        const int s = col0 / kCols;
        int l = (col0 - s * kCols) >> kLogC;
        int k = (col0 - s * kCols) & (C - 1);
        const int r0s = max(0, s * kCols - band_hi);
        if constexpr (CHECKED) {
            if (i <= r0s || i > min(m, s * kCols + kCols + span_lo)) return -3;
        }
        int t = i - r0s - 1 + l;
        const int gw = t >> 4, lw = l;
#pragma unroll
        for (int r = 0; r < C; ++r) {
            const int x = kWave * r + lane;
            const int gq = gw - 3 + (x >> (4 + kLogC));
            const int lk = x & (16 * C - 1);
            if (gq >= 0 && (lw - 15) * C + lk >= 0)
                win[r] = dirs[((size_t)s * G + gq) * kCols + (lw - 15) * C + lk];
        }
        const int tmin = 16 * (gw - 3), lmin = max(lw - 15, 0);
        const int xo = ((3 - gw) << (4 + kLogC)) + ((15 - lw) << kLogC);
        bool diag = true;
        for (;;) {
            if (diag) {
                // Diagonal run (tried at a new window and after a diagonal
                // move, so runs of gap moves pay nothing for it): lane d reads
                // the tag of the cell d diagonal moves on (from the window,
                // across lanes with ds_bpermute); the moves up to the first
                // lane that does not hold a diagonal tag inside the window
                // are all diagonal.
                const int c = (l << kLogC) + k;
                const int cd = c - lane;
                const int ld = cd >> kLogC, kd = cd & (C - 1);
                const int td = t - lane - (l - ld);
                const bool inside = cd >= 0 && ld >= lmin && td >= tmin && td >= 0 && i - lane >= 1 &&
                                    j - lane >= 1 && (!CHECKED || i - lane > r0s);
                const int xd = ((td >> 4) << (4 + kLogC)) + (ld << kLogC) + kd + xo;
                uint32_t wd = 0;
#pragma unroll
                for (int r = 0; r < C; ++r) {
                    const uint32_t v = (uint32_t)__builtin_amdgcn_ds_bpermute((xd & 63) << 2, (int)win[r]);
                    wd = ((xd >> 6) == r) ? v : wd;
                }
                const uint32_t tagd = inside ? (wd >> (2 * (td & 15))) & 3u : 0u;
                const uint64_t stop = __builtin_amdgcn_ballot_w64(tagd != 3u);
                const int run = stop ? __builtin_ctzll(stop) : kWave;
                if (run > 0) {
                    const int q0 = (int)(q & 63);
                    const int e1 = min(kWave, q0 + run);
                    buf = (lane >= q0 && lane < e1) ? 1u : buf;
                    if (e1 == kWave) rev[(q & ~(int64_t)63) + lane] = (uint8_t)buf;
                    const int rest = q0 + run - kWave;
                    if (rest > 0) buf = (lane < rest) ? 1u : buf;
                    q += run;
                    i -= run;
                    j -= run;
                    const int cn = c - run;
                    const int ln = cn >> kLogC;
                    t -= run + (l - ln);
                    l = ln;
                    k = cn & (C - 1);
                    if constexpr (CHECKED) {
                        if ((i > 0) & (i <= r0s)) return -3;
                    }
                    if ((i <= 0) | (j <= 0) | (t < tmin) | (l < lmin)) break;
                }
            }
            // Lookahead round: lane 0 holds the current cell, lanes 1..39 the
            // cells one, two and three moves on along every possible move
            // sequence (la, lb: the rows and columns the lane's moves take).
            // Each lane reads its cell's tag from the window (ds_bpermute);
            // four dependent v_readlanes then follow the actual path for up
            // to four moves, stopping at a cell outside the window.
            const int c = (l << kLogC) + k;
            const int cd = c - lb;
            const int ld = cd >> kLogC, kd = cd & (C - 1);
            const int td = t - la - (l - ld);
            const bool ok = lvl < 4 && cd >= 0 && ld >= lmin && td >= tmin && td >= 0 && i - la >= 1 &&
                            j - lb >= 1 && (!CHECKED || i - la > r0s);
            const int xd = ((td >> 4) << (4 + kLogC)) + (ld << kLogC) + kd + xo;
            uint32_t wd = 0;
#pragma unroll
            for (int r = 0; r < C; ++r) {
                const uint32_t v = (uint32_t)__builtin_amdgcn_ds_bpermute((xd & 63) << 2, (int)win[r]);
                wd = ((xd >> 6) == r) ? v : wd;
            }
            const int tg = ok ? (int)((wd >> (2 * (td & 15))) & 3u) : 0;
            const int t0 = __builtin_amdgcn_readlane(tg, 0);
            if (__builtin_expect(t0 == 0, 0)) return -1;  // the current cell is always in the window
            const int t1 = __builtin_amdgcn_readlane(tg, t0);
            const int t2 = __builtin_amdgcn_readlane(tg, 3 * t0 + t1);
            const int t3 = __builtin_amdgcn_readlane(tg, 9 * t0 + 3 * t1 + t2);
            const int nres = (t1 == 0) ? 1 : (t2 == 0) ? 2 : (t3 == 0) ? 3 : 4;
            const int s1 = nres > 1 ? t1 : 0, s2 = nres > 2 ? t2 : 0, s3 = nres > 3 ? t3 : 0;
            const int a = (t0 >> 1) + (s1 >> 1) + (s2 >> 1) + (s3 >> 1);
            const int b = (t0 & 1) + (s1 & 1) + (s2 & 1) + (s3 & 1);
            {
                // moves q .. q+nres-1 go to lanes (q+d) % 64, the block flushed
                // once it fills
                const int q0 = (int)(q & 63);
                const int dd = (lane - q0) & 63;
                const uint32_t mv = (uint32_t)(4 - (dd == 0 ? t0 : dd == 1 ? t1 : dd == 2 ? t2 : t3));
                const int e1 = min(kWave, q0 + nres);
                buf = (lane >= q0 && lane < e1) ? mv : buf;
                if (e1 == kWave) rev[(q & ~(int64_t)63) + lane] = (uint8_t)buf;
                buf = (lane < q0 + nres - kWave) ? mv : buf;
                q += nres;
            }
            diag = (nres == 1 ? t0 : nres == 2 ? t1 : nres == 3 ? t2 : t3) == 3;
            i -= a;
            j -= b;
            const int cn = c - b;
            const int ln = cn >> kLogC;
            t -= a + (l - ln);
            l = ln;
            k = cn & (C - 1);
            if constexpr (CHECKED) {
                if ((i > 0) & (i <= r0s)) return -3;
            }
            if ((i <= 0) | (j <= 0) | (t < tmin) | (l < lmin)) break;
        }
    }
    if ((q & 63) != 0 && lane < (int)(q & 63)) rev[(q & ~(int64_t)63) + lane] = (uint8_t)buf;
    for (int x = lane; x < i; x += kWave) rev[q + x] = 2;
    q += i;
    for (int x = lane; x < j; x += kWave) rev[q + x] = 3;
    q += j;
    return q;
}

}  // namespace nw
