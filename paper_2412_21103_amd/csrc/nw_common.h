// Shared device-side definitions for the libnw kernels (gfx950, wave64).
//
// Value domain.  The fill keeps, for every cell, an offset score
//     V(i,j) = 4*(H(i,j) - gap*(i+j)) + 1           (direction-recording fill)
//     W(i,j) =    H(i,j) - gap*(i+j)                (score-only fill)
// Both domains make the first row and column constant (V = 1, W = 0; paper
// Sec. 2.2) and turn the recurrence of Sec. 2.3 (Eq. 1, linear gap) into
//     W(i,j) = max( W(i-1,j-1) + (s - 2*gap), W(i-1,j), W(i,j-1) )
// so the horizontal candidate needs no add.  In the V domain the two low bits
// carry a tie-break tag: the diagonal candidate V(i-1,j-1) + 4(s-2gap) + 2 ends
// in 3, the vertical candidate V(i-1,j) + 1 ends in 2 and the horizontal
// candidate V(i,j-1) ends in 1, so one signed max3 returns the best score and,
// among equal scores, the first of diagonal > vertical > horizontal.  The tag
// t gives the paper's direction code 4 - t (Sec. 3.1: 1 diagonal, 2 vertical,
// 3 horizontal).  Clearing the tag to 1 gives the cell's own V.
//
// Both domains are monotone along a row (V(i,j) >= V(i,j-1) because
// H(i,j) >= H(i,j-1) + gap), which the kernels use to freeze lanes outside the
// matrix: a substitution term of -128 makes the vertical candidate win, and
// the vertical candidate reproduces the lane's own value.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace nw {

constexpr int kWave = 64;
constexpr int8_t kSentinelKd = -128;          // substitution term outside 1..m
constexpr uint32_t kSentinelWord = 0x80808080u;

// DPP controls (GFX9 encoding)
constexpr int kDppWaveShl1 = 0x130;  // lane l <- lane l+1
constexpr int kDppWaveShr1 = 0x138;  // lane l <- lane l-1

__device__ __forceinline__ int32_t dpp_from_left(int32_t old, int32_t src) {
    // lanes 1..63 take src of lane-1; lane 0 keeps old
    return __builtin_amdgcn_update_dpp(old, src, kDppWaveShr1, 0xF, 0xF, false);
}

// Lane 0 takes `first`; lanes 1..63 take src of lane-1.  Written as a
// zero-filled DPP shift and a lane-0 select so the compiler can fold both into
// one v_cndmask_b32 with a DPP source (no copy of `first` is needed).
__device__ __forceinline__ int32_t shift_in_from_left(int32_t first, int32_t src, bool lane0) {
    const int32_t sh = __builtin_amdgcn_update_dpp(0, src, kDppWaveShr1, 0xF, 0xF, true);
    return lane0 ? first : sh;
}

__device__ __forceinline__ int32_t dpp_from_right(int32_t old, int32_t src) {
    // lanes 0..62 take src of lane+1; lane 63 keeps old
    return __builtin_amdgcn_update_dpp(old, src, kDppWaveShl1, 0xF, 0xF, false);
}

__device__ __forceinline__ int32_t imax3(int32_t a, int32_t b, int32_t c) {
    return max(max(a, b), c);
}

__device__ __forceinline__ uint32_t shift_in_tag(uint32_t r, uint32_t acc) {
    // (acc >> 2) | (r << 30): the newest tag enters at bits 31:30
    return __builtin_amdgcn_alignbit(r, acc, 2u);
}

// (r & ~3) | 1 as one v_and_or_b32.  Written as asm so the compiler keeps the
// cell value in this form instead of also materialising (r & ~3) | 2 for the
// vertical candidate, which costs an extra instruction per cell.
__device__ __forceinline__ int32_t clear_tag(int32_t r) {
    int32_t v;
    asm("v_and_or_b32 %0, %1, -4, 1" : "=v"(v) : "v"(r));
    return v;
}

__device__ __forceinline__ int lane_id() { return __lane_id(); }

__device__ __forceinline__ int32_t uniform(int32_t x) {
    return __builtin_amdgcn_readfirstlane(x);
}

// Row table word for symbol code x: byte y = (x == y ? kdm : kdx).
__device__ __forceinline__ uint32_t row_word(uint32_t x, int32_t kdm, int32_t kdx) {
    uint32_t base = (uint32_t)(kdx & 0xFF) * 0x01010101u;
    return base ^ ((uint32_t)((kdm ^ kdx) & 0xFF) << (8u * (x & 3u)));
}

// Symbol codes.  Only equality of bytes matters (a match or a mismatch), and
// the substitution lookup above handles four codes.  A pair whose bytes take
// at most four distinct values that one two-bit field, bits k and k+1, tells
// apart is swept with code (x >> k) & 3: k = 0 for nucleotide codes 0..3,
// k = 1 for the letters ACGT, ACGU or acgt.  Other pairs compare bytes.
__device__ __forceinline__ uint32_t sym_code(uint32_t x, uint32_t shift) { return (x >> shift) & 3u; }

// The field offset k for a pair from its two byte-presence masks (eight words
// each, bit x set when byte x occurs), or -1 if the pair needs the
// byte-comparing sweep (more than four distinct bytes, or no separating field).
__device__ __forceinline__ int code_shift(const uint32_t* ma, const uint32_t* mb) {
    uint32_t sy = 0;  // up to four distinct bytes, one per byte of sy
    int count = 0;
    for (int i = 0; i < 8; ++i) {
        uint32_t u = ma[i] | mb[i];
        while (u != 0) {
            if (count == 4) return -1;
            sy |= (32u * (uint32_t)i + (uint32_t)__builtin_ctz(u)) << (8 * count);
            ++count;
            u &= u - 1;
        }
    }
    for (int k = 0; k < 7; ++k) {
        uint32_t seen = 0;
#pragma unroll
        for (int c = 0; c < 4; ++c)
            if (c < count) seen |= 1u << (((sy >> (8 * c)) >> k) & 3u);
        if (__popc(seen) == count) return k;
    }
    return -1;
}

// Pairs with more than four distinct bytes compare bytes instead.  The row
// word holds the row's byte in bits 0..8 (0x100 outside 1..m, which equals no
// byte) and, above them, the term a mismatch adds: kdx, or -128 outside 1..m
// (which freezes the lane as above).  A cell's diagonal candidate is then
// diag + (byte == b_j ? kdm : that term).
__device__ __forceinline__ uint32_t wide_word(bool valid, uint32_t x, int32_t kdx) {
    return valid ? ((x & 0xFFu) | ((uint32_t)kdx << 9)) : (0x100u | ((uint32_t)(int32_t)kSentinelKd << 9));
}

// Byte-presence mask (eight words, bit x for byte x) of bytes p[0..len), by
// one wave; the result is in lane l's `mask` for l < 8.  One pass ORs the
// bytes (16 at a time where the address allows); if they are all nucleotide
// codes 0..3 the mask lists all four (a superset, which still gives the field
// offset 0), otherwise a second pass sets each byte's bit in `bits` (eight LDS
// words of this wave).
__device__ __forceinline__ uint32_t chunk_mask(const uint8_t* p, int64_t len, uint32_t* bits) {
    const int lane = lane_id();
    uint32_t acc = 0;
    const int64_t head = min(len, (int64_t)((16u - ((uint32_t)(uintptr_t)p & 15u)) & 15u));
    if (lane < head) acc |= p[lane];
    const uint4* q = reinterpret_cast<const uint4*>(p + head);
    const int64_t nvec = (len - head) >> 4;
    for (int64_t v = lane; v < nvec; v += kWave) {
        const uint4 x = q[v];
        acc |= x.x | x.y | x.z | x.w;
    }
    const int64_t tail0 = head + (nvec << 4);
    if (tail0 + lane < len) acc |= p[tail0 + lane];
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) acc |= (uint32_t)__shfl_xor((int32_t)acc, d);
    if ((acc & 0xFCFCFCFCu) == 0) return lane == 0 ? 0xFu : 0u;
    if (lane < 8) bits[lane] = 0;
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    for (int64_t x = lane; x < len; x += kWave) {
        const uint32_t c = p[x];
        atomicOr(&bits[c >> 5], 1u << (c & 31u));
    }
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    return lane < 8 ? bits[lane] : 0u;
}

// The mask of a whole sequence by one wave, stored to out[0..8).
__device__ __forceinline__ void seq_mask(const uint8_t* p, int64_t len, uint32_t* out, uint32_t* bits) {
    const uint32_t m = chunk_mask(p, len, bits);
    if (lane_id() < 8) out[lane_id()] = m;
}

// Coherent (L1-bypassing) load of data written earlier by this or another
// wave on the same device.
__device__ __forceinline__ int32_t load_coherent(const int32_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint32_t load_coherent_u32(const uint32_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Record a device fault in the host-visible fault word (if the library has
// one): the next call on this device returns NW_EDEVICE.
__device__ __forceinline__ void report_fault(uint32_t* fault) {
    if (fault) __hip_atomic_store(fault, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}

__device__ __forceinline__ void fence_agent() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
}

}  // namespace nw
