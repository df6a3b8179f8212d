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
