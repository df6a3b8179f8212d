// Center-star multiple alignment (the paper's multiple-alignment extension,
// Sec. 3.2): the center is the sequence whose scores against all others sum
// highest (lowest index on ties), every other sequence is aligned to it by
// the batch engine (center in the rows), and the pairwise alignments are
// merged with the aligned center as the reference.
//
// The merge keeps every gap of every pairwise alignment: before center
// residue p (p = 0..Lc, slot Lc after the last residue) the alignment has as
// many columns as the longest insertion any sequence makes there, each row's
// inserted residues fill the first columns of that slot, and every column a
// row does not fill is a gap.  Merging the pairwise alignments one after
// another, each new insertion filling a free insertion column before opening
// a new one, gives exactly this alignment in any order; the kernels build it
// directly:
//   k_colsum / k_argmax  - off-diagonal score sums (column sums of the
//                          symmetric matrix, coalesced) and the center;
//   k_pairs              - the batch descriptors (center, sequence k);
//   (batch engine)       - scores and forward move strings;
//   k_ins                - per slot, the longest insertion (one wave per pair,
//                          a wave-wide scan over its moves, atomicMax per run);
//   k_cols               - prefix sums: first column of each slot and column
//                          of each center residue, and the width;
//   k_msa_fill / k_msa_center / k_msa_emit - gap-fill the rows, place the
//                          center's residues and every other row's residues.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "nw_common.h"
#include "nw_internal.h"

namespace nw {

namespace {

constexpr int kMoveD = 1, kMoveU = 2, kMoveL = 3;

__global__ void k_zero32(int32_t* p, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0;
}

__global__ void k_colsum(int32_t nseq, const int32_t* __restrict__ S, int64_t* __restrict__ sums) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nseq) return;
    int64_t t = 0;
    for (int j = 0; j < nseq; ++j)
        if (j != i) t += S[(int64_t)j * nseq + i];
    sums[i] = t;
}

// One block: the index of the largest sum, the lowest on ties.
__global__ __launch_bounds__(1024) void k_argmax(int32_t nseq, const int64_t* __restrict__ sums,
                                                 int32_t* __restrict__ center, int32_t* __restrict__ center_out) {
    __shared__ int64_t bv[1024];
    __shared__ int32_t bi[1024];
    int64_t v = INT64_MIN;
    int32_t idx = INT32_MAX;
    for (int i = threadIdx.x; i < nseq; i += blockDim.x) {
        if (sums[i] > v) {  // i increases within a thread, so > keeps the lowest index
            v = sums[i];
            idx = i;
        }
    }
    bv[threadIdx.x] = v;
    bi[threadIdx.x] = idx;
    __syncthreads();
    for (int d = blockDim.x / 2; d > 0; d >>= 1) {
        if ((int)threadIdx.x < d) {
            const int64_t ov = bv[threadIdx.x + d];
            const int32_t oi = bi[threadIdx.x + d];
            if (ov > bv[threadIdx.x] || (ov == bv[threadIdx.x] && oi < bi[threadIdx.x])) {
                bv[threadIdx.x] = ov;
                bi[threadIdx.x] = oi;
            }
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const int32_t c = nseq > 0 ? bi[0] : 0;
        center[0] = c;
        if (center_out) center_out[0] = c;
    }
}

struct PairArgs {
    int32_t nseq;
    const int64_t* off;
    const int32_t* len;
    const int32_t* center;
    int64_t path_stride;
    int64_t* a_off;
    int32_t* a_len;
    int64_t* b_off;
    int32_t* b_len;
    int64_t* path_off;
    int32_t* row;
};

__global__ void k_pairs(PairArgs P) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= P.nseq - 1) return;
    const int c = P.center[0];
    const int k = q < c ? q : q + 1;
    P.a_off[q] = P.off[c];
    P.a_len[q] = P.len[c];
    P.b_off[q] = P.off[k];
    P.b_len[q] = P.len[k];
    P.path_off[q] = (int64_t)q * P.path_stride;
    P.row[q] = k;
}

// Per chunk of 64 moves of a path (lane = move): how many center residues
// the moves before it consumed (slot), how many b residues (j), and where
// its run of insertions began.  Carries move from chunk to chunk.
struct MoveScan {
    int32_t slot;    // center residues consumed before this move
    int32_t jb;      // residues of b consumed before this move
    int32_t t;       // for an insertion: its index within the run (0 = first)
    int32_t mv;
};

__device__ __forceinline__ MoveScan scan_moves(const uint8_t* path, int64_t base, int64_t len, int32_t& c_slot,
                                               int32_t& c_jb, int64_t& c_last) {
    const int lane = lane_id();
    const int64_t x = base + lane;
    const int mv = x < len ? (int)path[x] : 0;
    const int fc = (mv == kMoveD || mv == kMoveU) ? 1 : 0;  // consumes a center residue
    const int fb = (mv == kMoveD || mv == kMoveL) ? 1 : 0;  // consumes a residue of b
    // inclusive prefix sums over the wave
    int sc = fc, sb = fb;
    int64_t last = fc ? x : -1;  // index of the latest center-consuming move so far
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        const int yc = __shfl_up(sc, d);
        const int yb = __shfl_up(sb, d);
        const int64_t yl = __shfl_up(last, d);
        if (lane >= d) {
            sc += yc;
            sb += yb;
            last = max(last, yl);
        }
    }
    const int64_t prev = __shfl_up(last, 1);   // every lane takes part
    const int64_t last_excl = lane > 0 ? prev : (int64_t)-1;
    MoveScan r;
    r.mv = mv;
    r.slot = c_slot + sc - fc;
    r.jb = c_jb + sb - fb;
    // an insertion's index within its run: moves since the last center residue
    r.t = (int32_t)(x - max(c_last, last_excl) - 1);
    // carries for the next chunk
    c_slot += __shfl(sc, kWave - 1);
    c_jb += __shfl(sb, kWave - 1);
    c_last = max(c_last, __shfl(last, kWave - 1));
    return r;
}

struct MsaArgs {
    int32_t npairs;
    const uint8_t* pool;
    const int64_t* off;
    const int32_t* len;
    const int32_t* center;
    const uint8_t* paths;
    const int64_t* path_off;
    const int32_t* path_len;
    const int32_t* row;
    int32_t* ins;        // [max_len + 1]: longest insertion per slot
    int32_t* slot_col;   // [max_len + 1]: first column of each slot
    int32_t* res_col;    // [max_len]: column of each center residue
    int64_t* width;      // device copy of the width
    int64_t* width_out;
    int32_t* error;      // a path inconsistent with its pair's lengths
    uint32_t* fault;     // host-visible device-fault word (may be null)
    uint8_t* msa;
    int64_t width_cap;
    uint8_t gap;
    int32_t nseq;
};

// One wave per pair: the longest insertion per slot.
__global__ __launch_bounds__(kWave) void k_ins(MsaArgs A) {
    const int q = blockIdx.x;
    if (q >= A.npairs) return;
    const int64_t len = A.path_len[q];
    if (len < 0) {
        if (lane_id() == 0) __hip_atomic_store(A.error, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        return;
    }
    const uint8_t* path = A.paths + A.path_off[q];
    const int lc = A.len[A.center[0]];
    int32_t c_slot = 0, c_jb = 0;
    int64_t c_last = -1;
    for (int64_t base = 0; base < len; base += kWave) {
        const MoveScan r = scan_moves(path, base, len, c_slot, c_jb, c_last);
        const int64_t x = base + lane_id();
        if (r.mv == kMoveL && r.slot <= lc) {
            const bool run_end = (x + 1 >= len) || (path[x + 1] != kMoveL);
            if (run_end) atomicMax(&A.ins[r.slot], r.t + 1);
        }
    }
}

// One block: first column of every slot, column of every center residue,
// and the width.
__global__ __launch_bounds__(1024) void k_cols(MsaArgs A) {
    __shared__ int64_t part[1024];
    const int lc = A.len[A.center[0]];
    const int nslot = lc + 1;
    int64_t carry = 0;  // columns before the current chunk
    for (int base = 0; base < nslot; base += blockDim.x) {
        const int p = base + threadIdx.x;
        // slot p and (if p < lc) residue p take ins[p] + 1 columns
        const int64_t w = p < nslot ? (int64_t)A.ins[p] + (p < lc ? 1 : 0) : 0;
        part[threadIdx.x] = w;
        __syncthreads();
        for (int d = 1; d < (int)blockDim.x; d <<= 1) {
            const int64_t y = (int)threadIdx.x >= d ? part[threadIdx.x - d] : 0;
            __syncthreads();
            part[threadIdx.x] += y;
            __syncthreads();
        }
        if (p < nslot) {
            const int64_t start = carry + part[threadIdx.x] - w;
            A.slot_col[p] = (int32_t)start;
            if (p < lc) A.res_col[p] = (int32_t)(start + A.ins[p]);
        }
        carry += part[blockDim.x - 1];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const bool bad = __hip_atomic_load(A.error, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0;
        A.width[0] = carry;
        if (A.width_out) A.width_out[0] = bad ? -1 : carry;
        if (bad) report_fault(A.fault);
    }
}

__global__ void k_msa_fill(MsaArgs A) {
    const int64_t w = A.width[0];
    if (w > A.width_cap || __hip_atomic_load(A.error, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return;
    const int64_t total = (int64_t)A.nseq * w;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r = e / w, x = e - r * w;
        A.msa[r * A.width_cap + x] = A.gap;
    }
}

__global__ void k_msa_center(MsaArgs A) {
    if (A.width[0] > A.width_cap || __hip_atomic_load(A.error, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return;
    const int c = A.center[0];
    const int lc = A.len[c];
    const uint8_t* s = A.pool + A.off[c];
    uint8_t* row = A.msa + (int64_t)c * A.width_cap;
    for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < lc; p += gridDim.x * blockDim.x) row[A.res_col[p]] = s[p];
}

// One wave per pair: place the pair's residues in its row.
__global__ __launch_bounds__(kWave) void k_msa_emit(MsaArgs A) {
    const int q = blockIdx.x;
    if (q >= A.npairs) return;
    if (A.width[0] > A.width_cap || __hip_atomic_load(A.error, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return;
    const int64_t len = A.path_len[q];
    const int k = A.row[q];
    const int lc = A.len[A.center[0]], lk = A.len[k];
    const int64_t w = A.width[0];
    const uint8_t* path = A.paths + A.path_off[q];
    const uint8_t* s = A.pool + A.off[k];
    uint8_t* row = A.msa + (int64_t)k * A.width_cap;
    int32_t c_slot = 0, c_jb = 0;
    int64_t c_last = -1;
    for (int64_t base = 0; base < len; base += kWave) {
        const MoveScan r = scan_moves(path, base, len, c_slot, c_jb, c_last);
        // the bounds hold for any path of the pair; they only guard the writes
        if (r.mv == kMoveD && r.slot < lc && r.jb < lk) {
            row[A.res_col[r.slot]] = s[r.jb];
        } else if (r.mv == kMoveL && r.slot <= lc && r.jb < lk) {
            const int64_t x = (int64_t)A.slot_col[r.slot] + r.t;
            if (x < w) row[x] = s[r.jb];
        }
    }
}

}  // namespace

// Workspace: [center, width, error | sums | pair descriptors | paths |
// ins, slot_col, res_col | batch engine workspace]
struct MsaLayout {
    int64_t path_stride;
    size_t off_sums, off_pairs, off_paths, off_cols, off_batch, total;
};

static MsaLayout msa_layout(int32_t nseq, int32_t max_len, const DeviceInfo& di) {
    MsaLayout L{};
    const int64_t np = std::max(nseq - 1, 1);
    const int64_t ml = std::max(max_len, 1);
    L.path_stride = (int64_t)align_up((size_t)(2 * ml), 64);
    size_t off = 256;
    L.off_sums = off;
    off = align_up(off + (size_t)std::max(nseq, 1) * 8, 256);
    L.off_pairs = off;
    off = align_up(off + (size_t)np * (8 + 4 + 8 + 4 + 8 + 4 + 4 + 4), 256);
    L.off_paths = off;
    off = align_up(off + (size_t)np * L.path_stride, 256);
    L.off_cols = off;
    off = align_up(off + (size_t)(3 * ml + 2) * 4, 256);
    L.off_batch = off;
    L.total = off + batch_workspace_bytes((int32_t)np, (int32_t)ml, true, di);
    return L;
}

size_t center_star_workspace_bytes(int32_t nseq, int32_t max_len, const DeviceInfo& di) {
    return msa_layout(nseq, max_len, di).total;
}

int launch_center_star(int32_t nseq, const uint8_t* pool, const int64_t* off, const int32_t* len, int32_t max_len,
                       const nw_scoring& sc, const int32_t* scores, uint8_t gap, int32_t* center_out, uint8_t* msa,
                       int64_t width_cap, int64_t* width_out, void* ws, size_t ws_bytes, hipStream_t st,
                       const DeviceInfo& di) {
    const MsaLayout L = msa_layout(nseq, max_len, di);
    if (ws_bytes < L.total) return NW_ENOSPC;
    uint8_t* base = (uint8_t*)ws;
    int32_t* center = (int32_t*)base;
    int64_t* width = (int64_t*)(base + 8);
    int32_t* error = (int32_t*)(base + 16);
    int64_t* sums = (int64_t*)(base + L.off_sums);
    const int32_t np = nseq - 1;
    const int64_t npa = std::max(np, 1);
    uint8_t* pd = base + L.off_pairs;
    int64_t* a_off = (int64_t*)pd;
    int64_t* b_off = a_off + npa;
    int64_t* path_off = b_off + npa;
    int32_t* a_len = (int32_t*)(path_off + npa);
    int32_t* b_len = a_len + npa;
    int32_t* path_len = b_len + npa;
    int32_t* pscores = path_len + npa;
    int32_t* rowi = pscores + npa;
    uint8_t* paths = base + L.off_paths;
    const int64_t ml = std::max(max_len, 1);
    int32_t* ins = (int32_t*)(base + L.off_cols);
    int32_t* slot_col = ins + (ml + 1);
    int32_t* res_col = slot_col + (ml + 1);

    {
        ProfScope ps("nw_msa_center", st);
        hipLaunchKernelGGL(k_zero32, dim3(1), dim3(64), 0, st, (int32_t*)base, (int64_t)64);
        hipLaunchKernelGGL(k_zero32, dim3((unsigned)std::min<int64_t>(di.cus, (ml + 1 + 255) / 256)), dim3(256), 0,
                           st, ins, ml + 1);
        hipLaunchKernelGGL(k_colsum, dim3((unsigned)((nseq + 255) / 256)), dim3(256), 0, st, nseq, scores, sums);
        hipLaunchKernelGGL(k_argmax, dim3(1), dim3(1024), 0, st, nseq, sums, center, center_out);
    }
    if (np > 0) {
        PairArgs P{nseq, off, len, center, L.path_stride, a_off, a_len, b_off, b_len, path_off, rowi};
        hipLaunchKernelGGL(k_pairs, dim3((unsigned)((np + 255) / 256)), dim3(256), 0, st, P);
        BatchJob J{};
        J.njobs = np;
        J.pool = pool;
        J.a_off = a_off;
        J.a_len = a_len;
        J.b_off = b_off;
        J.b_len = b_len;
        J.max_len = (int32_t)ml;
        J.sc = sc;
        J.dirs = true;
        J.scores = pscores;
        J.paths = paths;
        J.path_off = path_off;
        J.path_len = path_len;
        const int r = launch_batch(J, base + L.off_batch, ws_bytes - L.off_batch, st, di);
        if (r) return r;
    }
    MsaArgs A{};
    A.npairs = np;
    A.pool = pool;
    A.off = off;
    A.len = len;
    A.center = center;
    A.paths = paths;
    A.path_off = path_off;
    A.path_len = path_len;
    A.row = rowi;
    A.ins = ins;
    A.slot_col = slot_col;
    A.res_col = res_col;
    A.width = width;
    A.width_out = width_out;
    A.error = error;
    A.fault = di.fault;
    A.msa = msa;
    A.width_cap = width_cap;
    A.gap = gap;
    A.nseq = nseq;
    {
        ProfScope ps("nw_msa_merge", st);
        if (np > 0) hipLaunchKernelGGL(k_ins, dim3((unsigned)np), dim3(kWave), 0, st, A);
        hipLaunchKernelGGL(k_cols, dim3(1), dim3(1024), 0, st, A);
        hipLaunchKernelGGL(k_msa_fill,
                           dim3((unsigned)std::min<int64_t>(4 * di.cus, std::max<int64_t>(1, nseq * ml / 256 + 1))),
                           dim3(256), 0, st, A);
        hipLaunchKernelGGL(k_msa_center, dim3((unsigned)std::min<int64_t>(di.cus, ml / 256 + 1)), dim3(256), 0, st, A);
        if (np > 0) hipLaunchKernelGGL(k_msa_emit, dim3((unsigned)np), dim3(kWave), 0, st, A);
    }
    return hipGetLastError() == hipSuccess ? NW_OK : NW_EDEVICE;
}

}  // namespace nw
