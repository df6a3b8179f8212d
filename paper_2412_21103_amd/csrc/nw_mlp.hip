// Band model: k-mer features, a 259-64-64-1 ReLU network with bfloat16
// weights and float32 arithmetic, its training step (pinball loss, Adam) and
// the certified-band labels it learns.
//
// The model only proposes each pair's first band half-width; the certificate
// of the banded fill decides, so the model changes speed, never results.
//
// Parameter vector (float32 master; bfloat16 copy with the same layout):
//   W1[64][259] (row = hidden unit), b1[64], W2[64][64], b2[64], w3[64], b3.
// Forward and backward passes read W1, W2 and w3 from the bfloat16 copy and
// the biases from the float32 master; the gradient passes straight through
// the rounding.  Adam updates the master and rewrites the copy.
//
// The layers are small (about 21k weights, one evaluation per pair), so they
// run as plain VALU FMAs with float32 activations; no matrix cores.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "nw_common.h"
#include "nw_internal.h"

namespace nw {

constexpr int kIn = NW_MLP_INPUTS;
constexpr int kH = NW_MLP_HIDDEN;
constexpr int kOffB1 = kH * kIn;
constexpr int kOffW2 = kOffB1 + kH;
constexpr int kOffB2 = kOffW2 + kH * kH;
constexpr int kOffW3 = kOffB2 + kH;
constexpr int kOffB3 = kOffW3 + kH;
static_assert(kOffB3 + 1 == NW_MLP_PARAMS, "parameter layout");
static_assert(kH == kWave, "one lane per hidden unit");

constexpr float kLenScale = 20000.f;

__device__ __forceinline__ float bf16_to_f32(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// float32 -> bfloat16, round to nearest, ties to even; NaN stays NaN
__device__ __forceinline__ uint16_t f32_to_bf16(float f) {
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7F800000u) == 0x7F800000u && (u & 0x007FFFFFu)) return 0x7FC0;
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

// ------------------------------------------------------------- features
// One block per pair: the 4-mer count difference of the two sequences in an
// LDS histogram (a counts +1, b counts -1).
// x[k] = [m, n, m - n] / 20000, then (count_a - count_b) / max(m, n, 1)
// for the 256 4-mers, index = sum_t c_t 4^(3-t) (first base most significant).
__global__ __launch_bounds__(256) void k_features(int32_t npairs, const uint8_t* pool, const int64_t* a_off,
                                                  const int32_t* a_len, const int64_t* b_off,
                                                  const int32_t* b_len, float* x) {
    __shared__ int32_t hist[256];
    const int k = blockIdx.x;
    const int t = threadIdx.x;
    hist[t] = 0;
    __syncthreads();
    const int m = a_len[k], n = b_len[k];
    for (int s = 0; s < 2; ++s) {
        const uint8_t* q = pool + (s ? b_off[k] : a_off[k]);
        const int len = s ? n : m;
        const int inc = s ? -1 : 1;
        // thread t takes the 4-mers starting at 4 consecutive positions; it
        // reads bytes p .. p+6 as three aligned 32-bit words (a word that
        // holds at least one byte of the sequence lies within the sequence's
        // pages) and extracts the 2-bit codes of its bytes; bytes past the end
        // only reach 4-mers that are not counted
        const uint32_t* qa = reinterpret_cast<const uint32_t*>((uintptr_t)q & ~(uintptr_t)3);
        const int sh = (int)((uintptr_t)q & 3);
        auto word_at = [&](int wi) -> uint32_t {
            const int first = 4 * wi - sh;  // its first byte, relative to q
            return (first + 3 >= 0 && first < len) ? qa[wi] : 0u;
        };
        for (int p = 4 * t; p + 3 < len; p += 4 * 256) {
            const int b0 = p + sh;
            const int wi = b0 >> 2;
            const uint32_t r = (uint32_t)(b0 & 3);
            const uint32_t w0 = word_at(wi), w1 = word_at(wi + 1), w2 = word_at(wi + 2);
            const uint32_t lo = __builtin_amdgcn_alignbyte(w1, w0, r);  // bytes p .. p+3
            const uint32_t hi = __builtin_amdgcn_alignbyte(w2, w1, r);  // bytes p+4 .. p+7
            uint32_t w = 0;  // codes of bytes p .. p+6, 2 bits each
#pragma unroll
            for (int e = 0; e < 4; ++e) w |= ((lo >> (8 * e)) & 3u) << (2 * e);
#pragma unroll
            for (int e = 0; e < 3; ++e) w |= ((hi >> (8 * e)) & 3u) << (2 * e + 8);
            const int nk = min(4, len - 3 - p);
            for (int e = 0; e < nk; ++e) {
                const uint32_t c = w >> (2 * e);
                const int idx = ((c & 3) << 6) | (((c >> 2) & 3) << 4) | (((c >> 4) & 3) << 2) | ((c >> 6) & 3);
                atomicAdd(&hist[idx], inc);
            }
        }
    }
    __syncthreads();
    float* xk = x + (int64_t)k * kIn;
    const float denom = (float)max(max(m, n), 1);
    xk[3 + t] = (float)hist[t] / denom;
    if (t == 0) {
        xk[0] = (float)m / kLenScale;
        xk[1] = (float)n / kLenScale;
        xk[2] = (float)(m - n) / kLenScale;
    }
}

// -------------------------------------------------------------- forward
// Each block stages W1 and W2 transposed in LDS (bfloat16, hidden unit
// fastest) once and then runs rows grid-strided, one wave per row, lane j =
// hidden unit j.  rows_idx (optional) gathers x rows: row r of this call reads
// x[rows_idx[r]].  z1, z2 (pre-activations, [rows][64]) are written when not
// null, for the backward pass.
constexpr int kFwdWaves = 4;

__global__ __launch_bounds__(256) void k_mlp_forward(int32_t rows, const float* x, const int32_t* rows_idx,
                                                     const float* params, const uint16_t* wq, float* yhat,
                                                     float* z1, float* z2) {
    __shared__ uint16_t w1t[kIn * kH];
    __shared__ uint16_t w2t[kH * kH];
    __shared__ float xs[kFwdWaves][kIn + 1];
    __shared__ float hs[kFwdWaves][kH];
    for (int q = threadIdx.x; q < kIn * kH; q += 256) {
        const int i = q / kH, j = q - i * kH;
        w1t[q] = wq[j * kIn + i];
    }
    for (int q = threadIdx.x; q < kH * kH; q += 256) {
        const int k = q / kH, j = q - k * kH;
        w2t[q] = wq[kOffW2 + j * kH + k];
    }
    __syncthreads();
    const int wave = threadIdx.x >> 6;
    const int lane = lane_id();
    const float bias1 = params[kOffB1 + lane];
    const float bias2 = params[kOffB2 + lane];
    const float w3 = bf16_to_f32(wq[kOffW3 + lane]);
    const float bias3 = params[kOffB3];
    for (int r = blockIdx.x * kFwdWaves + wave; r < rows; r += gridDim.x * kFwdWaves) {
        const int64_t src = rows_idx ? rows_idx[r] : r;
        const float* xr = x + src * kIn;
        for (int i = lane; i < kIn; i += kWave) xs[wave][i] = xr[i];
        __builtin_amdgcn_wave_barrier();
        float acc = bias1;
        for (int i = 0; i < kIn; ++i) acc = fmaf(bf16_to_f32(w1t[i * kH + lane]), xs[wave][i], acc);
        if (z1) z1[(int64_t)r * kH + lane] = acc;
        hs[wave][lane] = fmaxf(acc, 0.f);
        __builtin_amdgcn_wave_barrier();
        float acc2 = bias2;
        for (int k = 0; k < kH; ++k) acc2 = fmaf(bf16_to_f32(w2t[k * kH + lane]), hs[wave][k], acc2);
        if (z2) z2[(int64_t)r * kH + lane] = acc2;
        float y = w3 * fmaxf(acc2, 0.f);
        for (int d = 32; d >= 1; d >>= 1) y += __shfl_xor(y, d);
        if (lane == 0) yhat[r] = y + bias3;
        __builtin_amdgcn_wave_barrier();  // xs/hs are rewritten by the next row
    }
}

// ------------------------------------------------------------ half-width
// w = ceil(expm1(max(yhat, 0)) * (1 + margin)), clamped to [0, max(m, n)];
// evaluated in double so the ceiling matches a float64 reference.
__global__ void k_widths(int32_t n, const float* yhat, const int32_t* a_len, const int32_t* b_len,
                         float margin, int32_t* w) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const double y = fmax((double)yhat[k], 0.0);
    const double v = ceil(expm1(y) * (1.0 + (double)margin));
    const int cap = max(a_len[k], b_len[k]);
    w[k] = (v >= (double)cap) ? cap : (v > 0.0 ? (int)v : 0);
}

// ---------------------------------------------------------- band labels
// w_cert = the smallest w >= 0 with S > cd*(min - w - 1) + gap*(|D| + 2w + 2),
// capped at min(m, n) (where the banded fill falls back to the full grid).
// Solving for w: w > (cd*(min-1) + gap*(|D|+2) - S) / (cd - 2 gap).
__global__ void k_band_labels(int32_t n, const int32_t* scores, const int32_t* a_len,
                              const int32_t* b_len, int32_t cd, int32_t gap, int32_t* w_cert,
                              float* target) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const int64_t m = a_len[k], nn = b_len[k];
    const int64_t mn = m < nn ? m : nn;
    const int64_t d = m > nn ? m - nn : nn - m;
    const int64_t num = (int64_t)cd * (mn - 1) + (int64_t)gap * (d + 2) - scores[k];
    const int64_t den = (int64_t)cd - 2 * (int64_t)gap;  // > 0 (checked on the host)
    int64_t w = num >= 0 ? num / den + 1 : 0;
    w = w > mn ? mn : w;
    if (w_cert) w_cert[k] = (int32_t)w;
    if (target) target[k] = log1pf((float)w);
}

// w_path: how far path k strays outside the corridor of diagonals between
// (0,0) and (m,n), [min(0,D), max(0,D)] with D = n - m, i.e. the band
// half-width it needs (the maximum diagonal offset of the optimal path beyond
// the straight band).  A diagonal move keeps the offset j - i, a vertical move
// lowers it by one, a horizontal move raises it.  One wave per path: lane l
// scans the l-th contiguous chunk of moves for its net offset and the highest
// and lowest running offsets inside the chunk; an exclusive scan of the net
// offsets across the wave gives each chunk's starting offset.
__global__ __launch_bounds__(256) void k_path_labels(int32_t n, const uint8_t* paths, const int64_t* path_off,
                                                     const int32_t* path_len, const int32_t* a_len,
                                                     const int32_t* b_len, int32_t* w_path, float* target) {
    const int k = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (k >= n) return;
    const int lane = lane_id();
    const int64_t len = path_len[k] > 0 ? path_len[k] : 0;
    const int64_t chunk = (len + kWave - 1) / kWave;
    const int64_t lo_i = min(len, chunk * lane), hi_i = min(len, lo_i + chunk);
    const uint8_t* p = paths + path_off[k];
    int32_t off = 0, top = 0, bot = 0;  // relative to the chunk's start
    for (int64_t x = lo_i; x < hi_i; ++x) {
        const uint8_t mv = p[x];
        off += (mv == 3) - (mv == 2);
        top = max(top, off);
        bot = min(bot, off);
    }
    // exclusive scan of the chunks' net offsets
    int32_t incl = off;
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        const int32_t y = __shfl_up(incl, d);
        if (lane >= d) incl += y;
    }
    const int32_t start = incl - off;
    const int32_t dd = b_len[k] - a_len[k];
    const int32_t corr_lo = min(0, dd), corr_hi = max(0, dd);
    int32_t e = max(0, max(start + top - corr_hi, corr_lo - (start + bot)));
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) e = max(e, __shfl_xor(e, d));
    if (lane == 0) {
        if (w_path) w_path[k] = e;
        if (target) target[k] = log1pf((float)e);
    }
}

// ------------------------------------------------------- training pieces
// Output error of the mean pinball loss and the two hidden-layer errors,
// one wave per row.  u = target - yhat; dL/dyhat = -(u < 0 ? tau - 1 : tau)/B.
__global__ __launch_bounds__(256) void k_mlp_backward_act(int32_t rows, const float* target,
                                                          const int32_t* rows_idx, const float* yhat,
                                                          const float* z1, const float* z2,
                                                          const uint16_t* wq, float tau, float* dy,
                                                          float* dz1, float* dz2, float* loss_row) {
    __shared__ float d2s[4][kH];
    const int wave = threadIdx.x >> 6;
    const int lane = lane_id();
    const int r = blockIdx.x * 4 + wave;
    if (r >= rows) return;
    const int64_t src = rows_idx ? rows_idx[r] : r;
    const float u = target[src] - yhat[r];
    const float slope = (u < 0.f) ? (tau - 1.f) : tau;
    const float g = -slope / (float)rows;
    if (lane == 0) {
        dy[r] = g;
        loss_row[r] = slope * u;
    }
    const float e2 = (z2[(int64_t)r * kH + lane] > 0.f) ? g * bf16_to_f32(wq[kOffW3 + lane]) : 0.f;
    dz2[(int64_t)r * kH + lane] = e2;
    d2s[wave][lane] = e2;
    __builtin_amdgcn_wave_barrier();
    // lane k: sum_j dz2[j] * W2[j][k]   (row j of W2 is contiguous in k)
    float acc = 0.f;
    for (int j = 0; j < kH; ++j) acc = fmaf(d2s[wave][j], bf16_to_f32(wq[kOffW2 + j * kH + lane]), acc);
    dz1[(int64_t)r * kH + lane] = (z1[(int64_t)r * kH + lane] > 0.f) ? acc : 0.f;
}

// Parameter gradients in two passes, both in a fixed order (deterministic,
// no atomics): kRowChunks partial sums over consecutive row chunks, one
// thread per (parameter, chunk), then their sum per parameter.
constexpr int kRowChunks = 8;

__global__ __launch_bounds__(256) void k_mlp_wgrad_part(int32_t rows, const float* x, const int32_t* rows_idx,
                                                        const float* z1, const float* z2, const float* dy,
                                                        const float* dz1, const float* dz2, float* part) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    const int chunk = blockIdx.y;
    if (p >= NW_MLP_PARAMS) return;
    const int per = (rows + kRowChunks - 1) / kRowChunks;
    const int r_lo = chunk * per, r_hi = min(rows, r_lo + per);
    float acc = 0.f;
    if (p < kOffB1) {
        const int j = p / kIn, i = p - j * kIn;
        for (int r = r_lo; r < r_hi; ++r) {
            const int64_t src = rows_idx ? rows_idx[r] : r;
            acc = fmaf(dz1[(int64_t)r * kH + j], x[src * kIn + i], acc);
        }
    } else if (p < kOffW2) {
        const int j = p - kOffB1;
        for (int r = r_lo; r < r_hi; ++r) acc += dz1[(int64_t)r * kH + j];
    } else if (p < kOffB2) {
        const int q = p - kOffW2, j = q / kH, k = q - j * kH;
        for (int r = r_lo; r < r_hi; ++r)
            acc = fmaf(dz2[(int64_t)r * kH + j], fmaxf(z1[(int64_t)r * kH + k], 0.f), acc);
    } else if (p < kOffW3) {
        const int j = p - kOffB2;
        for (int r = r_lo; r < r_hi; ++r) acc += dz2[(int64_t)r * kH + j];
    } else if (p < kOffB3) {
        const int j = p - kOffW3;
        for (int r = r_lo; r < r_hi; ++r) acc = fmaf(dy[r], fmaxf(z2[(int64_t)r * kH + j], 0.f), acc);
    } else {
        for (int r = r_lo; r < r_hi; ++r) acc += dy[r];
    }
    part[(int64_t)chunk * NW_MLP_PARAMS + p] = acc;
}

__global__ __launch_bounds__(256) void k_mlp_wgrad_sum(const float* part, float* grad) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= NW_MLP_PARAMS) return;
    float acc = 0.f;
#pragma unroll
    for (int c = 0; c < kRowChunks; ++c) acc += part[(int64_t)c * NW_MLP_PARAMS + p];
    grad[p] = acc;
}

// Mean of the per-row losses (one block, fixed reduction order).
__global__ __launch_bounds__(256) void k_mean(int32_t rows, const float* v, float* out) {
    __shared__ float part[256];
    float s = 0.f;
    for (int r = threadIdx.x; r < rows; r += 256) s += v[r];
    part[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w >= 1; w >>= 1) {
        if ((int)threadIdx.x < w) part[threadIdx.x] += part[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = part[0] / (float)rows;
}

// Adam (beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected) on the float32
// master; the bfloat16 copy is rewritten from the new master.
__global__ void k_adam(const float* grad, float* params, uint16_t* wq, float* mom, float* vel, float lr,
                       float bc1, float bc2) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= NW_MLP_PARAMS) return;
    const float g = grad[p];
    const float m = 0.9f * mom[p] + 0.1f * g;
    const float v = 0.999f * vel[p] + 0.001f * (g * g);
    mom[p] = m;
    vel[p] = v;
    const float np = params[p] - lr * (m / bc1) / (sqrtf(v / bc2) + 1e-8f);
    params[p] = np;
    wq[p] = f32_to_bf16(np);
}

__global__ void k_quantize(const float* params, uint16_t* wq) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p < NW_MLP_PARAMS) wq[p] = f32_to_bf16(params[p]);
}

// ------------------------------------------------------------ launchers

static unsigned blocks_for(int64_t n, int per) { return (unsigned)((n + per - 1) / per); }

static int launched() { return hipGetLastError() == hipSuccess ? NW_OK : NW_EDEVICE; }

int launch_features(int32_t npairs, const uint8_t* pool, const int64_t* a_off, const int32_t* a_len,
                    const int64_t* b_off, const int32_t* b_len, float* x, hipStream_t st) {
    if (npairs == 0) return NW_OK;
    ProfScope ps("nw_features", st);
    hipLaunchKernelGGL(k_features, dim3(npairs), dim3(256), 0, st, npairs, pool, a_off, a_len, b_off, b_len, x);
    return launched();
}

static unsigned forward_grid(int32_t rows, const DeviceInfo& di) {
    // enough waves to cover the rows, at most two blocks per CU (each block
    // stages the weights once)
    return std::max(1u, std::min(blocks_for(rows, kFwdWaves), (unsigned)(2 * di.cus)));
}

int launch_mlp_forward(int32_t rows, const float* x, const float* params, const uint16_t* wq, float* yhat,
                       hipStream_t st, const DeviceInfo& di) {
    if (rows == 0) return NW_OK;
    ProfScope ps("nw_mlp_forward", st);
    hipLaunchKernelGGL(k_mlp_forward, dim3(forward_grid(rows, di)), dim3(256), 0, st, rows, x,
                       (const int32_t*)nullptr, params, wq, yhat, (float*)nullptr, (float*)nullptr);
    return launched();
}

int launch_widths(int32_t n, const float* yhat, const int32_t* a_len, const int32_t* b_len, float margin,
                  int32_t* w, hipStream_t st) {
    if (n == 0) return NW_OK;
    ProfScope ps("nw_mlp_widths", st);
    hipLaunchKernelGGL(k_widths, dim3(blocks_for(n, 256)), dim3(256), 0, st, n, yhat, a_len, b_len, margin, w);
    return launched();
}

int launch_band_labels(int32_t n, const int32_t* scores, const int32_t* a_len, const int32_t* b_len,
                       int32_t cd, int32_t gap, int32_t* w_cert, float* target, hipStream_t st) {
    if (n == 0) return NW_OK;
    ProfScope ps("nw_band_labels", st);
    hipLaunchKernelGGL(k_band_labels, dim3(blocks_for(n, 256)), dim3(256), 0, st, n, scores, a_len, b_len, cd,
                       gap, w_cert, target);
    return launched();
}

int launch_path_labels(int32_t n, const uint8_t* paths, const int64_t* path_off, const int32_t* path_len,
                       const int32_t* a_len, const int32_t* b_len, int32_t* w_path, float* target, hipStream_t st) {
    if (n == 0) return NW_OK;
    ProfScope ps("nw_path_labels", st);
    hipLaunchKernelGGL(k_path_labels, dim3((unsigned)((n + 3) / 4)), dim3(256), 0, st, n, paths, path_off, path_len,
                       a_len, b_len, w_path, target);
    return launched();
}

int launch_quantize(const float* params, uint16_t* wq, hipStream_t st) {
    hipLaunchKernelGGL(k_quantize, dim3(blocks_for(NW_MLP_PARAMS, 256)), dim3(256), 0, st, params, wq);
    return launched();
}

size_t mlp_train_workspace_bytes(int32_t batch) {
    const size_t b = (size_t)std::max(batch, 1);
    // yhat, dy, loss_row: b each; z1, z2, dz1, dz2: b*64 each; grad; partial sums
    return align_up((3 * b + 4 * b * kH + (1 + kRowChunks) * (size_t)NW_MLP_PARAMS) * sizeof(float), 256);
}

int launch_mlp_train_step(nw_mlp* mlp, int32_t batch, const float* x, const float* target,
                          const int32_t* rows_idx, float tau, float lr, float* loss, float* grad_out,
                          void* ws, hipStream_t st, const DeviceInfo& di) {
    float* f = (float*)ws;
    float* yhat = f;
    float* dy = yhat + batch;
    float* loss_row = dy + batch;
    float* z1 = loss_row + batch;
    float* z2 = z1 + (size_t)batch * kH;
    float* dz1 = z2 + (size_t)batch * kH;
    float* dz2 = dz1 + (size_t)batch * kH;
    float* grad_ws = dz2 + (size_t)batch * kH;
    float* part = grad_ws + NW_MLP_PARAMS;
    float* grad = grad_out ? grad_out : grad_ws;
    {
        ProfScope ps("nw_mlp_train_forward", st);
        hipLaunchKernelGGL(k_mlp_forward, dim3(forward_grid(batch, di)), dim3(256), 0, st, batch, x, rows_idx,
                           (const float*)mlp->params, (const uint16_t*)mlp->params_bf16, yhat, z1, z2);
    }
    {
        ProfScope ps("nw_mlp_backward", st);
        hipLaunchKernelGGL(k_mlp_backward_act, dim3(blocks_for(batch, 4)), dim3(256), 0, st, batch, target,
                           rows_idx, yhat, z1, z2, (const uint16_t*)mlp->params_bf16, tau, dy, dz1, dz2,
                           loss_row);
        hipLaunchKernelGGL(k_mlp_wgrad_part, dim3(blocks_for(NW_MLP_PARAMS, 256), kRowChunks), dim3(256), 0, st,
                           batch, x, rows_idx, z1, z2, dy, dz1, dz2, part);
        hipLaunchKernelGGL(k_mlp_wgrad_sum, dim3(blocks_for(NW_MLP_PARAMS, 256)), dim3(256), 0, st, part, grad);
    }
    if (loss) hipLaunchKernelGGL(k_mean, dim3(1), dim3(256), 0, st, batch, loss_row, loss);
    if (lr > 0.f) {
        const int64_t t = mlp->step + 1;
        const double bc1 = 1.0 - std::pow(0.9, (double)t);
        const double bc2 = 1.0 - std::pow(0.999, (double)t);
        ProfScope ps("nw_mlp_adam", st);
        hipLaunchKernelGGL(k_adam, dim3(blocks_for(NW_MLP_PARAMS, 256)), dim3(256), 0, st, grad, mlp->params,
                           mlp->params_bf16, mlp->adam_m, mlp->adam_v, lr, (float)bc1, (float)bc2);
        mlp->step = t;
    }
    return launched();
}

}  // namespace nw
