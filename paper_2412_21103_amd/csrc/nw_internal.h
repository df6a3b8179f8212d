// Host-side internals shared by the libnw translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "../../include/nw.h"

namespace nw {

// Substitution-table bytes for the two value domains (see nw_common.h).
struct Consts {
    int32_t kdm, kdx;  // per-cell diagonal term for match / mismatch
    int32_t gap;
};

Consts dirs_consts(const nw_scoring& sc);   // V domain: 4(s - 2 gap) + 2
Consts score_consts(const nw_scoring& sc);  // W domain: s - 2 gap

// The one-hot lookup holds a cell's diagonal terms as signed bytes (-128 is
// the sentinel of rows outside the grid).  Constants outside -127..127 send
// every pair of the call to the byte-comparing sweep, whose row word holds
// the mismatch term in 23 bits and which takes the match term whole.
inline bool needs_wide(const Consts& K) {
    return K.kdm < -127 || K.kdm > 127 || K.kdx < -127 || K.kdx > 127;
}
constexpr int32_t kWideTermLimit = 1 << 22;  // |term| below this for the byte-comparing sweep

// Device facts needed to size persistent grids, and the per-call settings
// every launch carries: the device-fault word and the polls a bounded wait
// makes before it gives up.
struct DeviceInfo {
    int device;
    int cus;
    bool supported;
    uint32_t* fault;     // device view of this device's fault word (nullptr before nw_init)
    int32_t spin_limit;  // polls before a boundary wait gives up
    int64_t walk_limit;  // nw_align: longest path (m + n) traced back by one wave
};
// Fills *out for the current device.  With may_allocate (the default) the
// pinned fault words are set up on first use; without, a library that was
// never initialised reports no faults (fault = nullptr).
int device_info(DeviceInfo* out, bool may_allocate = true);

// Default polls before a boundary wait gives up: far beyond any legitimate
// wait (the last strip of a long pair waits for the whole pipeline to reach
// it, milliseconds for 65,536 columns), about 0.4 s of LDS polls or a few
// seconds of L2 polls.
constexpr int32_t kDefaultSpinLimit = 1 << 22;

// Default longest path (m + n moves) that nw_align traces back with one wave
// instead of the per-strip parallel walk.
constexpr int64_t kDefaultWalkLimit = 1 << 12;

// Device faults (a bounded wait that gave up, a corrupt direction tag) are
// reported by the kernels in a word of pinned host memory per device; the
// next entry point on that device, or nw_sync, returns NW_EDEVICE and clears
// it.  Kernels write it with report_fault (nw_common.h).
int take_fault(int device);

inline size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// Optional per-kernel timing (nw_profile_begin / nw_profile_end).  Construct
// a ProfScope right before a launch and let it go out of scope right after:
// while profiling is on it records a HIP event pair on the launch's stream.
struct ProfScope {
    ProfScope(const char* name, hipStream_t st);
    ~ProfScope();
    const char* name;
    hipStream_t st;
    int slot;
};

// Persistent batch engine (nw_batch.hip).
struct BatchJob {
    // pairs: explicit arrays; all-pairs: nseq sequences, jobs are i <= j
    bool allpairs;
    int32_t njobs;
    int32_t nseq;
    const uint8_t* pool;
    const int64_t* a_off;
    const int32_t* a_len;
    const int64_t* b_off;
    const int32_t* b_len;
    int32_t max_len;
    nw_scoring sc;
    bool dirs;
    int32_t* scores;     // pairs mode
    uint8_t* paths;
    const int64_t* path_off;
    int32_t* path_len;
    int64_t* path_len64; // single-pair calls report an int64 length
    int32_t* matrix;     // all-pairs mode
    // certified band
    bool banded;
    bool band_doubling;  // widen a failed band by doubling instead of to its certified width
    bool band_one_launch;  // no separate launch of the score-only first passes
    const int32_t* w_init;
    int32_t w_default;
    int32_t frac_1024;
    int32_t* w_used;
    uint8_t* status;
    int64_t* cells;
    int64_t* cells_so;  // of those, swept score-only
    // 0: sweep width per pass from the cost table; 2, 4 or 8: that width
    // always (used by the autotuner)
    int force_cols;
};

// Cooperative single-pair engine (nw_single.hip): used for one pair with at
// least kCoopMinCols columns.
constexpr int64_t kCoopMinCols = 512;
size_t coop_workspace_bytes(int64_t m, int64_t n, bool dirs);
int launch_coop(const uint8_t* a, int64_t m, const uint8_t* b, int64_t n, const nw_scoring& sc,
                bool dirs, int32_t* score, uint8_t* path, int64_t* path_len, void* ws,
                size_t ws_bytes, hipStream_t stream, const DeviceInfo& di);

// Workspace for full occupancy (one slot per resident wave, within the
// library's HBM budget); launch_batch runs with fewer waves when given less,
// down to one block of slots.
size_t batch_workspace_bytes(int32_t njobs, int32_t max_len, bool dirs, const DeviceInfo& di);
int launch_batch(const BatchJob& job, void* ws, size_t ws_bytes, hipStream_t stream,
                 const DeviceInfo& di);

// Center-star multiple alignment (nw_msa.hip).
size_t center_star_workspace_bytes(int32_t nseq, int32_t max_len, const DeviceInfo& di);
int launch_center_star(int32_t nseq, const uint8_t* pool, const int64_t* off, const int32_t* len, int32_t max_len,
                       const nw_scoring& sc, const int32_t* scores, uint8_t gap, int32_t* center, uint8_t* msa,
                       int64_t width_cap, int64_t* width, void* ws, size_t ws_bytes, hipStream_t st,
                       const DeviceInfo& di);

// Co-optimal alignment counts and enumeration (nw_coopt.hip).
size_t cooptimal_workspace_bytes(int32_t npairs, int32_t max_len, int32_t k, const DeviceInfo& di);
int launch_cooptimal(int32_t npairs, const uint8_t* pool, const int64_t* a_off, const int32_t* a_len,
                     const int64_t* b_off, const int32_t* b_len, int32_t max_len, const nw_scoring& sc,
                     int32_t* scores, uint64_t* counts, uint8_t* saturated, int32_t k, uint8_t* paths,
                     const int64_t* path_off, int32_t* path_len, int32_t* n_paths, void* ws, size_t ws_bytes,
                     hipStream_t st, const DeviceInfo& di);

// Sweep-width cost table (per device), filled by nw_autotune.
void set_step_costs(int device, const int32_t dirs[3], const int32_t score[3]);
void step_costs(int device, bool dirs, int32_t out[3]);
bool tuned_costs(int device);
void reset_step_costs();

// Band model (nw_mlp.hip).
int launch_features(int32_t npairs, const uint8_t* pool, const int64_t* a_off, const int32_t* a_len,
                    const int64_t* b_off, const int32_t* b_len, float* x, hipStream_t st);
int launch_mlp_forward(int32_t rows, const float* x, const float* params, const uint16_t* wq, float* yhat,
                       hipStream_t st, const DeviceInfo& di);
int launch_widths(int32_t n, const float* yhat, const int32_t* a_len, const int32_t* b_len, float margin,
                  int32_t* w, hipStream_t st);
int launch_band_labels(int32_t n, const int32_t* scores, const int32_t* a_len, const int32_t* b_len,
                       int32_t cd, int32_t gap, int32_t* w_cert, float* target, hipStream_t st);
int launch_path_labels(int32_t n, const uint8_t* paths, const int64_t* path_off, const int32_t* path_len,
                       const int32_t* a_len, const int32_t* b_len, int32_t* w_path, float* target, hipStream_t st);
int launch_quantize(const float* params, uint16_t* wq, hipStream_t st);
size_t mlp_train_workspace_bytes(int32_t batch);
int launch_mlp_train_step(nw_mlp* mlp, int32_t batch, const float* x, const float* target,
                          const int32_t* rows_idx, float tau, float lr, float* loss, float* grad_out,
                          void* ws, hipStream_t st, const DeviceInfo& di);

}  // namespace nw
