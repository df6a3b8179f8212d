/*
 * libnw -- global (Needleman-Wunsch) alignment with a linear gap on AMD
 * Instinct MI355X (gfx950).
 *
 * Method (paper Section 2): the score grid has one extra row and column
 * ((m+1) x (n+1) cells, Sec. 2.1); H(0,0) = 0 and the first row and column
 * fall by one gap per cell (Sec. 2.2); every other cell takes
 *     H(i,j) = max( H(i-1,j-1) + s(a_i,b_j), H(i-1,j) + gap, H(i,j-1) + gap )
 * (Sec. 2.3, Eq. 1, read as the standard linear-gap recurrence), with
 * s = match when a_i == b_j and mismatch otherwise.  Backtracking starts in
 * the bottom-right cell and follows the argmax (Sec. 2.4); moves use the
 * paper's direction codes (Sec. 3.1): 1 diagonal, 2 vertical (a_i against a
 * gap), 3 horizontal (a gap against b_j).  Among tied moves the library
 * always takes diagonal, then vertical, then horizontal, so every call
 * returns one fixed optimal path.
 *
 * Conventions shared by every entry point:
 *  - Sequence a (length m) labels rows, sequence b (length n) labels columns.
 *  - Symbols are bytes, one per position, and any byte value is legal: only
 *    equality matters (a match or a mismatch).  Nucleotide codes 0..3, or
 *    any pair whose bytes take at most four values that one two-bit field
 *    tells apart (the letters ACGT, ACGU, acgt...), run the fastest sweep;
 *    other pairs (protein letters, N, arbitrary bytes) are swept by
 *    comparing bytes, at about 7 instead of 5 operations per cell.  The band
 *    model's k-mer features read the two low bits only, which affects its
 *    widths (speed), never results.
 *  - Unless stated otherwise every pointer is a DEVICE pointer (memory from
 *    hipMalloc or a torch CUDA tensor on the current device), and every call
 *    is asynchronous on `stream` (a hipStream_t; NULL = the null stream).
 *    Outputs are valid once the stream has been synchronised.
 *  - The caller owns every buffer, including the workspace `ws`, which must
 *    stay allocated and untouched until the call's work on `stream` is done.
 *    Query its size with the matching *_workspace_size function.  The
 *    library allocates no device memory in these calls.
 *  - Paths are written in forward order, from (0,0) to (m,n).  A path has
 *    between max(m,n) and m+n moves.
 *  - Scores are int32.  Arguments are checked on the host before any GPU
 *    work is queued; a non-zero status means nothing was queued.
 *  - Overflow guard: (max(|match|,|mismatch|) + |gap|) * (m + n) must stay
 *    below 2^27, |match|, |mismatch| and |gap| at most 2^20, and the cell's
 *    diagonal term 4*(s - 2*gap) + 2 (s - 2*gap in score-only calls) below
 *    2^22 in magnitude for s = match and s = mismatch, else NW_ERANGE.  When
 *    a term does not fit in a signed byte (-127..127), the call sweeps every
 *    pair by comparing bytes (about 7 instead of 5 operations per cell);
 *    results are the same.
 *  - Calls on distinct streams with distinct workspaces may run concurrently.
 */
#ifndef NW_H
#define NW_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Scoring constants (paper Sec. 2.3): match +1, mismatch -1, gap -1. */
typedef struct nw_scoring {
    int32_t match;
    int32_t mismatch;
    int32_t gap;
} nw_scoring;

/* Move codes (paper Sec. 3.1). */
enum { NW_MOVE_D = 1, NW_MOVE_U = 2, NW_MOVE_L = 3 };

/* Status codes. */
enum {
    NW_OK = 0,
    NW_EINVAL = -1,  /* null pointer, negative length or count, bad flag   */
    NW_ERANGE = -2,  /* lengths or constants exceed the overflow guard      */
    NW_ENOSPC = -3,  /* path capacity or workspace too small                */
    NW_EDEVICE = -4, /* HIP error while queueing work, or a device fault     */
                     /* reported by earlier work (see Device faults below)  */
    NW_ENOTSUP = -5  /* no supported GPU (not gfx950) on the current device */
};

/* Device faults.  Work that has already been queued cannot return a status,
 * so the kernels report the failures only a device fault can cause -- a
 * bounded wait between waves that gave up (its watchdog), a stored direction
 * tag that is not a move -- in a host-visible word per device.  The next
 * libnw call on that device (any entry point, including the workspace-size
 * queries) returns NW_EDEVICE, queues nothing and clears the word; nw_sync
 * does the same after synchronising.  The affected outputs also carry the
 * failure:
 *   nw_align:            *score = INT32_MIN and *path_len = -3 (a wait gave
 *                        up) or -2 (a corrupt direction tag);
 *   nw_align_batch, nw_align_batch_banded, nw_align_batch_learned, and the
 *   alignments inside nw_center_star:
 *                        path_len[k] = -2 (a corrupt direction tag); these
 *                        engines have no waits between waves;
 *   nw_cooptimal:        scores[k] = INT32_MIN, counts[k] = 0,
 *                        saturated[k] = 0 for a pair whose team wait gave up;
 *   nw_center_star:      *width = -1 when some alignment was unusable.
 * Independently of faults, path_len[k] = -1 (with scores[k] = INT32_MIN)
 * marks a pair skipped because it exceeds max_len. */

/* One-time set-up of the library on the current device: the pinned host word
 * that device faults are reported in.  Optional -- every entry point does it
 * on first use -- but a caller that must not have the library allocate
 * during later calls (graph capture, allocation-free loops) calls it first.
 * Returns NW_OK, NW_ENOTSUP, or NW_EDEVICE (including a pending fault). */
int nw_init(void);

/* Synchronise `stream` (a hipStream_t; NULL = the null stream), then report
 * a pending device fault on the current device as NW_EDEVICE (and clear it). */
int nw_sync(void *stream);

/* Testing hook for the fault path: the number of polls a bounded wait between
 * waves makes before it gives up (default 2^22, far beyond any legitimate
 * wait; 0 restores the default).  Applies to calls queued afterwards.  A tiny
 * limit makes the waits of multi-wave calls (nw_align with n >= 512,
 * nw_cooptimal team pairs) give up early: every kernel still drains and exits
 * normally, the outputs carry the failure values above, and the fault is
 * reported.  polls < 0 is NW_EINVAL. */
int nw_set_wait_limit(int32_t polls);

/* Tuning hook of nw_align's traceback (multi-wave engine, n >= 512): paths of
 * at most `moves` moves (m + n) are walked back from (m, n) by one wave;
 * longer ones by every strip in parallel from guessed entry rows, then
 * merged (Sec. 3.1 and 4.1: the traceback follows the stored directions from
 * the last cell).  Both give the same path.  Default 4096; 0 restores the
 * default, 1 sends every such pair to the parallel walk.  Applies to calls
 * queued afterwards; moves < 0 is NW_EINVAL. */
int nw_set_walk_limit(int64_t moves);

/* Flags. */
#define NW_SCORE_ONLY 0x1u /* no traceback: paths, path_off, path_len may be NULL */
/* NW_GRAPH (nw_align_batch, nw_align_batch_banded, nw_align_batch_learned):
 * the first call with a given set of arguments (every pointer, count, size,
 * constant, flag and the stream) captures its launches into a HIP graph;
 * later calls with the same arguments replay that graph, which saves the
 * per-launch overhead of the planning kernels.  A replay reads every input
 * in place, so the caller may change the input bytes (not the addresses or
 * counts) between calls.  The stream must not be the null stream.  When the
 * caller's stream is already being captured the launches go into the
 * caller's graph instead.  The library owns the cached graphs (at most 256;
 * calls beyond that run without a graph) until nw_release_caches(). */
#define NW_GRAPH 0x2u
/* Banded and learned batch calls: widen a failed band by doubling it rather
 * than to the width its score certifies (see nw_align_batch_banded). */
#define NW_BAND_DOUBLING 0x4u
/* Banded and learned batch calls with paths: run every pass of a pair in one
 * launch, without the separate launch of the score-only first passes (see
 * nw_align_batch_banded).  The results are the same, every output included;
 * the call is slower.  For comparison and testing. */
#define NW_BAND_ONE_LAUNCH 0x8u

/* Human-readable text for a status code (static storage). */
const char *nw_strerror(int status);

/* Library version as 10000*major + 100*minor + patch. */
int nw_version(void);

/* ------------------------------------------------------------------------
 * One pair (paper Sec. 2; the single-alignment kernel of Sec. 3.1).
 *
 * nw_align_workspace_size: bytes of workspace nw_align needs for lengths
 * (m, n) and `flags`; written to *bytes (a host pointer).
 *
 * nw_align: a[m], b[n] (device, codes 0..3); *score (device int32) gets
 * H(m,n); unless NW_SCORE_ONLY, path[path_cap] (device) gets the moves and
 * *path_len (device int64) their number.  path_cap >= m + n is required
 * (NW_ENOSPC otherwise).  m == 0 or n == 0 is valid.  With n >= 512 the
 * columns are split into strips swept by different waves that hand their
 * boundaries over through bounded waits; a wait that gives up (which only a
 * device fault can cause) yields *score = INT32_MIN and *path_len = -3 and is
 * reported as a device fault (above).  The call may be captured into a HIP
 * graph: each launch, replays included, tags its boundary slots with a value
 * no earlier launch on the device used, so slots left in reused memory by
 * any earlier call never count as ready.
 * ------------------------------------------------------------------------ */
int nw_align_workspace_size(int64_t m, int64_t n, uint32_t flags, size_t *bytes);

int nw_align(const uint8_t *a, int64_t m, const uint8_t *b, int64_t n, nw_scoring sc,
             uint32_t flags, int32_t *score, uint8_t *path, int64_t path_cap,
             int64_t *path_len, void *ws, size_t ws_bytes, void *stream);

/* ------------------------------------------------------------------------
 * nw_align without a workspace, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid allocation).  Same arguments, outputs, checks and errors as
 * nw_align, minus ws/ws_bytes: the workspace is a fixed array of
 * NW_SCRATCH_BYTES in the library's device code, one per device, allocated
 * when the library is loaded on that device and held until the process ends.
 * The call makes no hipMalloc, hipFree or other allocating call (nw_init,
 * called once beforehand, does the library's own set-up; without it, device
 * faults are not reported through the fault word).  A pair whose nw_align
 * workspace exceeds NW_SCRATCH_BYTES returns NW_ENOSPC before any work is
 * queued; nw_align_noalloc_fits(m, n, flags) answers the same question
 * (NW_OK or NW_ENOSPC) without queueing anything.  With 64 MiB, full
 * alignments with paths fit up to about 14,000 x 14,000.
 * Every call on a device uses the same array and leaves its contents behind
 * (each call clears what it needs cleared): calls that overlap in time on one
 * device -- on different streams, or from different host threads -- race and
 * give wrong results; serialise them on one stream.
 * ------------------------------------------------------------------------ */
#define NW_SCRATCH_BYTES ((size_t)64 << 20)

int nw_align_noalloc(const uint8_t *a, int64_t m, const uint8_t *b, int64_t n, nw_scoring sc,
                     uint32_t flags, int32_t *score, uint8_t *path, int64_t path_cap,
                     int64_t *path_len, void *stream);

int nw_align_noalloc_fits(int64_t m, int64_t n, uint32_t flags);

/* ------------------------------------------------------------------------
 * Many independent pairs in one persistent launch (the data-parallel form of
 * the paper's multiple-alignment workload, Sec. 3.2).
 *
 * Pair k is a = pool[a_off[k] .. a_off[k]+a_len[k]) against
 * b = pool[b_off[k] .. b_off[k]+b_len[k]).  pool, a_off, a_len, b_off,
 * b_len are device arrays.  max_len (host) bounds every a_len[k] and
 * b_len[k]; the workspace is sized for it.  A pair that exceeds max_len is
 * skipped: scores[k] = INT32_MIN and path_len[k] = -1.
 *
 * Outputs (device): scores[npairs]; unless NW_SCORE_ONLY, pair k's moves go
 * to paths[path_off[k] ..] (path_off: device int64, caller-computed, with
 * room for a_len[k] + b_len[k] moves) and their count to path_len[k].
 * ------------------------------------------------------------------------ */
int nw_align_batch_workspace_size(int32_t npairs, int32_t max_len, uint32_t flags, size_t *bytes);

int nw_align_batch(int32_t npairs, const uint8_t *pool, const int64_t *a_off,
                   const int32_t *a_len, const int64_t *b_off, const int32_t *b_len,
                   int32_t max_len, nw_scoring sc, uint32_t flags, int32_t *scores,
                   uint8_t *paths, const int64_t *path_off, int32_t *path_len, void *ws,
                   size_t ws_bytes, void *stream);

/* ------------------------------------------------------------------------
 * Certified band (the paper's future-work aim of never missing an optimal
 * alignment, Sec. 5, made exact).  Same inputs and outputs as
 * nw_align_batch, and bit-identical results, but each pair first fills only
 * the staircase of strips that covers
 *     band(w) = { (i,j) : min(0,D) - w <= j - i <= max(0,D) + w },  D = n - m,
 * with every cell outside it taken as -infinity.  The region's score S_R is
 * certified when it beats the best score any path leaving band(w) can reach:
 *     S_R > U_out(w) = c_d*(min(m,n) - w - 1) + gap*(|D| + 2w + 2),
 *     c_d = max(match, mismatch)   (valid when 2*gap < c_d),
 * which forces every optimal path inside the band, so score and tie-break
 * path equal the full grid's.  Otherwise the band widens to the width S_R
 * itself certifies, w' = the smallest w' with S_R > U_out(w') (> w): the next
 * region contains this one, so its score is at least S_R and the second pass
 * always certifies.  Because the first pass serves mostly to find S_R, it
 * runs score-only (no directions); if it certifies after all, the same band
 * is swept again with directions.  With paths requested, the call runs every
 * pair's score-only first pass in a launch of its own before the others,
 * then orders the pairs again by the cost of their remaining passes; the
 * results are the same as if each pair ran its passes in one go.  The
 * widened pass records directions only
 * in the rows of band(1.5 w + 16) (w the first pass's width), where the path
 * most likely runs, and sweeps the rest of its band score-only; the
 * traceback checks that it stays in those rows, and if it would leave them
 * the pass is swept again with directions in a band four times as wide (+64),
 * or everywhere once that covers the certified band.  The traceback never
 * reads a direction that was not recorded, so results do not depend on w.
 * With the flag NW_BAND_DOUBLING, w doubles instead (0 becomes 1), every
 * pass records directions, and a pair may take more passes.  The full
 * grid is used directly once w >= min(m,n), when 2*gap >= c_d, or once the
 * band's height 128 + |D| + 2w reaches fallback_frac of m -- for a first pass
 * or any doubled one; a widened pass, which is certain to certify, takes the
 * full grid only once that height reaches m.  A first
 * half-width past the height limit (but below min(m,n)) is first lowered to
 * the widest band under the limit, so a pair reaches the full grid only after
 * a band has failed.  Each pass sweeps 128, 256 or 512 columns per wave,
 * whichever the library's cost model rates fastest for its height.
 *
 * w_init (device int32[npairs], may be NULL: then w_default for all) gives
 * each pair's first half-width, e.g. the band model's prediction.  Optional
 * device outputs (NULL to skip): w_used[k] = final half-width (-1 = full
 * grid); status[k] = bit 0 certified on the first pass, bits 1..5 number of
 * passes after the first, bit 6 full grid, bit 7 certificate not applicable;
 * cells[k] =
 * cells swept over all passes; cells_score_only[k] = those of them swept
 * score-only (the first pass's, when it ran without directions, and the
 * rows of later passes that recorded none).  A pair with m == 0 or n == 0 reports
 * w_used -1, the full-grid bit and 0 cells; a pair over max_len reports
 * w_used -1, status 0 and 0 cells.
 * ------------------------------------------------------------------------ */
int nw_align_batch_banded_workspace_size(int32_t npairs, int32_t max_len, uint32_t flags,
                                         size_t *bytes);

int nw_align_batch_banded(int32_t npairs, const uint8_t *pool, const int64_t *a_off,
                          const int32_t *a_len, const int64_t *b_off, const int32_t *b_len,
                          int32_t max_len, nw_scoring sc, uint32_t flags, const int32_t *w_init,
                          int32_t w_default, float fallback_frac, int32_t *scores, uint8_t *paths,
                          const int64_t *path_off, int32_t *path_len, int32_t *w_used,
                          uint8_t *status, int64_t *cells, int64_t *cells_score_only, void *ws,
                          size_t ws_bytes, void *stream);

/* ------------------------------------------------------------------------
 * All-pairs score matrix for the centre-star multiple alignment front end
 * (paper Sec. 3.2, Eq. 2): out[i*nseq + j] (device int32, nseq x nseq,
 * row-major) = score of sequence i (rows) against sequence j (columns) for
 * all i != j, computed once per unordered pair (n(n-1)/2 alignments) and
 * mirrored; out[i*nseq + i] is the score of sequence i against itself,
 * computed by the same recurrence (len[i] * match whenever match >= mismatch
 * and match >= 2*gap).  Sequence k = pool[off[k] .. off[k]+len[k]); max_len
 * (host) bounds every len[k]; an entry whose sequence exceeds it is
 * INT32_MIN.  nseq*(nseq+1)/2 must fit in int32 (NW_ERANGE otherwise).
 * ------------------------------------------------------------------------ */
int nw_allpairs_workspace_size(int32_t nseq, int32_t max_len, size_t *bytes);

int nw_allpairs_scores(int32_t nseq, const uint8_t *pool, const int64_t *off,
                       const int32_t *len, int32_t max_len, nw_scoring sc, int32_t *out,
                       void *ws, size_t ws_bytes, void *stream);

/* ------------------------------------------------------------------------
 * Centre-star multiple alignment (paper Sec. 3.2, Multiple Alignment): the
 * centre is the sequence whose scores against the other sequences sum
 * highest in `scores` (device int32 nseq x nseq, as nw_allpairs_scores writes
 * it; the diagonal is ignored; the lowest index wins ties).  Every other
 * sequence is aligned to the centre (centre in the rows, the single-path
 * traceback of nw_align), and the pairwise alignments are merged with the
 * centre as the reference, keeping all their gaps: before each centre
 * residue (and after the last) the alignment has as many columns as the
 * longest insertion any sequence makes there, a row's inserted residues fill
 * the first of those columns, and every column a row does not fill holds
 * gap_byte (which should not occur in the sequences).
 *
 * Outputs (device): *center (int32), *width (int64: the alignment's width,
 * or -1 if a pairwise alignment failed), and msa rows r = 0..nseq-1 (row r is
 * sequence r, row stride width_cap bytes, first *width bytes of each row).
 * The rows are written only if *width <= width_cap; the width never exceeds
 * the sum of all lengths, so width_cap = sum(len) always suffices.  Sequence
 * k = pool[off[k] .. off[k]+len[k]); max_len (host) bounds every len[k];
 * nseq * max_len must stay below 2^31 (NW_ERANGE).  nseq = 0 writes nothing.
 * The workspace holds the pairwise alignments and the batch engine's slots;
 * the call is asynchronous on `stream` and not meant for graph capture.
 * ------------------------------------------------------------------------ */
int nw_center_star_workspace_size(int32_t nseq, int32_t max_len, size_t *bytes);

int nw_center_star(int32_t nseq, const uint8_t *pool, const int64_t *off, const int32_t *len,
                   int32_t max_len, nw_scoring sc, const int32_t *scores, uint8_t gap_byte,
                   int32_t *center, uint8_t *msa, int64_t width_cap, int64_t *width, void *ws,
                   size_t ws_bytes, void *stream);

/* ------------------------------------------------------------------------
 * Co-optimal alignments (Sec. 2.4: backtracking keeps every path that
 * reaches the optimal score).
 *
 * For pair k (a = pool[a_off[k] ..+a_len[k]) in the rows, b = pool[b_off[k]
 * ..+b_len[k]) in the columns, all device arrays as in nw_align_batch):
 *   scores[k]    (int32)  H(m,n);
 *   counts[k]    (uint64) the number of optimal paths modulo 2^64;
 *   saturated[k] (uint8)  1 if that number is 2^64 or more, else 0.
 * The number follows the fill: one path to every cell of the first row and
 * column, elsewhere the sum over the neighbours whose candidate equals the
 * cell's score.
 *
 * With k > 0 the call also lists the first min(k, count) optimal paths in the
 * order of a depth-first search from (m,n) that tries the diagonal, then the
 * vertical, then the horizontal move at each cell; path 0 is nw_align_batch's
 * path.  Path r of pair q goes to paths[path_off[q] + r*(a_len[q]+b_len[q])
 * ..] (moves 1/2/3 from (0,0) to (m,n), caller-computed int64 path_off with
 * room for k*(a_len+b_len) bytes), its length to path_len[q*k + r] (int32),
 * and the number listed to n_paths[q] (int32).  With k = 0, paths, path_off,
 * path_len and n_paths may be NULL.  npairs*k must fit in int32 (NW_ERANGE).
 *
 * A pair longer than max_len is skipped: scores = INT32_MIN, counts 0,
 * saturated 0, n_paths 0.  With k = 0, pairs of 2^16 cells or more are filled
 * by the four waves of a block handing strip boundaries to each other; those
 * waits are bounded, and a pair whose wait gave up (which only a device
 * fault can cause) also reports INT32_MIN, 0, 0.  The workspace (caller-owned device memory) holds
 * the job order and one slot per resident wave: the boundary column, and
 * with k > 0 the tie bits of a whole pair (half a byte per cell) and the
 * walk's state.  Smaller workspaces run fewer waves, down to one block of
 * slots (NW_ENOSPC below that).  Asynchronous on `stream`.
 * ------------------------------------------------------------------------ */
int nw_cooptimal_workspace_size(int32_t npairs, int32_t max_len, int32_t k, size_t *bytes);

int nw_cooptimal(int32_t npairs, const uint8_t *pool, const int64_t *a_off, const int32_t *a_len,
                 const int64_t *b_off, const int32_t *b_len, int32_t max_len, nw_scoring sc,
                 int32_t *scores, uint64_t *counts, uint8_t *saturated, int32_t k, uint8_t *paths,
                 const int64_t *path_off, int32_t *path_len, int32_t *n_paths, void *ws,
                 size_t ws_bytes, void *stream);

/* ------------------------------------------------------------------------
 * Band model: a learned first half-width for the certified band.
 *
 * The paper closes (Sec. 5) by naming efficiency without missing an optimal
 * alignment as the aim of further work.  The certified band above never
 * misses one; this small network only predicts, per pair, the half-width at
 * which the certificate will first succeed, so that most pairs pass on the
 * first banded sweep.  Its outputs change speed, never scores or paths.
 *
 * Features (NW_MLP_INPUTS = 259 per pair, float32):
 *   x[0..2] = m/20000, n/20000, (m-n)/20000;
 *   x[3+c]  = (count of 4-mer c in a - count in b) / max(m, n, 1), where the
 *             4-mer with codes c0 c1 c2 c3 has index 64 c0 + 16 c1 + 4 c2 + c3.
 * Network: 259 -> 64 ReLU -> 64 ReLU -> 1.  Parameters are one flat vector of
 * NW_MLP_PARAMS floats in this order: W1[64][259] (row = hidden unit), b1[64],
 * W2[64][64], b2[64], w3[64], b3.  The layers use the bfloat16 copy of W1, W2
 * and w3 (round to nearest even) and the float32 biases; activations and
 * sums are float32.
 * Target: log1p(w_cert), w_cert = the smallest half-width the certificate
 * of nw_align_batch_banded accepts for the pair's score S (capped at
 * min(m,n)).  Loss: mean pinball loss with quantile tau over the batch
 * (tau near 1 makes under-prediction, which costs a doubling, rare).
 * Optimiser: Adam, beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected.
 * ------------------------------------------------------------------------ */
#define NW_MLP_INPUTS 259
#define NW_MLP_HIDDEN 64
#define NW_MLP_PARAMS 20865

/* Model state.  Every pointer is a device array of NW_MLP_PARAMS entries owned
 * by the caller.  adam_m and adam_v (zero-initialised by the caller) are only
 * read by the training calls and may be NULL otherwise.  step (host) counts
 * the Adam updates taken; each training update increments it. */
typedef struct nw_mlp {
    float *params;         /* float32 master weights                     */
    uint16_t *params_bf16; /* bfloat16 copy (bit patterns), same layout  */
    float *adam_m;         /* Adam first moments                         */
    float *adam_v;         /* Adam second moments                        */
    int64_t step;
} nw_mlp;

/* Rewrite params_bf16 from params (after the caller sets or loads the master
 * weights). */
int nw_mlp_sync(const nw_mlp *mlp, void *stream);

/* Features of npairs pairs (same pair description as nw_align_batch) into
 * x[npairs][NW_MLP_INPUTS] (device). */
int nw_mlp_features(int32_t npairs, const uint8_t *pool, const int64_t *a_off,
                    const int32_t *a_len, const int64_t *b_off, const int32_t *b_len, float *x,
                    void *stream);

/* yhat[r] (device float32) = network output for row x[r] (r < rows). */
int nw_mlp_forward(const nw_mlp *mlp, int32_t rows, const float *x, float *yhat, void *stream);

/* Half-widths from predictions of log1p(w): w[k] = ceil(expm1(max(yhat[k],0)) *
 * (1 + margin)) clamped to [0, max(a_len[k], b_len[k])], evaluated in double.
 * margin >= 0. */
int nw_mlp_widths(int32_t npairs, const float *yhat, const int32_t *a_len, const int32_t *b_len,
                  float margin, int32_t *w, void *stream);

/* Training labels from full-grid scores (e.g. nw_align_batch with
 * NW_SCORE_ONLY): w_cert[k] (device int32, may be NULL) and target[k] =
 * log1pf(w_cert[k]) (device float32, may be NULL).  Needs a scoring for
 * which the certificate applies (2*gap < max(match, mismatch)), else
 * NW_EINVAL. */
int nw_band_labels(int32_t npairs, const int32_t *scores, const int32_t *a_len,
                   const int32_t *b_len, nw_scoring sc, int32_t *w_cert, float *target,
                   void *stream);

/* Training labels from full-grid paths (the network's target: the maximum
 * diagonal offset of the optimal path, measured beyond the straight band).
 * paths, path_off, path_len (device) as nw_align_batch returns them, with
 * a_len/b_len of the same pairs.  w_path[k] (device int32, may be NULL) =
 * the largest excursion of path k outside the corridor [min(0,D), max(0,D)],
 * D = b_len[k] - a_len[k]: the half-width of the smallest band(w) that holds
 * the path (Sec. 5's aim: a band that keeps the optimal alignment);
 * target[k] = log1pf(w_path[k]) (device float32, may be NULL).  A pair with
 * path_len[k] <= 0 gets 0. */
int nw_path_labels(int32_t npairs, const uint8_t *paths, const int64_t *path_off,
                   const int32_t *path_len, const int32_t *a_len, const int32_t *b_len,
                   int32_t *w_path, float *target, void *stream);

/* Workspace for nw_mlp_train_step / nw_mlp_train_epoch at minibatch size
 * `batch`. */
int nw_mlp_train_workspace_size(int32_t batch, size_t *bytes);

/* One training step on the minibatch rows[0..batch) of (x, target) (rows:
 * device int32 indices into x and target; NULL = rows 0..batch-1).  Computes
 * the mean pinball loss and its gradient, then, when lr > 0, one Adam update
 * of params (and params_bf16, adam_m, adam_v; mlp->step is incremented).
 * lr == 0 computes loss and gradient only.  Optional device outputs: *loss
 * (float32) and grad[NW_MLP_PARAMS] (float32).  batch >= 1; 0 < tau < 1. */
int nw_mlp_train_step(nw_mlp *mlp, int32_t batch, const float *x, const float *target,
                      const int32_t *rows, float tau, float lr, float *loss, float *grad,
                      void *ws, size_t ws_bytes, void *stream);

/* One pass over n examples in the order given by order[n] (device int32, a
 * permutation or any index list; the caller draws it): minibatch b holds
 * order[b*batch .. min(n, (b+1)*batch)).  losses (device float32
 * [ceil(n/batch)], may be NULL) gets each minibatch's loss before its update.
 * lr > 0. */
int nw_mlp_train_epoch(nw_mlp *mlp, int32_t n, const float *x, const float *target,
                       const int32_t *order, int32_t batch, float tau, float lr, float *losses,
                       void *ws, size_t ws_bytes, void *stream);

/* Learned band: nw_mlp_features, nw_mlp_forward and nw_mlp_widths (with
 * `margin`) give w_init, then nw_align_batch_banded runs with it.  Same
 * arguments and outputs as nw_align_batch_banded otherwise; scores and paths
 * equal nw_align_batch's for any model. */
int nw_align_batch_learned_workspace_size(int32_t npairs, int32_t max_len, uint32_t flags,
                                          size_t *bytes);

int nw_align_batch_learned(int32_t npairs, const uint8_t *pool, const int64_t *a_off,
                           const int32_t *a_len, const int64_t *b_off, const int32_t *b_len,
                           int32_t max_len, nw_scoring sc, uint32_t flags, const nw_mlp *mlp,
                           float margin, float fallback_frac, int32_t *scores, uint8_t *paths,
                           const int64_t *path_off, int32_t *path_len, int32_t *w_used,
                           uint8_t *status, int64_t *cells, int64_t *cells_score_only, void *ws,
                           size_t ws_bytes, void *stream);

/* ------------------------------------------------------------------------
 * Autotuner for the batch engine (nw_align_batch, nw_align_batch_banded,
 * nw_align_batch_learned, nw_allpairs_scores).  Each pass of a pair sweeps
 * 128, 256 or 512 columns per wave, whichever minimises
 *     strips x (rows per strip + 64) x step_cost(width)
 * for its height.  The built-in step costs are instruction counts of the
 * compiled loops; nw_autotune measures them instead.  It runs the given
 * sample batch (same description and buffers as nw_align_batch with paths,
 * paper scoring) with each width forced, with and without directions,
 * 3 times each, and stores the measured time per strip-row of each width,
 * normalised to 1000 for 512 columns, as the current device's cost table.
 * Synchronises `stream`; results of later calls do not depend on the table,
 * only their speed.  costs (host int32[6], may be NULL) receives the table:
 * widths 128/256/512 with directions, then score-only.  npairs >= 1.
 * nw_release_caches() restores the built-in costs.
 * ------------------------------------------------------------------------ */
int nw_autotune(int32_t npairs, const uint8_t *pool, const int64_t *a_off, const int32_t *a_len,
                const int64_t *b_off, const int32_t *b_len, int32_t max_len, int32_t *scores,
                uint8_t *paths, const int64_t *path_off, int32_t *path_len, void *ws,
                size_t ws_bytes, int32_t *costs, void *stream);

/* The current device's sweep-width cost table (host int32[6]: widths
 * 128/256/512 with directions, then score-only) and whether it was set by
 * nw_autotune or nw_set_sweep_costs (*tuned, may be NULL). */
int nw_sweep_costs(int32_t *costs, int32_t *tuned);

/* Install a cost table on the current device (host int32[6], each 1..2^20),
 * e.g. one measured by nw_autotune in an earlier process and kept by the
 * caller.  Only speed depends on it: every width gives identical results. */
int nw_set_sweep_costs(const int32_t *costs);

/* Release host-side caches: the NW_GRAPH graphs and the autotuned cost
 * tables.  Call only when no library work is in flight on any stream. */
void nw_release_caches(void);

/* ------------------------------------------------------------------------
 * Kernel timing for benchmarks.  Between nw_profile_begin() and
 * nw_profile_end() the library records a HIP event before and after every
 * kernel it launches, on that call's stream.  Call nw_profile_end() only
 * after those streams have been synchronised: it writes up to `cap` records
 * (one per kernel name: launch count and summed milliseconds) to out (host
 * memory), the number of distinct kernels to *count (host), and stops
 * recording.  Not thread-safe; meant for single-threaded benchmark drivers.
 * ------------------------------------------------------------------------ */
typedef struct nw_kernel_time {
    const char *name;   /* static storage */
    int32_t launches;
    double total_ms;
} nw_kernel_time;

int nw_profile_begin(void);
int nw_profile_end(nw_kernel_time *out, int32_t cap, int32_t *count);

#ifdef __cplusplus
}
#endif

#endif /* NW_H */
