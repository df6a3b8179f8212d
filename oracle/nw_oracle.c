/*
 * Plain CPU oracle for global (Needleman-Wunsch) alignment with a linear gap.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file; only the tests, the smoke check and the benchmark's CPU
 * baseline do.  It shares no code, header or table with the HIP library.
 *
 * What it computes (paper, Section 2):
 *  - Grid construction (Sec. 2.1): a score grid with one extra row and column,
 *    i.e. (m+1) x (n+1) cells; sequence a (length m) labels rows i, sequence b
 *    (length n) labels columns j.
 *  - Initial data (Sec. 2.2): H(0,0) = 0, and the first row and column fall by
 *    one gap penalty per cell: H(i,0) = i*g, H(0,j) = j*g.
 *  - Scoring (Sec. 2.3, Eq. 1, read as the standard linear-gap recurrence):
 *        H(i,j) = max( H(i-1,j-1) + s(a_i,b_j),  H(i-1,j) + g,  H(i,j-1) + g )
 *    with s = match if a_i == b_j else mismatch.  The paper's constants are
 *    match = +1, mismatch = -1, gap = -1.
 *  - Backtracking (Sec. 2.4): from the bottom-right cell follow the argmax.
 *    A vertical step (i-1,j) is a gap in b, a horizontal step (i,j-1) a gap in
 *    a, a diagonal step a match or mismatch.  Among tied moves the oracle takes
 *    one fixed path: diagonal, then vertical, then horizontal.  Move codes are
 *    the paper's direction codes (Sec. 3.1): 1 diagonal, 2 vertical,
 *    3 horizontal.
 *  - Multiple alignment front end (Sec. 3.2, Eq. 2): all n(n-1)/2 pairwise
 *    scores of a sequence set, as a symmetric matrix.
 *  - Co-optimal alignments (Sec. 2.4 keeps every optimal path): the number
 *    of optimal paths of a pair, modulo 2^64 with a flag for counts of 2^64
 *    and more.
 *
 * The traceback re-derives each move from H by re-evaluating the three
 * candidates (it stores no directions), except in the memory-saving mode,
 * which keeps two score rows and one direction byte per cell decided by the
 * same comparisons in the same order.
 *
 * Plain C99, -O2, no intrinsics; OpenMP only across independent pairs.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_D 1
#define ORC_U 2
#define ORC_L 3

static int32_t subst(uint8_t x, uint8_t y, int32_t match, int32_t mismatch)
{
    return x == y ? match : mismatch;
}

static int32_t max3i(int32_t d, int32_t u, int32_t l)
{
    int32_t r = d;
    if (u > r) r = u;
    if (l > r) r = l;
    return r;
}

/* Fill the full (m+1) x (n+1) int32 score matrix, row-major. */
void orc_fill(const uint8_t *a, int64_t m, const uint8_t *b, int64_t n,
              int32_t match, int32_t mismatch, int32_t gap, int32_t *H)
{
    const int64_t W = n + 1;
    H[0] = 0;
    for (int64_t j = 1; j <= n; ++j) H[j] = (int32_t)(j * gap);
    for (int64_t i = 1; i <= m; ++i) {
        int32_t *row = H + i * W;
        const int32_t *up = H + (i - 1) * W;
        row[0] = (int32_t)(i * gap);
        for (int64_t j = 1; j <= n; ++j) {
            int32_t d = up[j - 1] + subst(a[i - 1], b[j - 1], match, mismatch);
            int32_t u = up[j] + gap;
            int32_t l = row[j - 1] + gap;
            row[j] = max3i(d, u, l);
        }
    }
}

/* Move chosen at cell (i,j) > (0,0), re-derived from H. */
static int move_at(const int32_t *H, int64_t W, const uint8_t *a, const uint8_t *b,
                   int64_t i, int64_t j, int32_t match, int32_t mismatch, int32_t gap)
{
    int32_t h = H[i * W + j];
    if (i > 0 && j > 0) {
        int32_t d = H[(i - 1) * W + (j - 1)] + subst(a[i - 1], b[j - 1], match, mismatch);
        if (h == d) return ORC_D;
    }
    if (i > 0) {
        int32_t u = H[(i - 1) * W + j] + gap;
        if (h == u) return ORC_U;
    }
    return ORC_L;
}

/* Traceback from (m,n) to (0,0) over a full H; moves written in forward
 * order (from (0,0) to (m,n)).  Returns the number of moves. */
int64_t orc_traceback(const int32_t *H, const uint8_t *a, int64_t m, const uint8_t *b, int64_t n,
                      int32_t match, int32_t mismatch, int32_t gap, uint8_t *path)
{
    const int64_t W = n + 1;
    int64_t i = m, j = n, k = 0;
    while (i > 0 || j > 0) {
        int mv = move_at(H, W, a, b, i, j, match, mismatch, gap);
        path[k++] = (uint8_t)mv;
        if (mv == ORC_D) { --i; --j; }
        else if (mv == ORC_U) { --i; }
        else { --j; }
    }
    for (int64_t p = 0, q = k - 1; p < q; ++p, --q) {
        uint8_t t = path[p]; path[p] = path[q]; path[q] = t;
    }
    return k;
}

/* Per-cell move codes of the whole grid (debug dump): 0 at (0,0), 2 on
 * column 0, 3 on row 0, else the move the traceback would take there. */
void orc_dirs(const int32_t *H, const uint8_t *a, int64_t m, const uint8_t *b, int64_t n,
              int32_t match, int32_t mismatch, int32_t gap, uint8_t *codes)
{
    const int64_t W = n + 1;
    for (int64_t i = 0; i <= m; ++i)
        for (int64_t j = 0; j <= n; ++j)
            codes[i * W + j] = (i == 0 && j == 0) ? 0
                               : (uint8_t)move_at(H, W, a, b, i, j, match, mismatch, gap);
}

/* Score only, two rows. */
int32_t orc_score(const uint8_t *a, int64_t m, const uint8_t *b, int64_t n,
                  int32_t match, int32_t mismatch, int32_t gap)
{
    int32_t *prev = (int32_t *)malloc((size_t)(n + 1) * sizeof(int32_t));
    int32_t *cur = (int32_t *)malloc((size_t)(n + 1) * sizeof(int32_t));
    if (!prev || !cur) { free(prev); free(cur); return INT32_MIN; }
    for (int64_t j = 0; j <= n; ++j) prev[j] = (int32_t)(j * gap);
    for (int64_t i = 1; i <= m; ++i) {
        cur[0] = (int32_t)(i * gap);
        for (int64_t j = 1; j <= n; ++j) {
            int32_t d = prev[j - 1] + subst(a[i - 1], b[j - 1], match, mismatch);
            int32_t u = prev[j] + gap;
            int32_t l = cur[j - 1] + gap;
            cur[j] = max3i(d, u, l);
        }
        int32_t *t = prev; prev = cur; cur = t;
    }
    int32_t s = prev[n];
    free(prev); free(cur);
    return s;
}

/* Memory-saving alignment: two score rows plus one direction byte per cell,
 * decided by the same comparisons in the same order as move_at(). */
static int orc_align_tworow(const uint8_t *a, int64_t m, const uint8_t *b, int64_t n,
                            int32_t match, int32_t mismatch, int32_t gap,
                            int32_t *score, uint8_t *path, int64_t *path_len)
{
    const int64_t W = n + 1;
    int32_t *prev = (int32_t *)malloc((size_t)W * sizeof(int32_t));
    int32_t *cur = (int32_t *)malloc((size_t)W * sizeof(int32_t));
    uint8_t *dir = (uint8_t *)malloc((size_t)((m + 1) * W));
    if (!prev || !cur || !dir) { free(prev); free(cur); free(dir); return -1; }
    for (int64_t j = 0; j <= n; ++j) { prev[j] = (int32_t)(j * gap); dir[j] = ORC_L; }
    dir[0] = 0;
    for (int64_t i = 1; i <= m; ++i) {
        uint8_t *drow = dir + i * W;
        cur[0] = (int32_t)(i * gap);
        drow[0] = ORC_U;
        for (int64_t j = 1; j <= n; ++j) {
            int32_t d = prev[j - 1] + subst(a[i - 1], b[j - 1], match, mismatch);
            int32_t u = prev[j] + gap;
            int32_t l = cur[j - 1] + gap;
            int32_t h = max3i(d, u, l);
            cur[j] = h;
            drow[j] = (h == d) ? ORC_D : (h == u) ? ORC_U : ORC_L;
        }
        int32_t *t = prev; prev = cur; cur = t;
    }
    *score = prev[n];
    int64_t i = m, j = n, k = 0;
    while (i > 0 || j > 0) {
        int mv = dir[i * W + j];
        path[k++] = (uint8_t)mv;
        if (mv == ORC_D) { --i; --j; }
        else if (mv == ORC_U) { --i; }
        else { --j; }
    }
    for (int64_t p = 0, q = k - 1; p < q; ++p, --q) {
        uint8_t t = path[p]; path[p] = path[q]; path[q] = t;
    }
    *path_len = k;
    free(prev); free(cur); free(dir);
    return 1;
}

/* Score and traceback path of one pair.  Uses the full int32 matrix when it
 * needs at most full_limit_bytes, else the two-row mode.  Returns the mode
 * used (0 = full matrix, 1 = two rows + direction bytes) or -1 if out of
 * memory.  path needs room for m + n moves. */
int orc_align(const uint8_t *a, int64_t m, const uint8_t *b, int64_t n,
              int32_t match, int32_t mismatch, int32_t gap,
              int32_t *score, uint8_t *path, int64_t *path_len, int64_t full_limit_bytes)
{
    const int64_t cells = (m + 1) * (n + 1);
    if (cells * 4 <= full_limit_bytes) {
        int32_t *H = (int32_t *)malloc((size_t)cells * sizeof(int32_t));
        if (H) {
            orc_fill(a, m, b, n, match, mismatch, gap, H);
            *score = H[cells - 1];
            *path_len = orc_traceback(H, a, m, b, n, match, mismatch, gap, path);
            free(H);
            return 0;
        }
    }
    return orc_align_tworow(a, m, b, n, match, mismatch, gap, score, path, path_len);
}

/* Pairs in order of decreasing m*n (ties by index), so that OpenMP's dynamic
 * schedule starts the largest pairs first. */
static int64_t *order_by_cost(int32_t npairs, const int32_t *a_len, const int32_t *b_len)
{
    int64_t *ord = (int64_t *)malloc((size_t)(npairs > 0 ? npairs : 1) * sizeof(int64_t));
    for (int32_t k = 0; k < npairs; ++k) ord[k] = k;
    /* insertion sort is too slow for 1e5 pairs: use a simple merge sort */
    int64_t *tmp = (int64_t *)malloc((size_t)(npairs > 0 ? npairs : 1) * sizeof(int64_t));
    for (int64_t w = 1; w < npairs; w *= 2) {
        for (int64_t lo = 0; lo < npairs; lo += 2 * w) {
            int64_t mid = lo + w < npairs ? lo + w : npairs;
            int64_t hi = lo + 2 * w < npairs ? lo + 2 * w : npairs;
            int64_t p = lo, q = mid, r = lo;
            while (p < mid && q < hi) {
                int64_t cp = (int64_t)a_len[ord[p]] * b_len[ord[p]];
                int64_t cq = (int64_t)a_len[ord[q]] * b_len[ord[q]];
                if (cp > cq || (cp == cq && ord[p] < ord[q])) tmp[r++] = ord[p++];
                else tmp[r++] = ord[q++];
            }
            while (p < mid) tmp[r++] = ord[p++];
            while (q < hi) tmp[r++] = ord[q++];
        }
        memcpy(ord, tmp, (size_t)npairs * sizeof(int64_t));
    }
    free(tmp);
    return ord;
}

/* Batch of independent pairs.  paths == NULL gives scores only.  Returns the
 * number of pairs that ran in two-row mode, or -1 on allocation failure. */
int64_t orc_align_batch(int32_t npairs, const uint8_t *pool,
                        const int64_t *a_off, const int32_t *a_len,
                        const int64_t *b_off, const int32_t *b_len,
                        int32_t match, int32_t mismatch, int32_t gap,
                        int32_t *scores, uint8_t *paths, const int64_t *path_off,
                        int32_t *path_len, int32_t nthreads, int64_t full_limit_bytes)
{
    int64_t *ord = order_by_cost(npairs, a_len, b_len);
    int64_t tworow = 0, fail = 0;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
#pragma omp parallel for schedule(dynamic, 1) reduction(+ : tworow, fail)
    for (int64_t q = 0; q < npairs; ++q) {
        int64_t k = ord[q];
        const uint8_t *a = pool + a_off[k];
        const uint8_t *b = pool + b_off[k];
        if (paths) {
            int32_t s;
            int64_t len;
            int mode = orc_align(a, a_len[k], b, b_len[k], match, mismatch, gap,
                                 &s, paths + path_off[k], &len, full_limit_bytes);
            if (mode < 0) { fail += 1; continue; }
            tworow += mode;
            scores[k] = s;
            path_len[k] = (int32_t)len;
        } else {
            scores[k] = orc_score(a, a_len[k], b, b_len[k], match, mismatch, gap);
        }
    }
    free(ord);
    return fail ? -1 : tworow;
}

/* All-pairs similarity matrix (paper Sec. 3.2): out[i*nseq+j] = score of
 * sequence i (rows) against sequence j (columns) for i < j, mirrored to
 * j > i; the diagonal is the score of a sequence against itself, computed
 * by the same recurrence. */
void orc_allpairs(int32_t nseq, const uint8_t *pool, const int64_t *off, const int32_t *len,
                  int32_t match, int32_t mismatch, int32_t gap, int32_t *out, int32_t nthreads)
{
    const int64_t npairs = (int64_t)nseq * (nseq - 1) / 2;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t p = 0; p < npairs + nseq; ++p) {
        int64_t i, j;
        if (p < npairs) {
            /* unrank p into (i, j), i < j, row-major over the upper triangle */
            i = 0;
            int64_t rem = p;
            while (rem >= nseq - 1 - i) { rem -= nseq - 1 - i; ++i; }
            j = i + 1 + rem;
        } else {
            i = j = p - npairs;
        }
        int32_t s = orc_score(pool + off[i], len[i], pool + off[j], len[j], match, mismatch, gap);
        out[i * nseq + j] = s;
        out[j * nseq + i] = s;
    }
}

int orc_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/*
 * Co-optimal alignments (Sec. 2.4 keeps every path that reaches the optimal
 * score).  N(i,j), the number of optimal paths from (0,0) to (i,j), follows
 * the fill: N(0,0) = 1; a cell of the first row or column has one path;
 * elsewhere N(i,j) is the sum of N over the neighbours whose candidate
 * (H(i-1,j-1) + s, H(i-1,j) + g, H(i,j-1) + g) equals H(i,j).  Counts are
 * kept modulo 2^64 together with a flag F(i,j) = [true count >= 2^64]: it is
 * set when a summed neighbour has it set or when the sum wraps.
 * Two rows of H, N and F.  Returns 0, or -1 if memory runs out.
 */
int orc_count(const uint8_t *a, int64_t m, const uint8_t *b, int64_t n,
              int32_t match, int32_t mismatch, int32_t gap,
              int32_t *score, uint64_t *count, uint8_t *saturated)
{
    int32_t *H0 = malloc((size_t)(n + 1) * sizeof(int32_t));
    int32_t *H1 = malloc((size_t)(n + 1) * sizeof(int32_t));
    uint64_t *N0 = malloc((size_t)(n + 1) * sizeof(uint64_t));
    uint64_t *N1 = malloc((size_t)(n + 1) * sizeof(uint64_t));
    uint8_t *F0 = malloc((size_t)(n + 1));
    uint8_t *F1 = malloc((size_t)(n + 1));
    if (!H0 || !H1 || !N0 || !N1 || !F0 || !F1) {
        free(H0); free(H1); free(N0); free(N1); free(F0); free(F1);
        return -1;
    }
    for (int64_t j = 0; j <= n; ++j) {
        H0[j] = (int32_t)(j * gap);
        N0[j] = 1;
        F0[j] = 0;
    }
    for (int64_t i = 1; i <= m; ++i) {
        H1[0] = (int32_t)(i * gap);
        N1[0] = 1;
        F1[0] = 0;
        for (int64_t j = 1; j <= n; ++j) {
            int32_t d = H0[j - 1] + subst(a[i - 1], b[j - 1], match, mismatch);
            int32_t u = H0[j] + gap;
            int32_t l = H1[j - 1] + gap;
            int32_t h = max3i(d, u, l);
            uint64_t s = 0;
            uint8_t f = 0;
            if (d == h) {
                uint64_t t = s + N0[j - 1];
                f |= (uint8_t)(F0[j - 1] | (t < s));
                s = t;
            }
            if (u == h) {
                uint64_t t = s + N0[j];
                f |= (uint8_t)(F0[j] | (t < s));
                s = t;
            }
            if (l == h) {
                uint64_t t = s + N1[j - 1];
                f |= (uint8_t)(F1[j - 1] | (t < s));
                s = t;
            }
            H1[j] = h;
            N1[j] = s;
            F1[j] = f;
        }
        int32_t *th = H0; H0 = H1; H1 = th;
        uint64_t *tn = N0; N0 = N1; N1 = tn;
        uint8_t *tf = F0; F0 = F1; F1 = tf;
    }
    *score = H0[n];
    *count = N0[n];
    *saturated = F0[n];
    free(H0); free(H1); free(N0); free(N1); free(F0); free(F1);
    return 0;
}

/* orc_count over a batch of pairs, OpenMP across pairs.  Returns -1 if any
 * pair ran out of memory, else 0. */
int orc_count_batch(int32_t npairs, const uint8_t *pool,
                    const int64_t *a_off, const int32_t *a_len,
                    const int64_t *b_off, const int32_t *b_len,
                    int32_t match, int32_t mismatch, int32_t gap,
                    int32_t *scores, uint64_t *counts, uint8_t *saturated, int32_t nthreads)
{
    int64_t *ord = order_by_cost(npairs, a_len, b_len);
    int64_t fail = 0;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
#pragma omp parallel for schedule(dynamic, 1) reduction(+ : fail)
    for (int64_t q = 0; q < npairs; ++q) {
        int64_t k = ord[q];
        if (orc_count(pool + a_off[k], a_len[k], pool + b_off[k], b_len[k], match, mismatch, gap,
                      &scores[k], &counts[k], &saturated[k]) < 0)
            fail += 1;
    }
    free(ord);
    return fail ? -1 : 0;
}
