/*
 * ssh.h -- C ABI of the SSH (Sketch, Shingle & Hash) hot path on MI355X (gfx950).
 *
 * Luo & Shrivastava, "SSH (Sketch, Shingle, & Hash) for Indexing Massive-Scale
 * Time Series", arXiv 1610.07328.  The library computes, for a batch of time
 * series held in device memory:
 *
 *   ssh_sketch     sign stream B_X of a sliding random filter   (Section 4.1)
 *   ssh_shingle    weighted set S_X of length-n bit shingles     (Section 4.2)
 *   ssh_cws        weighted MinHash values by consistent weighted sampling
 *                  (Section 4.3; Section 2, eqs. WJaccardDef / CollProb)
 *   ssh_band_keys  one key per hash table from K hash values     (Algorithm 1)
 *   ssh_cws_band_keys  the two above in one pass
 *   ssh_wmh_int    weighted MinHash by integer replication, integer only
 *                  (Section 2, eq. CollProb; Section 4, one-pass hashing)
 *   ssh_table_build  the L hash tables                           (Algorithm 1)
 *   ssh_table_insert / ssh_table_delete  the tables updated without a rebuild
 *   ssh_probe      retrieved set R of each query, ranked         (Algorithm 2)
 *   dtw_rerank     top-k of R by banded DTW distance             (Section 2.1,
 *                  last step of Algorithm 2)
 *   dtw_rerank_lb  the same, LB_Keogh bounds skipping far candidates
 *
 * Conventions shared by every entry point:
 *   - Pointers are DEVICE pointers unless marked [host].  The caller owns every
 *     buffer; the library never allocates device memory.  Buffers that hold
 *     per-series data are indexed by series id 0..N-1.
 *   - `stream` is a hipStream_t (NULL for the null stream).  Work is enqueued
 *     asynchronously on it; nothing is synchronised.  Errors raised by a kernel
 *     after launch surface at the caller's next synchronisation.
 *   - Validation is synchronous: on a bad argument the call returns SSH_EINVAL
 *     (or SSH_EUNSUPPORTED for a shape outside the implemented range) and
 *     enqueues nothing.  A failed launch returns SSH_EDEVICE.  The reason is
 *     available from ssh_last_error() on the calling thread.  Outputs are
 *     undefined after an error.
 *   - Ragged batches use CSR offsets: series s occupies [off[s], off[s+1]) of
 *     its value array, off has N + 1 entries, off[0] = 0, non-decreasing.
 *   - Edge cases are not errors: a series shorter than the filter has no bits,
 *     a stream shorter than n has no shingles, and a series without shingles
 *     gets SSH_HV_EMPTY hash values and SSH_KEY_EMPTY keys (it never matches a
 *     query).
 */
#ifndef SSH_H_
#define SSH_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t ssh_status;
#define SSH_OK 0
#define SSH_EINVAL (-1)
#define SSH_EUNSUPPORTED (-2)
#define SSH_EDEVICE (-3)
#define SSH_ECAPACITY (-4)

#define SSH_HV_EMPTY UINT64_MAX  /* hash value of a series without shingles */
#define SSH_KEY_EMPTY UINT64_MAX /* band key of a series without shingles   */
#define SSH_MAX_W 256            /* longest supported filter                */
#define SSH_MAX_N 16             /* longest supported shingle               */
#define SSH_LNS_ENTRIES 65536    /* entries of the prepared ln-count table  */
#define SSH_CWS_KEY_WEIGHTS 31   /* weights keyed for every token code      */
#define SSH_CWS_RUN_CAP 4096     /* counts keyed for the codes 0 and 2^n-1  */
#define SSH_MAX_C 4096           /* largest candidate cap of ssh_probe      */
#define SSH_MAX_K 1024           /* largest k of dtw_rerank                 */
#define SSH_MAX_BAND 255         /* largest Sakoe-Chiba radius of a dtw_rerank pair */
#define SSH_NOALLOC_SCRATCH_BYTES (32u << 20) /* static scratch of dtw_rerank_noalloc, per device */

/* [host] Name of a status code, and the detail of the last error raised on the
 * calling thread ("" if none).  Both strings are owned by the library. */
const char* ssh_status_str(ssh_status s);
const char* ssh_last_error(void);

/* [host] Size helpers.
 * ssh_num_bits: length N_B of the sign stream of a series of length m, i.e. the
 *   number of window starts i*delta with i*delta + W <= m: (m - W)/delta + 1,
 *   or 0 when m < W (Section 4.1; the paper's N_B = (m-W)/delta is read with
 *   the +1 its worked example needs).
 * ssh_num_shingles: number of length-n shingles of a stream of nbits bits:
 *   nbits - n + 1, or 0 when nbits < n (Section 4.2). */
int32_t ssh_num_bits(int64_t m, int32_t W, int32_t delta);
int32_t ssh_num_shingles(int32_t nbits, int32_t n);

/* [host] Layout plan of a ragged batch.  From the series offsets x_off[N+1]
 * (host copy) it fills, all [host]:
 *   bit_word_off[N+1]  offsets (in uint64 words) of each series' packed sign
 *                      stream: ceil(N_B / 64) words per series;
 *   hist_off[N+1]      offsets of each series' weighted-set slots: capacity
 *                      ssh_num_shingles(N_B, n) per series;
 *   max_nbits          largest N_B in the batch (may be NULL).
 * Returns SSH_EINVAL on bad sizes or decreasing offsets. */
ssh_status ssh_plan(const int64_t* x_off, int64_t N, int32_t W, int32_t delta, int32_t n,
                    int64_t* bit_word_off, int64_t* hist_off, int32_t* max_nbits);

/* Sliding-window sign sketch (Section 4.1, definition of B_X and its worked
 * example).  For series s with values x[x_off[s] .. x_off[s+1]) and window i in
 * [0, N_B), bit i is 1 when r . x[i*delta .. i*delta + W) >= 0 and 0 otherwise
 * (+1 / -1 of the paper).  The sign is that of the float64 sum of the exact
 * float32 products taken in ascending filter index; windows whose fast
 * half-precision dot product is within a proven error margin of zero are
 * recomputed that way, so the bits are exact whatever the input.
 *   x            float32 values (finite; non-finite windows take the float64
 *                path, whose comparison with NaN yields 0)
 *   x_off        int64 [N+1] series offsets
 *   r            [host] float32 [W] filter, 1 <= W <= SSH_MAX_W, finite
 *   delta        step, >= 1
 *   bits         uint64 packed streams: bit i of series s is bit (i & 63) of
 *                word bit_word_off[s] + (i >> 6); unused high bits are 0
 *   bit_word_off int64 [N+1] from ssh_plan (same x_off, W, delta)
 *   nbits        int32 [N] output: N_B of each series
 *   repair_count uint64 [1] or NULL: incremented by the number of windows
 *                recomputed in float64 */
ssh_status ssh_sketch(const float* x, const int64_t* x_off, int64_t N, const float* r, int32_t W,
                      int32_t delta, uint64_t* bits, const int64_t* bit_word_off, int32_t* nbits,
                      uint64_t* repair_count, void* stream);

/* Weighted set of length-n shingles (Section 4.2, eq. "set").  Every one of the
 * N_B - n + 1 length-n substrings of a series' stream is a token with weight =
 * its number of occurrences.  A token is the integer whose binary digits, most
 * significant first, are the n bits in stream order.
 *   bits, bit_word_off, nbits   as produced by ssh_sketch
 *   n            1..SSH_MAX_N
 *   codes        uint32 output: series s writes its distinct tokens in
 *                ascending order to codes[hist_off[s] .. + n_distinct[s])
 *   counts       uint32 output, parallel to codes (>= 1)
 *   hist_off     int64 [N+1] from ssh_plan (capacity N_B - n + 1 per series)
 *   n_distinct   int32 [N] output */
ssh_status ssh_shingle(const uint64_t* bits, const int64_t* bit_word_off, const int32_t* nbits,
                       int64_t N, int32_t n, uint32_t* codes, uint32_t* counts,
                       const int64_t* hist_off, int32_t* n_distinct, void* stream);

/* Random numbers of consistent weighted sampling, one triple per (token k,
 * hash j), code-major: element [k * H + j] of each array.  They are inputs,
 * drawn by the caller: r ~ Gamma(2,1) (0 < r < 1e5), lnc = ln c with
 * c ~ Gamma(2,1), beta ~ U[0,1).  a1, lnS, k16 and rb are scratch tables the
 * caller allocates and fills once with ssh_cws_prepare. */
typedef struct {
  int32_t n;          /* token length; tables have 2^n rows */
  int32_t H;          /* hashes per series, >= 1 */
  const double* r;    /* [2^n * H] */
  const double* lnc;  /* [2^n * H] */
  const double* beta; /* [2^n * H] */
  double* a1;         /* [2^n * H] prepared: ln a of a token of weight 1 */
  double* lnS;        /* [SSH_LNS_ENTRIES] prepared: correctly rounded ln s */
  uint16_t* k16;      /* [ssh_cws_key_table_elems(n, H)]: prepared 16-bit
                         monotone keys of ln a, R = SSH_CWS_KEY_WEIGHTS * 2^n +
                         2 * SSH_CWS_RUN_CAP + 1 rows: one per (code, weight
                         1..SSH_CWS_KEY_WEIGHTS), then the codes 0 and 2^n - 1 at
                         weights 1..SSH_CWS_RUN_CAP, then one padding row; stored
                         in column chunks of 128 hashes, chunk by chunk, each
                         row-major (see ssh_cws_key_table_elems); the table must
                         stay below 2^31 bytes */
  double* rb;         /* [2^n * H * 2] prepared: r and beta of (k, j) side by side at
                         [2 (k * H + j)] and [2 (k * H + j) + 1], so that a winner's
                         t takes one 16-byte read */
} ssh_cws_tables;

/* Elements (uint16) of the key table tab->k16 for token length n and H
 * hashes: R rows times the chunks' widths, chunk q holding hashes
 * 128 q .. min(128 (q + 1), H) - 1 at a row width of that count rounded up
 * to even, or of 128 when that is above 96 (a row then starts on a 256-byte
 * boundary of its chunk).  Returns 0 for n outside 1..SSH_MAX_N or H < 1. */
int64_t ssh_cws_key_table_elems(int32_t n, int32_t H);

/* Fill tab->a1, tab->lnS, tab->k16 and tab->rb from the draws (device work on
 * `stream`).  tab is a [host] struct of device pointers.  A draw outside the
 * ranges above raises a device flag that ssh_check_device_errors reports.
 * Returns SSH_EINVAL for n outside 1..SSH_MAX_N, H < 1 or a null pointer. */
ssh_status ssh_cws_prepare(const ssh_cws_tables* tab, void* stream);

/* Weighted MinHash of every weighted set (Section 4.3), by Ioffe's improved
 * consistent weighted sampling.  For hash j and every token k of weight S_k:
 *     t = floor(ln S_k / r + beta),  ln y = r (t - beta),  ln a = ln c - ln y - r
 * each step one correctly rounded float64 operation in this order, ln S_k
 * correctly rounded.  The sample is k* = argmin_k ln a (ties to the smaller k)
 * with its t*, stored as hv = min(t*, 2^47 - 1) << 16 | k* (at most 2^63 - 1,
 * so never SSH_HV_EMPTY, whatever k* is).  The probability
 * that two sets agree on hv equals their weighted Jaccard similarity
 * (eq. CollProb).
 *   codes, counts, hist_off, n_distinct  as produced by ssh_shingle
 *   tab          [host] struct of device tables, prepared
 *   hv           uint64 [N * H] output, series-major; SSH_HV_EMPTY for a
 *                series with no token */
ssh_status ssh_cws(const uint32_t* codes, const uint32_t* counts, const int64_t* hist_off,
                   const int32_t* n_distinct, int64_t N, const ssh_cws_tables* tab, uint64_t* hv,
                   void* stream);

/* Weighted MinHash by integer replication (Section 2, eqs. WJaccardDef and
 * CollProb; the tokens hashed with a running minimum, Section 4, Discussions
 * and Practical Issues).  A token of
 * integer weight n_c stands for the n_c pairs (c, j), j = 1..n_c, and hash k
 * keeps the pair of smallest
 *     v_k(c, j) = mix(s_k ^ (c << 32 | j)),  s_k = mix(seed + (k + 1) * 0x9E3779B97F4A7C15),
 * mix the SplitMix64 output function (as in ssh_band_keys).  Equal v_k resolve
 * to the pair met first in input order (tokens as stored, then j ascending).
 * The value stored is hv = c << 32 | j.  Two sets agree on hv with probability
 * equal to their generalized Jaccard similarity, as for ssh_cws, with integer
 * arithmetic only; the work is sum of counts x H per series.
 *   codes, counts, hist_off, n_distinct  as for ssh_cws (any token order)
 *   H            hashes per series, 1..65536
 *   hv           uint64 [N * H] output, series-major; SSH_HV_EMPTY for a
 *                series whose counts sum to zero
 * Returns SSH_EINVAL for N < 0, H out of range or a null pointer (N > 0). */
ssh_status ssh_wmh_int(const uint32_t* codes, const uint32_t* counts, const int64_t* hist_off,
                       const int32_t* n_distinct, int64_t N, int32_t H, uint64_t seed, uint64_t* hv,
                       void* stream);

/* Band keys (Algorithm 1, one key per hash table).  Table l is keyed by the K
 * hash values hv[s*H + l*K .. + K) (H = K*L) folded with the SplitMix64 output
 * function mix: h = mix(seed + (l+1) * 0x9E3779B97F4A7C15); h = mix(h ^ hv_j)
 * for each j in order; key = h, moved to SSH_KEY_EMPTY - 1 if it equals
 * SSH_KEY_EMPTY.  A series with SSH_HV_EMPTY values gets SSH_KEY_EMPTY.
 *   keys         uint64 [N * L] output, series-major */
ssh_status ssh_band_keys(const uint64_t* hv, int64_t N, int32_t K, int32_t L, uint64_t seed,
                         uint64_t* keys, void* stream);

/* ssh_cws and ssh_band_keys in one pass (Section 4.3, then Algorithm 1): hv
 * and keys are exactly what ssh_cws followed by ssh_band_keys(hv, N, K, L,
 * seed) write, with the keys folded from the hash values while the CWS kernel
 * still holds them, so hv is not read back.  Shapes with H > 256 run the two
 * steps as separate kernels.  Arguments as for those two calls; additionally
 * returns SSH_EINVAL unless K * L == tab->H. */
ssh_status ssh_cws_band_keys(const uint32_t* codes, const uint32_t* counts,
                             const int64_t* hist_off, const int32_t* n_distinct, int64_t N,
                             const ssh_cws_tables* tab, int32_t K, int32_t L, uint64_t seed,
                             uint64_t* hv, uint64_t* keys, void* stream);

/* [host] Workspace bytes needed by ssh_table_build for N series and L tables. */
size_t ssh_table_workspace_bytes(int64_t N, int32_t L);

/* Hash tables (Algorithm 1).  Table l lists every (key, id) pair of the batch
 * ordered by the top B bits of the key, B = 24 when N <= 2^24 and 32
 * otherwise, ids ascending among equal top bits (a stable sort of ids
 * 0..N-1).  A bucket is the set of ids with one full key; ssh_probe finds it
 * inside the run of its top B bits.
 *   keys         uint64 [N * L] from ssh_band_keys; N <= 2^32 - 1
 *   tab_keys     uint64 [L * N] output, table-major
 *   tab_ids      uint32 [L * N] output, table-major
 *   ws, ws_bytes device workspace, at least ssh_table_workspace_bytes(N, L) */
ssh_status ssh_table_build(const uint64_t* keys, int64_t N, int32_t L, uint64_t* tab_keys,
                           uint32_t* tab_ids, void* ws, size_t ws_bytes, void* stream);

/* [host] Workspace bytes needed by ssh_table_insert for M new series. */
size_t ssh_table_insert_workspace_bytes(int64_t M, int32_t L);

/* Insert M new series into built tables (Algorithm 1's tables, updated in
 * place of a rebuild: with data-independent hashing, Section 1, new series
 * need no change to the hash functions or the other entries).  The new series
 * get ids id_base .. id_base+M-1, above every id in the tables (id_base = N
 * for tables that never lost a series); their band keys are new_keys
 * (series-major [M * L], from ssh_band_keys or ssh_cws_band_keys).  The output
 * tables are exactly what ssh_table_build writes for the N + M series when
 * id_base = N: the new entries are sorted by themselves and merged.  The probe
 * needs their keys and hash values at rows id_base .. of db_keys and db_hv.
 *   tab_keys, tab_ids   [L * N] tables of N entries
 *   out_keys, out_ids   [L * (N + M)] output tables, not aliasing the inputs
 *   ws, ws_bytes        at least ssh_table_insert_workspace_bytes(M, L)
 * Returns SSH_EUNSUPPORTED when N and N + M lie on different sides of 2^24
 * (the tables' sort width changes there: build them again). */
ssh_status ssh_table_insert(const uint64_t* tab_keys, const uint32_t* tab_ids, int64_t N,
                            const uint64_t* new_keys, int64_t M, int32_t L, int64_t id_base,
                            uint64_t* out_keys, uint32_t* out_ids, void* ws, size_t ws_bytes,
                            void* stream);

/* [host] Workspace bytes needed by ssh_table_delete for tables of N entries. */
size_t ssh_table_delete_workspace_bytes(int64_t N, int32_t L);

/* Delete series from built tables: every table keeps, in order, the entries
 * whose id is not marked dead, so the result is the tables a build over the
 * surviving series would give, with the surviving series keeping their ids
 * (ids are not renumbered; the probe reads db_keys and db_hv by id, so their
 * rows stay in place).  Probe the result with N = n_live.
 *   tab_keys, tab_ids  [L * N] tables
 *   dead               uint8 [id_bound]: 1 for a series to delete
 *   n_live             number of entries every table keeps (N minus the
 *                      number of deleted series present); a table that keeps
 *                      another number raises a device flag
 *   out_keys, out_ids  [L * n_live] output tables, not aliasing the inputs
 *   ws, ws_bytes       at least ssh_table_delete_workspace_bytes(N, L)
 * Returns SSH_EUNSUPPORTED when N and n_live lie on different sides of 2^24. */
ssh_status ssh_table_delete(const uint64_t* tab_keys, const uint32_t* tab_ids, int64_t N, int32_t L,
                            const uint8_t* dead, int64_t id_bound, int64_t n_live,
                            uint64_t* out_keys, uint32_t* out_ids, void* ws, size_t ws_bytes,
                            void* stream);

/* [host] Workspace bytes needed by ssh_probe for nq queries, L tables and C
 * candidates. */
size_t ssh_probe_workspace_bytes(int32_t nq, int32_t L, int32_t C);

/* Probe (Algorithm 2).  For query q the retrieved set R is the union over
 * tables l of the bucket with key q_keys[q*L + l].  Members of R are ranked by
 * the number of the H hash values they share with the query (ties to the
 * smaller id) and the first min(|R|, C) are returned.  A query without
 * shingles retrieves nothing.
 *   tab_keys, tab_ids  from ssh_table_build over db_keys
 *   db_keys      uint64 [N * L], db_hv uint64 [N * H]: the indexed series
 *   q_keys       uint64 [nq * L], q_hv uint64 [nq * H]: the queries
 *   C            1..SSH_MAX_C
 *   cand         int64 [nq * C] output: ranked ids, -1 after ncand[q]
 *   ncand        int32 [nq] output: min(|R|, C)
 *   r_size       int64 [nq] output: |R|
 *   ws, ws_bytes device workspace, at least ssh_probe_workspace_bytes(nq, L, C);
 *                each query's entries are split over several workgroups whose
 *                partial rankings are merged there */
ssh_status ssh_probe(const uint64_t* tab_keys, const uint32_t* tab_ids, int64_t N, int32_t L,
                     const uint64_t* db_keys, const uint64_t* db_hv, int32_t H,
                     const uint64_t* q_keys, const uint64_t* q_hv, int32_t nq, int32_t C,
                     int64_t* cand, int32_t* ncand, int64_t* r_size, void* ws, size_t ws_bytes,
                     void* stream);

/* ssh_probe for callers that want no silent truncation: the same outputs
 * (cand truncated at C, r_size the full |R|), then the call synchronises
 * `stream`, reads r_size back and returns SSH_ECAPACITY when some query
 * retrieved more than C series (the count and the largest |R| are in
 * ssh_last_error()); SSH_OK otherwise.  Blocks the host until the probe ends. */
ssh_status ssh_probe_strict(const uint64_t* tab_keys, const uint32_t* tab_ids, int64_t N,
                            int32_t L, const uint64_t* db_keys, const uint64_t* db_hv, int32_t H,
                            const uint64_t* q_keys, const uint64_t* q_hv, int32_t nq, int32_t C,
                            int64_t* cand, int32_t* ncand, int64_t* r_size, void* ws,
                            size_t ws_bytes, void* stream);

/* [host] Workspace bytes needed by dtw_rerank for nq queries of C candidates. */
size_t ssh_rerank_workspace_bytes(int32_t nq, int32_t C);

/* DTW re-rank (Section 2.1; last step of Algorithm 2).  For each query q and
 * each of its ncand[q] candidates X = cand[q*C + c], the banded DTW distance:
 * cost (q_i - x_j)^2, steps (1,0), (0,1), (1,1) from (0,0) to (lq-1, lx-1),
 * Sakoe-Chiba band |i - j| <= r with r = floor(band_frac * max(lq, lx)) taken
 * per pair from that pair's own lengths, distance = sqrt of the least total
 * cost (+inf when |lq - lx| > r or a length is 0).  Accumulated in float32.
 * Queries and candidates may all have different lengths.  The k nearest by
 * (distance, id) are returned.
 *   q, q_off     float32 query values and int64 [nq+1] offsets (ragged)
 *   db, db_off   float32 series values and int64 [N+1] offsets (ragged); N series
 *   cand, ncand  from ssh_probe (C columns); ids must lie in [0, N)
 *   band_frac    in [0, 1]; a pair whose radius exceeds SSH_MAX_BAND gets +inf
 *                and raises a device flag (ssh_check_device_errors)
 *   k            1..SSH_MAX_K, k <= C; nq * C must stay below 2^31
 *   out_id       int64 [nq * k] output, -1 padding
 *   out_dist     float32 [nq * k] output, +inf padding
 *   ws, ws_bytes at least ssh_rerank_workspace_bytes(nq, C); on return (after
 *                the stream is synchronised) its first nq * C float32 values
 *                are every pair's distance, [q][c], +inf past ncand[q]
 * An invalid candidate id raises a device flag and gets +inf. */
ssh_status dtw_rerank(const float* q, const int64_t* q_off, int32_t nq, const float* db,
                      const int64_t* db_off, int64_t N, const int64_t* cand, const int32_t* ncand,
                      int32_t C, float band_frac, int32_t k, int64_t* out_id, float* out_dist,
                      void* ws, size_t ws_bytes, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): dtw_rerank
 * with the same arguments and results, minus the workspace.  Its workspace is
 * a static array of SSH_NOALLOC_SCRATCH_BYTES (32 MiB) that every device the
 * library runs on holds until the process ends; the call itself allocates and
 * frees nothing.
 *   Limit: ssh_rerank_workspace_bytes(nq, C) must not exceed the array (about
 *   3.5 million pairs nq * C); a larger call returns SSH_ECAPACITY and enqueues
 *   nothing.
 *   Concurrency: every call on one device shares that device's array, so calls
 *   that overlap on one GPU (other threads, or other streams whose work is not
 *   ordered after this call's) race and give undefined results.  Calls on one
 *   stream are ordered and safe.  The array's contents after a call are the
 *   pair distances as for dtw_rerank's workspace (read by no other entry
 *   point); nothing in it needs to start at zero. */
ssh_status dtw_rerank_noalloc(const float* q, const int64_t* q_off, int32_t nq, const float* db,
                              const int64_t* db_off, int64_t N, const int64_t* cand,
                              const int32_t* ncand, int32_t C, float band_frac, int32_t k,
                              int64_t* out_id, float* out_dist, void* stream);

/* [host] Workspace bytes needed by dtw_rerank_lb; q_values = q_off[nq], the
 * number of query values of the batch. */
size_t ssh_rerank_lb_workspace_bytes(int32_t nq, int32_t C, int64_t q_values);

/* dtw_rerank with lower-bound pruning and early abandoning (Section 2.1: DTW
 * is costly, so cheap lower bounds discard candidates first).  Same arguments
 * and the same outputs, bit for bit, as dtw_rerank; only the work differs.
 * Each candidate gets a bound on its squared distance: LB_Kim (first and last
 * cells, which every warping path visits) and, when the candidate is not
 * longer than the query, LB_Keogh (squared distance of x_j to the envelope of
 * the query values it may be aligned with).  Each query's k candidates of
 * smallest bound are computed first; tau, the largest of their distances,
 * bounds the k-th best.  A candidate whose bound exceeds tau^2 times a factor
 * covering every float32 rounding (about 1 + (lq + 2 lx) 2^-23) is not
 * computed, and the DTW of the others stops as soon as every cell of a row
 * front exceeds that cut: either way its distance is above the k-th best.
 * Pays off when many candidates are far from the query; the two dependent DTW
 * passes make it slower on small batches.
 *   ws, ws_bytes at least ssh_rerank_lb_workspace_bytes(nq, C, q_off[nq]); a
 *                smaller workspace that still holds the fixed part leaves the
 *                queries past its envelope capacity with LB_Kim alone and
 *                raises a device flag.  The distances of skipped or abandoned
 *                candidates in the workspace are +inf. */
ssh_status dtw_rerank_lb(const float* q, const int64_t* q_off, int32_t nq, const float* db,
                         const int64_t* db_off, int64_t N, const int64_t* cand,
                         const int32_t* ncand, int32_t C, float band_frac, int32_t k,
                         int64_t* out_id, float* out_dist, void* ws, size_t ws_bytes,
                         void* stream);

/* Same contract as ssh_sketch, always through the kernel that handles any W
 * and delta (ssh_sketch picks a register-blocked kernel for the filter shapes
 * it specialises).  Both must produce identical bits. */
ssh_status ssh_sketch_generic(const float* x, const int64_t* x_off, int64_t N, const float* r,
                              int32_t W, int32_t delta, uint64_t* bits,
                              const int64_t* bit_word_off, int32_t* nbits, uint64_t* repair_count,
                              void* stream);

/* ssh_sketch with the size of the matrix-core path's work item chosen by the
 * caller (Section 4.1; the same bits whatever the choice): an item is
 * tile_rows rows of 16 windows of one series, tile_rows in {8, 12, 16, 20},
 * for the (W, delta) shapes that have a matrix-core kernel: (80, 3), (64, 4),
 * (128, 4), (30, 5).  Smaller items waste less of a series' last item, larger
 * ones amortise more per item; ssh_sketch uses 20 rows for (80, 3) and 16
 * otherwise.  Returns SSH_EUNSUPPORTED for any other shape or row count. */
ssh_status ssh_sketch_tiled(const float* x, const int64_t* x_off, int64_t N, const float* r,
                            int32_t W, int32_t delta, uint64_t* bits, const int64_t* bit_word_off,
                            int32_t* nbits, uint64_t* repair_count, int32_t tile_rows,
                            void* stream);

/* Sign sketches of F random filters at once (Section 4.1's sketch with F
 * filters r_1 .. r_F in place of one).  Stream f of a series is exactly what
 * ssh_sketch gives for filter r_f: bit i is 1 when r_f . x[i*delta ..
 * i*delta + W) >= 0, the sign of the float64 sum of exact float32 products in
 * ascending filter index.  The inner products of 256 windows with the filters
 * form one matrix product (windows x taps times taps x filters) computed on
 * the matrix cores in fp16 with fp32 accumulation; pairs within a proven
 * margin of zero are recomputed in float64, so every bit is exact.
 * Shapes: (W, delta) in {(80, 3), (64, 4), (128, 4), (30, 5)} and F in
 * {16, 32, 48, 64}; anything else returns SSH_EUNSUPPORTED (shape) or
 * SSH_EINVAL (F).
 *
 * ssh_sketch_multi_workspace_bytes: bytes of the prepared filter block.
 *
 * ssh_sketch_multi_prepare [host]: checks the filters and writes the block.
 *   R            [host] float32 [F][W] filters, row-major; every entry finite
 *                with |r| < 2^14, and none in fp16's subnormal range
 *                (0 < |r| < 2^-14: SSH_EUNSUPPORTED)
 *   ws           device memory of ws_bytes >= the size above; written on
 *                `stream`, and the call returns after the copy completes
 *
 * ssh_sketch_multi: the streams.
 *   x, x_off, N, W, delta, bit_word_off, nbits   as for ssh_sketch
 *   ws           a block written by ssh_sketch_multi_prepare for the same F,
 *                W and delta (read only; another block gives other bits)
 *   bits         uint64 [F * total_words]: stream f of series s starts at
 *                word f * total_words + bit_word_off[s]
 *   total_words  bit_word_off[N] (or more)
 *   repair_count uint64 [1] or NULL: incremented by the number of (window,
 *                filter) pairs recomputed in float64
 *   kdepth       taps per matrix instruction: 16, 32, or 0 for the default
 *                (32 when W is a multiple of 32, else 16); the bits do not
 *                depend on it */
size_t ssh_sketch_multi_workspace_bytes(int32_t F, int32_t W);
ssh_status ssh_sketch_multi_prepare(const float* R, int32_t F, int32_t W, int32_t delta, void* ws,
                                    size_t ws_bytes, void* stream);
ssh_status ssh_sketch_multi(const float* x, const int64_t* x_off, int64_t N, const void* ws,
                            int32_t F, int32_t W, int32_t delta, uint64_t* bits,
                            int64_t total_words, const int64_t* bit_word_off, int32_t* nbits,
                            uint64_t* repair_count, int32_t kdepth, void* stream);

/* [host] Synchronise the device and collect the error flags that kernels raise
 * for inconsistent device-side arguments since the last call (offsets whose
 * capacity is too small, candidate ids outside [0, N), a DTW band radius above
 * SSH_MAX_BAND, an undersized pruned re-rank workspace, CWS draws outside their
 * ranges, table ids or live counts that do not match ssh_table_delete's
 * arguments).  The flags are cleared.  Returns SSH_OK when none was raised, else SSH_EINVAL with the
 * detail in ssh_last_error(). */
ssh_status ssh_check_device_errors(void);

#ifdef __cplusplus
}
#endif
#endif /* SSH_H_ */
