// C ABI of the SSH library: argument validation, size helpers, error strings,
// and dispatch to the kernels.  Every entry point validates synchronously and
// enqueues nothing when it rejects its arguments.
#include <string>
#include <vector>

#include "common.hpp"

namespace ssh {

static thread_local std::string t_last_error;

void set_error(const std::string& msg) { t_last_error = msg; }

ssh_status fail(ssh_status code, const std::string& msg) {
  t_last_error = msg;
  return code;
}

ssh_status check_launch(const char* what) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(SSH_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
  return SSH_OK;
}

// kernels (other translation units)
ssh_status sketch_launch(const float* x, const int64_t* x_off, int64_t N, const float* r, int W,
                         int delta, uint64_t* bits, const int64_t* bit_word_off, int32_t* nbits,
                         uint64_t* repair_count, hipStream_t stream, bool force_generic,
                         int tile_rows);
bool sketch_tile_supported(int W, int delta, int rows);
size_t sketch_multi_workspace_bytes(int F, int W);
bool sketch_multi_supported(int W, int delta);
ssh_status sketch_multi_prepare(const float* R, int F, int W, int delta, void* ws,
                                size_t ws_bytes, hipStream_t stream);
ssh_status sketch_multi_launch(const float* x, const int64_t* x_off, int64_t N, const void* ws,
                               int F, int W, int delta, uint64_t* bits, int64_t total_words,
                               const int64_t* bit_word_off, int32_t* nbits,
                               uint64_t* repair_count, int kdepth, hipStream_t stream);
ssh_status shingle_launch(const uint64_t* bits, const int64_t* bit_word_off, const int32_t* nbits,
                          int64_t N, int n, uint32_t* codes, uint32_t* counts,
                          const int64_t* hist_off, int32_t* n_distinct, hipStream_t stream);
ssh_status cws_prepare_launch(const ssh_cws_tables* tab, hipStream_t stream);
int64_t cws_key_table_elems(int n, int H);
ssh_status cws_launch(const uint32_t* codes, const uint32_t* counts, const int64_t* hist_off,
                      const int32_t* n_distinct, int64_t N, const ssh_cws_tables* tab, uint64_t* hv,
                      uint64_t* keys, int K, int L, uint64_t seed, hipStream_t stream);
ssh_status band_keys_launch(const uint64_t* hv, int64_t N, int K, int L, uint64_t seed,
                            uint64_t* keys, hipStream_t stream);
size_t table_workspace_bytes(int64_t N, int L);
ssh_status table_build_launch(const uint64_t* keys, int64_t N, int L, uint64_t* tab_keys,
                              uint32_t* tab_ids, void* ws, size_t ws_bytes, hipStream_t stream,
                              int sort_bits = 0);
size_t table_insert_workspace_bytes(int64_t M, int L);
ssh_status table_insert_launch(const uint64_t* tab_keys, const uint32_t* tab_ids, int64_t N,
                               const uint64_t* new_keys, int64_t M, int L, int64_t id_base,
                               uint64_t* out_keys, uint32_t* out_ids, void* ws, size_t ws_bytes,
                               hipStream_t stream);
size_t table_delete_workspace_bytes(int64_t N, int L);
ssh_status table_delete_launch(const uint64_t* tab_keys, const uint32_t* tab_ids, int64_t N, int L,
                               const uint8_t* dead, int64_t id_bound, int64_t n_live,
                               uint64_t* out_keys, uint32_t* out_ids, void* ws, size_t ws_bytes,
                               hipStream_t stream);
ssh_status probe_launch(const uint64_t* tab_keys, const uint32_t* tab_ids, int64_t N, int L,
                        const uint64_t* db_keys, const uint64_t* db_hv, int H,
                        const uint64_t* q_keys, const uint64_t* q_hv, int nq, int C, int64_t* cand,
                        int32_t* ncand, int64_t* r_size, void* ws, size_t ws_bytes,
                        hipStream_t stream);
size_t probe_workspace_bytes(int nq, int L, int C);
size_t rerank_workspace_bytes(int nq, int C);
size_t rerank_lb_workspace_bytes(int nq, int C, int64_t q_values);
ssh_status rerank_lb_launch(const float* q, const int64_t* q_off, int nq, const float* db,
                            const int64_t* db_off, int64_t Ndb, const int64_t* cand,
                            const int32_t* ncand, int C, float band_frac, int k, int64_t* out_id,
                            float* out_dist, void* ws, size_t ws_bytes, hipStream_t stream);
ssh_status rerank_launch(const float* q, const int64_t* q_off, int nq, const float* db,
                         const int64_t* db_off, int64_t Ndb, const int64_t* cand,
                         const int32_t* ncand, int C, float band_frac, int k, int64_t* out_id,
                         float* out_dist, void* ws, size_t ws_bytes, hipStream_t stream);
ssh_status rerank_noalloc_launch(const float* q, const int64_t* q_off, int nq, const float* db,
                                 const int64_t* db_off, int64_t Ndb, const int64_t* cand,
                                 const int32_t* ncand, int C, float band_frac, int k,
                                 int64_t* out_id, float* out_dist, hipStream_t stream);

ssh_status wmh_int_launch(const uint32_t* codes, const uint32_t* counts, const int64_t* hist_off,
                          const int32_t* n_distinct, int64_t N, int H, uint64_t seed, uint64_t* hv,
                          hipStream_t stream);

int take_sketch_err();
int take_shingle_err();
int take_cws_err();
int take_dtw_err();
int take_table_err();

}  // namespace ssh

using namespace ssh;

#define SSH_REQUIRE(cond, msg)                 \
  do {                                         \
    if (!(cond)) return fail(SSH_EINVAL, msg); \
  } while (0)

extern "C" {

const char* ssh_status_str(ssh_status s) {
  switch (s) {
    case SSH_OK: return "SSH_OK";
    case SSH_EINVAL: return "SSH_EINVAL";
    case SSH_EUNSUPPORTED: return "SSH_EUNSUPPORTED";
    case SSH_EDEVICE: return "SSH_EDEVICE";
    case SSH_ECAPACITY: return "SSH_ECAPACITY";
    default: return "SSH_UNKNOWN";
  }
}

const char* ssh_last_error(void) { return t_last_error.c_str(); }

int32_t ssh_num_bits(int64_t m, int32_t W, int32_t delta) {
  if (W < 1 || delta < 1 || m < W) return 0;
  return (int32_t)((m - W) / delta + 1);
}

int32_t ssh_num_shingles(int32_t nbits, int32_t n) {
  if (n < 1 || nbits < n) return 0;
  return nbits - n + 1;
}

ssh_status ssh_plan(const int64_t* x_off, int64_t N, int32_t W, int32_t delta, int32_t n,
                    int64_t* bit_word_off, int64_t* hist_off, int32_t* max_nbits) {
  SSH_REQUIRE(N >= 0, "ssh_plan: N < 0");
  SSH_REQUIRE(x_off && bit_word_off && hist_off, "ssh_plan: null pointer");
  SSH_REQUIRE(W >= 1 && W <= SSH_MAX_W, "ssh_plan: W out of [1, SSH_MAX_W]");
  SSH_REQUIRE(delta >= 1, "ssh_plan: delta < 1");
  SSH_REQUIRE(n >= 1 && n <= SSH_MAX_N, "ssh_plan: n out of [1, SSH_MAX_N]");
  SSH_REQUIRE(x_off[0] == 0, "ssh_plan: x_off[0] != 0");
  bit_word_off[0] = 0;
  hist_off[0] = 0;
  int32_t mx = 0;
  for (int64_t s = 0; s < N; ++s) {
    const int64_t m = x_off[s + 1] - x_off[s];
    SSH_REQUIRE(m >= 0, "ssh_plan: decreasing offsets");
    SSH_REQUIRE(m <= (int64_t)1 << 31, "ssh_plan: series longer than 2^31");
    const int32_t nb = ssh_num_bits(m, W, delta);
    mx = nb > mx ? nb : mx;
    bit_word_off[s + 1] = bit_word_off[s] + (nb + 63) / 64;
    hist_off[s + 1] = hist_off[s] + ssh_num_shingles(nb, n);
  }
  if (max_nbits) *max_nbits = mx;
  return SSH_OK;
}

ssh_status ssh_sketch(const float* x, const int64_t* x_off, int64_t N, const float* r, int32_t W,
                      int32_t delta, uint64_t* bits, const int64_t* bit_word_off, int32_t* nbits,
                      uint64_t* repair_count, void* stream) {
  SSH_REQUIRE(N >= 0 && N <= (int64_t)UINT32_MAX, "ssh_sketch: N out of [0, 2^32)");
  SSH_REQUIRE(W >= 1 && W <= SSH_MAX_W, "ssh_sketch: W out of [1, SSH_MAX_W]");
  SSH_REQUIRE(delta >= 1, "ssh_sketch: delta < 1");
  SSH_REQUIRE(r, "ssh_sketch: null filter");
  if (N == 0) return SSH_OK;
  SSH_REQUIRE(x && x_off && bits && bit_word_off && nbits, "ssh_sketch: null pointer");
  return sketch_launch(x, x_off, N, r, W, delta, bits, bit_word_off, nbits, repair_count,
                       as_stream(stream), false, 0);
}

// Same as ssh_sketch but always through the generic kernel (any W, delta);
// exposed so that tests can compare both paths.
ssh_status ssh_sketch_generic(const float* x, const int64_t* x_off, int64_t N, const float* r,
                              int32_t W, int32_t delta, uint64_t* bits,
                              const int64_t* bit_word_off, int32_t* nbits, uint64_t* repair_count,
                              void* stream) {
  SSH_REQUIRE(N >= 0 && N <= (int64_t)UINT32_MAX, "ssh_sketch: N out of [0, 2^32)");
  SSH_REQUIRE(W >= 1 && W <= SSH_MAX_W, "ssh_sketch: W out of [1, SSH_MAX_W]");
  SSH_REQUIRE(delta >= 1, "ssh_sketch: delta < 1");
  SSH_REQUIRE(r, "ssh_sketch: null filter");
  if (N == 0) return SSH_OK;
  SSH_REQUIRE(x && x_off && bits && bit_word_off && nbits, "ssh_sketch: null pointer");
  return sketch_launch(x, x_off, N, r, W, delta, bits, bit_word_off, nbits, repair_count,
                       as_stream(stream), true, 0);
}

ssh_status ssh_sketch_tiled(const float* x, const int64_t* x_off, int64_t N, const float* r,
                            int32_t W, int32_t delta, uint64_t* bits, const int64_t* bit_word_off,
                            int32_t* nbits, uint64_t* repair_count, int32_t tile_rows,
                            void* stream) {
  SSH_REQUIRE(N >= 0 && N <= (int64_t)UINT32_MAX, "ssh_sketch_tiled: N out of [0, 2^32)");
  SSH_REQUIRE(W >= 1 && W <= SSH_MAX_W, "ssh_sketch_tiled: W out of [1, SSH_MAX_W]");
  SSH_REQUIRE(delta >= 1, "ssh_sketch_tiled: delta < 1");
  SSH_REQUIRE(r, "ssh_sketch_tiled: null filter");
  if (!sketch_tile_supported(W, delta, tile_rows))
    return fail(SSH_EUNSUPPORTED, "ssh_sketch_tiled: no matrix-core work item of that many rows "
                                  "for this (W, delta)");
  if (N == 0) return SSH_OK;
  SSH_REQUIRE(x && x_off && bits && bit_word_off && nbits, "ssh_sketch_tiled: null pointer");
  return sketch_launch(x, x_off, N, r, W, delta, bits, bit_word_off, nbits, repair_count,
                       as_stream(stream), false, tile_rows);
}

size_t ssh_sketch_multi_workspace_bytes(int32_t F, int32_t W) {
  if (F < 1 || F > 64 || W < 1 || W > SSH_MAX_W) return 0;
  return sketch_multi_workspace_bytes(F, W);
}

ssh_status ssh_sketch_multi_prepare(const float* R, int32_t F, int32_t W, int32_t delta, void* ws,
                                    size_t ws_bytes, void* stream) {
  SSH_REQUIRE(W >= 1 && W <= SSH_MAX_W, "ssh_sketch_multi_prepare: W out of [1, SSH_MAX_W]");
  SSH_REQUIRE(delta >= 1, "ssh_sketch_multi_prepare: delta < 1");
  SSH_REQUIRE(R && ws, "ssh_sketch_multi_prepare: null pointer");
  return sketch_multi_prepare(R, F, W, delta, ws, ws_bytes, as_stream(stream));
}

ssh_status ssh_sketch_multi(const float* x, const int64_t* x_off, int64_t N, const void* ws,
                            int32_t F, int32_t W, int32_t delta, uint64_t* bits,
                            int64_t total_words, const int64_t* bit_word_off, int32_t* nbits,
                            uint64_t* repair_count, int32_t kdepth, void* stream) {
  SSH_REQUIRE(N >= 0 && N <= (int64_t)UINT32_MAX, "ssh_sketch_multi: N out of [0, 2^32)");
  SSH_REQUIRE(W >= 1 && W <= SSH_MAX_W, "ssh_sketch_multi: W out of [1, SSH_MAX_W]");
  SSH_REQUIRE(delta >= 1, "ssh_sketch_multi: delta < 1");
  SSH_REQUIRE(total_words >= 0, "ssh_sketch_multi: total_words < 0");
  if (!sketch_multi_supported(W, delta))
    return fail(SSH_EUNSUPPORTED, "ssh_sketch_multi: no matrix-core kernel for this (W, delta)");
  SSH_REQUIRE(F >= 16 && F <= 64 && F % 16 == 0, "ssh_sketch_multi: F must be 16, 32, 48 or 64");
  SSH_REQUIRE(kdepth == 0 || kdepth == 16 || kdepth == 32,
              "ssh_sketch_multi: kdepth must be 0, 16 or 32");
  if (N == 0) return SSH_OK;
  SSH_REQUIRE(x && x_off && ws && bits && bit_word_off && nbits, "ssh_sketch_multi: null pointer");
  return sketch_multi_launch(x, x_off, N, ws, F, W, delta, bits, total_words, bit_word_off, nbits,
                             repair_count, kdepth, as_stream(stream));
}

ssh_status ssh_shingle(const uint64_t* bits, const int64_t* bit_word_off, const int32_t* nbits,
                       int64_t N, int32_t n, uint32_t* codes, uint32_t* counts,
                       const int64_t* hist_off, int32_t* n_distinct, void* stream) {
  SSH_REQUIRE(N >= 0, "ssh_shingle: N < 0");
  SSH_REQUIRE(n >= 1 && n <= SSH_MAX_N, "ssh_shingle: n out of [1, SSH_MAX_N]");
  if (N == 0) return SSH_OK;
  SSH_REQUIRE(bits && bit_word_off && nbits && codes && counts && hist_off && n_distinct,
              "ssh_shingle: null pointer");
  return shingle_launch(bits, bit_word_off, nbits, N, n, codes, counts, hist_off, n_distinct,
                        as_stream(stream));
}

static ssh_status check_tables(const ssh_cws_tables* tab, const char* who) {
  if (!tab) return fail(SSH_EINVAL, std::string(who) + ": null tables");
  if (tab->n < 1 || tab->n > SSH_MAX_N) return fail(SSH_EINVAL, std::string(who) + ": n out of [1, SSH_MAX_N]");
  if (tab->H < 1) return fail(SSH_EINVAL, std::string(who) + ": H < 1");
  if (!tab->r || !tab->lnc || !tab->beta || !tab->a1 || !tab->lnS || !tab->k16 || !tab->rb)
    return fail(SSH_EINVAL, std::string(who) + ": null table pointer");
  return SSH_OK;
}

int64_t ssh_cws_key_table_elems(int32_t n, int32_t H) { return cws_key_table_elems(n, H); }

ssh_status ssh_cws_prepare(const ssh_cws_tables* tab, void* stream) {
  ssh_status st = check_tables(tab, "ssh_cws_prepare");
  if (st != SSH_OK) return st;
  return cws_prepare_launch(tab, as_stream(stream));
}

ssh_status ssh_cws(const uint32_t* codes, const uint32_t* counts, const int64_t* hist_off,
                   const int32_t* n_distinct, int64_t N, const ssh_cws_tables* tab, uint64_t* hv,
                   void* stream) {
  ssh_status st = check_tables(tab, "ssh_cws");
  if (st != SSH_OK) return st;
  SSH_REQUIRE(N >= 0, "ssh_cws: N < 0");
  if (N == 0) return SSH_OK;
  SSH_REQUIRE(codes && counts && hist_off && n_distinct && hv, "ssh_cws: null pointer");
  return cws_launch(codes, counts, hist_off, n_distinct, N, tab, hv, nullptr, 0, 0, 0,
                    as_stream(stream));
}

ssh_status ssh_cws_band_keys(const uint32_t* codes, const uint32_t* counts,
                             const int64_t* hist_off, const int32_t* n_distinct, int64_t N,
                             const ssh_cws_tables* tab, int32_t K, int32_t L, uint64_t seed,
                             uint64_t* hv, uint64_t* keys, void* stream) {
  ssh_status st = check_tables(tab, "ssh_cws_band_keys");
  if (st != SSH_OK) return st;
  SSH_REQUIRE(N >= 0, "ssh_cws_band_keys: N < 0");
  SSH_REQUIRE(K >= 1 && L >= 1, "ssh_cws_band_keys: K or L < 1");
  SSH_REQUIRE((int64_t)K * L == tab->H, "ssh_cws_band_keys: K * L != H");
  if (N == 0) return SSH_OK;
  SSH_REQUIRE(codes && counts && hist_off && n_distinct && hv && keys,
              "ssh_cws_band_keys: null pointer");
  return cws_launch(codes, counts, hist_off, n_distinct, N, tab, hv, keys, K, L, seed,
                    as_stream(stream));
}

ssh_status ssh_wmh_int(const uint32_t* codes, const uint32_t* counts, const int64_t* hist_off,
                       const int32_t* n_distinct, int64_t N, int32_t H, uint64_t seed, uint64_t* hv,
                       void* stream) {
  SSH_REQUIRE(N >= 0, "ssh_wmh_int: N < 0");
  SSH_REQUIRE(H >= 1 && H <= 65536, "ssh_wmh_int: H out of [1, 65536]");
  if (N == 0) return SSH_OK;
  SSH_REQUIRE(codes && counts && hist_off && n_distinct && hv, "ssh_wmh_int: null pointer");
  return wmh_int_launch(codes, counts, hist_off, n_distinct, N, H, seed, hv, as_stream(stream));
}

ssh_status ssh_band_keys(const uint64_t* hv, int64_t N, int32_t K, int32_t L, uint64_t seed,
                         uint64_t* keys, void* stream) {
  SSH_REQUIRE(N >= 0, "ssh_band_keys: N < 0");
  SSH_REQUIRE(K >= 1 && L >= 1, "ssh_band_keys: K or L < 1");
  if (N == 0) return SSH_OK;
  SSH_REQUIRE(hv && keys, "ssh_band_keys: null pointer");
  return band_keys_launch(hv, N, K, L, seed, keys, as_stream(stream));
}

size_t ssh_table_workspace_bytes(int64_t N, int32_t L) {
  if (N < 0 || L < 1) return 0;
  return table_workspace_bytes(N, L);
}

ssh_status ssh_table_build(const uint64_t* keys, int64_t N, int32_t L, uint64_t* tab_keys,
                           uint32_t* tab_ids, void* ws, size_t ws_bytes, void* stream) {
  SSH_REQUIRE(N >= 0 && N <= (int64_t)UINT32_MAX - 1, "ssh_table_build: N out of [0, 2^32 - 1)");
  SSH_REQUIRE(L >= 1 && L <= 65535, "ssh_table_build: L out of range");
  if (N == 0) return SSH_OK;
  SSH_REQUIRE(keys && tab_keys && tab_ids && ws, "ssh_table_build: null pointer");
  return table_build_launch(keys, N, L, tab_keys, tab_ids, ws, ws_bytes, as_stream(stream));
}

size_t ssh_table_insert_workspace_bytes(int64_t M, int32_t L) {
  if (M < 0 || L < 1) return 0;
  return table_insert_workspace_bytes(M, L);
}

ssh_status ssh_table_insert(const uint64_t* tab_keys, const uint32_t* tab_ids, int64_t N,
                            const uint64_t* new_keys, int64_t M, int32_t L, int64_t id_base,
                            uint64_t* out_keys, uint32_t* out_ids, void* ws, size_t ws_bytes,
                            void* stream) {
  SSH_REQUIRE(N >= 0 && M >= 0 && N + M <= (int64_t)UINT32_MAX,
              "ssh_table_insert: N + M out of [0, 2^32)");
  SSH_REQUIRE(id_base >= N && id_base + M <= (int64_t)UINT32_MAX,
              "ssh_table_insert: id_base below N or ids past 2^32 - 1");
  SSH_REQUIRE(L >= 1, "ssh_table_insert: L < 1");
  if (N + M == 0) return SSH_OK;
  SSH_REQUIRE(out_keys && out_ids && ws, "ssh_table_insert: null pointer");
  SSH_REQUIRE(N == 0 || (tab_keys && tab_ids), "ssh_table_insert: null table pointer");
  SSH_REQUIRE(M == 0 || new_keys, "ssh_table_insert: null key pointer");
  return table_insert_launch(tab_keys, tab_ids, N, new_keys, M, L, id_base, out_keys, out_ids, ws,
                             ws_bytes, as_stream(stream));
}

size_t ssh_table_delete_workspace_bytes(int64_t N, int32_t L) {
  if (N < 0 || L < 1) return 0;
  return table_delete_workspace_bytes(N, L);
}

ssh_status ssh_table_delete(const uint64_t* tab_keys, const uint32_t* tab_ids, int64_t N, int32_t L,
                            const uint8_t* dead, int64_t id_bound, int64_t n_live,
                            uint64_t* out_keys, uint32_t* out_ids, void* ws, size_t ws_bytes,
                            void* stream) {
  SSH_REQUIRE(N >= 0 && N <= (int64_t)UINT32_MAX, "ssh_table_delete: N out of [0, 2^32)");
  SSH_REQUIRE(L >= 1, "ssh_table_delete: L < 1");
  SSH_REQUIRE(n_live >= 0 && n_live <= N, "ssh_table_delete: n_live out of [0, N]");
  SSH_REQUIRE(id_bound >= 0, "ssh_table_delete: id_bound < 0");
  if (N == 0 || n_live == 0) return SSH_OK;
  SSH_REQUIRE(tab_keys && tab_ids && dead && out_keys && out_ids && ws,
              "ssh_table_delete: null pointer");
  return table_delete_launch(tab_keys, tab_ids, N, L, dead, id_bound, n_live, out_keys, out_ids, ws,
                             ws_bytes, as_stream(stream));
}

size_t ssh_probe_workspace_bytes(int32_t nq, int32_t L, int32_t C) {
  if (nq < 0 || L < 1 || C < 1 || C > SSH_MAX_C) return 0;
  return probe_workspace_bytes(nq, L, C);
}

ssh_status ssh_probe(const uint64_t* tab_keys, const uint32_t* tab_ids, int64_t N, int32_t L,
                     const uint64_t* db_keys, const uint64_t* db_hv, int32_t H,
                     const uint64_t* q_keys, const uint64_t* q_hv, int32_t nq, int32_t C,
                     int64_t* cand, int32_t* ncand, int64_t* r_size, void* ws, size_t ws_bytes,
                     void* stream) {
  SSH_REQUIRE(N >= 0 && N <= (int64_t)UINT32_MAX - 1, "ssh_probe: N out of range");
  SSH_REQUIRE(L >= 1 && H >= 1 && nq >= 0, "ssh_probe: L, H or nq out of range");
  SSH_REQUIRE(C >= 1 && C <= SSH_MAX_C, "ssh_probe: C out of [1, SSH_MAX_C]");
  if (nq == 0) return SSH_OK;
  SSH_REQUIRE(q_keys && q_hv && cand && ncand && r_size && ws, "ssh_probe: null pointer");
  SSH_REQUIRE(N == 0 || (tab_keys && tab_ids && db_keys && db_hv), "ssh_probe: null table pointer");
  return probe_launch(tab_keys, tab_ids, N, L, db_keys, db_hv, H, q_keys, q_hv, nq, C, cand, ncand,
                      r_size, ws, ws_bytes, as_stream(stream));
}

ssh_status ssh_probe_strict(const uint64_t* tab_keys, const uint32_t* tab_ids, int64_t N,
                            int32_t L, const uint64_t* db_keys, const uint64_t* db_hv, int32_t H,
                            const uint64_t* q_keys, const uint64_t* q_hv, int32_t nq, int32_t C,
                            int64_t* cand, int32_t* ncand, int64_t* r_size, void* ws,
                            size_t ws_bytes, void* stream) {
  const ssh_status st = ssh_probe(tab_keys, tab_ids, N, L, db_keys, db_hv, H, q_keys, q_hv, nq, C,
                                  cand, ncand, r_size, ws, ws_bytes, stream);
  if (st != SSH_OK || nq == 0) return st;
  std::vector<int64_t> rs((size_t)nq);
  if (hipMemcpyAsync(rs.data(), r_size, (size_t)nq * sizeof(int64_t), hipMemcpyDeviceToHost,
                     as_stream(stream)) != hipSuccess ||
      hipStreamSynchronize(as_stream(stream)) != hipSuccess)
    return fail(SSH_EDEVICE, "ssh_probe_strict: reading r_size back failed");
  int64_t over = 0, worst = 0;
  for (int32_t q = 0; q < nq; ++q) {
    if (rs[(size_t)q] > C) {
      ++over;
      worst = rs[(size_t)q] > worst ? rs[(size_t)q] : worst;
    }
  }
  if (over > 0)
    return fail(SSH_ECAPACITY, "ssh_probe_strict: " + std::to_string(over) +
                                   " queries retrieved more than C candidates (largest |R| = " +
                                   std::to_string(worst) + ")");
  return SSH_OK;
}

size_t ssh_rerank_workspace_bytes(int32_t nq, int32_t C) {
  if (nq < 0 || C < 1) return 0;
  return rerank_workspace_bytes(nq, C);
}

ssh_status dtw_rerank(const float* q, const int64_t* q_off, int32_t nq, const float* db,
                      const int64_t* db_off, int64_t N, const int64_t* cand, const int32_t* ncand,
                      int32_t C, float band_frac, int32_t k, int64_t* out_id, float* out_dist,
                      void* ws, size_t ws_bytes, void* stream) {
  SSH_REQUIRE(nq >= 0 && N >= 0, "dtw_rerank: nq or N < 0");
  SSH_REQUIRE(C >= 1 && C <= SSH_MAX_C, "dtw_rerank: C out of [1, SSH_MAX_C]");
  SSH_REQUIRE(k >= 1 && k <= SSH_MAX_K && k <= C, "dtw_rerank: k out of [1, min(C, SSH_MAX_K)]");
  SSH_REQUIRE(band_frac >= 0.0f && band_frac <= 1.0f, "dtw_rerank: band_frac out of [0, 1]");
  if (nq == 0) return SSH_OK;
  SSH_REQUIRE(q && q_off && cand && ncand && out_id && out_dist && ws, "dtw_rerank: null pointer");
  SSH_REQUIRE(N == 0 || (db && db_off), "dtw_rerank: null series pointer");
  return rerank_launch(q, q_off, nq, db, db_off, N, cand, ncand, C, band_frac, k, out_id, out_dist,
                       ws, ws_bytes, as_stream(stream));
}

ssh_status dtw_rerank_noalloc(const float* q, const int64_t* q_off, int32_t nq, const float* db,
                              const int64_t* db_off, int64_t N, const int64_t* cand,
                              const int32_t* ncand, int32_t C, float band_frac, int32_t k,
                              int64_t* out_id, float* out_dist, void* stream) {
  SSH_REQUIRE(nq >= 0 && N >= 0, "dtw_rerank_noalloc: nq or N < 0");
  SSH_REQUIRE(C >= 1 && C <= SSH_MAX_C, "dtw_rerank_noalloc: C out of [1, SSH_MAX_C]");
  SSH_REQUIRE(k >= 1 && k <= SSH_MAX_K && k <= C,
              "dtw_rerank_noalloc: k out of [1, min(C, SSH_MAX_K)]");
  SSH_REQUIRE(band_frac >= 0.0f && band_frac <= 1.0f, "dtw_rerank_noalloc: band_frac out of [0, 1]");
  if (nq == 0) return SSH_OK;
  SSH_REQUIRE(q && q_off && cand && ncand && out_id && out_dist, "dtw_rerank_noalloc: null pointer");
  SSH_REQUIRE(N == 0 || (db && db_off), "dtw_rerank_noalloc: null series pointer");
  return rerank_noalloc_launch(q, q_off, nq, db, db_off, N, cand, ncand, C, band_frac, k, out_id,
                               out_dist, as_stream(stream));
}

size_t ssh_rerank_lb_workspace_bytes(int32_t nq, int32_t C, int64_t q_values) {
  if (nq < 0 || C < 1 || q_values < 0) return 0;
  return rerank_lb_workspace_bytes(nq, C, q_values);
}

ssh_status dtw_rerank_lb(const float* q, const int64_t* q_off, int32_t nq, const float* db,
                         const int64_t* db_off, int64_t N, const int64_t* cand,
                         const int32_t* ncand, int32_t C, float band_frac, int32_t k,
                         int64_t* out_id, float* out_dist, void* ws, size_t ws_bytes,
                         void* stream) {
  SSH_REQUIRE(nq >= 0 && N >= 0, "dtw_rerank_lb: nq or N < 0");
  SSH_REQUIRE(C >= 1 && C <= SSH_MAX_C, "dtw_rerank_lb: C out of [1, SSH_MAX_C]");
  SSH_REQUIRE(k >= 1 && k <= SSH_MAX_K && k <= C, "dtw_rerank_lb: k out of [1, min(C, SSH_MAX_K)]");
  SSH_REQUIRE(band_frac >= 0.0f && band_frac <= 1.0f, "dtw_rerank_lb: band_frac out of [0, 1]");
  if (nq == 0) return SSH_OK;
  SSH_REQUIRE(q && q_off && cand && ncand && out_id && out_dist && ws, "dtw_rerank_lb: null pointer");
  SSH_REQUIRE(N == 0 || (db && db_off), "dtw_rerank_lb: null series pointer");
  return rerank_lb_launch(q, q_off, nq, db, db_off, N, cand, ncand, C, band_frac, k, out_id,
                          out_dist, ws, ws_bytes, as_stream(stream));
}

ssh_status ssh_check_device_errors(void) {
  if (hipDeviceSynchronize() != hipSuccess) return fail(SSH_EDEVICE, "device synchronisation failed");
  const int a = take_sketch_err(), b = take_shingle_err(), c = take_cws_err(), d = take_dtw_err();
  const int t = take_table_err();
  if (a < 0 || b < 0 || c < 0 || d < 0 || t < 0)
    return fail(SSH_EDEVICE, "cannot read device error flags");
  std::string msg;
  if (a) msg += "ssh_sketch: bit_word_off capacity below ceil(N_B/64); ";
  if (b) msg += "ssh_shingle: hist_off or bit_word_off capacity too small; ";
  if (c & 2) msg += "ssh_cws_prepare: a draw is outside its range (0 < r < 1e5, beta in [0,1), finite ln c); ";
  if (c & 4) msg += "ssh_cws: internal error, a minimum pointed past the token list; ";
  if (d & 1) msg += "dtw_rerank: candidate id outside [0, N); ";
  if (d & 2) msg += "dtw_rerank: a pair's band radius is above SSH_MAX_BAND (its distance is +inf); ";
  if (d & 4) msg += "dtw_rerank: a series or query length is negative or above 2^30; ";
  if (d & 8) msg += "dtw_rerank_lb: workspace holds fewer query values than q_off[nq] (bounds fell back to LB_Kim); ";
  if (t & 1) msg += "ssh_table_delete: a table id is not below id_bound; ";
  if (t & 2) msg += "ssh_table_delete: a table keeps a number of entries other than n_live; ";
  if (!msg.empty()) return fail(SSH_EINVAL, msg);
  return SSH_OK;
}

}  // extern "C"
