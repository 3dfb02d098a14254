/*
 * lvs.h -- C ABI of liblvs, an MI355X (gfx950) implementation of the
 * Leuvenshtein encrypted edit distance (Legiest, D'Anvers, Spasic, Tran,
 * Verbauwhede, arXiv 2508.14568).
 *
 * Conventions common to every call:
 *   - Return value: LVS_OK (0) on success, a negative LVS_E_* code on failure;
 *     lvs_last_error() returns a text for the calling thread's last failure.
 *   - A ciphertext is a big-key LWE vector of N+1 = 2049 little-endian 64-bit
 *     words (a_0..a_{N-1}, b) over the torus Z/2^64 with a 5-bit plaintext
 *     space: value x in Z_32 sits at x * 2^59 (Section 2.2 of the paper).
 *   - An encrypted string of length L is an array [L][nsym][N+1] words,
 *     nsym = 2 for 7-bit ASCII (symbols c & 15 and c >> 4, Section 4.3) and 1
 *     for 2-bit DNA bases (codes 0..3).
 *   - Pointers named d_* are device pointers on the context's device, h_* and
 *     other pointers are host pointers.  The library never allocates device
 *     memory: the caller passes the context arena and per-call workspaces
 *     whose sizes the *_bytes queries return.  Input buffers are borrowed for
 *     the duration of the call; device work is enqueued on the context's
 *     stream and the call returns without waiting for it unless stated.
 *   - Handles are opaque and released with lvs_free (NULL is ignored).
 *   - Calls on one context must not overlap (one context per device).
 */
#ifndef LVS_H
#define LVS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    LVS_OK = 0,
    LVS_E_INVAL = -1,        /* bad argument (NULL, size, alignment)           */
    LVS_E_ALPHABET = -2,     /* symbol outside the alphabet of the encoding   */
    LVS_E_NOISE_BUDGET = -3, /* min(m, n) past the bound with refresh off     */
    LVS_E_NOMEM_HOST = -4,   /* host allocation failed                        */
    LVS_E_NOMEM_DEVICE = -5, /* caller-provided device memory too small       */
    LVS_E_DEVICE = -6,       /* HIP runtime error                             */
    LVS_E_PARAMS = -7        /* parameter set not supported by the kernels    */
};

typedef enum { LVS_ENC_ASCII7 = 0, LVS_ENC_DNA2 = 1 } lvs_encoding;

/* Lookup-table slots of a context.  EQ = [1,0,..] (Eq. eq_eqlut), EQ9 =
 * [9,0,..] (Eq. eq_eqlut9), MIN = 1 + min(-eq, dv, dh) under the key
 * (1 - dv) + 3 (1 + dh) + 9 eq (Eq. eq_keyeq2, Algorithms 1 and 4), REFRESH =
 * the identity on the differences -1, 0, 1 ([0,1,0,..,0,1]; -1 reads -f(15)),
 * the noise refresh of Section 3.1.  MAX = [0,..,0,1] and MAX9 = [0,..,0,9]
 * test whether a merging sum of the wide-symbol equality reached its maximum
 * (Algorithm 2, with the sum offset so that the maximum reads 15).  Slots from
 * LVS_LUT_USER are free for lvs_context_set_lut. */
enum {
    LVS_LUT_EQ = 0,
    LVS_LUT_EQ9 = 1,
    LVS_LUT_MIN = 2,
    LVS_LUT_REFRESH = 3,
    LVS_LUT_MAX = 4,
    LVS_LUT_MAX9 = 5,
    LVS_LUT_USER = 6,
    LVS_LUT_SLOTS = 8
};

/* Noise refresh (Section 3.1: the differences are bootstrapped again before
 * their noise reaches the decoding threshold, Fig. noise5).  The error of a
 * difference grows with the number of cell updates since its last bootstrap
 * through the refresh table, one per two anti-diagonals along the diagonal
 * of the matrix.  With an interval R, the v and h written on anti-diagonals
 * s = R, 2R, ... (s < m + n) are refreshed in place before anti-diagonal
 * s + 1 reads them (2 bootstraps per cell of such a diagonal), which bounds
 * that count by R / 2.  A context starts at LVS_REFRESH_DEFAULT; R = 0 turns
 * refresh off, and then every DP entry point returns LVS_E_NOISE_BUDGET when
 * min(m, n) exceeds LVS_MAX_DEPTH_NO_REFRESH.  Strings are at most
 * LVS_MAX_LEN symbols long (LVS_E_INVAL past it).  The *_workspace_bytes
 * functions size for the shortest interval, so one workspace serves every
 * setting. */
enum {
    LVS_REFRESH_DEFAULT = 256,
    LVS_REFRESH_MIN = 4,
    LVS_REFRESH_MAX = 512,
    LVS_MAX_DEPTH_NO_REFRESH = 256,
    LVS_MAX_LEN = 1 << 20
};

/* TFHE parameter set; noise standard deviations are given as sigma * 2^64. */
typedef struct {
    uint32_t n_lwe, glwe_k, poly_N, pbs_base_log, pbs_level, ks_base_log, ks_level;
    uint64_t lwe_noise_q64, glwe_noise_q64;
} lvs_params;

typedef struct lvs_client_key lvs_client_key;
typedef struct lvs_server_key lvs_server_key;
typedef struct lvs_context lvs_context;

/* Text of the calling thread's last error (never NULL). */
const char* lvs_last_error(void);

/* The parameter set the kernels implement: n = 742, k = 1, N = 2048,
 * bootstrap gadget 2^23 x 1, key switch 2^3 x 5, noise 7.0698e-6 / 2.9404e-16
 * of q (the TFHE parameter set for 4-bit messages that the paper's
 * implementation runs on, Section 6.2). */
int lvs_params_default(lvs_params* out);

/* Words per ciphertext (N + 1). */
size_t lvs_ct_words(void);

/* ----------------------------------------------------------- host crypto */

/* Key generation from one seed (Section 2.2: TFHE's keys; the client keeps
 * the secret keys, the server gets the bootstrapping and key-switching keys
 * that let it evaluate blind).  The client draws the small LWE key, the GLWE
 * key, the bootstrapping key GGSW(s_i) and the key-switching key with a
 * counter-based SplitMix64 stream per object.  Both handles are owned by the
 * caller.  Cost: about a second of host time. */
int lvs_keygen(const lvs_params* params, uint64_t seed, lvs_client_key** ck, lvs_server_key** sk);

/* Encrypts symbol value mu (0..31) as ciphertext number `index` of the
 * encryption seed `seed` into h_ct (N+1 words): Section 2.2's plaintext space
 * of 4 message bits and a padding bit, mu encoded as mu * 2^59 under the big
 * key, with Gaussian noise. */
int lvs_lwe_encrypt(const lvs_client_key* ck, uint32_t mu, uint64_t seed, uint64_t index, uint64_t* h_ct);

/* Decrypts h_ct (Section 2.2): the phase rounded to the nearest multiple of
 * 2^59 gives *mu in 0..31 and, if phase_err is not NULL, the signed distance
 * of the phase from mu * 2^59. */
int lvs_lwe_decrypt(const lvs_client_key* ck, const uint64_t* h_ct, uint32_t* mu, int64_t* phase_err);

/* Encrypts a string (Section 2.1 notation a_1..a_m, split into symbols
 * a_i^(r)).  Symbol r of character i is ciphertext number i * nsym + r of
 * `seed`.  h_out holds len * nsym * (N+1) words.  LVS_E_ALPHABET if a
 * character is >= 128 (ASCII) or >= 4 (DNA codes 0..3). */
int lvs_encrypt_string(const lvs_client_key* ck, const uint8_t* s, size_t len, int encoding, uint64_t seed,
                       uint64_t* h_out);

/* Decrypts the result of an edit distance: h_last holds the n bottom-row
 * difference ciphertexts h[m, 1..n]; *out = m + sum_j dec(h[m, j]) with dec
 * in {-1, 0, 1} (Fig. fig_myers: the bottom-row differences sum to the
 * distance; Algorithm 4 returns m plus that row). */
int lvs_decrypt_distance(const lvs_client_key* ck, const uint64_t* h_last, size_t m, size_t n, int64_t* out);

/* Copies key material out for inspection by tests: kind 0 = small key
 * (n bytes), 1 = GLWE key (N bytes), 2 = bootstrapping key (n*2*2*N words,
 * [i][row][mask|body][N]), 3 = key-switching key (N*5*(n+1) words).  With
 * buf == NULL only *len (bytes) is set. */
int lvs_key_export(const lvs_client_key* ck, const lvs_server_key* sk, int kind, void* buf, size_t* len);

/* ------------------------------------------------------------ wire format */

/* Records for moving keys and ciphertexts between the client, which encrypts
 * and alone holds the secret key, and the server, which computes on the
 * ciphertexts with the server key (the outsourcing setting of the paper's
 * introduction).  A record is self-describing and little-endian: "LVS1", the
 * kind, the parameter set (lvs_params), a count, the payload length, the
 * payload and an FNV-1a checksum of the payload.  Payloads: client key = n
 * small-key bits then N GLWE-key bits, one byte each; server key = the
 * bootstrapping key then the key-switching key, as u64 words; ciphertexts =
 * count x (N+1) u64 words (an encrypted string, [len][nsym], or result rows). */
enum { LVS_WIRE_CLIENT_KEY = 1, LVS_WIRE_SERVER_KEY = 2, LVS_WIRE_CIPHERTEXTS = 3 };

/* Writes the record of obj: a client key (lvs_client_key*), a server key
 * (lvs_server_key*) or `count` host ciphertexts (const uint64_t*, [count][N+1];
 * count is ignored for keys).  buf == NULL: only *len is set to the record's
 * size; otherwise *len is the capacity on entry and the record's size on
 * return (LVS_E_INVAL if the buffer is too small). */
int lvs_export(int kind, const void* obj, size_t count, uint8_t* buf, size_t* len);

/* Reads a key record into a new handle (*out: lvs_client_key* or
 * lvs_server_key*, as *kind says; release with lvs_free).  LVS_E_INVAL for a
 * malformed record (magic, length, checksum, payload size, key bits outside
 * {0, 1}); LVS_E_PARAMS for a parameter set the kernels do not support. */
int lvs_import_key(const uint8_t* buf, size_t len, int* kind, void** out);

/* Reads a ciphertext record: out == NULL sets *count to the number of
 * ciphertexts; otherwise *count is the capacity of out (in ciphertexts) on
 * entry and the number written on return.  Errors as for lvs_import_key. */
int lvs_import_ciphertexts(const uint8_t* buf, size_t len, uint64_t* out, size_t* count);

/* --------------------------------------------------------- device context */

/* Bytes of device memory lvs_context_create needs (bootstrapping key in NTT
 * form, key-switching key, twiddles, lookup tables). */
int lvs_context_bytes(const lvs_params* params, size_t* bytes);

/* Uploads the server key into d_arena (at least lvs_context_bytes, 256-byte
 * aligned, owned by the caller and kept alive while the context lives),
 * converts the bootstrapping key to the NTT domain, and binds hip_stream (a
 * hipStream_t; NULL = default stream) on device `device`.  Synchronous. */
int lvs_context_create(const lvs_server_key* sk, int device, void* hip_stream, void* d_arena, size_t arena_bytes,
                       lvs_context** out);

/* Replaces the stream work is enqueued on. */
int lvs_context_set_stream(lvs_context* ctx, void* hip_stream);

/* Installs a 16-entry lookup table f: Z_16 -> Z_32 in slot >= LVS_LUT_USER
 * (inputs 16..31 read -f(x-16), Section 2.2).  Synchronous. */
int lvs_context_set_lut(lvs_context* ctx, int slot, const int32_t f16[16]);

/* Sets the refresh interval R of the DP entry points (plans built later,
 * servers created later): 0 (off) or LVS_REFRESH_MIN..LVS_REFRESH_MAX, else
 * LVS_E_INVAL. */
int lvs_context_set_refresh(lvs_context* ctx, size_t every);
int lvs_context_get_refresh(const lvs_context* ctx, size_t* every);

/* Waits for all work enqueued on the context's stream. */
int lvs_sync(lvs_context* ctx);

/* ----------------------------------------------------------------- tuning */

/* Launch shape of the blind rotation kernel (the dominant cost of every
 * bootstrap, Section 2.2).  br_grid: workgroups per launch, each looping over
 * the batch (0: one workgroup per bootstrap).  latency_form_max: batches of
 * at most this many bootstraps use a one-workgroup-per-CU form; larger
 * batches use a two-workgroups-per-CU form.  latency_waves picks the
 * one-per-CU form: 8 (512 threads, two waves per prime) or 16 (1024 threads,
 * four waves per prime, first and last three transform stages in the digit
 * and CRT steps).  throughput_waves picks the two-per-CU form: 8 (the
 * eight-wave form with one LDS buffer and at most 128 registers per thread)
 * or 4 (256 threads, one wave per prime).  ks_tile: job inputs per
 * key-switch workgroup, each key-switching key row read once per tile.  A new
 * context starts at {0, INT32_MAX, 8, 8, 8}.  Plans captured as graphs keep the shape they were
 * captured with. */
typedef struct lvs_tuning {
    int32_t br_grid;
    int32_t latency_form_max;
    int32_t latency_waves;      /* 8 or 16: wavefronts per bootstrap of the one-per-CU form (0 = 8) */
    int32_t throughput_waves;   /* 8 or 4: wavefronts per bootstrap of the two-per-CU form (0 = 8) */
    int32_t ks_tile;            /* 4, 8 or 16: ciphertexts per key-switch workgroup (0 = 8) */
} lvs_tuning;

int lvs_context_get_tuning(const lvs_context* ctx, lvs_tuning* out);
/* Rejects negative values, latency_waves other than 0, 8, 16,
 * throughput_waves other than 0, 4, 8 and ks_tile other than 0, 4, 8, 16
 * (LVS_E_INVAL). */
int lvs_context_set_tuning(lvs_context* ctx, const lvs_tuning* t);

/* One timing of the autotuner: mean duration (ms) of a launch over `batch`
 * bootstraps: the blind rotation in `form` 1 to 4 (1: eight-wave, one
 * workgroup per CU; 2: four-wave, two per CU; 3: sixteen-wave, one per CU;
 * 4: eight-wave with one LDS buffer, two per CU) with `grid` workgroups, or
 * the key switch (form 5) with tiles of `grid` ciphertexts. */
typedef struct lvs_tune_sample {
    int32_t batch;
    int32_t form;
    int32_t grid;
    double ms;
} lvs_tune_sample;

/* Device workspace bytes of lvs_autotune (256-byte aligned, caller-owned). */
size_t lvs_autotune_workspace_bytes(size_t max_batch);

/* Times the four forms (form 1 / 3: one eight- / sixteen-wave workgroup per
 * CU; 2 / 4: two four- / eight-wave workgroups per CU), and the two-per-CU
 * forms with a persistent grid of twice the CU count, on batches from half
 * to four times the CU count (at most max_batch, 1..65536) of zero
 * ciphertexts, installs the fastest shape in the context (of each kind the
 * form with the smaller total time; the one-per-CU form up to the batch
 * before the first one at which the two-per-CU form is more than 1% faster)
 * and returns it in *best; the key switch is timed at tiles of 4, 8 and 16
 * on the same batches and the tile with the smallest total time is
 * installed.  Up to max_samples timings go to samples (may be NULL); *n_samples
 * (may be NULL) receives how many were taken.  Synchronous; uses the
 * context's stream.  Errors: LVS_E_INVAL, LVS_E_NOMEM_DEVICE (workspace too
 * small), LVS_E_DEVICE. */
int lvs_autotune(lvs_context* ctx, size_t max_batch, void* d_work, size_t work_bytes, lvs_tuning* best,
                 lvs_tune_sample* samples, size_t max_samples, size_t* n_samples);

/* ------------------------------------------------------------- bootstraps */

/* Workspace bytes for lvs_pbs_batch with B ciphertexts. */
size_t lvs_pbs_workspace_bytes(size_t B);

/* B independent programmable bootstraps (Section 2.2): d_out[b] =
 * PBS(d_in[b]; table lut(b)) with lut(b) = lut_ids[b] if lut_ids (host bytes,
 * each < LVS_LUT_SLOTS) is not NULL, else lut_id.  Each runs key switch ->
 * modulus switch -> blind rotation -> sample extraction; results are
 * bit-identical to the schoolbook definition.  d_in and d_out are [B][N+1]
 * and must not overlap.  Waits for earlier work on the stream before
 * enqueueing (its job list is staged through host memory). */
int lvs_pbs_batch(lvs_context* ctx, const uint64_t* d_in, const uint8_t* lut_ids, int lut_id, size_t B,
                  uint64_t* d_out, void* d_work, size_t work_bytes);

/* For callers that cannot allocate device memory (code under stream capture,
 * serving loops, harnesses that forbid allocation): lvs_pbs_batch without a
 * workspace, bit-identical to it.  The job list and the key switch's partial
 * sums live in a device array of the library (about 12.3 MB per device, held
 * by every device a context was created on until the process ends); the call
 * allocates no memory, stages nothing through the host and does not wait on
 * the stream.  B is at most LVS_PBS_STATIC_MAX (LVS_E_INVAL past it); d_in
 * and d_out as for lvs_pbs_batch.  All calls on one device share the array:
 * calls that overlap on a device (other streams, other threads, other
 * contexts of the device) race and must be serialised by the caller.  The
 * array needs no clearing: each call writes every word it reads.  Errors:
 * LVS_E_INVAL, LVS_E_DEVICE (HIP error, or no context created on the
 * device). */
enum { LVS_PBS_STATIC_MAX = 1024 };
int lvs_pbs_batch_static(lvs_context* ctx, const uint64_t* d_in, const uint8_t* lut_ids, int lut_id, size_t B,
                         uint64_t* d_out);

/* --------------------------------------------------------- edit distance */

/* Workspace bytes for lvs_equality. */
size_t lvs_equality_workspace_bytes(size_t m, size_t n, int encoding);

/* Equality of every character pair, all m*n pairs independent of the DP
 * (Section 4): ASCII follows Algorithm 3 with the eq9 table of Algorithm 4,
 * eq1 = PBS(x1 - y1; LUT_eq), eq9 = PBS(2 (x2 - y2) + (1 - eq1); LUT_eq9);
 * DNA uses one bootstrap, eq9 = PBS(x - y; LUT_eq9).  d_eq9 receives the
 * [m][n] matrix of Enc(9 [a_i = b_j]) (row i = character of a). */
int lvs_equality(lvs_context* ctx, const uint64_t* d_a, size_t m, const uint64_t* d_b, size_t n, int encoding,
                 uint64_t* d_eq9, void* d_work, size_t work_bytes);

/* Workspace bytes for lvs_edit_distance_eq9. */
size_t lvs_edit_distance_eq9_workspace_bytes(size_t m, size_t n);

/* Algorithm 1 over every cell (exact distance, no band) given the [m][n]
 * eq9 matrix: key = (1 - v[i,j-1]) + 3 (1 + h[i-1,j]) + eq9[i,j]
 * (Eq. eq_keyeq2), M = PBS(key; LUT_min), v[i,j] = M - h[i-1,j],
 * h[i,j] = M - v[i,j-1], boundary v[i,0] = h[0,j] = Enc(1), evaluated one
 * anti-diagonal per batch.  d_h_last receives h[m, 1..n].  d_trace, if not
 * NULL, receives every M as an [m][n] ciphertext matrix (for checking). */
int lvs_edit_distance_eq9(lvs_context* ctx, const uint64_t* d_eq9, size_t m, size_t n, uint64_t* d_h_last,
                          uint64_t* d_trace, void* d_work, size_t work_bytes);

/* Workspace bytes for lvs_edit_distance on an m x n problem. */
size_t lvs_edit_distance_workspace_bytes(size_t m, size_t n, int encoding);

/* Algorithm 4 (Appendix) on two encrypted strings: the equality of every
 * character pair (Algorithm 3: 2 PBS for ASCII, 1 PBS for DNA, Section 4),
 * then the single-PBS cell update of Eq. (mye_eq_2) with key
 * (1 - v) + 3 (1 + h) + eq9 over every cell, anti-diagonal by anti-diagonal
 * (Section 6.2: cells on one anti-diagonal are independent).  d_a is the
 * encrypted [m][nsym][N+1] string, d_b [n][nsym][N+1]; d_h_last receives the n
 * ciphertexts h[m, 1..n].  m = 0 or n = 0 returns n noise-free encryptions of
 * 1 (distance max(m, n)).  The context's refresh interval applies (see
 * LVS_REFRESH_DEFAULT), as in every DP entry point below. */
int lvs_edit_distance(lvs_context* ctx, const uint64_t* d_a, size_t m, const uint64_t* d_b, size_t n, int encoding,
                      uint64_t* d_h_last, void* d_work, size_t work_bytes);

/* Workspace bytes for lvs_preprocess. */
size_t lvs_preprocess_workspace_bytes(size_t m, size_t alphabet_len, int encoding);

/* Section 5 preprocessing of an encrypted string against a cleartext
 * alphabet S: d_table[c][i] = Enc(9 [a_i = S_c]) ([alen][m][N+1] words), at a
 * cost of nsym * alen * m bootstraps. */
int lvs_preprocess(lvs_context* ctx, const uint64_t* d_a, size_t m, int encoding, const uint8_t* alphabet,
                   size_t alen, uint64_t* d_table, void* d_work, size_t work_bytes);

/* Workspace bytes for lvs_edit_distance_clear. */
size_t lvs_edit_distance_clear_workspace_bytes(size_t m, size_t n);

/* Main pass with one cleartext string b (Section 5): eq9[i,j] is read from
 * the preprocessing table row of b_j, so every cell costs one bootstrap.
 * LVS_E_ALPHABET if some b_j is not in the table's alphabet. */
int lvs_edit_distance_clear(lvs_context* ctx, const uint64_t* d_table, size_t m, const uint8_t* alphabet,
                            size_t alen, const uint8_t* b, size_t n, uint64_t* d_h_last, void* d_work,
                            size_t work_bytes);

/* ------------------------------------------------------------ band modes */

/* Skipping irrelevant cells (Section 3.2, Algorithm 1): only the cells with
 * |i - j| <= ell are bootstrapped (and, with both strings encrypted, only
 * their character pairs get equality bootstraps); a neighbour outside the
 * band reads as the noise-free 1 of Algorithm 1's set-up.  The last row is
 * then incomplete, so the result is the diagonal path of differences
 * d_path ([m+n][N+1]): v[k,k-1], h[k,k] for k = 1..min(m, n) (v[1,0] is the
 * noise-free boundary 1), then h[m, j] for j = m+1..n or v[i, n] for
 * i = n+1..m.  The distance is the sum of their decryptions,
 * lvs_decrypt_distance(ck, path, 0, m + n, &d).
 *
 * With ell >= lvs_band_exact(m, n) the result is the exact distance
 * (ceil(m / 2) for m = n, Section 3.2; for m != n the band has to reach the
 * corner: max(m, n) - floor(min(m, n) / 2)).  For m = n, a smaller ell gives
 * a value never below the distance and equal to it whenever the distance is
 * at most 2 ell + 1 (approximate mode).  ell past m + n is clamped. */
size_t lvs_band_exact(size_t m, size_t n);

/* Cells with |i - j| <= ell (m (2 ell + 1) - ell^2 - ell for m = n, ell < m;
 * Eq. eq_skip). */
size_t lvs_band_cells(size_t m, size_t n, size_t ell);

size_t lvs_edit_distance_band_workspace_bytes(size_t m, size_t n, int encoding, size_t ell);

/* Algorithm 4's pipeline (equality, then the wavefront) restricted to the
 * band.  Buffers as lvs_edit_distance; d_path receives m + n ciphertexts.
 * Errors as lvs_edit_distance. */
int lvs_edit_distance_band(lvs_context* ctx, const uint64_t* d_a, size_t m, const uint64_t* d_b, size_t n,
                           int encoding, size_t ell, uint64_t* d_path, void* d_work, size_t work_bytes);

size_t lvs_edit_distance_clear_band_workspace_bytes(size_t m, size_t n, size_t ell);

/* The cleartext-string variant (Section 5 table, no bootstrap for equality)
 * restricted to the band.  Arguments as lvs_edit_distance_clear. */
int lvs_edit_distance_clear_band(lvs_context* ctx, const uint64_t* d_table, size_t m, const uint8_t* alphabet,
                                 size_t alen, const uint8_t* b, size_t n, size_t ell, uint64_t* d_path, void* d_work,
                                 size_t work_bytes);

/* ----------------------------------------------------------- wide symbols */

/* Section 4.2's hybrid equality for symbols wider than a character (up to
 * 64 bits, e.g. 21-bit Unicode code points).  A symbol of `width` bits is
 * encrypted as c = ceil(width / 4) ciphertexts of its 4-bit chunks (chunk k
 * holds bits 4k .. 4k + 3).  Equality of two symbols costs one bootstrap per
 * chunk pair, PBS(x_k - y_k; LUT_eq), then Algorithm 2's merging: groups of
 * at most 15 sub-equalities are summed, a group of g offset by 15 - g, and
 * bootstrapped through LUT_max (LUT_max9 at the last level) until one
 * ciphertext, Enc(9 [x = y]), is left; a single chunk (width <= 4) reads
 * LUT_eq9 at once.  lvs_wide_pbs_per_pair gives the count: c plus the
 * merges. */
size_t lvs_wide_chunks(unsigned width);          /* c, or 0 unless 1 <= width <= 64 */
size_t lvs_wide_pbs_per_pair(unsigned width);    /* bootstraps per symbol pair, 0 if width is invalid */

/* h_out ([len][c][N+1] words, host): chunk k of syms[i] is ciphertext number
 * i * c + k under the encryption seed.  LVS_E_ALPHABET if a symbol does not
 * fit in width bits. */
int lvs_encrypt_symbols(const lvs_client_key* ck, const uint64_t* syms, size_t len, unsigned width, uint64_t seed,
                        uint64_t* h_out);

/* Equality of every pair of two encrypted symbol strings ([m][c][N+1] and
 * [n][c][N+1], device): d_eq9 ([m][n][N+1]) receives Enc(9 [a_i = b_j]). */
size_t lvs_equality_wide_workspace_bytes(size_t m, size_t n, unsigned width);
int lvs_equality_wide(lvs_context* ctx, const uint64_t* d_a, size_t m, const uint64_t* d_b, size_t n, unsigned width,
                      uint64_t* d_eq9, void* d_work, size_t work_bytes);

/* Edit distance of two encrypted symbol strings: the single-bootstrap main
 * loop of Algorithm 1 over the wide equality of every pair (with the
 * context's refresh interval), the equality bootstraps running inside the
 * loop as in lvs_plan_create_wide; d_h_last as for lvs_edit_distance. */
size_t lvs_edit_distance_wide_workspace_bytes(size_t m, size_t n, unsigned width);
int lvs_edit_distance_wide(lvs_context* ctx, const uint64_t* d_a, size_t m, const uint64_t* d_b, size_t n,
                           unsigned width, uint64_t* d_h_last, void* d_work, size_t work_bytes);

/* Section 5's preprocessing for wide symbols: d_table[s][i] =
 * Enc(9 [a_i = alphabet[s]]) ([alen][m][N+1]), c + merges bootstraps per
 * entry; the main pass is lvs_edit_distance_clear_wide. */
size_t lvs_preprocess_wide_workspace_bytes(size_t m, size_t alen, unsigned width);
int lvs_preprocess_wide(lvs_context* ctx, const uint64_t* d_a, size_t m, unsigned width, const uint64_t* alphabet,
                        size_t alen, uint64_t* d_table, void* d_work, size_t work_bytes);

/* Main pass with a cleartext symbol string b (host, n symbols, each in the
 * alphabet the table was built for, else LVS_E_ALPHABET): as
 * lvs_edit_distance_clear.  Workspace: lvs_edit_distance_clear_workspace_bytes. */
int lvs_edit_distance_clear_wide(lvs_context* ctx, const uint64_t* d_table, size_t m, const uint64_t* alphabet,
                                 size_t alen, const uint64_t* b, size_t n, uint64_t* d_h_last, void* d_work,
                                 size_t work_bytes);

/* ------------------------------------------------------------ batch plans */

/* One edit distance of a batch.  Both strings encrypted: d_a ([m][nsym][N+1])
 * and d_b ([n][nsym][N+1]).  One cleartext string (Section 5): d_b = NULL,
 * d_table = lvs_preprocess output of a over `alphabet` (host, alen symbols),
 * b_clear = the cleartext string (host, n symbols).  d_h_last receives
 * h[m, 1..n] ([n][N+1]).  banded != 0 restricts the query to the band
 * |i - j| <= ell (see lvs_edit_distance_band); its result goes to d_path
 * ([m+n][N+1]) and d_h_last is not used.  A zero-initialised query is the
 * full matrix.  Optional outputs, for checking (NULL: not kept): d_trace
 * receives every cell's bootstrap output M as an [m][n][N+1] matrix; with
 * both strings encrypted, d_eq9 receives the [m][n][N+1] matrix of
 * Enc(9 [a_i = b_j]) and (ASCII) d_eq1 the first-stage outputs
 * Enc([x1_i = y1_j]) of Algorithm 3, and the plan then needs no workspace for
 * them.  Entries outside a band are left untouched.  d_eq1 and d_eq9 must be
 * NULL for a cleartext query and for wide-symbol plans. */
typedef struct {
    const uint64_t* d_a;
    size_t m;
    const uint64_t* d_b;
    size_t n;
    const uint64_t* d_table;
    const uint8_t* alphabet;
    size_t alen;
    const uint8_t* b_clear;
    uint64_t* d_h_last;
    int32_t banded;
    size_t ell;
    uint64_t* d_path;
    uint64_t* d_trace;
    uint64_t* d_eq1;
    uint64_t* d_eq9;
} lvs_query;

typedef struct lvs_plan lvs_plan;

enum { LVS_PLAN_GRAPH = 1 };   /* capture the whole schedule as one HIP graph */

/* Workspace bytes of lvs_plan_create for these queries. */
int lvs_plan_workspace_bytes(const lvs_query* queries, size_t nq, int encoding, size_t* bytes);

/* Batch of edit distances (batch input matching, Section 6.2): the equality
 * bootstraps of every pair of every query form the first step(s); then step
 * s = 2 .. max(m + n) bootstraps every ready cell (i, s - i) of every query
 * in one key-switch launch and one blind-rotation launch, together with the
 * equality bootstraps of the next diagonals (and, to fill the device's last
 * partial round of the step, of later ones).  The
 * schedule is static (no data-dependent branch exists under encryption), so
 * it is built and uploaded once into d_work and, with LVS_PLAN_GRAPH,
 * captured as one HIP graph.  Query buffers are referenced, not copied: they
 * must stay valid while the plan is used.  Results are bit-identical to
 * computing each query alone. */
int lvs_plan_create(lvs_context* ctx, const lvs_query* queries, size_t nq, int encoding, int flags, void* d_work,
                    size_t work_bytes, lvs_plan** out);

/* Batch plan over wide symbols (Section 4.2): every query has both strings
 * encrypted by lvs_encrypt_symbols with the same width (d_a [m][c][N+1],
 * d_b [n][c][N+1]; d_table must be NULL).  Step t runs the cells of
 * anti-diagonal t of every query, as in lvs_plan_create (full or banded; the
 * context's refresh interval), together with the hybrid equality of the
 * in-band pairs of later diagonals: a pair's chunk bootstraps by step
 * s - 1 - levels, each merging level one step later (its group sums run just
 * before the step), so the pair's eq9 is ready a step before its cell; chunk
 * bootstraps of later diagonals fill each step's last partial device round.
 * Run and free it like any plan. */
int lvs_plan_wide_workspace_bytes(const lvs_query* queries, size_t nq, unsigned width, size_t* bytes);
int lvs_plan_create_wide(lvs_context* ctx, const lvs_query* queries, size_t nq, unsigned width, int flags,
                         void* d_work, size_t work_bytes, lvs_plan** out);

/* Host-side check of the schedule lvs_plan_create_wide builds for these
 * queries (no device, nothing dereferenced), as lvs_plan_verify does for
 * lvs_plan_create: round is the device's round (the schedule fills partial
 * rounds with chunk sub-equalities of later diagonals), refresh the interval
 * (0 = off).  Violations count reads of a word the plan writes (by a
 * bootstrap or a group sum) before an earlier step wrote it, in-step races
 * and steps above the workspace's bound. */
int lvs_plan_verify_wide(const lvs_query* queries, size_t nq, unsigned width, size_t round, size_t refresh,
                         size_t* steps, size_t* jobs, size_t* rounds, size_t* violations);

/* Host-side check of the schedule lvs_plan_create builds for these queries
 * (no device, nothing dereferenced: the query pointers only name buffers).
 * round: bootstraps the device runs at once (>= 1); with fill != 0 the
 * schedule fills the last partial round of each step with equality
 * bootstraps of later diagonals, as lvs_plan_create does with the device's
 * round.  Returns the steps, bootstraps, device rounds (sum over steps of
 * ceil(count / round)) and violations: reads of a word the plan writes
 * before an earlier step has written it, subtrahend reads or writes of a
 * word another job of the same step writes, and steps larger than the
 * workspace bound.  refresh: the refresh interval (0 = off; the noise bound
 * is not checked here). */
int lvs_plan_verify(const lvs_query* queries, size_t nq, int encoding, size_t round, int fill, size_t refresh,
                    size_t* steps, size_t* jobs, size_t* rounds, size_t* violations);

/* Enqueues one execution of the plan on the context's stream. */
int lvs_plan_run(lvs_plan* plan);

/* Steps, bootstraps and the largest step of a plan (any may be NULL). */
int lvs_plan_info(const lvs_plan* plan, size_t* steps, size_t* bootstraps, size_t* max_step);

/* Enqueues steps first .. first + count - 1 of one execution of the plan as
 * separate launches (never the captured graph), so that a caller can time a
 * range of steps; an execution starts at step 0 (which also resets the
 * plan's boundary rows) and must run its steps in order.  LVS_E_INVAL past
 * the last step. */
int lvs_plan_run_steps(lvs_plan* plan, size_t first, size_t count);

/* Bootstraps of each of the plan's first n steps (0 for a step of linear
 * group sums) into counts[]. */
int lvs_plan_step_bootstraps(const lvs_plan* plan, size_t* counts, size_t n);

/* ------------------------------------------ continuous batching of queries */

/* Continuous batching of general queries (Section 6.2: the cells at one
 * distance from the first cell are independent, so the ready cells of many
 * queries form one batch): lvs_submit queues lvs_query items (both strings
 * encrypted, or one cleartext string with its Section 5 table; full or
 * banded) and returns at once; a worker thread of the engine admits them in
 * arrival order while their device state (what lvs_plan_create would carve
 * from its workspace for the query: V, the row state, eq1, eq9) fits a
 * first-fit pool in the caller's arena (admission by device memory), and at
 * every engine step runs the next plan step of every admitted query, in
 * arrival order up to max_step bootstraps and trimmed to whole device rounds,
 * as one key-switch launch and one blind-rotation launch on the engine's own
 * stream.  A query runs the steps its lone lvs_plan_create would run, one
 * after the other, so its results are bit-identical alone and in any mix.
 * The arena holds lvs_engine_fixed_bytes(max_step) bytes of job list and
 * key-switch partials, then the pool.
 *
 * Buffers: every device buffer of a query (d_a, d_b, d_table, d_h_last,
 * d_path) must be ready when lvs_submit is called (the engine's stream does
 * not wait for the caller's stream) and stay valid, untouched, until lvs_poll
 * reports the query done; then its results are complete in d_h_last (d_path
 * for a banded query).  d_trace, d_eq1 and d_eq9 must be NULL.  Host buffers
 * (alphabet, b_clear) are read during lvs_submit.  The context's refresh
 * interval at submission applies; its launch shape (lvs_context_set_tuning)
 * must not change while an engine runs, and engines are released before
 * their context. */
typedef struct lvs_engine lvs_engine;

/* Job list and key-switch partials for at most max_step bootstraps per step. */
size_t lvs_engine_fixed_bytes(size_t max_step);

/* Pool bytes the engine keeps for query q while it runs. */
int lvs_engine_query_bytes(const lvs_query* q, int encoding, size_t* bytes);

/* Engine for queries of one encoding; d_arena (256-byte aligned) is borrowed
 * for the engine's lifetime.  Starts the worker thread and a stream of the
 * context's device.  Released with lvs_free, which finishes the step in
 * flight and stops the worker (queries not yet done are abandoned). */
int lvs_engine_create(lvs_context* ctx, int encoding, size_t max_step, void* d_arena, size_t arena_bytes,
                      lvs_engine** out);

/* Queues nq queries (non-blocking) and writes one ticket per query.
 * LVS_E_NOMEM_DEVICE if a query could never fit in the pool; LVS_E_ALPHABET,
 * LVS_E_INVAL and LVS_E_NOISE_BUDGET as for lvs_plan_create; nothing is queued
 * when any query is refused.  May be called from any thread. */
int lvs_submit(lvs_engine* eng, const lvs_query* q, size_t nq, uint64_t* tickets);

/* *done = 1 once the query's results are complete (wait != 0 blocks until
 * then); a done ticket is released and its pool space returns to the engine.
 * An error of the worker (LVS_E_DEVICE for its device work, LVS_E_NOMEM_HOST
 * for host memory while admitting a query) stops the engine and is returned
 * by every later lvs_submit and lvs_poll. */
int lvs_poll(lvs_engine* eng, uint64_t ticket, int wait, int* done);

/* Engine steps and bootstraps run so far, queries running and queued (any
 * pointer may be NULL). */
int lvs_engine_stats(lvs_engine* eng, uint64_t* steps, uint64_t* bootstraps, size_t* active, size_t* queued);

/* --------------------------------------------------------------- serving */

/* Continuous batching of encrypted name queries against a cleartext name
 * list (Section 5: an encrypted query against an unencrypted database; the
 * query is preprocessed once, then every name costs one bootstrap per cell).
 * The caller passes one device arena: lvs_server_fixed_bytes(max_step) bytes
 * for the job list and key-switch partials, the rest is the pool requests are
 * admitted into (admission by device memory). */
typedef struct lvs_server lvs_server;

/* Fixed part of the arena for at most max_step bootstraps per launch. */
size_t lvs_server_fixed_bytes(size_t max_step);

/* Pool bytes one request of length m occupies: its ciphertexts, the eq1 and
 * preprocessing tables over the alphabet, and one DP frontier plus result
 * row per name. */
size_t lvs_server_request_bytes(const uint8_t* names, const size_t* name_lens, size_t n_names, size_t alen,
                                size_t m);

/* Server over n_names cleartext names (concatenated in `names`, lengths in
 * name_lens, each at most 4096, every symbol in `alphabet`, 7-bit ASCII).
 * d_arena is borrowed for the server's lifetime (256-byte aligned).  The
 * context's refresh interval at creation applies to every request. */
int lvs_server_create(lvs_context* ctx, const uint8_t* names, const size_t* name_lens, size_t n_names,
                      const uint8_t* alphabet, size_t alen, size_t max_step, void* d_arena, size_t arena_bytes,
                      lvs_server** out);

/* The same engine over wide symbols (Section 4.2): names and alphabet are
 * symbols of `width` bits (1..64) as uint64_t, and each request's
 * preprocessing is the table of lvs_preprocess_wide (the chunk
 * sub-equalities, then one bootstrap round per merging level, each level's
 * group sums run by the engine just before its round).  Queries are
 * lvs_encrypt_symbols output of the same width.  Everything else (arena,
 * admission, the main pass, results) is as for lvs_server_create.
 * LVS_E_ALPHABET for an alphabet symbol wider than width bits or a name
 * symbol outside the alphabet; LVS_E_INVAL for a bad width. */
int lvs_server_create_wide(lvs_context* ctx, const uint64_t* names, const size_t* name_lens, size_t n_names,
                           const uint64_t* alphabet, size_t alen, unsigned width, size_t max_step, void* d_arena,
                           size_t arena_bytes, lvs_server** out);

/* Pool bytes of one request of length m on a wide server: its chunk
 * ciphertexts, the merging levels' buffers, the table, one DP frontier per
 * name and the result rows.  0 for a bad width. */
size_t lvs_server_request_bytes_wide(const size_t* name_lens, size_t n_names, size_t alen, size_t m,
                                     unsigned width);

/* Queues a request: h_query is the encrypted query (ASCII: [m][2][N+1]; a
 * wide server: [m][ceil(width / 4)][N+1]; host, copied, 1 <= m <= 4096).  Requests are admitted in arrival order at the
 * next step that has room.  LVS_E_NOMEM_DEVICE if it could never fit;
 * LVS_E_NOISE_BUDGET with refresh off and min(m, longest name) above
 * LVS_MAX_DEPTH_NO_REFRESH. */
int lvs_server_submit(lvs_server* srv, const uint64_t* h_query, size_t m, uint64_t* ticket);

/* One engine step: admits queued requests while their buffers fit, then runs
 * one batched launch over the ready bootstraps of the admitted requests
 * (preprocessing rounds of new requests and the current anti-diagonal of
 * running ones), taken in arrival order up to max_step bootstraps, and
 * advances every request whose round is complete.  The bootstraps of one
 * round are independent, so the last request taken may run part of its
 * round (the rest runs in the next step first); a step larger than one device
 * round (one bootstrap per CU, two in the four-wave form) is trimmed to a
 * whole number of rounds, the trimmed bootstraps taken off the latest
 * requests.  A smaller max_step shortens the steps and so the latency of the
 * requests in front, at some cost in throughput.  Waits for the step to
 * finish.  Reports the requests still running, still queued, and the step's
 * bootstraps (any may be NULL). */
int lvs_server_step(lvs_server* srv, size_t* active, size_t* queued, size_t* step_jobs);

/* *done = 1 once the request has finished; then, if h_out is not NULL, copies
 * its results (for every name k in order, the n_k ciphertexts h[m, 1..n_k],
 * [sum n_k][N+1]) and releases the request. */
int lvs_server_poll(lvs_server* srv, uint64_t ticket, uint64_t* h_out, int* done);

/* Steps run and bootstraps executed so far (any may be NULL). */
int lvs_server_stats(const lvs_server* srv, uint64_t* steps, uint64_t* bootstraps);

/* ------------------------------------------------------------ measurement */

#define LVS_KERNEL_BLIND_ROTATE 0            /* every form together */
#define LVS_KERNEL_KEYSWITCH 1
#define LVS_KERNEL_GRAPH 2                   /* a graph-captured plan, whole */
#define LVS_KERNEL_BLIND_ROTATE_LATENCY 3    /* eight-wave form, one workgroup per CU */
#define LVS_KERNEL_BLIND_ROTATE_THROUGHPUT 4 /* four-wave form, two workgroups per CU */
#define LVS_KERNEL_BLIND_ROTATE_W16 5        /* sixteen-wave form, one workgroup per CU */

/* Kernel timing for measurement: while enabled, every launch of the blind
 * rotation, of the key switch and of a plan's graph is bracketed by HIP
 * events on the context's stream (ids above).  Enabling (or disabling) waits
 * for the stream and clears earlier records. */
int lvs_profile_enable(lvs_context* ctx, int enable);

/* Sum of the recorded launch durations of `kernel` (milliseconds), the
 * number of launches and the bootstraps they processed.  Waits for the
 * recorded events. */
int lvs_profile_read(lvs_context* ctx, int kernel, double* total_ms, uint64_t* launches, uint64_t* units);

/* Microbenchmarks of the two ceilings the blind rotation is measured
 * against.  lvs_microbench_modmul runs the forward-butterfly instruction
 * sequence (Shoup product by a twiddle: three 32-bit multiplies and three
 * adds) on 16 independent register chains per thread in eight resident waves
 * per SIMD on every CU, `iters` rounds, and returns the duration (ms) and the number of
 * 32-bit multiplies executed.  d_work (>= lvs_microbench_workspace_bytes(),
 * device) receives per-thread checksums.  lvs_microbench_copy copies `bytes`
 * (a multiple of 16, device buffers, 16-byte aligned) `reps` times with
 * 16-byte vector loads and stores and returns the mean ms per copy.
 * Synchronous; use the context's stream.  Errors: LVS_E_INVAL, LVS_E_DEVICE. */
size_t lvs_microbench_workspace_bytes(const lvs_context* ctx);
int lvs_microbench_modmul(lvs_context* ctx, int iters, void* d_work, size_t work_bytes, double* ms,
                          double* int_muls);
int lvs_microbench_copy(lvs_context* ctx, const void* d_src, void* d_dst, size_t bytes, int reps, double* ms);

/* Releases a handle created by the library (keys, contexts, plans, servers). */
void lvs_free(void* handle);

#ifdef __cplusplus
}
#endif

#endif /* LVS_H */
