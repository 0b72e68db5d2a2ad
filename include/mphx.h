/*
 * mphx.h -- C ABI of the MI355X (gfx950) MWHC build library: hypergraph peeling and minimal
 * perfect hashing after Belazzougui, Boldi, Ottaviano, Venturini, Vigna, "Cache-Oblivious
 * Peeling of Random Hypergraphs" (arXiv 1312.0526).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Pointers marked (dev) are device pointers on the current HIP device; (host) are host
 *    pointers.  The caller allocates and owns every buffer, including the workspace; the
 *    library never frees caller memory and allocates no device memory in these calls (the
 *    server API is the exception: it owns a pool sized by its budget).
 *  - `stream` is a hipStream_t passed as void*; all device work is enqueued on it.  Calls
 *    that return data-dependent results (status, info) synchronise that stream once or a
 *    few times before returning; the others only enqueue.
 *  - Status: 0 = MPHX_OK; negative = error (MPHX_EINVAL bad argument, MPHX_ERANGE a limit
 *    exceeded, MPHX_ENOMEM workspace too small, MPHX_EDEVICE a HIP runtime error); positive
 *    = the method's own failure outcomes (MPHX_ECORE a 2-core remained after every try,
 *    MPHX_EDUP duplicate keys).  mphx_last_error() returns a message for the calling thread.
 *    No C++ exception crosses the ABI.
 *  - Vertex layout of the tripartite hypergraph (Section 4.3, "Exploiting the
 *    tripartition"): P = ceil(n * gamma_num / (3 * gamma_den)) vertices per part, m = 3P;
 *    vertex k of every key's edge lies in part k, i.e. in [k*P, (k+1)*P).
 *  - Hashing (Section 3; SplitMix64 stands in for the paper's Jenkins hash): a u64 key x
 *    under seed s has state a = b = x XOR s; a byte string has the 128-bit digest (a, b)
 *    (two lanes, each the sum over the key's little-endian 8-byte words w_j, tail padded
 *    with zeros, of fin(w_j XOR (s_lane + j*GAMMA)), then fin(sum XOR s_lane XOR length),
 *    s_A = SplitMix64 output 1 at state s, s_B = output 2).  Vertex k is
 *    k*P + floor(z_k * P / 2^64) with z_0 = fin(a + GAMMA), z_1 = fin(a + 2 GAMMA),
 *    z_2 = fin(b + 3 GAMMA); fin is SplitMix64's output function, GAMMA = 0x9E3779B97F4A7C15.
 */
#ifndef MPHX_H
#define MPHX_H

#include <stddef.h>
#include <stdint.h>

#if defined(__GNUC__)
#define MPHX_API __attribute__((visibility("default")))
#else
#define MPHX_API
#endif

#ifdef __cplusplus
extern "C" {
#endif

#define MPHX_OK 0
#define MPHX_EINVAL (-1)
#define MPHX_ERANGE (-2)
#define MPHX_ENOMEM (-3)
#define MPHX_EDEVICE (-4)
#define MPHX_ECANCELED (-5) /* server: the request was not started before the server was destroyed */
#define MPHX_ECORE 1
#define MPHX_EDUP 2

/* round[] value of an edge that stays in the 2-core */
#define MPHX_ROUND_CORE 0xFFFFFFFFu
/* largest degree a vertex may reach (degrees are 8-bit quantities) */
#define MPHX_MAX_DEGREE 255u

typedef struct mphx_peel_info {
    uint64_t n_peeled;       /* edges removed; n - n_peeled edges form the 2-core */
    uint32_t n_rounds;       /* number of non-empty layers */
    uint32_t reserved;
    uint64_t frontier_total; /* frontier entries over all rounds (vertices that reached degree 1) */
    uint64_t claims;         /* (vertex, edge) pairs where the vertex had degree 1 at round start */
    uint64_t frontier0;      /* vertices of degree 1 before round 0 */
} mphx_peel_info;

typedef struct mphx_mphf_info {
    uint64_t P;          /* vertices per part */
    uint64_t m;          /* 3P vertices */
    uint64_t seed_used;  /* seed of the successful (or last) try */
    uint32_t tries;      /* tries made: seed, seed+1, ... */
    uint32_t n_rounds;   /* peeling rounds of the last try */
    uint64_t n_core;     /* 2-core edges left on the last try (0 on success) */
    uint64_t frontier_total; /* last try: frontier entries over all rounds */
    uint64_t claims;         /* last try: (vertex, edge) claims over all rounds */
    uint64_t frontier0;      /* last try: vertices of degree 1 before round 0 */
    uint64_t update_deletes; /* last try: deletes applied through update lists */
    uint64_t update_records; /* last try: vertex records those deletes changed */
    uint64_t layer0;         /* last try: edges removed in round 0 */
} mphx_mphf_info;

/* Message describing the last failure on the calling thread ("" if none). */
MPHX_API const char* mphx_last_error(void);

/* Vertices per part, P = ceil(n * gamma_num / (3 * gamma_den)) (Section 3: gamma*n vertices,
 * Section 4.3: three equal parts). */
MPHX_API uint64_t mphx_part_size(uint64_t n, uint32_t gamma_num, uint32_t gamma_den);

/* ---------------------------------------------------------------------------------------
 * Peeling (Section 1 definition of a peeling order and 2-core; Section 4.2 layered peeling;
 * Section 4.1 packed incidence lists).
 *
 * Synchronous rounds: round r removes every edge that has a vertex of degree 1 at the start
 * of round r.  Outputs, per edge e (all (dev), length n):
 *   round[e]     round that removed e, or MPHX_ROUND_CORE if e is in the 2-core;
 *   core_mask[e] 1 if e is in the 2-core, else 0;
 *   hinge[e]     lowest tuple position (0..2) among e's vertices that had degree 1 at the
 *                start of its round; 0xFF for 2-core edges.  May be NULL;
 *   order        edge ids sorted by round, ascending id inside a round, then the 2-core
 *                edges in ascending id (a peeling order of the peeled prefix).
 * Input edges (dev): n x 3 row-major uint32 vertex ids, each < m, three distinct ids per
 * edge.  n < 2^32, m <= 2^32.  Duplicate edges are legal (they end in the 2-core).
 * A non-empty 2-core is a result, not an error.
 * Errors: MPHX_EINVAL (null pointer, vertex >= m, a repeated vertex in an edge, sizes out of
 * range, misaligned workspace), MPHX_ERANGE (a degree above 255, or more rounds than the
 * workspace holds: mphx_peel_workspace_bytes reserves min(n, 2^22) + 2 rounds),
 * MPHX_ENOMEM (ws_bytes too small), MPHX_EDEVICE.
 * ws (dev): at least mphx_peel_workspace_bytes(n, m) bytes, 256-byte aligned, contents
 * ignored on entry.
 * --------------------------------------------------------------------------------------- */
MPHX_API size_t mphx_peel_workspace_bytes(uint64_t n, uint64_t m);
MPHX_API int mphx_peel(const uint32_t* edges, uint64_t n, uint64_t m, uint32_t* order, uint32_t* round,
              uint8_t* core_mask, uint8_t* hinge, void* ws, size_t ws_bytes, void* stream,
              mphx_peel_info* info /* host, may be NULL */);

/* The same peel for r-hypergraphs, 2 <= r <= 8 (Section 2 defines r-hypergraphs; the paper
 * works with r = 3 and notes that the generalization is direct): edges (dev) n x r row-major
 * uint32 vertex ids, each < m, r distinct ids per edge; hinge[e] in 0..r-1.  Same outputs,
 * conditions and errors as mphx_peel, plus MPHX_EINVAL for r outside [2, 8];
 * mphx_peel_r_workspace_bytes returns 0 for such r.  For r >= 3 a random r-hypergraph with
 * more than 1/c*_r vertices per edge peels completely with high probability (c*_3 = 0.818,
 * c*_4 = 0.772). */
MPHX_API size_t mphx_peel_r_workspace_bytes(uint64_t n, uint64_t m, uint32_t r);
MPHX_API int mphx_peel_r(const uint32_t* edges, uint64_t n, uint64_t m, uint32_t r, uint32_t* order,
                         uint32_t* round, uint8_t* core_mask, uint8_t* hinge, void* ws, size_t ws_bytes,
                         void* stream, mphx_peel_info* info);

/* ---------------------------------------------------------------------------------------
 * MWHC minimal perfect hash build (Section 3): hash the keys to a tripartite 3-hypergraph,
 * peel it (retrying with seed+1, seed+2, ... while a 2-core remains, up to max_tries),
 * assign g in {0,1,2} to the hinge vertices by backward substitution along the layers in
 * reverse round order (Section 4.3, "Avoiding backward scans"), and build the ranking table.
 *
 * Outputs (dev, caller-allocated):
 *   codes  ceil(m/32) uint64 words; vertex v's 2-bit code sits at bits 2*(v%32) of word
 *          v/32: 0 = not a hinge, 1 or 2 = hinge with g = 1 or 2, 3 = hinge with g = 0;
 *   rank   ceil(m/512) uint64; rank[b] = number of hinge vertices in [0, 512*b).
 * The MPHF of a key with edge (v0, v1, v2) is rank(v_i), i = (g0 + g1 + g2) mod 3 with
 * g = code mod 3, rank(h) = rank[h/512] + non-zero codes in [512*(h/512), h)  (Section 5
 * broadword ranking); it maps the n keys onto [0, n) bijectively.
 * gamma = gamma_num / gamma_den (1.23 = 123/100).  max_tries >= 1.
 * Byte-string keys: bytes (dev, 4-byte aligned), offs (dev) n+1 uint64 offsets, key i is
 * bytes[offs[i], offs[i+1]).
 * Errors: as mphx_peel, plus MPHX_ECORE (a 2-core remained on every try; info->n_core says
 * how large on the last) and MPHX_EDUP (on the last try the 2-core held two identical edges
 * from equal keys, which no seed can separate).
 * ws (dev): at least mphx_mphf_workspace_bytes(n, ...) bytes, 256-byte aligned.
 * --------------------------------------------------------------------------------------- */
#define MPHX_KEYS_U64 0
#define MPHX_KEYS_STR 1
MPHX_API size_t mphx_mphf_workspace_bytes(uint64_t n, uint32_t gamma_num, uint32_t gamma_den, int key_kind);
MPHX_API int mphx_mphf_build_u64(const uint64_t* keys, uint64_t n, uint64_t seed, uint32_t gamma_num,
                        uint32_t gamma_den, uint32_t max_tries, uint64_t* codes, uint64_t* rank,
                        void* ws, size_t ws_bytes, void* stream, mphx_mphf_info* info);
MPHX_API int mphx_mphf_build_str(const uint8_t* bytes, const uint64_t* offs, uint64_t n, uint64_t seed,
                        uint32_t gamma_num, uint32_t gamma_den, uint32_t max_tries, uint64_t* codes,
                        uint64_t* rank, void* ws, size_t ws_bytes, void* stream, mphx_mphf_info* info);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc): mphx_mphf_build_u64 without the ws argument.  Its
 * workspace is a device array of 128 MiB (134,217,728 bytes) that the library
 * holds on every device it runs on until the process ends; the call allocates nothing.  It
 * takes keys with a workspace up to that size (at gamma = 1.23, n <= 1,917,869 u64 keys) and
 * returns MPHX_ENOMEM, with a message, beyond it.  Arguments, outputs and results are those of
 * mphx_mphf_build_u64 (the same codes, rank and info).  Every call on a device shares that
 * device's array: calls that overlap on one device (other host threads, other streams) race
 * and must be serialized by the caller. */
MPHX_API int mphx_mphf_build_u64_static(const uint64_t* keys, uint64_t n, uint64_t seed, uint32_t gamma_num,
                                        uint32_t gamma_den, uint32_t max_tries, uint64_t* codes, uint64_t* rank,
                                        void* stream, mphx_mphf_info* info);

/* Evaluate a built MPHF (Section 3 definition; Section 5 lookup): out[i] = f(key i) (dev,
 * n uint64).  P and seed are the build's info->P and info->seed_used.  Enqueue only. */
MPHX_API int mphx_mphf_lookup_u64(const uint64_t* codes, const uint64_t* rank, uint64_t P, uint64_t seed,
                         const uint64_t* keys, uint64_t n, uint64_t* out, void* stream);
MPHX_API int mphx_mphf_lookup_str(const uint64_t* codes, const uint64_t* rank, uint64_t P, uint64_t seed,
                         const uint8_t* bytes, const uint64_t* offs, uint64_t n, uint64_t* out,
                         void* stream);

/* ---------------------------------------------------------------------------------------
 * Static functions (Section 3: MWHC stores any f: S -> [sigma]).  Keys are hashed, built and
 * peeled exactly as for the MPHF; then u in [sigma]^m is solved along the layers in reverse
 * round order so that f(x) = u[v0] + u[v1] + u[v2] (mod sigma) for every key, with u = 0 on
 * vertices that are no hinge.  Each u is stored in b = mphx_sf_bits(sigma) bits (the bits of
 * sigma - 1; 0 when sigma = 1): vertex v's field at bits [v*b, v*b + b) of the little-endian
 * bit string of the uint64 words.
 *   values (dev) n uint32, each below sigma (key i's value); sigma in [1, 2^32].
 *   words  (dev, caller-allocated) mphx_sf_words(n, gamma_num, gamma_den, sigma) uint64
 *          (may be null when that is 0).
 *   ws     (dev) at least mphx_sf_workspace_bytes(n, ...) bytes, 256-byte aligned.
 *   info   as for the MPHF (P and seed_used are needed for lookups).
 * Errors: as mphx_mphf_build_*, plus MPHX_EINVAL for sigma outside [1, 2^32] or a value not
 * below sigma (checked on the device before any try).  Synchronises the stream.
 * mphx_sf_lookup_*: out[i] = f(key i) (dev, n uint64).  Enqueue only.
 * --------------------------------------------------------------------------------------- */
MPHX_API uint32_t mphx_sf_bits(uint64_t sigma);
MPHX_API uint64_t mphx_sf_words(uint64_t n, uint32_t gamma_num, uint32_t gamma_den, uint64_t sigma);
MPHX_API size_t mphx_sf_workspace_bytes(uint64_t n, uint32_t gamma_num, uint32_t gamma_den, int key_kind);
MPHX_API int mphx_sf_build_u64(const uint64_t* keys, const uint32_t* values, uint64_t n, uint64_t sigma,
                               uint64_t seed, uint32_t gamma_num, uint32_t gamma_den, uint32_t max_tries,
                               uint64_t* words, void* ws, size_t ws_bytes, void* stream, mphx_mphf_info* info);
MPHX_API int mphx_sf_build_str(const uint8_t* bytes, const uint64_t* offs, const uint32_t* values, uint64_t n,
                               uint64_t sigma, uint64_t seed, uint32_t gamma_num, uint32_t gamma_den,
                               uint32_t max_tries, uint64_t* words, void* ws, size_t ws_bytes, void* stream,
                               mphx_mphf_info* info);
MPHX_API int mphx_sf_lookup_u64(const uint64_t* words, uint64_t sigma, uint64_t P, uint64_t seed,
                                const uint64_t* keys, uint64_t n, uint64_t* out, void* stream);
MPHX_API int mphx_sf_lookup_str(const uint64_t* words, uint64_t sigma, uint64_t P, uint64_t seed,
                                const uint8_t* bytes, const uint64_t* offs, uint64_t n, uint64_t* out,
                                void* stream);

/* ---------------------------------------------------------------------------------------
 * Static functions in the ranked layout (Section 3: ceil(log sigma) n + gamma n + o(n) bits
 * through a ranking structure).  The keys, values, hash, peel and u are exactly those of
 * mphx_sf_build_*; u is zero off the hinges, and only the vertices whose u is not zero keep a
 * field (at most n):
 *   marks (dev, caller-allocated) mphx_sfr_mark_words(n, gamma_num, gamma_den) uint64: bit
 *          v % 64 of word v / 64 is set iff u[v] != 0 (m = 3P bits).
 *   rank  (dev) mphx_sfr_rank_words(n, gamma_num, gamma_den) uint64: rank[j] = the number of
 *          marked vertices below vertex 1024 j, j = 0 .. ceil(m / 1024); the last entry is the
 *          number of fields.
 *   vals  (dev) mphx_sfr_val_words(n, sigma) uint64 (may be null when that is 0): the fields of
 *          the marked vertices in vertex order, field i at bits [i b, i b + b) of the
 *          little-endian bit string, b = mphx_sf_bits(sigma); the words after the last field,
 *          up to mphx_sfr_val_words(n, sigma), are 0.
 *   ws    (dev) at least mphx_sf_workspace_bytes(n, ...) bytes, 256-byte aligned.
 * Space: m + 64 (m / 1024 + 2) + fields * b bits, against b m for mphx_sf_build_*.  A lookup
 * reads the mark word, one rank sample, up to 15 more mark words of the same block (two 64-byte
 * lines) and the field.  Errors, info and synchronisation as mphx_sf_build_*; n = 0 writes
 * nothing.  mphx_sfr_lookup_*: out[i] = f(key i) (dev, n uint64).  Enqueue only.
 * --------------------------------------------------------------------------------------- */
MPHX_API uint64_t mphx_sfr_mark_words(uint64_t n, uint32_t gamma_num, uint32_t gamma_den);
MPHX_API uint64_t mphx_sfr_rank_words(uint64_t n, uint32_t gamma_num, uint32_t gamma_den);
MPHX_API uint64_t mphx_sfr_val_words(uint64_t n, uint64_t sigma);
MPHX_API int mphx_sfr_build_u64(const uint64_t* keys, const uint32_t* values, uint64_t n, uint64_t sigma,
                                uint64_t seed, uint32_t gamma_num, uint32_t gamma_den, uint32_t max_tries,
                                uint64_t* marks, uint64_t* rank, uint64_t* vals, void* ws, size_t ws_bytes,
                                void* stream, mphx_mphf_info* info);
MPHX_API int mphx_sfr_build_str(const uint8_t* bytes, const uint64_t* offs, const uint32_t* values, uint64_t n,
                                uint64_t sigma, uint64_t seed, uint32_t gamma_num, uint32_t gamma_den,
                                uint32_t max_tries, uint64_t* marks, uint64_t* rank, uint64_t* vals, void* ws,
                                size_t ws_bytes, void* stream, mphx_mphf_info* info);
MPHX_API int mphx_sfr_lookup_u64(const uint64_t* marks, const uint64_t* rank, const uint64_t* vals, uint64_t sigma,
                                 uint64_t P, uint64_t seed, const uint64_t* keys, uint64_t n, uint64_t* out,
                                 void* stream);
MPHX_API int mphx_sfr_lookup_str(const uint64_t* marks, const uint64_t* rank, const uint64_t* vals, uint64_t sigma,
                                 uint64_t P, uint64_t seed, const uint8_t* bytes, const uint64_t* offs, uint64_t n,
                                 uint64_t* out, void* stream);

/* Hash keys to edges (Section 3 / Section 4.3), edges (dev) n x 3 uint32.  Enqueue only. */
MPHX_API int mphx_hash_u64(const uint64_t* keys, uint64_t n, uint64_t seed, uint64_t P, uint32_t* edges,
                  void* stream);
MPHX_API int mphx_hash_str(const uint8_t* bytes, const uint64_t* offs, uint64_t n, uint64_t seed, uint64_t P,
                  uint32_t* edges, void* stream);

/* Check that vals (dev, n uint64) is a permutation of [0, n) (the MPHF definition,
 * Section 1).  scratch (dev, 256-byte aligned) must hold mphx_bijection_scratch_bytes(n)
 * bytes.  Returns the number of out-of-range or repeated values in *n_bad (host).
 * Synchronises the stream. */
MPHX_API size_t mphx_bijection_scratch_bytes(uint64_t n);
MPHX_API int mphx_check_bijection(const uint64_t* vals, uint64_t n, void* scratch, uint64_t* n_bad,
                         void* stream);

/* ---------------------------------------------------------------------------------------
 * Batched builds: B independent u64 key buckets (bucket b = keys[bucket_off[b],
 * bucket_off[b+1])), each an MWHC MPHF of its own exactly as mphx_mphf_build_u64 would build
 * it with the same seed, gamma and max_tries (Section 3 / 4.2 / 4.3 per bucket; independent
 * buckets as in the HEM scheme of Section 3).  One persistent launch: every workgroup takes
 * the next bucket from a device queue (the `order` array, largest first) and builds it alone,
 * including the retries, so nothing returns to the host between buckets.
 *
 * mphx_batch_layout (all host arrays): from the B+1 bucket offsets, writes code_off / rank_off
 * (B+1 entries each: where bucket b's ceil(m_b/32) code words and ceil(m_b/512) rank samples
 * start in the concatenated outputs; the last entry is the total), order (B bucket ids by
 * decreasing size) and *max_bucket.  Returns MPHX_EINVAL if offsets decrease or a bucket
 * needs 3P > 2^32 vertices.
 * mphx_build_batch_u64: device arrays keys, bucket_off, order, code_off, rank_off, codes,
 * rank, results (B entries); ws (dev, 256-byte aligned) of mphx_batch_workspace_bytes(...)
 * bytes for the same B, max_bucket and tuning.  Enqueues only (no synchronisation, no host
 * read-back), so the call can be captured into a HIP graph.  A bucket larger than max_bucket
 * gets status MPHX_EINVAL and is left untouched.  Per-bucket status: MPHX_OK, MPHX_ECORE
 * (2-core after max_tries; duplicate keys also end here), MPHX_ERANGE (degree above 255).
 * tuning may be NULL (block 1024, one workgroup per compute unit).
 * mphx_graph_capture_batch_u64 records the same work into an instantiated graph (*graph);
 * mphx_graph_launch replays it on a stream; mphx_graph_destroy frees it.
 * --------------------------------------------------------------------------------------- */
typedef struct mphx_bucket_result {
    uint64_t seed_used;
    uint32_t tries;
    int32_t status;
    uint32_t n_rounds;
    uint32_t reserved;
} mphx_bucket_result;

typedef struct mphx_batch_tuning {
    uint32_t block;  /* threads per workgroup: 256, 512 or 1024 (0 = 1024) */
    uint32_t grid;   /* workgroups in the persistent launch (0 = one per compute unit) */
    uint32_t scope;  /* atomics on a bucket's state: 0 = workgroup scope (one workgroup owns a
                        bucket), 1 = device scope; results are identical */
    uint32_t reserved;
} mphx_batch_tuning;

MPHX_API int mphx_batch_layout(const uint64_t* bucket_off, uint32_t B, uint32_t gamma_num, uint32_t gamma_den,
                               uint64_t* code_off, uint64_t* rank_off, uint32_t* order, uint64_t* max_bucket);
MPHX_API size_t mphx_batch_workspace_bytes(uint32_t B, uint64_t max_bucket, uint32_t gamma_num,
                                           uint32_t gamma_den, const mphx_batch_tuning* tuning);
MPHX_API int mphx_build_batch_u64(const uint64_t* keys, const uint64_t* bucket_off, const uint32_t* order,
                                  uint32_t B, uint64_t max_bucket, uint64_t seed, uint32_t gamma_num,
                                  uint32_t gamma_den, uint32_t max_tries, const uint64_t* code_off,
                                  const uint64_t* rank_off, uint64_t* codes, uint64_t* rank,
                                  mphx_bucket_result* results, void* ws, size_t ws_bytes,
                                  const mphx_batch_tuning* tuning, void* stream);
MPHX_API int mphx_graph_capture_batch_u64(const uint64_t* keys, const uint64_t* bucket_off, const uint32_t* order,
                                          uint32_t B, uint64_t max_bucket, uint64_t seed, uint32_t gamma_num,
                                          uint32_t gamma_den, uint32_t max_tries, const uint64_t* code_off,
                                          const uint64_t* rank_off, uint64_t* codes, uint64_t* rank,
                                          mphx_bucket_result* results, void* ws, size_t ws_bytes,
                                          const mphx_batch_tuning* tuning, void** graph);
/* Autotuning the batched launch.  The workgroup size fixes the per-workgroup LDS budget and
 * the vertex tile the records are built in (1024 threads: 158 KB, tiles of 8192 vertices,
 * one workgroup per compute unit; 512: 78 KB, 4096 vertices; 256: 48 KB, 4096 vertices), and
 * the grid how many workgroups share a compute unit; every tuning builds the same outputs.
 * mphx_batch_tuning_candidates writes up to `cap` candidate tunings to `out` (host; NULL
 * with cap 0 to ask for the count) and returns how many there are: (1024, 1 per CU),
 * (512, 1 per CU), (512, 2 per CU), (256, 2 per CU), (256, 3 per CU).
 * mphx_batch_autotune_u64 runs mphx_build_batch_u64 with each of the ncand tunings in
 * `cands` (host) on the given buckets -- a sample of the workload, which the caller chooses
 * -- once untimed and then `reps` times (1..100), timed by HIP events on `stream`, and writes
 * the index of the fastest to *best (host) and each candidate's best time in ms to ms[i]
 * (host, nullable; -1 for a candidate whose workspace, mphx_batch_workspace_bytes with that
 * tuning, exceeds ws_bytes, which is then skipped).  The other arguments are those of
 * mphx_build_batch_u64, and the outputs hold the build afterwards.  Synchronises (not for
 * graph capture).  Errors: MPHX_EINVAL for a bad argument or candidate (before any device
 * work), MPHX_ENOMEM if no candidate fits, MPHX_EDEVICE if a launch failed.  B = 0 returns
 * MPHX_OK with *best = 0 and no device work. */
MPHX_API uint32_t mphx_batch_tuning_candidates(mphx_batch_tuning* out, uint32_t cap);
MPHX_API int mphx_batch_autotune_u64(const uint64_t* keys, const uint64_t* bucket_off, const uint32_t* order,
                                     uint32_t B, uint64_t max_bucket, uint64_t seed, uint32_t gamma_num,
                                     uint32_t gamma_den, uint32_t max_tries, const uint64_t* code_off,
                                     const uint64_t* rank_off, uint64_t* codes, uint64_t* rank,
                                     mphx_bucket_result* results, void* ws, size_t ws_bytes,
                                     const mphx_batch_tuning* cands, uint32_t ncand, uint32_t reps, float* ms,
                                     uint32_t* best, void* stream);

/* The general form: B buckets described one by one (dev array `buckets`), each with its own
 * keys (u64 `keys`, or 4-byte-aligned string `bytes` + n+1 `offs` with keys == NULL), seed,
 * output buffers (codes ceil(m_b/32) words, rank ceil(m_b/512)) and result slot.  order (dev,
 * nullable) gives the processing order (largest first is best).  ws (dev, 256-byte aligned):
 * mphx_batch_desc_workspace_bytes(max_bucket, ...) bytes.  Enqueue only. */
typedef struct mphx_bucket {
    const uint64_t* keys;
    const uint8_t* bytes;
    const uint64_t* offs;
    uint64_t n;
    uint64_t seed;
    uint64_t* codes;
    uint64_t* rank;
    mphx_bucket_result* result;
} mphx_bucket;

MPHX_API size_t mphx_batch_desc_workspace_bytes(uint64_t max_bucket, uint32_t gamma_num, uint32_t gamma_den,
                                                const mphx_batch_tuning* tuning);
MPHX_API int mphx_build_batch(const mphx_bucket* buckets, uint32_t B, const uint32_t* order, uint64_t max_bucket,
                              uint32_t gamma_num, uint32_t gamma_den, uint32_t max_tries, void* ws, size_t ws_bytes,
                              const mphx_batch_tuning* tuning, void* stream);
MPHX_API int mphx_graph_launch(void* graph, void* stream);
MPHX_API int mphx_graph_destroy(void* graph);

/* ---------------------------------------------------------------------------------------
 * HEM split of one key set (Section 3, "Practical workarounds", with signatures that no two
 * keys share): a u64 key's signature is fin(s + 4*GAMMA), s = key XOR seed (64 bits, a
 * bijection); a string key's is its whole 128-bit digest (a, b) under seed (two distinct
 * strings share one with probability about n^2 / 2^129).  The top k bits of the signature's
 * first word pick one of 2^k buckets; inside it the key is the digest pair (swap(first word),
 * second word) -- (swap(sig), swap(sig)) for u64 keys, (swap(a), b) for strings, swap
 * exchanging the 32-bit halves -- whose edge under seed t is that of the digest (x XOR t,
 * y XOR t) (for u64 keys: the MWHC hash of the key swap(sig)).  Each bucket gets the MWHC MPHF
 * of its keys (hash seed `seed`, retries seed+1, ... per bucket) built by the batched kernel.
 * f(x) = bucket_off[b] + the bucket MPHF's value.
 *   k in [9, 20] (2^k buckets; beyond 2^18 each of the 2^18 buckets of the top 18 bits is split
 *   by the next k - 18 bits); outputs (dev, caller-allocated): bucket_off, code_off, rank_off
 *   (2^k + 1 each: where bucket b's keys, ceil(m_b/32) code words and ceil(m_b/512) rank
 *   samples start), seeds (2^k: each bucket's seed used), codes and rank (at least the
 *   mphx_hem_capacity words).  ws (dev, 256-byte aligned): mphx_hem_workspace_bytes bytes
 *   (key_kind MPHX_KEYS_U64: 8-byte signature records; MPHX_KEYS_STR: 16-byte ones);
 *   it admits buckets up to n/2^k + 8 sqrt(n/2^k) + 64 keys (MPHX_ENOMEM beyond).  Pick k so
 *   that buckets hold hundreds of keys or more: at gamma < 1.5 a bucket of exactly two keys
 *   has parts of one vertex, both edges are (0, 1, 2), and it fails under every seed.
 * Errors: MPHX_EINVAL for bad arguments; MPHX_ECORE (MPHX_ERANGE) when some bucket failed --
 * a 2-core on every try (or two equal keys) -- info->n_core then counts the failed buckets:
 * build again with another seed.  info->tries / n_rounds are the largest over the buckets.  Synchronises.
 * mphx_hem_lookup_*: out[i] = f(key i) (dev, n uint64); seed and k as built.  Enqueue only.
 * --------------------------------------------------------------------------------------- */
MPHX_API size_t mphx_hem_workspace_bytes(uint64_t n, uint32_t k, uint32_t gamma_num, uint32_t gamma_den,
                                         int key_kind);
MPHX_API int mphx_hem_capacity(uint64_t n, uint32_t k, uint32_t gamma_num, uint32_t gamma_den, uint64_t* code_words,
                               uint64_t* rank_words);
MPHX_API int mphx_hem_build_u64(const uint64_t* keys, uint64_t n, uint32_t k, uint64_t seed, uint32_t gamma_num,
                                uint32_t gamma_den, uint32_t max_tries, uint64_t* bucket_off, uint64_t* code_off,
                                uint64_t* rank_off, uint64_t* seeds, uint64_t* codes, uint64_t* rank, void* ws,
                                size_t ws_bytes, void* stream, mphx_mphf_info* info);
MPHX_API int mphx_hem_build_str(const uint8_t* bytes, const uint64_t* offs, uint64_t n, uint32_t k, uint64_t seed,
                                uint32_t gamma_num, uint32_t gamma_den, uint32_t max_tries, uint64_t* bucket_off,
                                uint64_t* code_off, uint64_t* rank_off, uint64_t* seeds, uint64_t* codes,
                                uint64_t* rank, void* ws, size_t ws_bytes, void* stream, mphx_mphf_info* info);
/* ---------------------------------------------------------------------------------------
 * The HEM split with the keys in HOST memory, for key sets larger than device memory (the
 * paper's key sets reach 7.6 * 10^9 keys, Table 1).  The result -- every output
 * above, bit for bit -- equals mphx_hem_build_* on the same keys, seed, k and gamma; the
 * lookups are mphx_hem_lookup_* (device keys, in batches of any size).
 *   keys (host, n uint64) or bytes + offs (host: key i is bytes[offs[i], offs[i+1]), offs
 *   non-decreasing, n + 1 entries): read by hipMemcpyAsync in chunks of at most chunk_keys keys
 *   (strings: and at most chunk_bytes bytes from the 256-byte boundary below the chunk's first
 *   key, so every key must be shorter than chunk_bytes - 255).  Pinned memory (hipHostMalloc)
 *   gives the full PCIe rate; pageable memory works, slower.  Device memory: 8 bytes per key
 *   (u64 keys) or 16 (strings) for the grouped signatures plus chunk and batch buffers:
 *   mphx_hem_host_workspace_bytes
 *   (kind = MPHX_KEYS_U64 or MPHX_KEYS_STR; chunk_bytes ignored for u64; 0 for bad
 *   arguments).  Each chunk's signatures are grouped by their top k - 8 bits; then batches of
 *   consecutive groups holding at most batch_keys keys are gathered from every chunk,
 *   partitioned into their buckets and built.  Outputs, seeds and errors as above;
 *   MPHX_ENOMEM also when one group holds more than batch_keys keys (groups hold about
 *   n / 2^(k-8): take batch_keys at least twice that).  chunk_keys, batch_keys in
 *   [1, 2^31 - 1), chunk_bytes >= 512.  Synchronises.
 * --------------------------------------------------------------------------------------- */
MPHX_API size_t mphx_hem_host_workspace_bytes(uint64_t n, uint32_t k, uint32_t gamma_num, uint32_t gamma_den,
                                              int kind, uint64_t chunk_keys, uint64_t chunk_bytes,
                                              uint64_t batch_keys);
MPHX_API int mphx_hem_build_host_u64(const uint64_t* keys, uint64_t n, uint32_t k, uint64_t seed,
                                     uint32_t gamma_num, uint32_t gamma_den, uint32_t max_tries,
                                     uint64_t chunk_keys, uint64_t batch_keys, uint64_t* bucket_off,
                                     uint64_t* code_off, uint64_t* rank_off, uint64_t* seeds, uint64_t* codes,
                                     uint64_t* rank, void* ws, size_t ws_bytes, void* stream, mphx_mphf_info* info);
MPHX_API int mphx_hem_build_host_str(const uint8_t* bytes, const uint64_t* offs, uint64_t n, uint32_t k,
                                     uint64_t seed, uint32_t gamma_num, uint32_t gamma_den, uint32_t max_tries,
                                     uint64_t chunk_keys, uint64_t chunk_bytes, uint64_t batch_keys,
                                     uint64_t* bucket_off, uint64_t* code_off, uint64_t* rank_off, uint64_t* seeds,
                                     uint64_t* codes, uint64_t* rank, void* ws, size_t ws_bytes, void* stream,
                                     mphx_mphf_info* info);
MPHX_API int mphx_hem_lookup_u64(const uint64_t* bucket_off, const uint64_t* code_off, const uint64_t* rank_off,
                                 const uint64_t* seeds, const uint64_t* codes, const uint64_t* rank, uint32_t k,
                                 uint32_t gamma_num, uint32_t gamma_den, uint64_t seed, const uint64_t* keys,
                                 uint64_t n, uint64_t* out, void* stream);
MPHX_API int mphx_hem_lookup_str(const uint64_t* bucket_off, const uint64_t* code_off, const uint64_t* rank_off,
                                 const uint64_t* seeds, const uint64_t* codes, const uint64_t* rank, uint32_t k,
                                 uint32_t gamma_num, uint32_t gamma_den, uint64_t seed, const uint8_t* bytes,
                                 const uint64_t* offs, uint64_t n, uint64_t* out, void* stream);

/* ---------------------------------------------------------------------------------------
 * Build server: continuous admission of MPHF builds of mixed sizes under an HBM budget.
 *
 * mphx_server_create allocates one device pool of hbm_budget bytes on `device` (the only
 * device allocation the library makes) and starts `slots` worker threads (1..64), each with its
 * own HIP stream.  With batch_max_keys > 0 it also reserves, inside the pool, a workspace for
 * batched launches (when the budget leaves room for it): requests of at most that many keys
 * then go to one more worker that builds every such request waiting at that moment together,
 * in one persistent batched launch (mphx_build_batch); the others take the plain path.  mphx_server_submit queues a request and returns a ticket at once; the
 * request's keys and output buffers are caller-owned device memory that must stay valid until
 * the ticket completes.  Requests are admitted in arrival order as workers and pool memory
 * free up (a later request that fits may pass the queue head a bounded number of times);
 * admitted builds run concurrently.  A request whose workspace exceeds what the pool can give
 * a build (the budget less the batching lane's reservation, if any) completes at once with
 * MPHX_ENOMEM; smaller ones wait and never fail for lack of memory: the queue head is passed
 * at most 8 times by later requests that fit, then admitted before any of them.
 * Each result (status, tries, seed, codes, rank) is exactly what mphx_mphf_build_u64/_str
 * returns for the request alone.  Times are seconds of mphx_server_clock() (steady clock):
 * t_submit at submission, t_start at admission, t_done when the outputs are complete.
 * mphx_server_poll returns 0 (done, *res filled) or 1 (pending); mphx_server_wait blocks.
 * mphx_server_destroy completes every request not admitted yet with MPHX_ECANCELED, waits for
 * the admitted builds to finish, then frees the pool; no other call on the server may overlap
 * or follow it.
 * --------------------------------------------------------------------------------------- */
typedef struct mphx_server mphx_server;

typedef struct mphx_request {
    int32_t key_kind;        /* MPHX_KEYS_U64 or MPHX_KEYS_STR */
    uint32_t max_tries;
    const uint64_t* keys;    /* dev, n u64 keys (MPHX_KEYS_U64) */
    const uint8_t* bytes;    /* dev, 4-byte aligned (MPHX_KEYS_STR) */
    const uint64_t* offs;    /* dev, n + 1 offsets into bytes (MPHX_KEYS_STR) */
    uint64_t n;
    uint64_t seed;
    uint32_t gamma_num, gamma_den;
    uint64_t* codes;         /* dev, ceil(m/32) words */
    uint64_t* rank;          /* dev, ceil(m/512) entries */
} mphx_request;

typedef struct mphx_request_result {
    int32_t status;
    uint32_t tries;
    uint32_t n_rounds;
    uint32_t reserved;
    uint64_t seed_used, P, m;
    double t_submit, t_start, t_done;
} mphx_request_result;

typedef struct mphx_server_stats_t {
    uint32_t pending, running;
    uint64_t completed;
    size_t budget, in_use, peak_in_use;
} mphx_server_stats_t;

MPHX_API int mphx_server_create(int device, size_t hbm_budget, uint32_t slots, uint64_t batch_max_keys,
                                mphx_server** server);
MPHX_API int mphx_server_submit(mphx_server* server, const mphx_request* req, uint64_t* ticket);
MPHX_API int mphx_server_poll(mphx_server* server, uint64_t ticket, mphx_request_result* res);
MPHX_API int mphx_server_wait(mphx_server* server, uint64_t ticket, mphx_request_result* res);
MPHX_API int mphx_server_stats(mphx_server* server, mphx_server_stats_t* stats);
MPHX_API double mphx_server_clock(void);
MPHX_API int mphx_server_destroy(mphx_server* server);

/* ---------------------------------------------------------------------------------------
 * Streamed MWHC build of u64 keys held in HOST memory, for key sets whose in-HBM build does
 * not fit the device (the paper builds 7.6 * 10^9 keys, Section 5).  The result -- codes and
 * rank -- is the MWHC MPHF of Section 3 exactly as mphx_mphf_build_u64 defines it (the same
 * hash, the same synchronous rounds and hinges, the same g), for any n with
 * P = ceil(gamma n / 3) <= 2^32 (about 1.04 * 10^10 keys at gamma = 1.23; vertex positions
 * k P + local beyond 2^32 are fine).
 * The vertex record is the packed incidence list of Section 4.1 for r = 3: a degree byte and the
 * XOR of the other two endpoints' part-local ids (Section 4.3's tripartition), from which a
 * vertex of degree 1 reads its edge; no edge array and no edge ids exist.  Each round scans the
 * degrees, appends the layer hinge first (runs by hinge part) and deletes it (Section 4.2); the
 * assignment walks the layers in reverse round order (Section 4.3).
 *   keys (host, n uint64; pinned gives the full PCIe rate) are copied in chunks of at most
 *   chunk_keys keys, once per try.
 *   layer_slots: slots of 12 bytes the device keeps for layers.  At least n: every layer stays
 *   in device memory.  Less: each round's layer is copied to host_layers (host, 12 n bytes,
 *   caller-owned) after its deletes and copied back, last round first, for the assignment; the
 *   largest layer (round 0's, about 0.24 n at gamma 1.23) must fit, else MPHX_ENOMEM.
 *   ws (dev, 256-byte aligned): mphx_stream_workspace_bytes(n, ...) bytes, about 9 bytes per
 *   vertex + 12 per layer slot + 16 per chunk key (two chunks: one is copied in on a stream of
 *   the library's own while the records are built from the other).  codes (dev) ceil(m/32) words, rank (dev)
 *   ceil(m/512) samples, as for mphx_mphf_build_u64.
 * Errors: MPHX_EINVAL (bad arguments, n = 0, P > 2^32, layer_slots < n without host_layers),
 * MPHX_ERANGE (a degree above 255), MPHX_ENOMEM (workspace, or a layer larger than the layer
 * area), MPHX_ECORE (a 2-core on every try; equal keys also end here), MPHX_EDEVICE.
 * Synchronises.  mphx_stream_workspace_bytes returns 0 for bad arguments.
 * mphx_mphf_lookup_wide_u64: f(key) for MPHFs of any P <= 2^32 (out: dev, n uint64; keys dev).
 * mphx_check_stream_u64: streams host keys through the evaluation and counts the values that
 * are >= n or repeated (0 = the MPHF is a bijection onto [0, n), Section 1); ws:
 * mphx_check_stream_workspace_bytes(n, chunk_keys) bytes (an n-bit map and one chunk).
 * --------------------------------------------------------------------------------------- */
MPHX_API size_t mphx_stream_workspace_bytes(uint64_t n, uint32_t gamma_num, uint32_t gamma_den, uint64_t chunk_keys,
                                            uint64_t layer_slots);
MPHX_API int mphx_mphf_build_stream_u64(const uint64_t* keys, uint64_t n, uint64_t seed, uint32_t gamma_num,
                                        uint32_t gamma_den, uint32_t max_tries, uint64_t chunk_keys,
                                        uint64_t layer_slots, void* host_layers, size_t host_layer_bytes,
                                        uint64_t* codes, uint64_t* rank, void* ws, size_t ws_bytes, void* stream,
                                        mphx_mphf_info* info);
MPHX_API int mphx_mphf_lookup_wide_u64(const uint64_t* codes, const uint64_t* rank, uint64_t P, uint64_t seed,
                                       const uint64_t* keys, uint64_t n, uint64_t* out, void* stream);
MPHX_API size_t mphx_check_stream_workspace_bytes(uint64_t n, uint64_t chunk_keys);
MPHX_API int mphx_check_stream_u64(const uint64_t* codes, const uint64_t* rank, uint64_t P, uint64_t seed,
                                   const uint64_t* keys, uint64_t n, uint64_t chunk_keys, void* ws, size_t ws_bytes,
                                   void* stream, uint64_t* n_bad);

/* ---------------------------------------------------------------------------------------
 * Synthetic key sets on the device (benchmark inputs; the same definitions as the host-side
 * generators that the tests use).  GAMMA and fin as above; S(s, t) = fin(s + t*GAMMA).
 *   u64 keys:     key_i = S(gen_seed, i + 1), i in [start, start + n).
 *   string keys:  with x_i the u64 key i: length = qtable[S(x_i, 1) >> 48]; bytes 0..4 are
 *                 0x20 + the base-95 digits of i (least significant first); byte j >= 5 is
 *                 0x20 + ((b * 95) >> 8) with b byte (j-5)%8 (little-endian) of S(x_i, 2 + (j-5)/8).
 * mphx_gen_str_lengths writes the n lengths (dev uint32) and mphx_gen_str_offsets their
 * exclusive prefix sums (dev, n+1 uint64; scratch (dev) >= mphx_scan_scratch_bytes(n+1));
 * mphx_gen_str_bytes then fills bytes (dev) from the offsets.  qtable (dev): 65536 uint16.
 * --------------------------------------------------------------------------------------- */
MPHX_API int mphx_gen_keys_u64(uint64_t* keys, uint64_t n, uint64_t gen_seed, uint64_t start, void* stream);
/* Bucketed u64 key sets: bucket b (keys[off[b], off[b+1]), off (dev) B+1 entries) is the u64
 * key set of generator seed S(0, b + 1). */
MPHX_API int mphx_gen_buckets_u64(uint64_t* keys, const uint64_t* off, uint32_t B, void* stream);
MPHX_API int mphx_gen_str_lengths(uint32_t* lens, uint64_t n, uint64_t gen_seed, uint64_t start,
                         const uint16_t* qtable, void* stream);
MPHX_API size_t mphx_scan_scratch_bytes(uint64_t count);
MPHX_API int mphx_gen_str_offsets(const uint32_t* lens, uint64_t n, uint64_t* offs, void* scratch,
                         size_t scratch_bytes, void* stream);
MPHX_API int mphx_gen_str_bytes(uint8_t* bytes, const uint64_t* offs, uint64_t n, uint64_t gen_seed,
                       uint64_t start, void* stream);

/* ---------------------------------------------------------------------------------------
 * Tuning and diagnostics.
 * mphx_set_option / mphx_get_option (process-wide):
 *   "grid"        blocks per launch of the grid-stride peeling kernels (0 = automatic: one
 *                 256-thread block per 256 edges of the layer, between 64 and 1024).
 *   "round_batch" peeling rounds enqueued before the first check of the termination flag
 *                 (default 64; later checks come every 16 rounds).  Empty rounds past the end
 *                 cost a launch each, a check a host round trip.
 *   "timing"      1 = record a HIP event pair on the caller's stream around every kernel
 *                 launch of mphx_peel / mphx_mphf_build_*, accumulated per phase.
 *   "part_build"  b in 0..32 (default 21): mphx_mphf_build_* with n >= 2^b keys builds the
 *                 vertex records by partitioning each part's (vertex, edge) incidences into
 *                 buckets of 2^14 vertices and accumulating each bucket in LDS; smaller key
 *                 sets (and every set with b = 0) use device atomics straight into the
 *                 records, one launch against the partition's dozen, faster while the
 *                 records stay in the caches (1 = always partitioned).  Both give identical
 *                 records; mphx_peel always uses the atomics.
 *   "claim_lists" b in 0..32 (default 26): mphx_mphf_build_* with n >= 2^b keys claims the
 *                 edges of each layer after the first by appending (edge, position) lists
 *                 that are radix-partitioned by edge and resolved in LDS, instead of one
 *                 device atomic per claim, and reads one count back per round.  0 = never.
 *                 The same codes either way; the workspace grows by 16 bytes per vertex, so
 *                 query mphx_mphf_workspace_bytes after setting it.
 *   "update_lists" p in 0..100 (default 16): in a claim-list build, a round whose claim count
 *                 c has 2c >= p% of the vertex count (and 2c <= m) deletes its layer through
 *                 a degree update list -- one (vertex, edge) record per delete, radix-
 *                 partitioned by vertex and applied per bucket of 2^14 records in LDS, the
 *                 sort-based round update of Section 4.2 -- instead of device atomics; the
 *                 claims of the next round then come from the updated records.  0 = never.
 *                 The same codes either way.
 *   "batch_lds"   1 (default) = in the batched kernel (mphx_build_batch*, the server's
 *                 batching lane, the HEM split) a bucket whose 4-byte records and edge states
 *                 fit in the workgroup's LDS budget (1024 threads: 158 KB, about 18,000 keys;
 *                 512: 78 KB, about 9,000; 256: 48 KB, about 5,500) is built and peeled
 *                 entirely in LDS; 0 = every bucket through device memory.
 *                 The same codes either way.
 *   "batch_sort_deletes" d in 0..1024 (default 4): in the batched kernel, a layer of a
 *                 bucket given by key words (at most 2^20 keys, built through device memory)
 *                 with 2 * layer * d >= m vertices, whose slots carry their hinges, deletes
 *                 through a list sorted by tile of vertices and applied in LDS instead of
 *                 device atomics; its claims clear part bits of the edge states and a scan
 *                 of the states appends the next layer; 0 = never.  The default takes layer
 *                 0 only (at gamma 1.23 it holds about a quarter of the edges).  The same
 *                 codes either way.
 *   "batch_claim_lists" 0 or 1 (default 1): in the batched kernel, the other layers of such
 *                 a bucket (those of at most 3n/8 edges: with sorted deletes off, all) record
 *                 their next-layer claims (and cancels of claims made stale within the
 *                 round) in a list that is grouped by tile of edges and resolved in LDS,
 *                 which also writes each winner's hinge part into its layer slot, instead
 *                 of one device atomicMin per claim and a state read per edge in the next
 *                 round; 0 = atomicMin.  The same codes either way.  A sparse round (at most
 *                 as many records as an LDS record tile has vertices) resolves in one LDS
 *                 hash table keyed by edge.
 *   "batch_clock" 0 or 1 (default 0): batched launches run the instantiation of the kernel
 *                 that adds its per-phase workgroup time and work counts to the device's
 *                 batch clock (mphx_batch_clock); 0 = the kernel without clocks.  The same
 *                 outputs either way; the clock costs a few registers and atomics per bucket.
 *   "hem_block"   256, 512 or 1024 (default 1024): workgroup size of the batched kernel that
 *                 builds the HEM split's buckets (mphx_hem_build_*, mphx_hem_build_host_*).
 *   "hem_grid"    0..65536 (default 0 = one workgroup per compute unit): its persistent grid.
 *                 Both shape the work only, never the result; the HEM workspaces depend on the
 *                 grid, so query them after setting it.
 *   "list_cap"    c >= 0 (default 0 = m): records a claim-list round may keep in its list (at
 *                 most m, the buffers' size).  A round with more claims, or a round 0 with
 *                 more deletes, makes the try start again with atomic claims (the same codes
 *                 either way); a small value exercises that fallback.
 *   "list_fallbacks" (read; set only to 0 to reset) tries redone with atomic claims after
 *                 a list overflowed, over the process.
 * Returns MPHX_EINVAL for an unknown key or value.
 *
 * mphx_phase_times copies the accumulated per-phase kernel time (ms) and launch counts of
 * the calling thread (phases: hash, build, frontier, apply, resolve, assign, rank, order, other,
 * update; mphx_phase_name(i) names phase i) and optionally resets them; returns the number of
 * phases.
 * --------------------------------------------------------------------------------------- */
MPHX_API int mphx_set_option(const char* key, int64_t value);
MPHX_API int64_t mphx_get_option(const char* key);
MPHX_API int mphx_phase_times(double* ms, uint64_t* launches, int max_phases, int reset);
MPHX_API const char* mphx_phase_name(int i);
/* mphx_batch_clock copies up to max_entries entries of the current device's batch clock to
 * out (host) and, if reset, zeroes it; returns the number of entries (MPHX_EDEVICE on a HIP
 * error, MPHX_EINVAL for a null out with max_entries > 0).  Entry 0 is the wall-clock tick
 * rate in Hz; then, summed over the workgroups of every launch made with option batch_clock=1
 * since the last reset: ticks spent in the record build (hashing, partition, records, layer 0),
 * the rounds' deletes, the grouping of claim lists, their resolve, rounds claiming by
 * atomicMin or sorted deletes, the assignment, code packing and rank, whole buckets of the LDS
 * path, the bucket queue, and the workgroups' lifetimes; then the device-path bucket and key
 * counts, tries, rounds, deletes issued in list rounds, claim-list records, and the LDS-path
 * bucket and key counts.  mphx_batch_clock_name(i) names entry i.  Phase ticks divided by the
 * grid give the average workgroup's time in that phase. */
MPHX_API int mphx_batch_clock(uint64_t* out, int max_entries, int reset);
MPHX_API const char* mphx_batch_clock_name(int i);

/* ---------------------------------------------------------------------------------------
 * Machine-ceiling probes (measurement only; none is on the build path).  The streaming copy
 * gives the practical HBM ceiling the build's streaming phases are compared against; the
 * random probes give the throughput of the access patterns that bound the degree build
 * (non-returning 8-byte atomic add), the peeling rounds (returning 8-byte atomic add), the
 * assignment (8-byte random loads, 1-byte random stores) and an LDS-resident build (8-byte
 * LDS atomic add), as a function of the table's footprint.
 *
 * mphx_probe_copy: dst[0, bytes) = src[0, bytes); both 16-byte aligned, bytes a multiple
 *   of 16 (else MPHX_EINVAL).  grid 0 = 8192 blocks of 256 threads.
 * mphx_probe_random: `count` operations at indices uniform in [0, slots) drawn from the
 *   SplitMix64 outputs of seed + (i+1)*0x9E3779B97F4A7C15.  The table (dev) holds `slots`
 *   entries of 8 bytes (1 byte for MPHX_PROBE_STORE1); for MPHX_PROBE_LDS_ATOMIC_ADD each
 *   workgroup keeps its own LDS table of `slots` <= 8192 entries and writes it to
 *   table[block_index * slots + j] at the end, so the table holds grid * slots entries.
 *   The table's contents afterwards are meaningless.  grid 0 = 8192; block a multiple of 64
 *   up to 1024.  Returns MPHX_EINVAL for a bad argument, MPHX_EDEVICE if the launch failed.
 * --------------------------------------------------------------------------------------- */
#define MPHX_PROBE_ATOMIC_ADD 1
#define MPHX_PROBE_ATOMIC_ADD_RET 2
#define MPHX_PROBE_LOAD8 3
#define MPHX_PROBE_STORE1 4
#define MPHX_PROBE_LDS_ATOMIC_ADD 5
#define MPHX_PROBE_ATOMIC_ADD32 6   /* 4-byte entries */
#define MPHX_PROBE_ATOMIC_ADD_WG 7  /* workgroup-scope 8-byte add: atomic only within a workgroup */
MPHX_API int mphx_probe_copy(const void* src, void* dst, uint64_t bytes, uint32_t grid, void* stream);
MPHX_API int mphx_probe_random(int op, void* table, uint64_t slots, uint64_t count, uint64_t seed, uint32_t grid,
                               uint32_t block, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* MPHX_H */
