/*
 * pmp.h — C ABI of libpmp, batched PM+32 / PM+64 hashing on AMD Instinct
 * MI355X (gfx950).
 *
 * The hash families are those of Ivanchykhin, Ignatchenko and Lemire,
 * "Regular and almost universal hashing: an efficient implementation"
 * (arXiv 1609.09840):
 *   - field Z_p with p = 2^32 + 15 (PM+32) or p = 2^64 + 13 (PM+64), the
 *     smallest primes above a word power (Sec. 5, Table "smallestprimes");
 *   - block function f_j(s) = (b_j + sum_{i<128} a_{j,i} s_i) mod p (Eq. (1)),
 *     keys a in (0, p - kappa) with kappa = 28 / 24, b in [0, 2^n)
 *     (Sec. 6.1, Table "parameters");
 *   - tree construction over blocks of m = 128 words, at most 8 levels
 *     (Algorithm 1, Sec. 4);
 *   - byte strings become n-bit little-endian words after appending a byte
 *     0x01 and zero bytes up to the next word boundary (end of Sec. 4);
 *   - output h mod 2^n (Sec. 5, after Lemma 9), then the avalanche mixer of
 *     Sec. 7 unless PMP_NO_MIX is given.
 *
 * Conventions the paper leaves open (fixed here, same in every entry point):
 *   leaves always use the level-1 keys (Algorithm 1, Fig. 1); at least one
 *   level is applied, also to strings of less than one word; the key table is
 *   a[8][128] (level-major) followed by b[8].
 *
 * Memory: "device" pointers are HIP device memory (hipMalloc or a torch CUDA
 * tensor on ROCm); "host" pointers are ordinary host memory. The caller owns
 * every buffer passed in. The library owns only plan workspaces.
 *
 * Errors: every entry point returns 0 (PMP_OK) or a negative PMP_E_* code and
 * sets a thread-local message readable with pmp_last_error(). Hash calls are
 * asynchronous on the given stream; problems that only the device can see
 * (offsets out of order or past the buffer) are recorded in the plan's status
 * word and reported by pmp_plan_status().
 */
#ifndef PMP_H_
#define PMP_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
#define PMP_OK 0
#define PMP_E_INVALID_ARG (-1) /* null pointer, negative count, bad flag     */
#define PMP_E_KEY_RANGE (-2)   /* a key a_{j,i} outside [0, p - kappa - 1]    */
#define PMP_E_TOO_LONG (-3)    /* a string needs more than 8 levels          */
#define PMP_E_OFFSETS (-4)     /* offsets decrease or point past buf_bytes   */
#define PMP_E_HIP (-5)         /* a HIP runtime call failed                  */
#define PMP_E_NOMEM (-6)       /* workspace allocation failed                */
#define PMP_E_INTERNAL (-7)    /* a tree-node accumulator index fell outside the plan workspace */

/* flags for the hash calls */
#define PMP_NO_MIX 1u    /* output h mod 2^n without the Sec. 7 mixer        */
#define PMP_OUT_FIELD 2u /* output the field element h itself (see below)    */

/* key table geometry */
#define PMP_LEVELS 8
#define PMP_BLOCK 128
#define PMP_KEYS (PMP_LEVELS * PMP_BLOCK + PMP_LEVELS) /* 1032 entries */

typedef struct pmp_plan pmp_plan; /* opaque: workspace + status + tuning */
typedef struct ihipStream_t* pmp_stream_t; /* a hipStream_t (0 = null stream) */

/* ---------------------------------------------------------------------- */
/* Key tables (Eq. (1) keys; generation is a project convention because the
 * paper only asks for keys drawn at random).
 *
 * pmp_expand_keys32 / pmp_expand_keys64: fill a HOST table of PMP_KEYS
 * entries from splitmix64 started at `seed`. Entries are drawn in storage
 * order: a[0][0..127], ..., a[7][0..127], then b[0..7]. PM+32 takes the top
 * 32 bits of each 64-bit draw. An `a` draw outside [1, p - kappa - 1]
 * (PM+32: [1, 2^32 - 14]; PM+64: [1, 2^64 - 12]) is discarded and drawn
 * again; b takes the next 8 draws as they are. Returns PMP_E_INVALID_ARG if
 * keys_out is NULL. Upload the table to the device once and keep it there. */
int pmp_expand_keys32(uint64_t seed, uint32_t* keys_out);
int pmp_expand_keys64(uint64_t seed, uint64_t* keys_out);

/* pmp_check_keys32 / pmp_check_keys64: check a HOST key table. Every a must
 * lie in [0, p - kappa - 1] so that a * s < 2^(2n) for every field element s
 * (Sec. 6.1); zero keys are accepted (they make a degenerate but well-defined
 * function, useful for tests). Returns PMP_OK or PMP_E_KEY_RANGE. */
int pmp_check_keys32(const uint32_t* keys);
int pmp_check_keys64(const uint64_t* keys);

/* ---------------------------------------------------------------------- */
/* Plans. A plan owns a device workspace (one tree-node accumulator per 128
 * words of buffer, a status word, a pinned descriptor staging buffer) sized
 * for a batch. Calls that share a plan must be
 * ordered on one stream. plan == NULL in a hash call selects a default plan
 * private to the (current device, stream) pair, created on first use.
 * Creating or growing a workspace allocates device memory; hash calls on a
 * plan reserved large enough do not allocate. */
int pmp_plan_create(int device, pmp_plan** plan_out);
int pmp_plan_destroy(pmp_plan* plan);
/* Size the workspace for batches whose buffers total at most max_buf_bytes
 * bytes over at most max_count strings (both variants together). */
int pmp_plan_reserve(pmp_plan* plan, uint64_t max_buf_bytes, int64_t max_count);
/* Synchronize `stream`, then return and clear the device-side status of
 * `plan` (NULL: the default plan of the current device and `stream`):
 * PMP_OK, PMP_E_OFFSETS or PMP_E_INTERNAL (a consistency check of the
 * workspace that a correct call never trips). A nonzero status also clears
 * the workspace so that the plan can be used again. */
int pmp_plan_status(pmp_plan* plan, pmp_stream_t stream);
/* Lanes per 128-word block for strings longer than one block, per variant
 * (wide = 0: PM+32, 1: PM+64; 0 = the default, 8 and 8). Compiled pairs:
 * (8,16) (8,8) (16,16) (4,16) (16,8) (4,8); others give PMP_E_INVALID_ARG.
 * Set by the autotuner or by hand. */
int pmp_plan_set_tile(pmp_plan* plan, int wide, int lanes_per_block);
/* Launch shape: waves per CU (0 = as many as stay resident), the per-string
 * work weight alpha in byte equivalents used to split a batch between waves
 * (0 = keep; a new plan has 768; PMP_ALPHA_BY_COUNT splits by string count
 * alone, which needs no search of the offsets and suits batches of strings
 * of similar lengths), the smallest share of work worth a wave
 * (0 = keep; a new plan has 8192), and the
 * number of shares each wave takes, spread over the batch (1..64, 0 = keep;
 * more shares even out regions of the batch that cost more per byte, at a
 * small search cost per share). */
#define PMP_ALPHA_BY_COUNT 0xFFFFFFFFu
int pmp_plan_tune(pmp_plan* plan, int waves_per_cu, uint32_t alpha, uint64_t wave_bytes, int shares_per_wave);

/* ---------------------------------------------------------------------- */
/* Hashing a batch (Algorithm 1 with Eq. (1) blocks, Sec. 4 byte padding,
 * Sec. 5 output, Sec. 7 mixer).
 *
 *   d_buf      device, concatenated string bytes; no alignment required
 *   buf_bytes  number of bytes at d_buf that hold the strings. The kernels
 *              read no other byte, except that the short-string path loads
 *              whole 16-byte-aligned granules: up to 15 bytes before a
 *              string and after it, within the granule of one of its bytes
 *              (a granule never crosses a page, so these loads cannot fault;
 *              bytes outside the strings never reach an output)
 *   d_offsets  device, int64[count + 1]: string i is
 *              d_buf[d_offsets[i] .. d_offsets[i+1]); offsets must be
 *              non-decreasing and lie in [0, buf_bytes]; empty strings are
 *              allowed. A string whose offsets break this gets no output and
 *              the plan's status becomes PMP_E_OFFSETS; since the work is
 *              split among waves by offset, strings near offsets that
 *              decrease may get no output either.
 *   count      number of strings (0 is a no-op)
 *   d_keys     device, key table of PMP_KEYS entries (layout above)
 *   d_out      device output:
 *                pmp_hash32: uint32[count]; with PMP_OUT_FIELD uint64[count]
 *                  holding h < 2^32 + 15
 *                pmp_hash64: uint64[count]; with PMP_OUT_FIELD
 *                  uint64[2 * count], pairs (h mod 2^64, h >> 64)
 *   flags      0, PMP_NO_MIX or PMP_OUT_FIELD
 *   stream     HIP stream the work is queued on; the call returns at once.
 *
 * One kernel launch processes the whole batch. The batch is cut into equal
 * shares of work (bytes plus a per-string weight) by a merge-path split over
 * the offsets, one share per wave. Strings of at most one block are hashed
 * one per lane, medium strings one per lane group, long strings a level-2
 * node (128 blocks) per wave; the levels above 2 are finished by whichever
 * wave completes a node's last child, through the plan's accumulators. */
int pmp_hash32(pmp_plan* plan, const uint8_t* d_buf, uint64_t buf_bytes, const int64_t* d_offsets,
               int64_t count, const uint32_t* d_keys, void* d_out, uint32_t flags, pmp_stream_t stream);
int pmp_hash64(pmp_plan* plan, const uint8_t* d_buf, uint64_t buf_bytes, const int64_t* d_offsets,
               int64_t count, const uint64_t* d_keys, void* d_out, uint32_t flags, pmp_stream_t stream);

/* One batch for pmp_hash_mixed: the arguments of pmp_hash32/64 in a struct.
 * keys points to uint32[PMP_KEYS] when wide == 0, uint64[PMP_KEYS] when
 * wide == 1. */
typedef struct pmp_batch {
  const uint8_t* buf;
  uint64_t buf_bytes;
  const int64_t* offsets;
  int64_t count;
  const void* keys;
  void* out;
  uint32_t flags;
  uint32_t wide; /* 0: PM+32, 1: PM+64 */
} pmp_batch;

/* Hash up to two batches (any mix of PM+32 and PM+64) in ONE kernel launch;
 * either pointer may be NULL. Same semantics per batch as pmp_hash32/64. */
int pmp_hash_mixed(pmp_plan* plan, const pmp_batch* b0, const pmp_batch* b1, pmp_stream_t stream);

/* For callers that cannot allocate device memory (code under stream capture,
 * tight serving loops, harnesses that forbid hipMalloc): pmp_hash_mixed
 * without a plan, with the same outputs. The node accumulators live in a
 * static device array of PMP_NOALLOC_SCRATCH_BYTES per device (16 bytes per
 * 128-word block of each batch's buffer, plus 2 per batch: up to about
 * 512 MiB of PM+32 or 1 GiB of PM+64 buffer), held until the process ends.
 * Batches that need more return PMP_E_NOMEM before anything is queued.
 * d_status: caller-owned device int32; the call sets it to 0, and the kernel
 * ORs in 1 for offsets out of order or past buf_bytes (those strings get no
 * output) and 2 for an internal workspace fault. The call queues a fill
 * kernel (it clears the accumulators it uses and *d_status) and the hash
 * kernel on `stream`, asynchronously, and allocates nothing. All calls on
 * one device share the array: calls that overlap on one device race (the
 * same stream orders them). Tiles and work weight are the library defaults. */
#define PMP_NOALLOC_SCRATCH_BYTES (16u << 20)
int pmp_hash_mixed_noalloc(const pmp_batch* b0, const pmp_batch* b1, int32_t* d_status, pmp_stream_t stream);
/* Hash any number of batches (a HOST array of nbatch descriptors) in ONE
 * kernel launch; each batch keeps its own buffer, offsets, keys, output and
 * flags. With more than two batches the descriptors are uploaded to the
 * device on `stream` first (through the plan's pinned staging buffer). */
int pmp_hash_many(pmp_plan* plan, const pmp_batch* batches, int32_t nbatch, pmp_stream_t stream);

/* Captured launches (hipGraph). pmp_graph_create captures the launch that
 * pmp_hash_many(plan, batches, nbatch, .) would make into a graph, with the
 * plan's current tiles and launch shape; pmp_graph_launch replays it on any
 * stream at the cost of one graph launch. The graph keeps the batch
 * descriptors (pointers, counts, flags) fixed; the CONTENTS of the buffers,
 * offsets, keys and outputs are read at each replay, so new data in the same
 * buffers is hashed by the next replay. The plan must not be used by other
 * calls while a replay runs, and must outlive the graph. Creation allocates
 * (workspace, descriptors); replays do not. Later calls on the plan that
 * need a larger workspace allocate a new one and keep the one the graphs
 * use until the plan's last graph is destroyed. */
typedef struct pmp_graph pmp_graph;
int pmp_graph_create(pmp_plan* plan, const pmp_batch* batches, int32_t nbatch, pmp_graph** graph_out);
int pmp_graph_launch(pmp_graph* graph, pmp_stream_t stream);
int pmp_graph_destroy(pmp_graph* graph);

/* Autotuner: times pmp_hash_many(plan, batches, nbatch, stream) over every
 * compiled lanes-per-block pair and per-string weight alpha in {256, 512, 768, 1024,
 * 1536, 2048, PMP_ALPHA_BY_COUNT},
 * then over 1, 2 and 4 shares per wave, then over launch widths of 4, 12 and
 * 16 waves per CU, each stage on the best of the one before (three launches
 * a setting), then times the four fastest again over ten launches each;
 * leaves the fastest setting in the plan and reports it in *best (may be
 * NULL). The
 * outputs are written by every timed launch (same values). The stream is
 * synchronized. */
typedef struct pmp_tuning {
  int32_t g32, g64;        /* lanes per block, PM+32 / PM+64 */
  uint32_t alpha;          /* per-string work weight, bytes */
  int32_t waves_per_cu;    /* 0: as many as stay resident */
  int32_t shares_per_wave; /* shares of the work per wave */
  float ms;                /* mean launch time of the chosen setting */
} pmp_tuning;
int pmp_plan_autotune(pmp_plan* plan, const pmp_batch* batches, int32_t nbatch, pmp_stream_t stream,
                      pmp_tuning* best);

/* ---------------------------------------------------------------------- */
/* Serving loop (continuous batching). A server owns `lanes` in-flight
 * positions, each a HIP stream with its own plan and a device arena of
 * lane_bytes (plus a pinned host twin). A dispatcher thread takes queued
 * requests in arrival order and hashes as many as fit one lane in ONE launch
 * (pmp_hash_many), while earlier launches still run on other lanes.
 *
 * A request is a batch of strings of one variant (wide 0: PM+32, 1: PM+64),
 * hashed with the server's key tables:
 *   device_resident = 1: buf, offsets, out are device pointers, used in
 *     place (the caller keeps them alive until the request completes);
 *   device_resident = 0: they are HOST pointers; payload and offsets are
 *     copied through the lane arena and the hashes copied back to `out`
 *     before the request counts as complete. Such a request must fit the
 *     arena (16-byte rounded payload + offsets + output <= lane_bytes), else
 *     submit returns PMP_E_NOMEM ("admission by memory"); a request that fits
 *     waits in the queue until a lane has room. Its offsets are checked at
 *     submit (PMP_E_OFFSETS if out of order or past buf_bytes).
 * Device-resident requests are admitted against max_inflight_bytes: the
 * payload bytes of the batches on the device never exceed it (a request
 * larger than the budget is refused at submit with PMP_E_NOMEM), and every
 * lane's plan is sized for it at creation, so the loop does not allocate.
 * Offsets of a device-resident request are checked by the kernel: a batch
 * that flags bad offsets is hashed again one request at a time, and only the
 * requests with bad offsets fail (pmp_server_wait returns PMP_E_OFFSETS);
 * the others complete with their correct outputs.
 * While a lane is busy or a request is queued, the dispatcher polls without
 * sleeping; when idle it polls for idle_spin_us before it sleeps.
 * Latency is measured from submit to completion (results visible in `out`).
 * Outputs are bit-identical to hashing the request alone with pmp_hash32/64. */
typedef struct pmp_server pmp_server;

typedef struct pmp_server_config {
  int device;                     /* HIP device index */
  int lanes;                      /* in-flight launches, 1..16 */
  uint64_t lane_bytes;            /* arena per lane for host requests (0: device-resident only) */
  const uint32_t* d_keys32;       /* device, PM+32 key table (PMP_KEYS entries) */
  const uint64_t* d_keys64;       /* device, PM+64 key table */
  int max_requests_per_batch;     /* >= 1 */
  int64_t max_batch_strings;      /* strings per launch before a lane closes (0: no limit) */
  uint64_t reserve_bytes;         /* pre-size each lane's plan for this much buffer (0: grow on use) */
  uint64_t max_inflight_bytes;    /* device-resident payload bytes in flight over all lanes (0: no limit) */
  int32_t idle_spin_us;           /* when idle, the dispatcher polls for work this long before it
                                     sleeps (0..1000000; 0: sleep at once) */
  int32_t reserved;
} pmp_server_config;

typedef struct pmp_request {
  const uint8_t* buf;
  uint64_t buf_bytes;
  const int64_t* offsets; /* int64[count + 1], rules as for pmp_hash32 */
  int64_t count;
  void* out;              /* as d_out of pmp_hash32/64 */
  uint32_t flags;
  uint32_t wide;
  uint32_t device_resident;
  uint32_t reserved;
} pmp_request;

typedef struct pmp_server_report {
  uint64_t completed, rejected, batches, bytes; /* bytes: payload bytes hashed */
  uint64_t failed;                              /* requests that completed with an error */
  double p50_us, p99_us, max_us, mean_us;       /* submit-to-completion latency */
  double span_us;                               /* first submit to last completion */
} pmp_server_report;

int pmp_server_create(const pmp_server_config* cfg, pmp_server** out);
/* Finish every queued request, then free the server. */
int pmp_server_destroy(pmp_server* server);
/* Queue a request (any thread). *ticket identifies it for pmp_server_wait. */
int pmp_server_submit(pmp_server* server, const pmp_request* req, uint64_t* ticket);
/* Wait for a request: timeout_us < 0 waits for ever. Returns 1 if it is still
 * pending at the timeout (the ticket stays valid), else its final status
 * (PMP_OK or a PMP_E_* code, PMP_E_OFFSETS for offsets the kernel found
 * bad) and releases the ticket. */
int pmp_server_wait(pmp_server* server, uint64_t ticket, int64_t timeout_us);
/* Latency and throughput over the requests completed since the last reset. */
int pmp_server_stats(pmp_server* server, pmp_server_report* stats);
int pmp_server_reset_stats(pmp_server* server);
/* Load generator: submit reqs[k] at arrival_us[k] microseconds after the
 * call starts (non-decreasing), wait for all, and write each latency to
 * latency_us[k] (may be NULL). Returns PMP_OK or the worst request status. */
int pmp_server_replay(pmp_server* server, const pmp_request* reqs, int64_t n, const double* arrival_us,
                      double* latency_us);
/* Device status of every lane's plan, as pmp_plan_status (synchronizes). */
int pmp_server_status(pmp_server* server);

/* ---------------------------------------------------------------------- */
/* PM+128: the same construction over p = 2^128 + 51, the smallest prime
 * above 2^128 (Table "smallestprimes"), with 16-byte words. The paper gives
 * only the prime for n = 128; the rest follows PM+32 / PM+64: words after
 * the 0x01 byte and zero padding to a multiple of 16 (end of Sec. 4),
 * Eq. (1) with 128-bit keys, the tree of Algorithm 1 (leaves on level-1
 * keys, at least one and at most 8 levels), output h mod 2^128 (Sec. 5).
 * Keys a in [1, 2^128 - 50] (p - kappa - 1 with kappa = 2 (k - 1) = 100,
 * extended from Table "parameters"), b in [0, 2^128). Sec. 7 defines no
 * mixer for n = 128: the output is never mixed and PMP_NO_MIX changes
 * nothing.
 *
 * Key table: PMP_KEYS entries of two uint64 (lo, hi), a[8][128] then b[8]
 * (2064 uint64). pmp_expand_keys128 fills a HOST table from splitmix64(seed),
 * two draws per entry (low half first), redrawing an `a` outside its range;
 * pmp_check_keys128 returns PMP_E_KEY_RANGE for an `a` above 2^128 - 50.
 *
 * pmp_hash128: string i = d_buf[d_offsets[i] .. d_offsets[i+1]) (device
 * memory, as pmp_hash32). d_out: count x 2 uint64 (lo, hi of h mod 2^128),
 * or with PMP_OUT_FIELD count x 3 uint64 (lo, hi, top bit of h < p). A pair
 * of offsets out of order or past buf_bytes is hashed as an empty string.
 * d_scratch: device memory of pmp_hash128_scratch_bytes(count, buf_bytes)
 * bytes at least. Seven launches on `stream` (string counts, a three-launch
 * scan, short strings, level-2 nodes, upper levels), asynchronous; no
 * allocation. */
int pmp_expand_keys128(uint64_t seed, uint64_t* keys_out);
int pmp_check_keys128(const uint64_t* keys);
uint64_t pmp_hash128_scratch_bytes(int64_t count, uint64_t buf_bytes);
int pmp_hash128(const uint8_t* d_buf, uint64_t buf_bytes, const int64_t* d_offsets, int64_t count,
                const uint64_t* d_keys, void* d_out, uint32_t flags, void* d_scratch, uint64_t scratch_bytes,
                pmp_stream_t stream);

/* ---------------------------------------------------------------------- */
/* Hash table of variable-length keys (Sec. 1 and Sec. 3: a randomly chosen
 * hash function picks each key's bucket; bucket = h mod M keeps the family
 * almost universal (Lemma 1) and regular (Lemma 8)). h is the n-bit output
 * of pmp_hash32/64 with the batch's flags (PMP_OUT_FIELD is refused).
 *
 * pmp_table_build: hashes the batch `keys` (key i = its string i) into
 * keys->out (count outputs), then builds a CSR table in caller-owned device
 * arrays: d_bucket_start[M + 1] (int64; bucket b holds entries
 * [start[b], start[b + 1])) and d_entries[count], one 32-byte record per key
 * (its index, its n-bit hash, its offset and length in keys->buf). The
 * order of the entries within a bucket is unspecified. d_work: device
 * scratch of at least
 * pmp_table_work_bytes(M) bytes. M = nbuckets in [1, 2^31]. Asynchronous on
 * `stream`; plan as for the hash calls.
 *
 * pmp_table_probe: hashes the batch `queries` into queries->out, then writes
 * d_result[q] = the smallest key index i whose bytes equal query q's, or -1.
 * `keys` is the batch given to the build (its buf is read; the entries hold
 * the rest); queries and keys must share wide, the key table pointer and the
 * flags. The byte comparison loads whole 16-byte-aligned granules that hold
 * a byte of the query or key compared (as the short-string path of the hash
 * does), never other memory. Returns PMP_E_INVALID_ARG on NULL pointers,
 * mismatched batches or M out of range. */
typedef struct pmp_table_entry {
  int64_t key;     /* key index in the build's batch */
  uint64_t hash;   /* its n-bit output (PM+32: zero-extended) */
  int64_t offset;  /* its first byte in the build's buf */
  int64_t length;  /* its length in bytes */
} pmp_table_entry;
uint64_t pmp_table_work_bytes(uint64_t nbuckets);
int pmp_table_build(pmp_plan* plan, const pmp_batch* keys, uint64_t nbuckets, int64_t* d_bucket_start,
                    pmp_table_entry* d_entries, void* d_work, uint64_t work_bytes, pmp_stream_t stream);
int pmp_table_probe(pmp_plan* plan, const pmp_batch* queries, const pmp_batch* keys, uint64_t nbuckets,
                    const int64_t* d_bucket_start, const pmp_table_entry* d_entries, int64_t* d_result,
                    pmp_stream_t stream);

/* ---------------------------------------------------------------------- */
/* Incremental hashing of ONE string delivered in pieces (Sec. 4: with its
 * words arriving in order, the tree of Algorithm 1 needs one open node per
 * level, so a string longer than any buffer, or still being produced, is
 * hashed in bounded memory). The digest of the pieces appended so far equals
 * pmp_hash32 / pmp_hash64 of their concatenation, with the same keys and
 * flags, bit for bit.
 *
 * pmp_incr_create: wide = 0 (PM+32) or 1 (PM+64); d_keys is the device key
 * table (1032 uint32 or uint64), which must stay valid and unchanged for
 * the object's life. Every call on the object is queued on `stream`, in
 * order. Allocates about 1.5 KiB of device state plus a workspace of 80
 * bytes per level-2 node of the largest piece (a node is 64 KiB of PM+32 or
 * 128 KiB of PM+64 input). Returns PMP_E_INVALID_ARG or PMP_E_NOMEM.
 *
 * pmp_incr_append: appends nbytes device bytes at d_piece (any alignment;
 * nbytes = 0 is a no-op). Asynchronous: the piece must stay unchanged until
 * the stream has passed the call. One launch, which also finishes the tree
 * levels of the previous append (an append's levels above 1 run at the start
 * of the next append or digest). A piece larger than any before
 * (beyond what pmp_incr_reserve set aside) first synchronizes the stream and
 * grows the workspace. Returns PMP_E_TOO_LONG if the string would need more
 * than 8 levels (more than 128^8 words after padding), leaving the state as
 * it was.
 *
 * pmp_incr_digest: writes the hash of everything appended so far to d_out
 * (one output in the layout of pmp_hash32 / pmp_hash64 for these flags).
 * More pieces may follow (the digest only runs the last append's pending
 * tree levels, as the next append would). One launch.
 *
 * pmp_incr_reset: starts a new string with the same keys.
 * pmp_incr_length: bytes appended since creation or the last reset.
 * pmp_incr_destroy: synchronizes the stream and frees the object (NULL is a
 * no-op). An object is used by one thread at a time. */
typedef struct pmp_incr pmp_incr;
int pmp_incr_create(int wide, const void* d_keys, pmp_stream_t stream, pmp_incr** out);
int pmp_incr_reserve(pmp_incr* h, uint64_t max_piece_bytes);
int pmp_incr_append(pmp_incr* h, const uint8_t* d_piece, uint64_t nbytes);
int pmp_incr_digest(pmp_incr* h, void* d_out, uint32_t flags);
int pmp_incr_reset(pmp_incr* h);
int pmp_incr_length(const pmp_incr* h, uint64_t* len);
int pmp_incr_destroy(pmp_incr* h);

/* ---------------------------------------------------------------------- */
/* Plain GPU form, kept as a baseline: one string at a time, one launch per
 * tree level, one thread per block of 128 words. h_offsets is a HOST copy of
 * the offsets (the baseline needs the lengths on the host to size its
 * launches); everything else as in pmp_hash32/64. Results are identical to
 * pmp_hash32/64. The call queues 1 + (levels - 1) launches per string and
 * returns; d_scratch must hold 16 * ceil((max string bytes / W + 1) / 128)
 * bytes (W = 4 or 8). */
int pmp_hash_plain(int wide, const uint8_t* d_buf, uint64_t buf_bytes, const int64_t* h_offsets,
                   int64_t count, const void* d_keys, void* d_out, uint32_t flags, void* d_scratch,
                   uint64_t scratch_bytes, pmp_stream_t stream);

/* ---------------------------------------------------------------------- */
/* Field reduction hook for tests (Sec. 6.2 fold and the corrected
 * Algorithm 2): for each i, reduce S = w0[i] + 2^n w1[i] + 2^(2n) w2[i]
 * (n = 32 or 64; w2[i] <= 128 as for any block sum) to z = S mod p in
 * [0, p), on the device. PM+32: device arrays of uint32 w0, w1, w2 and
 * uint64 z. PM+64: uint64 w0, w1, uint32 w2, and z as uint64 pairs
 * (lo, hi). Returns PMP_E_INVALID_ARG if some w2[i] > 128 would be
 * needed (checked on the device: such entries yield z = all ones). */
int pmp_debug_fold(int wide, const void* d_w0, const void* d_w1, const uint32_t* d_w2, void* d_z, int64_t n,
                   pmp_stream_t stream);

/* Measurement hook (not on the path): the rate of v_mad_u64_u32, the
 * 32x32->64 multiply-add that the level-1 sums of Eq. (1) are built from
 * (Sec. 6: one per PM+32 word, four per PM+64 word), on the current device,
 * in lane operations per second: 8 waves per CU's worth of 256-thread blocks
 * run independent chains. This is the multiply roofline the kernels are
 * compared with. Allocates and frees a small buffer and a stream;
 * synchronous (about a millisecond). */
int pmp_probe_mad_rate(double* mads_per_s);

/* Measurement hook (not on the path): the read bandwidth of a plain
 * streaming kernel (workgroups take 32 KiB chunks in turn, 16-byte loads,
 * eight in flight per thread) over `bytes` of device memory at d_buf
 * (at least 1 MiB, 16-byte aligned), in bytes per second: the achievable
 * HBM read rate the kernels are compared with beside the published peak.
 * Allocates and frees a small buffer and a stream; synchronous. */
int pmp_probe_read_bw(const void* d_buf, uint64_t bytes, double* bytes_per_s);

/* Message for the last error on this thread (never NULL). */
const char* pmp_last_error(void);
/* Library version string. */
const char* pmp_version(void);

#ifdef __cplusplus
}
#endif
#endif /* PMP_H_ */
