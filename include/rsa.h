/*
 * rsa.h -- C ABI of the MI355X (gfx950) library for random sequential
 * adsorption (RSA) of linear k-mers on an L x L torus, run to jamming with
 * first-wrap (percolation) tracking.
 *
 * Paper: Slutskii, Barash, Tarasevich, "Percolation and jamming of random
 * sequential adsorption samples of large linear k-mers on a square lattice",
 * arXiv:1810.06800.
 *
 * Problem statement (Sec. II.A): k-mers -- straight needles covering k
 * consecutive sites of one row (horizontal, H) or one column (vertical, V) --
 * are deposited on an L x L square lattice with periodic boundaries (a
 * torus) by isotropic RSA until jamming, i.e. until no k-mer fits.  Sec. II.B
 * draws each new k-mer among the placements where it still fits; Sec. II.C
 * labels clusters by union-find; Sec. II.D detects the first cluster that
 * wraps round the torus.  Each sample is one independent run (Sec. II.A).
 * The caller derives the concentrations p_c = n_wrap_any*k/L^2 (first wrap,
 * in one or both directions, Sec. II.D) and p_j = n_jam*k/L^2 (jamming).
 *
 * Canonical sampling (the paper's RNG cannot be reproduced, so it is fixed
 * here and every result is a deterministic function of the descriptor):
 *   placement p = (o, y, x), o = 0 (H: sites (y, x+i)) or 1 (V: (y+i, x)),
 *   i = 0..k-1 mod L; canonical index P = o*L*L + y*L + x;
 *   step t: (r0..r3) = Philox4x32-10(key = (seed mod 2^32, seed >> 32),
 *   counter = (t, sample, 0, 0)); u = r0 + 2^32*r1;
 *   rank = floor(u * A_t / 2^64) among the A_t available placements in
 *   canonical order.
 *
 * Threading: a context may be used from one host thread at a time.  All
 * functions return negative rsa_status codes on failure; no C++ exception
 * crosses this boundary.
 */
#ifndef RSA_H
#define RSA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define RSA_ABI_VERSION 1

/* Status codes (0 or negative). */
enum rsa_status {
    RSA_OK = 0,
    RSA_EINVAL = -1,    /* bad argument; nothing was enqueued               */
    RSA_ENOMEM = -2,    /* device memory budget or allocation exhausted     */
    RSA_EDEVICE = -3,   /* a HIP call failed; the context is poisoned       */
    RSA_ENOTREADY = -4, /* rsa_results(wait = 0) before the batch finished  */
    RSA_EBUSY = -5,     /* resource in use                                  */
    RSA_ENOTFOUND = -6  /* unknown or already collected batch id            */
};

/* Per-sample flags. */
enum rsa_flags {
    /* Vertical placements start unavailable: L independent rings of length L
     * (one-dimensional RSA).  Test mode. */
    RSA_FLAG_H_ONLY = 1u << 0,
    /* Also report the number of clusters and of non-wrapping clusters at
     * jamming (Appendix A: the latter is always 0).  Keeps cluster labelling
     * running to jamming instead of stopping once both wrap steps are known. */
    RSA_FLAG_TRACK_CLUSTERS = 1u << 1,
    /* Also report the contact census of the jammed state (Eq. 12): pairs of
     * nearest-neighbour sites in different k-mers, both horizontal, both
     * vertical or perpendicular.  Keeps the site map written to jamming and
     * adds one pass over it. */
    RSA_FLAG_CONTACTS = 1u << 2,
    /* rsa_run_batch only: also histogram the cluster sizes right after
     * deposit n_wrap_any, the percolation threshold (Eq. 11: n_s at p_c);
     * read them with rsa_batch_cluster_sizes.  The sample is run a second
     * time, inside the same batch, up to that deposit. */
    RSA_FLAG_CLUSTER_SIZES = 1u << 3
};

/* Bins of a cluster-size histogram: bin b counts the clusters whose size in
 * sites s satisfies 2^b <= s < 2^(b+1). */
#define RSA_SIZE_BINS 32

/* Opaque context.  Owns every device allocation made on its behalf. */
typedef struct rsa_ctx rsa_ctx;

/* One independent run (Sec. II.A).  1 <= k <= L <= 32768; flags from
 * rsa_flags.  (seed, sample) select the Philox stream described above. */
typedef struct {
    uint32_t L, k;
    uint64_t seed;
    uint32_t sample, flags;
} rsa_sample_t;

/* Result of one run (104 bytes).  Counts are 1-based deposit numbers; -1 means
 * "never" (possible for one direction on small tori).
 *   n_jam        k-mers on the lattice at jamming
 *   n_wrap_x/_y  deposit after which some cluster first wraps in x / in y
 *                (a closed path whose unwrapped displacement has a non-zero
 *                x / y component)
 *   n_wrap_any   the smaller of the defined wrap counts (the paper's p_c)
 *   occ_hash     sum over occupied sites s of mix64((s << 32) | id(s)) mod
 *                2^64, id(s) = deposit number of the k-mer covering s and
 *                mix64 the SplitMix64 finalizer (Steele, Lea, Flood 2014)
 *   seq_hash     sum over steps t of mix64((t << 32) | P_t) mod 2^64
 *   n_clusters_jam, n_nonwrapping_jam   cluster census at jamming, -1 unless
 *                RSA_FLAG_TRACK_CLUSTERS
 *   status       0, or a negative rsa_status for this sample
 *   tile         schedule the batch planner chose for this sample
 *   alg_bytes    algorithmic-byte model of the run: 4 B/site map
 *                initialisation and both availability bitmaps; per deposit
 *                4k (map) + 4(2k+2) (contacts) + 8*ceil(L/64) (select row)
 *                + 16 (k-mer record); 16 B per availability word changed
 *   wchg_words   availability words whose value changed, summed over steps
 *   n_contacts_x, n_contacts_y, n_contacts_xy   contact census at jamming,
 *                -1 unless RSA_FLAG_CONTACTS: over every site and its right
 *                and lower neighbour (mod L), pairs of occupied sites in
 *                different k-mers that are both horizontal / both vertical /
 *                of different orientations; n*_xy = n_xy / (n_x + n_y + n_xy)
 */
typedef struct {
    int64_t n_jam, n_wrap_x, n_wrap_y, n_wrap_any;
    uint64_t occ_hash, seq_hash;
    int32_t n_clusters_jam, n_nonwrapping_jam;
    int32_t status, tile;
    uint64_t alg_bytes, wchg_words;
    int64_t n_contacts_x, n_contacts_y, n_contacts_xy;
} rsa_result_t;

/* Optional device allocator.  alloc returns device memory of at least
 * `bytes` (256-byte aligned) or NULL; free releases it.  Both are called on
 * the thread that calls into the library, never from a device callback. */
typedef struct {
    void *(*alloc)(size_t bytes, void *user);
    void (*free)(void *ptr, size_t bytes, void *user);
    void *user;
} rsa_allocator_t;

/* Create a context on HIP device `device`.
 *   hbm_budget_bytes  upper bound on device memory the context may hold at
 *                     once (0 = 90 % of the device's memory)
 *   alloc             NULL = hipMalloc/hipFree; otherwise used for every
 *                     device allocation (the pointer is copied)
 * Writes the new context to *out.  RSA_EINVAL for a NULL out or a bad device,
 * RSA_EDEVICE if HIP fails. */
int rsa_create(rsa_ctx **out, int device, uint64_t hbm_budget_bytes,
               const rsa_allocator_t *alloc);

/* Device bytes one resident sample of shape (L, k) needs: two availability
 * bitmaps of L*ceil(L/64) words, the int32 site map, k-mer records for up to
 * L*L/k + 1 deposits, and 256-byte alignment.  0 for an invalid shape. */
size_t rsa_footprint_bytes(uint32_t L, uint32_t k);

/* Enqueue n independent samples on `hip_stream` (a hipStream_t; NULL = the
 * null stream) and return at once.  The descriptors are copied before the
 * call returns; the caller keeps ownership of `s`.  Results of one batch do
 * not depend on its composition, its order or the schedule chosen.
 * *batch_id receives a handle for rsa_results.
 * n == 0 is an empty batch.  RSA_EINVAL (nothing enqueued) for s == NULL with
 * n > 0, any invalid descriptor, a flag outside rsa_flags, or a lattice whose
 * row counts do not fit the workgroup's LDS; RSA_ENOMEM if the batch does not
 * fit the budget; RSA_EDEVICE on a HIP failure. */
int rsa_run_batch(rsa_ctx *ctx, const rsa_sample_t *s, uint32_t n, void *hip_stream,
                  uint64_t *batch_id);

/* ---------------------------------------------------------------------------
 * For callers that cannot allocate: code under HIP graph capture, tight
 * serving loops, harnesses that forbid allocation while they run.
 *
 * rsa_run_batch_static runs the samples of rsa_run_batch with the same
 * kernels and schedules and gives the same results, but allocates nothing:
 * no device, pinned or host-heap memory, no events, no graphs.  Its device
 * state (work-queue counters, kernel-side descriptors, one slab per resident
 * workgroup) lives in a static array of RSA_STATIC_SCRATCH_BYTES per device,
 * held from the library's load to the end of the process.  Descriptors reach
 * the device as kernel arguments.
 *   s          host array of n descriptors, read before the call returns
 *   d_results  DEVICE memory of n rsa_result_t, owned by the caller; written
 *              in descriptor order when the stream reaches the end of the
 *              call's kernels (no host copy; synchronise the stream first)
 *   hip_stream the caller's hipStream_t (NULL = null stream)
 * Samples sharing a kernel run in one persistent launch, launches one after
 * another on the stream.  Every call on a device shares that device's array
 * and leaves its contents behind; the call zeroes what must start at zero.
 * Calls that overlap on one device (other streams, other contexts) race and
 * give undefined results: the caller orders them.  RSA_EINVAL for a NULL
 * argument, an invalid descriptor, RSA_FLAG_CLUSTER_SIZES (a two-pass feature
 * of rsa_run_batch) or n > RSA_STATIC_MAX_SAMPLES; RSA_ENOMEM when one
 * sample's slab does not fit the array (the message names the sizes);
 * RSA_EDEVICE when the array's address could not be obtained at rsa_create
 * or a launch fails.  RSA_OPT_MODE, RSA_OPT_GRAPH and RSA_OPT_PROFILE do not
 * apply; tiles follow the context as in rsa_run_batch. */
#define RSA_STATIC_SCRATCH_BYTES (128u << 20)
#define RSA_STATIC_MAX_SAMPLES 2048
int rsa_run_batch_static(rsa_ctx *ctx, const rsa_sample_t *s, uint32_t n, rsa_result_t *d_results,
                         void *hip_stream);

/* Copy the n results of batch `batch_id` into out[0..n-1] (same order as the
 * descriptors) and release the batch's device memory.  wait = 1 blocks until
 * the batch is done; wait = 0 returns RSA_ENOTREADY if it is still running
 * (the batch stays valid).  RSA_ENOTFOUND for an unknown id, RSA_EINVAL if n
 * differs from the batch size. */
int rsa_results(rsa_ctx *ctx, uint64_t batch_id, rsa_result_t *out, uint32_t n, int wait);

/* Device time of batch `batch_id`'s kernels in milliseconds, from HIP events
 * recorded on its stream right before the first and after the last kernel
 * (descriptor and result copies excluded).  Blocks until the kernels are
 * done; valid until rsa_results collects the batch.  RSA_ENOTFOUND for an
 * unknown id. */
int rsa_batch_elapsed_ms(rsa_ctx *ctx, uint64_t batch_id, float *ms);

/* Diagnostic: per-sample phase counters of a batch run with RSA_OPT_PROFILE.
 * out receives n * (*slots) uint64 values, sample-major, in descriptor order;
 * *slots and *clock_khz (the tick rate) are written even on failure.  Slot
 * order: init, select-chain total / ring wait / select / clear, labelling
 * total / idle / map / gather / resolve / merge / write-back (ticks), then
 * labelling batches, edges, flushes, steps and rows read ahead correctly
 * (counts), then the select wave's read-ahead outside the clear (planning
 * and issuing the window's reads; 0 with the dense clear, which does both
 * inside) and its clear proper (reads, the deposit's hashes while they are
 * in flight, bits cleared, counts updated) (ticks), then, for the interval
 * clear of long k-mers, the select wave's line cuts, its wait for the other
 * selecting waves between the clear's two phases, and its row-count phase
 * (ticks).  Blocks until the kernels are done; valid until rsa_results.
 * RSA_EINVAL if the batch was not profiled or n differs from its size. */
int rsa_batch_profile(rsa_ctx *ctx, uint64_t batch_id, uint64_t *out, uint32_t n,
                      uint32_t *slots, uint32_t *clock_khz);

/* Cluster-size histograms of batch `batch_id` (RSA_FLAG_CLUSTER_SIZES):
 * out[i * RSA_SIZE_BINS + b], i in descriptor order, = the number of clusters
 * of sample i with 2^b <= size in sites < 2^(b+1), over the whole lattice
 * right after deposit n_wrap_any (n_s at the percolation threshold, Eq. 11,
 * is bin / (L*L) after averaging over samples).  Samples without the flag
 * read all zero; a sample whose rerun failed reads all ones.  Blocks until
 * the batch's kernels are done; valid until rsa_results.  RSA_EINVAL if no
 * sample of the batch has the flag or n differs from its size. */
int rsa_batch_cluster_sizes(rsa_ctx *ctx, uint64_t batch_id, uint64_t *out, uint32_t n);

/* Wait for all work of the context, free every allocation and the context.
 * NULL is ignored. */
void rsa_destroy(rsa_ctx *ctx);

/* Static description of a status code. */
const char *rsa_strerror(int code);

/* Message of the context's most recent failure ("" if none).  The string
 * stays valid until the next call on the context. */
const char *rsa_last_error(rsa_ctx *ctx);

/* Context options (rsa_set_option / rsa_get_option):
 *   RSA_OPT_MODE   RSA_MODE_BATCHED (default): one persistent launch per
 *                  batch pulls samples from a device work queue, longest
 *                  first; RSA_MODE_PLAIN: one launch per sample with a fixed
 *                  schedule, round-robin over four streams forked from and
 *                  joined back to the caller's stream (the comparison form)
 *   RSA_OPT_TILE   -1 (default) = schedule from the autotune table (see
 *                  rsa_set_tile_table), else a fixed schedule id in
 *                  [0, rsa_num_tiles())
 *   RSA_OPT_GRAPH  1 (default) = batched launches are captured into a
 *                  hipGraph once per shape signature and replayed; 0 = direct
 *   RSA_OPT_SLOTS  0 (default) = as many resident workgroups as fit, else
 *                  an upper bound on them
 *   RSA_OPT_PROFILE 0 (default); 1 = later batches record per-sample phase
 *                  counters (device wall-clock ticks), read by
 *                  rsa_batch_profile; results are unchanged
 *   RSA_OPT_IV_SLAB 0 (default); 1 = diagnostic: samples on the interval
 *                  clear keep its difference counts in the slab even where
 *                  they fit LDS (the layout large lattices use); results are
 *                  unchanged
 * Unknown options or values: RSA_EINVAL. */
enum rsa_option { RSA_OPT_MODE = 1, RSA_OPT_TILE = 2, RSA_OPT_GRAPH = 3, RSA_OPT_SLOTS = 4,
                  RSA_OPT_PROFILE = 5, RSA_OPT_IV_SLAB = 6 };
enum rsa_mode { RSA_MODE_BATCHED = 0, RSA_MODE_PLAIN = 1 };
int rsa_set_option(rsa_ctx *ctx, int option, int64_t value);
int rsa_get_option(rsa_ctx *ctx, int option, int64_t *value);

/* Schedules ("tiles").  A tile fixes the waves that share one sample's
 * select/clear (one more wave labels clusters), the height of the 128-byte
 * bitmap tiles (1..16 rows of 16..1 words), the height of the 128-byte
 * site-map tiles (1..32 rows of 32..1 sites), and the clear mode (0 dense:
 * every word of the blocked rectangles is read; 1 sparse: per-word summary
 * bits are read first and only words that are still non-zero are touched).
 * Results never depend on the tile.  rsa_num_tiles: how many exist;
 * rsa_tile_for_shape: the built-in heuristic's tile for (L, k) (RSA_EINVAL
 * for an invalid shape); rsa_tile_shape: decode a tile id (RSA_EINVAL if out
 * of range; NULL outputs are skipped). */
int rsa_num_tiles(void);
int rsa_tile_for_shape(uint32_t L, uint32_t k);
int rsa_tile_shape(int tile, int *waves, int *bitmap_tile_rows, int *map_tile_rows, int *sparse);

/* Autotune table of a context: entry i says that samples of shape
 * (L[i], k[i]) run with schedule tile[i] (measured fastest by the project's
 * autotuner; the arrays are copied).  It replaces the previous table; n = 0
 * clears it.  Shapes not in the table use the built-in heuristic, and
 * RSA_OPT_TILE >= 0 overrides both.  RSA_EINVAL (table unchanged) for an
 * invalid shape or tile id.  rsa_tile_for_sample: the tile a sample of
 * (L, k) gets on this context now. */
int rsa_set_tile_table(rsa_ctx *ctx, const uint32_t *L, const uint32_t *k, const int32_t *tile,
                       uint32_t n);
int rsa_tile_for_sample(rsa_ctx *ctx, uint32_t L, uint32_t k);

/* ---------------------------------------------------------------------------
 * Request server: continuous batching of independent runs (Sec. II.A: every
 * sample is one run of the problem above) submitted over time.
 *
 * Each sample of an admitted request gets its own device state (bitmaps, site
 * map, k-mer records: rsa_footprint_bytes) carved from an arena that the
 * server allocates once, and keeps it resident until it jams.  The device
 * runs in launches of one time quantum: every resident sample that a
 * workgroup reaches advances until the quantum is spent, then saves its row
 * counts and chain position next to its lattice and yields; the next launch
 * resumes it exactly there.  Between launches the host retires finished
 * samples (their arena space is reused) and admits queued samples, oldest
 * request first, as arena space and resident slots free up, so new requests
 * join work already on the device (a sample too large for the free space is
 * passed over by up to 256 later ones that fit).  Results are the same, bit for bit, as
 * rsa_run_batch's for the same descriptors, whatever else runs beside them.
 *
 * Two launches are kept in flight on the server's streams (forked from and
 * joined to the caller's stream), so the device never waits for the host's
 * bookkeeping.  A server is used from one host thread at a time, like its
 * context, and the context must outlive it.
 * ------------------------------------------------------------------------- */
typedef struct rsa_server rsa_server;

typedef struct {
    uint64_t arena_bytes;    /* device bytes for resident samples; 0 = half of the
                                context's budget                                  */
    uint32_t quantum_us;     /* device time per launch before samples yield;
                                0 = 2000 us                                       */
    uint32_t max_resident;   /* samples resident at once; 0 = 4096                */
} rsa_server_config_t;

typedef struct {
    uint64_t requests_submitted, requests_completed;
    uint64_t samples_queued;     /* submitted, not yet admitted                       */
    uint64_t samples_resident;   /* admitted, not yet retired                         */
    uint64_t samples_completed;
    uint64_t deposits_completed; /* n_jam summed over completed samples               */
    uint64_t deposits_in_progress; /* deposits made so far by resident samples that
                                      have not finished (as of the last retired launch) */
    uint64_t arena_bytes, arena_used, arena_peak;
    uint64_t launches;
} rsa_server_stats_t;

/* Create a server on `ctx` whose launches are ordered after work already on
 * `hip_stream` (a hipStream_t, NULL = null stream).  cfg NULL = defaults.
 * RSA_ENOMEM if the arena does not fit the context's budget, RSA_EINVAL for a
 * NULL ctx or out, RSA_EDEVICE on a HIP failure. */
int rsa_server_create(rsa_ctx *ctx, const rsa_server_config_t *cfg, void *hip_stream,
                      rsa_server **out);

/* Queue a request of n samples (copied; the caller keeps `samples`) and
 * return its id in *request_id.  Nothing is launched here; rsa_server_step
 * admits and runs.  RSA_EINVAL (nothing queued) for n == 0, an invalid
 * descriptor, RSA_FLAG_CLUSTER_SIZES (a batch feature), or a descriptor whose
 * row counts do not fit a workgroup's LDS; RSA_ENOMEM if one sample alone
 * needs more than the arena. */
int rsa_server_submit(rsa_server *srv, const rsa_sample_t *samples, uint32_t n,
                      uint64_t *request_id);

/* One round of the loop: retire launches that finished (wait = 1: block
 * until at least one has, when any is in flight), admit queued samples that
 * fit, and enqueue launches until two are in flight.  Returns the number of
 * requests that completed during the call (>= 0), or a negative status. */
int rsa_server_step(rsa_server *srv, int wait);

/* Ids of completed requests not yet reported by this call, oldest first: up
 * to `cap` are written to ids; returns how many were written. */
int rsa_server_completed(rsa_server *srv, uint64_t *ids, uint32_t cap);

/* Copy the n results of a completed request (descriptor order) and forget
 * it.  RSA_ENOTREADY if it has not completed (it stays queued or running),
 * RSA_ENOTFOUND for an unknown or already collected id, RSA_EINVAL if n
 * differs from the request's size. */
int rsa_server_results(rsa_server *srv, uint64_t request_id, rsa_result_t *out, uint32_t n);

/* Counters of the server so far. */
int rsa_server_stats(rsa_server *srv, rsa_server_stats_t *out);

/* Wait for the launches in flight, drop queued and resident samples, and
 * free the arena and the server.  NULL is ignored. */
void rsa_server_destroy(rsa_server *srv);

#ifdef __cplusplus
}
#endif
#endif
