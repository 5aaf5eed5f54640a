/*
 * xdrop.h -- C ABI of libxdrop: batched X-drop seed extension of read pairs on
 * one AMD Instinct MI355X (gfx950).
 *
 * What is computed (LOGAN, arXiv 2002.05200):
 *   - Each pair (A, B) carries an exact k-mer seed A[a_seed, a_seed+k) ~
 *     B[b_seed, b_seed+k) and is split at it into a right extension of the
 *     suffixes and a left extension of the reversed prefixes (Section IV-B).
 *   - Each extension is the semi-global X-drop alignment of Section III-A:
 *     anti-diagonal dynamic programming of the linear-gap recurrence from the
 *     origin, a running best score, cells scoring below best - X set to -inf,
 *     the -inf runs at both ends of each anti-diagonal trimmed, and the loop
 *     ending when an anti-diagonal has no surviving cell (Algorithms 1 and 2).
 *   - Readings where the paper is silent: best is updated once per
 *     anti-diagonal and pruning compares strictly (< best - X) against best as
 *     of the previous anti-diagonal; the next anti-diagonal spans
 *     [first live, last live + 1] clipped to the matrix; the reported end is
 *     the first anti-diagonal reaching the final best, smallest A index on it;
 *     both directions start from best = 0; "cells" counts every computed cell.
 *   - The pair score is left best + seed score + right best.
 *
 * Conventions:
 *   - All integers little-endian.  All buffers are owned by the caller; the
 *     library owns only its context's internal scratch.
 *   - Sequences are 2-bit packed, A=0 C=1 G=2 T=3, 16 bases per uint32, base
 *     g of an arena in bits [2*(g%16), 2*(g%16)+1] of word g/16 (see xd_pack).
 *   - No C++ exception crosses this boundary.  Call-level problems return an
 *     xd_status; problems with one pair set that pair's xd_result.status and
 *     leave the other pairs unaffected.
 *   - xd_last_error() returns a thread-local description of the last failure.
 */
#ifndef XDROP_H
#define XDROP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    XD_OK = 0,
    XD_EINVAL = 1,     /* bad argument (null pointer, bad score set, bad pair)       */
    XD_ENOMEM = 2,     /* device or host allocation failed                           */
    XD_EDEVICE = 3,    /* a HIP runtime call failed                                  */
    XD_EBUSY = 4,      /* serving: no admission capacity right now                   */
    XD_EOVERFLOW = 5,  /* pair: int32 score range could be exceeded (see xdrop_extend) */
    XD_ECANCELED = 6,  /* serving: request canceled                                  */
    XD_ENOTREADY = 7,  /* serving: result not complete yet                           */
    XD_ETIMEDOUT = 8   /* serving: the request's batch outran the server's watchdog   */
} xd_status;

/* Linear-gap scoring (Section III-A), signed and additive: a match adds
 * `match`, a mismatch adds `mismatch`, a gap adds `gap`.  Supported:
 * match >= mismatch, gap <= 0, mismatch - 2*gap in [-128, 127] and
 * match - mismatch <= 255; xdrop_extend returns XD_EINVAL otherwise. */
typedef struct {
    int32_t match, mismatch, gap;
} xd_scores;

/* One seeded pair.  a_off / b_off are base offsets of the reads in the packed
 * arenas; seeds are read-local.  x is the X-drop threshold, 0 <= x <= 2^29. */
typedef struct {
    uint64_t a_off, b_off;
    uint32_t a_len, b_len;
    uint32_t a_seed, b_seed;
    uint32_t k;
    int32_t x;
} xd_pair; /* 40 bytes */

/* Result of one pair.  Coordinates are read-local and half-open: the
 * alignment spans A[a_begin, a_end) and B[b_begin, b_end). */
typedef struct {
    int32_t score, left_score, right_score, seed_score;
    uint32_t a_begin, a_end, b_begin, b_end;
    uint64_t left_cells, right_cells; /* computed cells of each extension */
    int32_t status;                   /* xd_status of this pair            */
    int32_t reserved;
} xd_result; /* 56 bytes */

/* Batch execution strategy (Section IV-B inter-sequence parallelism). */
typedef enum {
    XD_SCHED_AUTO = 0,       /* persistent queue, longest estimated job first */
    XD_SCHED_PLAIN = 1,      /* one wavefront per job, grid = number of jobs  */
    XD_SCHED_PERSISTENT = 2  /* persistent waves popping a device job queue   */
} xd_sched;

typedef struct {
    int32_t sched;        /* xd_sched                                           */
    int32_t min_tier;     /* 0 = automatic; else start every job at this lane
                             width tier (cells per lane 2, 4, 8, 16, 32 for
                             1..5; 6 = straight to the global-memory tier)      */
    int32_t waves_per_cu; /* persistent grid: waves per compute unit (0 = auto) */
    int32_t sort_jobs;    /* persistent: 1 = longest estimated job first        */
    int32_t long_job;     /* 0 = off; else jobs with m + n >= long_job start
                             long_tier_bias tiers wider than X suggests         */
    int32_t long_tier_bias; /* 0..5, see long_job                              */
    int32_t profile;      /* 1 = time every stage with HIP events (see
                             xd_last_stats); not combined with graph            */
    int32_t impl;         /* 0 = hand-scheduled loops where available, 1 = the
                             portable C loops only (same results; for testing)  */
    int32_t graph;        /* 1 = capture the launch sequence in a hipGraph on
                             the first call and replay it while every argument
                             stays the same; needs a non-NULL stream            */
    int32_t multi_wave;   /* 1 / 2 = the tiers of 8, 16 and 32 cells per lane
                             run four / two wavefronts per job (shorter
                             anti-diagonal steps for very long jobs);
                             0 = one wavefront; others: XD_EINVAL             */
    int32_t max_save_slots; /* 0 = automatic; N > 0 = at most N escalation
                             saves per call.  A job whose band outgrows its
                             window stores its state in a save slot and the
                             next tier resumes from it; once the slots run
                             out, further escalating jobs start over in the
                             wider tier (same results, more work: see
                             xd_stats.restarted).  For tests and for callers
                             that cap memory                                   */
    int32_t reserved;     /* must be 0                                          */
} xd_opts; /* 48 bytes */

/* Statistics of the last xdrop_extend on a context.  Tier t in 0..5 runs C =
 * 2^t cells per lane (a window of 64*C diagonals); tier 6 keeps the band in
 * global memory. */
typedef struct {
    uint64_t jobs[7];      /* jobs finished at each tier                        */
    uint64_t cells[7];     /* cells computed by the jobs finished at each tier  */
    uint64_t escalated[7]; /* jobs whose band outgrew the tier's window          */
    uint64_t restarted[7]; /* of those, jobs that found no free save slot (or
                              outgrew the widest save) and start over in the
                              next tier                                        */
    uint64_t wasted_cells[7]; /* cells the restarted jobs had computed here   */
    float stage_ms[9];     /* plan, tiers 0..5, tier 6, combine (profile only)  */
    int32_t profiled;      /* 1 when stage_ms is valid                          */
} xd_stats;

typedef struct xd_ctx xd_ctx;

/* Host-side 2-bit packer.  Packs n ASCII bases (ACGT, upper or lower case)
 * into words[0 .. (n+15)/16); unused high bits of the last word are zero.
 * Returns XD_EINVAL (and packs nothing) if any character is not ACGT. */
xd_status xd_pack(const char *ascii, size_t n, uint32_t *words);

/* Same, from base codes 0..3 (one byte each) written at base offset
 * base_off of an arena already holding whole words (read-modify-write of the
 * words it touches).  Rejects codes > 3. */
xd_status xd_pack_codes(const uint8_t *codes, size_t n, uint32_t *words,
                        uint64_t base_off);

/* Context on HIP device `device`: kernels, internal scratch (job lists, tier
 * queues, global-memory band buffers, escalation saves) grown on demand.
 * mem_budget caps all of it (0 = no cap): under a budget the global-memory
 * band holds fewer cells per anti-diagonal (at least 16,388; wider bands give
 * XD_ENOMEM per pair) and fewer escalation saves are kept (jobs then start
 * over in the wider tier), and a call whose job scratch alone does not fit
 * returns XD_ENOMEM. */
xd_status xd_ctx_create(int device, size_t mem_budget, xd_ctx **out);
void xd_ctx_destroy(xd_ctx *ctx);

/* Device bytes the context holds now (scratch, band buffers, saves). */
xd_status xd_ctx_memory(const xd_ctx *ctx, uint64_t *bytes);

/*
 * Batched X-drop extension of n_pairs pairs, enqueued on `stream` (a
 * hipStream_t; NULL = the default stream).  Asynchronous: d_out is valid after
 * the stream is synchronised.
 *   d_a, d_b      device arenas of a_words / b_words packed words;
 *   d_pairs       device array of n_pairs xd_pair;
 *   d_out         device array of n_pairs xd_result;
 *   opts          NULL = automatic.
 * Per pair: XD_EINVAL if a seed runs past its read, k > read length, x
 * outside [0, 2^29] or a read runs past its arena; XD_EOVERFLOW if
 * (a_len + b_len) * (|match| + |mismatch| + 2|gap|) + x >= 2^29.
 * Returns XD_EINVAL for null pointers or an unsupported score set, XD_ENOMEM
 * when scratch cannot be allocated, XD_EDEVICE when a launch fails.
 */
xd_status xdrop_extend(xd_ctx *ctx, const uint32_t *d_a, uint64_t a_words,
                       const uint32_t *d_b, uint64_t b_words,
                       const xd_pair *d_pairs, size_t n_pairs, xd_scores scores,
                       xd_result *d_out, void *stream, const xd_opts *opts);

/*
 * The same batched extension with the diagonal step scored by a 4 x 4
 * substitution table instead of match/mismatch (Section III-A's recurrence
 * with the scoring generalised, as Section VIII proposes): aligning base p of
 * A with base q of B (codes A=0 C=1 G=2 T=3) adds matrix[4*p + q]; gaps add
 * `gap`.  matrix is a host array of 16 entries in [-2^20, 2^20], row-major by
 * the base of A; gap in [-2^20, 0].  seed_score sums the table over the seed.
 * Everything else -- pairs, results, seed split, readings, asynchrony,
 * per-pair errors -- is as in xdrop_extend; the int32 guard uses the table's
 * largest magnitude for both the match and the mismatch term.  Options: only
 * sched, waves_per_cu and sort_jobs apply (graph, profile, multi_wave,
 * min_tier and long_job give XD_EINVAL).  Bands up to 62 cells run one
 * wavefront per job in registers; wider ones start over in the
 * global-memory tier.
 */
xd_status xdrop_extend_matrix(xd_ctx *ctx, const uint32_t *d_a, uint64_t a_words,
                              const uint32_t *d_b, uint64_t b_words,
                              const xd_pair *d_pairs, size_t n_pairs,
                              const int32_t *matrix, int32_t gap,
                              xd_result *d_out, void *stream, const xd_opts *opts);

/* Seed of one read pair (xd_find_seeds). */
typedef struct {
    uint32_t a_seed, b_seed;  /* the chosen match: A[a_seed, +k) == B[b_seed, +k)
                                 (0, 0 when found == 0)                        */
    int32_t found;            /* 1 when the reads share at least one k-mer       */
    int32_t status;           /* XD_OK, or XD_EINVAL for a read past its arena   */
    uint64_t bin_matches;     /* exact k-mer matches in the winning bin          */
    uint64_t matches;         /* all exact k-mer matches of the pair             */
} xd_seed; /* 32 bytes */

/*
 * Seed choice for n_pairs read pairs, enqueued on `stream`: the k-mer each
 * extension starts from, picked by binning (the application of Section V,
 * where the positions of the k-mers two reads share are binned to estimate
 * their overlap and the consensus bin gives the seed).  Reading taken, as the
 * paper gives no formula: every exact match (p, q), A[p, p+k) == B[q, q+k),
 * lies on diagonal q - p and falls in bin floor((q - p) / width); the bin with
 * the most matches wins (the lower bin on a tie), and its match with the
 * smallest p, then the smallest q, is the seed.
 *   d_a, d_b    device arenas (2-bit packed, as for xdrop_extend);
 *   d_pairs     device xd_pair records: a_off, b_off, a_len, b_len are read;
 *               with set_pairs = 1, a_seed, b_seed and k of every pair with a
 *               seed are overwritten (pairs without one are left as they
 *               are), so the records can go straight to xdrop_extend;
 *   k           seed length, 1..31; width: bin width in diagonals, >= 1;
 *   d_seeds     device array of n_pairs xd_seed (caller-owned).
 * Reads shorter than k have no seed.  Returns XD_EINVAL for null pointers or
 * k / width / set_pairs out of range, XD_EDEVICE when the launch fails.  Uses
 * no context scratch: the hash table and bins of each pair live in LDS.
 */
xd_status xd_find_seeds(xd_ctx *ctx, const uint32_t *d_a, uint64_t a_words,
                        const uint32_t *d_b, uint64_t b_words, xd_pair *d_pairs,
                        size_t n_pairs, uint32_t k, uint32_t width, int32_t set_pairs,
                        xd_seed *d_seeds, void *stream);

/* Synchronous convenience: host arenas, pairs and results; copies in, runs
 * xdrop_extend on an internal stream, copies out. */
xd_status xdrop_extend_host(xd_ctx *ctx, const uint32_t *a, uint64_t a_words,
                            const uint32_t *b, uint64_t b_words,
                            const xd_pair *pairs, size_t n_pairs, xd_scores scores,
                            xd_result *out, const xd_opts *opts);

/*
 * xdrop_extend without a context and without any device allocation, for
 * callers that cannot allocate: code under hipGraph stream capture, tight
 * serving loops, harnesses that forbid hipMalloc.
 *   - Runs on HIP device `device`, which is made current for the call and
 *     restored afterwards; arguments, results and asynchrony are those of
 *     xdrop_extend.
 *   - Scratch is one fixed array in the library's device memory, of
 *     XD_NOALLOC_SCRATCH_BYTES on every GPU the library runs on, held until the
 *     process ends: job lists for at most XD_NOALLOC_MAX_PAIRS pairs,
 *     XD_NOALLOC_SAVE_SLOTS escalation saves (later escalations start over in
 *     the wider tier, as xd_opts.max_save_slots describes) and global-memory
 *     band buffers of XD_NOALLOC_BAND_CELLS cells per anti-diagonal (a job
 *     whose band is wider fails with XD_ENOMEM in its pair status).
 *   - Every call on one GPU uses that GPU's one array, which keeps the last
 *     call's contents (each call clears what must start at zero with a
 *     kernel).  Calls that overlap on one GPU -- on different streams, or from
 *     different threads -- race on it; serialise them.
 *   - Returns XD_EINVAL for n_pairs > XD_NOALLOC_MAX_PAIRS, for graph or
 *     profile options, and for everything xdrop_extend rejects; calls no
 *     hipMalloc, hipFree or other allocating routine.
 */
#define XD_NOALLOC_MAX_PAIRS 8192
#define XD_NOALLOC_SAVE_SLOTS 512
#define XD_NOALLOC_BAND_CELLS 16388
#define XD_NOALLOC_SCRATCH_BYTES (13u << 20)
xd_status xdrop_extend_noalloc(int device, const uint32_t *d_a, uint64_t a_words,
                               const uint32_t *d_b, uint64_t b_words,
                               const xd_pair *d_pairs, size_t n_pairs, xd_scores scores,
                               xd_result *d_out, void *stream, const xd_opts *opts);

/* Statistics of the last xdrop_extend on this context (synchronises the
 * context's device first). */
xd_status xd_last_stats(xd_ctx *ctx, xd_stats *out);

/* ---------------------------------------------------------------------------
 * Serving: a request loop with continuous batching.
 *
 * Requests (1 .. max_batch_pairs pairs with their own packed reads) are
 * submitted from any host thread and queue in arrival order.  A scheduler
 * thread owned by the server forms a batch as soon as one of its `slots` is
 * free: it admits the oldest queued request, then later requests with the
 * same scores (and, with group_by_class, the same cost class: the tier X
 * selects and the octave of the longest pair) while the batch's packed reads
 * and pair records fit in the slot's device memory.  It copies them to the
 * device, where they stay until the batch is done, and launches xdrop_extend
 * on the slot's own stream.  Requests that arrive while other batches run are
 * admitted into the next free slot, so their kernels overlap with the
 * batches already on the device.  Results are the same whether a request
 * runs alone or in a mix (every pair is an independent extension).
 *
 * Memory: every slot holds an equal share of mem_budget, and everything the
 * slot allocates on the device stays inside it: its extension context
 * (created under half the share and sized for a full batch up front: job
 * lists, global-memory band buffers, escalation saves), the pair records and
 * results of one batch, and two read arenas of what remains.
 * ------------------------------------------------------------------------- */
typedef struct xd_server xd_server;

typedef struct {
    int32_t device;
    int32_t slots;            /* batches in flight at once, 1..16 (0 = 4); each
                                 slot has its own stream, and HIP runs the
                                 streams of a process on GPU_MAX_HW_QUEUES
                                 hardware queues (4 unless the environment sets
                                 it before the runtime starts): slots beyond that
                                 share queues and their kernels serialise       */
    int32_t max_batch_pairs;  /* pairs per batch (0 = 2048)                         */
    int32_t graph;            /* 1 = every slot replays a captured hipGraph of
                                 xdrop_extend (batches padded to max_batch_pairs)  */
    uint64_t mem_budget;      /* device bytes for all slots (0 = 1 GiB); each
                                 slot holds an equal share                          */
    xd_opts extend_opts;      /* launch options of every batch (graph and
                                 profile are set by the server)                     */
    int32_t group_by_class;   /* 1 = a batch takes only requests of the oldest
                                 request's cost class; 0 = any, in arrival order    */
    int32_t watchdog_ms;      /* 0 = off; else a batch still running this many
                                 milliseconds after its launch fails its requests
                                 with XD_ETIMEDOUT at once (their polls return);
                                 its kernels still run to the end, and the slot
                                 takes new work only after they have             */
} xd_server_opts; /* 80 bytes */

/* One request: host buffers, read by xd_server_submit before it returns. */
typedef struct {
    const uint32_t *a;        /* packed reads A of this request (a_words words)    */
    uint64_t a_words;
    const uint32_t *b;        /* packed reads B (b_words words)                    */
    uint64_t b_words;
    const xd_pair *pairs;     /* n_pairs pairs; offsets into this request's reads  */
    uint32_t n_pairs;
    xd_scores scores;         /* batches only mix requests with equal scores        */
} xd_request; /* 56 bytes */

/* Creates a server and its scheduler thread.  XD_EINVAL for bad options,
 * XD_ENOMEM if the device memory of the slots cannot be allocated. */
xd_status xd_server_create(const xd_server_opts *opts, xd_server **out);

/* Queues a request (its data are copied) and returns its ticket.
 * XD_EINVAL if the request is empty, larger than one slot can hold, or its
 * scores are unsupported; pair-level problems are reported per pair. */
xd_status xd_server_submit(xd_server *srv, const xd_request *req, uint64_t *ticket);

/* Waits up to wait_ms (0 = do not wait, -1 = forever) for a ticket.  When it
 * is done, copies its n_pairs results to out, stores the host steady-clock
 * time (nanoseconds, CLOCK_MONOTONIC) at which the scheduler saw the batch
 * complete in done_ns (if not NULL), releases the ticket and returns XD_OK.
 * XD_ENOTREADY if not done in time; XD_EINVAL for an unknown ticket;
 * XD_EDEVICE if its batch failed; XD_ETIMEDOUT if its batch outran the
 * watchdog; XD_ECANCELED if it was canceled. */
xd_status xd_server_poll(xd_server *srv, uint64_t ticket, xd_result *out, int32_t wait_ms,
                         uint64_t *done_ns);

typedef struct {
    uint64_t requests, pairs, batches; /* completed                               */
    uint64_t cells;                    /* cells of completed requests             */
    uint64_t queued;                   /* requests waiting for admission now      */
    uint64_t max_inflight;             /* most batches on the device at once      */
    uint64_t canceled;                 /* requests canceled before admission      */
    uint64_t device_bytes;             /* device memory the slots hold (at most
                                          mem_budget)                             */
    uint64_t arena_words;              /* packed words of each read arena of a
                                          slot: the reads one batch can hold      */
    uint64_t waiting_polls;            /* xd_server_poll calls waiting inside the
                                          server now                              */
    uint64_t timed_out;                /* requests failed by the watchdog         */
} xd_server_stats;

xd_status xd_server_get_stats(xd_server *srv, xd_server_stats *out);

/* Cancels a request that is still waiting for admission: it leaves the queue
 * and its poll returns XD_ECANCELED.  XD_EBUSY if it is already on the device
 * or done (its poll then returns its results as usual); XD_EINVAL for an
 * unknown ticket. */
xd_status xd_server_cancel(xd_server *srv, uint64_t ticket);

/* Stops the scheduler after the batches on the device finish.  Requests not
 * yet admitted are canceled (their polls return XD_ECANCELED); polls waiting
 * inside the server are woken and return before the server is freed.  No
 * call on the server may start once destroy has begun.  Safe on NULL. */
void xd_server_destroy(xd_server *srv);

const char *xd_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
