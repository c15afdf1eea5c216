/*
 * pscl - CRC-aided list decoding of polar codes on AMD Instinct MI355X
 * (gfx950), after "Fast List Decoders for Polar Codes" (Sarkis, Giard, Vardy,
 * Thibeault, Gross).
 *
 * The decoder runs list decoding on the decoding tree of the code (Sec. II-D,
 * Sec. III): min-sum F (eq. (f)), G (eq. (g)) and Combine (eq. (combine)) on
 * every internal node of every active path; Rate-0, Rate-1 (Chase-II over two
 * least reliable bits), repetition and SPC (Chase-II over four least reliable
 * bits) list decoders at the leaves, each scoring its candidates with the
 * codeword metric of eq. (pm); candidate selection keeping the L best paths
 * (Alg. 1); and the final choice of the most reliable path that satisfies the
 * CRC (Sec. II-B).
 *
 * Conventions (all entry points):
 *  - frozen_mask: host array of N bytes, 1 = frozen (fixed to 0), 0 = carries
 *    a bit.  K = number of zero bytes.
 *  - The K unfrozen positions, in increasing position order, carry the K - r
 *    payload bits followed by the r CRC bits ("CRC inside K").
 *  - CRC: generator x^r + crc_poly (crc_poly in normal form, without the x^r
 *    term), register initialised to 0, bits fed most significant first, no
 *    reflection, no final XOR.  r = crc_len in [0, 64]; 0 = no CRC.
 *  - LLRs: positive favours bit 0 (Sec. II-A, eq. (sc:h)).  F x N row-major
 *    device array of float (PSCL_F32), int16 in [-32767, 32767] (PSCL_I16) or
 *    int8 in [-127, 127] (PSCL_I8).  Integer G results saturate to that range.
 *  - Ties: equal candidate metrics are ordered by enumeration index (source
 *    path slot, then candidate rank); the final pick prefers the lower slot.
 *
 * Ownership: the caller owns every device buffer passed in; a plan owns its
 * device schedule, tables and workspace.  Decoding is asynchronous on the
 * caller's HIP stream.  A plan's workspace is allocated by pscl_decode
 * for the workgroups a call needs (F frames use at most F) and enlarged when
 * a later call needs more (to the next power of two workgroups, at most the
 * full grid); pscl_plan_reserve allocates the full grid's, after which no
 * call allocates.  A plan's workspace serves one call at a time: calls on one plan must be
 * ordered (one stream, or synchronised); a group (below) keeps a workspace
 * per call in flight, so its calls may overlap on different streams, and so
 * may calls of the one-call form.  All device pointers must be accessible
 * from the device that was current when the plan was created.
 *
 * Integer inputs: the int8 / int16 domains are [-127, 127] / [-32767,
 * 32767]; an input of -128 / -32768 is read as -127 / -32767 (saturated on
 * load, as every G result is).
 *
 * Errors: every function returns a status code and never throws.  A HIP
 * failure reported by the runtime (including asynchronous faults of earlier
 * work) is returned as PSCL_E_HIP.  "No path satisfies the CRC" is not an
 * error: crc_ok = 0 and the most reliable path is returned.
 */
#ifndef PSCL_H
#define PSCL_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    PSCL_OK = 0,
    PSCL_E_INVALID = 1,     /* invalid argument */
    PSCL_E_UNSUPPORTED = 2, /* valid, but no kernel for this combination */
    PSCL_E_NOMEM = 3,       /* device allocation failed */
    PSCL_E_HIP = 4,         /* HIP runtime error */
    PSCL_E_NODEV = 5,       /* no usable gfx950 device */
    PSCL_E_BUSY = 6,        /* a server holds as many requests as it admits */
    PSCL_E_TIMEOUT = 7      /* a wait with a time limit ended before completion */
} pscl_status;

typedef enum { PSCL_F32 = 0, PSCL_I16 = 1, PSCL_I8 = 2 } pscl_dtype;

/* Decoding-tree modes (Table 1): PSCL_MODE_TREE uses the Rate-0, Rate-1,
 * repetition and SPC list decoders ("unrolled Dec-SPC-4" with spc_max = 4);
 * PSCL_MODE_SCL_LEAVES splits every node down to single bits ("unrolled
 * SC-list"). */
typedef enum { PSCL_MODE_TREE = 0, PSCL_MODE_SCL_LEAVES = 1 } pscl_mode;

/* Schedule operations, as reported by pscl_schedule. */
typedef enum {
    PSCL_OP_F = 0,    /* alpha_l = F(alpha_v), eq. (f) */
    PSCL_OP_G = 1,    /* alpha_r = G(alpha_v, beta_l), eq. (g) */
    PSCL_OP_COMB = 2, /* beta_v = Combine(beta_l, beta_r), eq. (combine) */
    PSCL_OP_R0 = 3,   /* Rate-0 list decoder, Sec. III-B */
    PSCL_OP_REP = 4,  /* repetition list decoder, Sec. III-E */
    PSCL_OP_R1 = 5,   /* Rate-1 list decoder, Sec. III-C */
    PSCL_OP_SPC = 6   /* SPC list decoder, Sec. III-D */
} pscl_op_type;

typedef struct pscl_plan pscl_plan;

/* Human-readable name of a status code (static string). */
const char* pscl_status_str(pscl_status s);

/* Library version, major * 10000 + minor * 100 + patch. */
int pscl_version(void);

/*
 * Host-only schedule compiler (Sec. II-D: tree optimisation; Listing 2: the
 * unrolled operation sequence).  Classifies every node of the decoding tree
 * of (N, frozen_mask) and emits the operations in decoding order.  Needs no
 * GPU.
 *   ops: host array of capacity cap entries, 4 int32 each:
 *        {pscl_op_type, log2(node size), side (0 = left child, 1 = right child
 *        or root), active paths after the operation}.
 *   *n_ops: number of operations (written even when cap is too small, in
 *   which case PSCL_E_INVALID is returned).
 * spc_max: largest SPC node (4 = Dec-SPC-4; up to N allowed; values below 4
 * disable SPC nodes).  L: list size in {1, 2, 4, ..., 128}.
 */
pscl_status pscl_schedule(int N, const uint8_t* frozen_mask, int L, int spc_max,
                          int mode, int32_t* ops, int cap, int* n_ops);

/*
 * Create a decoding plan on the current HIP device.
 *   N: power of two in [2, 4096].  K: number of unfrozen positions (1..N).
 *   crc_poly, crc_len: see the conventions above (crc_len <= K).
 *   L: list size in {1, 2, 4, 8, 16, 32, 64, 128} (Sec. VII-B uses 128 for
 *   the CRC-length comparison).  dtype: pscl_dtype.
 *   spc_max, mode: see pscl_schedule.
 * Allocates the device schedule and CRC tables; the decoding workspace
 * follows on first use (pscl_plan_reserve).
 * Returns PSCL_E_INVALID on bad arguments, PSCL_E_NODEV without a gfx950
 * device, PSCL_E_NOMEM / PSCL_E_HIP on runtime failures.  *out is set only on
 * success.
 */
pscl_status pscl_plan_create(int N, int K, const uint8_t* frozen_mask, uint64_t crc_poly,
                             int crc_len, int L, int dtype, int spc_max, int mode,
                             pscl_plan** out);

/*
 * Launch shape of a plan.  A zero field takes the library default for the
 * dtype (float32: 128 threads, 24 KiB; int16: 64 threads, 12 KiB; int8: 64
 * threads, 10 KiB, chosen by measurement at (2048,1723) L=32; for L = 64 /
 * 128: float32 128 / 256 threads with 32 / 48 KiB, int16 128 threads with
 * 20 / 32 KiB, int8 128 threads with 16 / 20 KiB), which the environment
 * variables PSCL_THREADS, PSCL_LDS_BUDGET and PSCL_MAX_WG_PER_CU override.
 *   threads: threads per workgroup (one frame per workgroup): 64, 128, 256,
 *            512 or 1024; at least 128 for L = 128 (one wavefront serves at
 *            most 64 paths), else PSCL_E_UNSUPPORTED.
 *   lds_budget: LDS bytes per workgroup (one frame) for the path tables, candidate
 *            scratch and the low tree levels' LLR stages and partial sums;
 *            the levels that do not fit go to the global workspace.  A
 *            budget too small for the tables alone is raised to what they
 *            need (every tree level then in the workspace).
 */
typedef struct {
    int threads;
    int lds_budget;
    int max_wg_per_cu; /* resident workgroups per CU at most (0 = as many as fit) */
    /* LLR stages below the root that are recomputed from the channel row
     * where they are read instead of being stored, when they would live in
     * the workspace and only F / G / Combine touch their levels: 1 = none,
     * 2 = the stage of level n - 1, 3 = those of levels n - 1 and n - 2
     * (int8: as 2) (0 = default: 2 for float32 and int16, 1 for int8). */
    int recompute;
    /* float32 with L <= 32 only: forking leaves of at most 2^fuse_log2
     * values are scored, ranked and written in one wavefront (-1 = never,
     * 1..5; 0 = default 5); ignored otherwise. */
    int fuse_log2;
    /* Tree levels one F / G pass descends (the unrolling of Sec. II-D at
     * the granularity of node operations): 1 = each F and G its own pass;
     * 2 = an F or G immediately followed by the F of its left child runs as
     * one pass that stores both outputs without re-reading the first
     * (float32: three levels when the grandchild's F follows as well), and
     * (float32, forking leaves run in one wavefront) a leaf right after the
     * F or G forming its input forms its values from that operation's input
     * instead of their being stored and read back (0 = default 2). */
    int unroll;
} pscl_launch_cfg;

/* pscl_plan_create with an explicit launch shape (cfg may be NULL).
 * Returns PSCL_E_INVALID for an unsupported thread count. */
pscl_status pscl_plan_create_cfg(int N, int K, const uint8_t* frozen_mask, uint64_t crc_poly,
                                 int crc_len, int L, int dtype, int spc_max, int mode,
                                 const pscl_launch_cfg* cfg, pscl_plan** out);

/*
 * Autotuner: times pscl_decode of the caller's F frames (llr: device, F x N,
 * as for pscl_decode, F >= 1) on the given stream and writes the fastest
 * launch configuration found to *best (and its time per call, in
 * milliseconds, to *best_ms when not NULL).  The search runs coordinate by
 * coordinate, each plan that differs from those already timed being timed
 * once: waves per frame (threads 64, 128, 256) x LDS budget (8 to 48 KiB:
 * which tree levels stay on chip); then the stages recomputed below the
 * root (recompute 1..3); then, for float32 with L <= 32, the largest fused
 * forking leaf (fuse_log2 -1, 3, 4, 5); then the tree levels per F / G
 * pass (unroll 1, 2); then a residency cap (2, 4, 8 workgroups per CU).  Allocates and frees plans and output buffers while
 * it runs, so it belongs to set-up, not to a decoding loop.  Same argument
 * rules and errors as pscl_plan_create.
 */
pscl_status pscl_autotune(int N, int K, const uint8_t* frozen_mask, uint64_t crc_poly,
                          int crc_len, int L, int dtype, int spc_max, int mode,
                          const void* llr, int64_t F, void* stream, pscl_launch_cfg* best,
                          float* best_ms);

/* Release a plan (NULL allowed).  Synchronises the device first. */
void pscl_plan_destroy(pscl_plan* plan);

/* The code and list a plan decodes (each output pointer may be NULL). */
pscl_status pscl_plan_code(const pscl_plan* plan, int* N, int* K, int* crc_len, int* L,
                           int* dtype);

/* Device bytes one frame of the plan occupies while it is decoded: its
 * global workspace and LDS, its LLR row and its outputs (K + 1 + 4 bytes).
 * Servers charge requests F times this against their admission budget. */
pscl_status pscl_plan_footprint(const pscl_plan* plan, int64_t* bytes_per_frame);

/* Allocate the plan's decoding workspace for its full grid now
 * (pscl_decode otherwise allocates what its calls need), so that every
 * pscl_decode on it is free of allocation, e.g. before capturing one in a
 * HIP graph.  Plans used only through groups or servers never need it.
 * Returns PSCL_E_NOMEM when the device is out of memory. */
pscl_status pscl_plan_reserve(const pscl_plan* plan);

/*
 * Decode F frames (Sec. III; Alg. 1; final CRC choice, Sec. II-B).
 *   llr: device, F x N row-major in the plan's dtype.
 *   u_hat: device, F x K bytes (0/1): the decided bits at the unfrozen
 *          positions in increasing position order (payload then CRC).
 *   crc_ok: device, F bytes or NULL: 1 if the chosen path satisfies the CRC
 *          (always 1 when crc_len = 0).
 *   pm: device, F entries or NULL: path metric of the chosen path, float for
 *       PSCL_F32, int32 for the integer dtypes.
 *   stream: hipStream_t or NULL for the default stream.
 * F = 0 is a no-op.  Returns PSCL_E_INVALID on null required pointers or
 * F < 0.  When the plan's workspace already serves the call's workgroups
 * (after pscl_plan_reserve, or an earlier call on at least as many frames,
 * up to the full grid) only kernel launches are issued (no allocation, copy
 * or memset), so a call can be captured in a HIP graph and replayed.
 */
pscl_status pscl_decode(const pscl_plan* plan, const void* llr, int64_t F, uint8_t* u_hat,
                        uint8_t* crc_ok, void* pm, void* stream);

/*
 * pscl_decode for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc).
 * Same arguments, outputs and errors as pscl_decode, but the plan's own
 * workspace is never used or allocated: the frame counter and the global
 * workspaces live in one static device array of the library, 128 MiB per
 * device (the counter in its first 256 bytes), held from the library's load
 * until the process ends.  The launch uses as many workgroups as have a
 * workspace there, at most the plan's own count, so a plan whose levels
 * spill to the workspace may run on fewer workgroups than pscl_decode uses.
 * Issues kernel launches only (no allocation, copy or memset).
 * Returns PSCL_E_UNSUPPORTED when one workgroup's workspace alone exceeds
 * 128 MiB - 256 bytes, PSCL_E_INVALID when the current device is not the
 * plan's.  Every call on a device shares that device's array, which keeps
 * the last call's contents: calls that overlap on one device (other
 * streams, other threads) race and must be ordered by the caller.
 */
pscl_status pscl_decode_noalloc(const pscl_plan* plan, const void* llr, int64_t F,
                                uint8_t* u_hat, uint8_t* crc_ok, void* pm, void* stream);

/*
 * One-call form decode(N, K, frozen_mask, crc_poly, L, llr) -> u_hat: builds
 * (or reuses from a per-process cache keyed by every argument that shapes the
 * plan) the plan for the Dec-SPC-4 tree, with a group of it holding two
 * workspaces, and decodes.  Calls may overlap on any threads and streams,
 * also for one code: each call in flight has its own workspace and frame
 * counter (a third overlapping call waits on the host for the oldest).
 * Same buffers and errors as pscl_plan_create + pscl_group_decode.
 */
pscl_status pscl_decode_oneshot(int N, int K, const uint8_t* frozen_mask, uint64_t crc_poly,
                                int crc_len, int L, int dtype, const void* llr, int64_t F,
                                uint8_t* u_hat, uint8_t* crc_ok, void* stream);

/*
 * Mixed launches: frames of several codes (N, K, L, CRC) of one dtype in one
 * persistent launch.  Workgroups take frames one at a time from a device
 * counter, most expensive code first, so frames of very different cost
 * share the GPU without a tail per code.
 *
 * A job is F frames of plans[plan] with its own buffers, each with the
 * layout and rules of pscl_decode (llr 16-byte aligned; crc_ok, pm may be
 * NULL).  Jobs with F = 0 are skipped.
 */
typedef struct {
    int plan;
    const void* llr;
    int64_t F;
    uint8_t* u_hat;
    uint8_t* crc_ok;
    void* pm;
} pscl_job;

typedef struct pscl_group pscl_group;

/*
 * A group of plans decoded together.  All plans must have one dtype and
 * belong to the current device (PSCL_E_UNSUPPORTED / PSCL_E_INVALID
 * otherwise) and must outlive the group.  max_jobs bounds the non-empty
 * jobs of one call; max_inflight (1..8) the calls in flight at once (4 for
 * the group pscl_decode_mixed keeps).  cfg (NULL allowed) sets the threads
 * per workgroup;
 * each plan keeps its own LDS layout, and the launch reserves the largest.
 * Allocates the concatenated schedules and, per call in flight, a workspace
 * for the largest plan and a pinned job table, so pscl_group_decode never
 * allocates.
 */
pscl_status pscl_group_create(const pscl_plan* const* plans, int n_plans, int max_jobs,
                              int max_inflight, const pscl_launch_cfg* cfg, pscl_group** out);

/*
 * Autotuner of a mixed launch: times pscl_group_decode of the caller's jobs
 * (job.plan indexes `plans`, whose codes define the trial plans; buffers as
 * for pscl_group_decode) on the stream, with every plan rebuilt under one
 * launch configuration at a time, searched coordinate by coordinate: group
 * threads (64, 128, 256) x LDS budget per plan (8 to 32 KiB); then the
 * stages recomputed below the root (recompute 1..3); then, for float32, the
 * largest fused forking leaf (fuse_log2 -1, 4, 5); then the tree levels per
 * F / G pass (unroll 1, 2).  Writes the fastest
 * configuration for each plan to cfgs[0 .. n_plans) (pass each to
 * pscl_plan_create_cfg), the group's threads to *threads (pass them to
 * pscl_group_create) and the time per call in milliseconds to *best_ms
 * when not NULL.  Allocates and frees plans and groups while it runs (set-up
 * work).  PSCL_E_INVALID for missing arguments, plans of different dtypes
 * or a job whose plan index is out of range.
 */
pscl_status pscl_autotune_group(const pscl_plan* const* plans, int n_plans, const pscl_job* jobs,
                                int n_jobs, void* stream, pscl_launch_cfg* cfgs, int* threads,
                                float* best_ms);

/* Release a group (NULL allowed) after its launches have finished. */
void pscl_group_destroy(pscl_group* group);

/*
 * Decode the jobs in one launch on the stream (asynchronous).  Up to
 * max_inflight calls may be in flight per group, on any streams (each has
 * its own job table and workspace, taken in turn); a further call waits on
 * the host for the oldest to finish.  Returns PSCL_E_INVALID for a bad plan index, F < 0,
 * null or misaligned required pointers, or more than max_jobs non-empty
 * jobs.  Results are identical to pscl_decode of each job with its plan.
 */
pscl_status pscl_group_decode(pscl_group* group, const pscl_job* jobs, int n_jobs, void* stream);

/*
 * The same without an explicit group: the group for this list of plans is
 * created on first use (allocating) and cached until one of its plans is
 * destroyed.
 */
pscl_status pscl_decode_mixed(const pscl_plan* const* plans, int n_plans, const pscl_job* jobs,
                              int n_jobs, void* stream);

/*
 * Serving.  A server decodes requests (one pscl_job each: F frames of one
 * of its codes, in the caller's device buffers) as they arrive.  A
 * dispatcher thread keeps up to `streams` launches in flight, one per
 * stream; whenever a stream is free it launches every pending request (up
 * to the batch limits) as one mixed launch, so requests that arrive while
 * others run join the next launch as soon as a stream frees up (continuous
 * batching), and launches on different streams overlap on the device.
 * Each request's results equal pscl_decode of it alone.  Latency runs from
 * submission (or, in pscl_replay, the scheduled arrival) to the moment the
 * dispatcher sees the launch that decoded it complete.
 *
 * Persistent mode (cfg.persistent = 1): instead of a launch per batch, the
 * dispatcher publishes each request, once its inputs are ready, into a ring
 * in coherent host memory (a record per frame: its rows, its request's
 * slot, ticket, plan and size; the count of published frames), and one
 * persistent kernel on the
 * server's stream, with as many workgroups as it can keep resident,
 * claims published frames one at a time and decodes them, so a request
 * starts as soon as any workgroup is free (continuous batching at frame
 * granularity); the last frame of a request writes its ticket to the
 * request's completion word.  Workgroups are ranked by start order on
 * their CU: the first active_per_cu of each CU take frames, or by default
 * the one of rank r while more than r x (CU count) frames are outstanding
 * (published, not yet finished), so that at low load few frames share a
 * CU (lower latency) and under load every resident workgroup works.  The
 * kernel ends after idle_us microseconds
 * without work (so it never outlives the server) and is relaunched when
 * requests are held.  `streams`, max_batch_frames and max_batch_requests
 * do not apply; at most 2^18 frames are published and unfinished at once
 * (a larger request is invalid, more are held back).
 *
 * Admission (pscl_server_submit returns PSCL_E_BUSY, the caller retries):
 * by request count, by queued frames, and by device footprint: a request of
 * F frames of plan p is charged F * pscl_plan_footprint(p) bytes from its
 * submission to its completion, and the charges held stay within
 * max_footprint_bytes.
 */
typedef struct pscl_server pscl_server;

typedef struct {
    const pscl_plan* const* plans; /* the codes served, one dtype; they must outlive the server */
    int n_plans;
    int streams;                /* launches in flight, 1..8 (0 = 2) */
    int max_requests;           /* requests held, queued or running (0 = 4096) */
    int64_t max_pending_frames; /* frames queued and not yet launched (0 = no limit) */
    int64_t max_batch_frames;   /* frames per launch (0 = no limit; one request at least) */
    int max_batch_requests;     /* requests per launch (0 = 1024) */
    int64_t max_footprint_bytes; /* device bytes of held requests (0 = no limit) */
    int persistent; /* 1 = persistent mode (below); 0 = launches per batch */
    int idle_us;    /* persistent mode: a launch ends after this long without work
                       (0 = 2000) */
    int wg_per_cu;  /* persistent mode: resident workgroups per CU at most (0 = as
                       many as fit) */
    int active_per_cu; /* persistent mode: resident workgroups per CU that take
                          frames (0 = by the frames outstanding, as above) */
} pscl_server_cfg;

/* Create a server on the current device (allocates one group, stream and
 * event per stream, and starts the dispatcher thread). */
pscl_status pscl_server_create(const pscl_server_cfg* cfg, pscl_server** out);

/* Finish every held request, stop the dispatcher and release the server
 * (NULL allowed). */
void pscl_server_destroy(pscl_server* server);

/*
 * Queue one request and return its ticket.  The job's buffers stay the
 * caller's and must stay valid until the request is done.  stream: the HIP
 * stream (NULL = the null stream) whose work issued before this call
 * produces the job's inputs; the request is decoded only after that work
 * (an event recorded on it now).  PSCL_E_BUSY when the server already holds
 * max_requests requests, or the request would take the queued frames beyond
 * max_pending_frames or the held footprint beyond max_footprint_bytes
 * (admission control: the caller retries later); PSCL_E_INVALID for a bad
 * job or one that exceeds either limit alone.  A failed launch is reported
 * by every later call.
 */
pscl_status pscl_server_submit(pscl_server* server, const pscl_job* job, void* stream,
                               uint64_t* ticket);

/* *done = 1 once the request's outputs are complete in device memory (and
 * its latency in microseconds to *latency_us when not NULL); a ticket is
 * forgotten once reported done. */
pscl_status pscl_server_poll(pscl_server* server, uint64_t ticket, int* done,
                             double* latency_us);

/* Block until the request is done (then as pscl_server_poll), or for at
 * most timeout_ms milliseconds (timeout_ms < 0: no limit), returning
 * PSCL_E_TIMEOUT if it is not done by then (the ticket stays valid). */
pscl_status pscl_server_wait(pscl_server* server, uint64_t ticket, double timeout_ms,
                             double* latency_us);

/* Requests, frames and launches completed, and the 50th / 99th percentile
 * latencies (microseconds) of those requests; reset != 0 clears them. */
pscl_status pscl_server_stats(pscl_server* server, int64_t* requests, int64_t* frames,
                              int64_t* launches, double* p50_us, double* p99_us, int reset);

/*
 * Replay a request trace: job i arrives arrival_us[i] microseconds after
 * the start (non-decreasing; the host clock is busy-waited).  Through
 * `server` (plans, n_plans and streams unused), or, when server is NULL, as
 * the plain baseline of one pscl_decode per request, issued in arrival order
 * round-robin on `streams` (1..8) streams of the replay's own: request i
 * runs on stream i % streams with plan plans[(i % streams) * n_plans +
 * job.plan], so `plans` holds `streams` sets of n_plans plans (one set per
 * stream: calls on one plan must not overlap).  The jobs' inputs must be
 * ready before the call.  Blocks until every request is done and writes
 * each request's latency (from its scheduled arrival, so queueing counts)
 * and the elapsed time from the start to the last completion.
 */
pscl_status pscl_replay(pscl_server* server, const pscl_plan* const* plans, int n_plans,
                        int streams, const pscl_job* jobs, const double* arrival_us, int n,
                        double* latency_us, double* elapsed_us);

/*
 * Adaptive decoding (Sec. VI): every frame is decoded first by `fast`, a
 * plan with L = 1 (Fast-SSC on the same tree), and only the frames whose
 * CRC fails are decoded again by `list`.  Both plans must be of the same
 * code (N, frozen set, K, CRC, which must be present) and dtype, and must
 * outlive the adaptive decoder; `fast` must have L = 1 (PSCL_E_INVALID
 * otherwise).  max_frames bounds F per call.  Allocates the index scratch.
 */
typedef struct pscl_adaptive pscl_adaptive;
pscl_status pscl_adaptive_create(const pscl_plan* fast, const pscl_plan* list, int64_t max_frames,
                                 pscl_adaptive** out);

/* Release (NULL allowed); synchronises the device first. */
void pscl_adaptive_destroy(pscl_adaptive* ad);

/*
 * Decode F frames (F <= max_frames) with the buffers and rules of
 * pscl_decode: a frame's outputs are the fast pass's if its CRC passes,
 * else the list pass's (crc_ok, pm then describe the list pass).  Nothing
 * returns to the host in between: the failing frames are gathered on the
 * device.  n_list (device int64, NULL allowed) receives the number of
 * frames list-decoded.  Calls on one adaptive decoder must be ordered
 * (they share its scratch and the plans' workspaces).
 */
pscl_status pscl_adaptive_decode(pscl_adaptive* ad, const void* llr, int64_t F, uint8_t* u_hat,
                                 uint8_t* crc_ok, void* pm, int64_t* n_list, void* stream);

/*
 * Synthetic frames on the device, the workload of Sec. VII-A: uniform
 * payload bits, the CRC appended inside K (conventions above), polar
 * encoding x = u F^{(x)n}, BPSK s = 1 - 2x over AWGN y = s + sigma n with
 * sigma^2 = 1 / (2 R 10^(EbN0/10)), R = (K - r) / N, LLR = 2y / sigma^2,
 * quantised for the integer dtypes (int8: rne(4 LLR) clipped to +-127;
 * int16: rne(64 LLR) clipped to +-32767).  Random numbers: Philox4x32-10
 * keyed by the seed, counters by frame index, so frame f is the same
 * whatever call produces it; normals by Box-Muller.  For throughput and
 * error-rate runs at scale.
 */
typedef struct pscl_generator pscl_generator;
pscl_status pscl_generator_create(int N, int K, const uint8_t* frozen_mask, uint64_t crc_poly,
                                  int crc_len, int dtype, pscl_generator** out);
void pscl_generator_destroy(pscl_generator* gen);

/* Frames first_frame .. first_frame + F - 1 into llr (device, F x N in the
 * dtype) and, when not NULL, their K information bits into info (device,
 * F x K bytes: payload then CRC), asynchronously on the stream.  The device
 * current at pscl_generator_create must be current (else PSCL_E_INVALID);
 * F = 0 does nothing. */
pscl_status pscl_generate(pscl_generator* gen, uint64_t seed, int64_t first_frame, int64_t F,
                          double ebn0_db, void* llr, uint8_t* info, void* stream);

/* Launch shape chosen for a plan: frames per workgroup, threads per
 * workgroup, workgroups, LDS bytes per workgroup, bytes of global workspace,
 * first tree level whose LLR stage lives in global memory (n = none). */
pscl_status pscl_plan_info(const pscl_plan* plan, int* frames_per_wg, int* threads,
                           int* workgroups, int* lds_bytes, int64_t* workspace_bytes,
                           int* first_global_stage);

#ifdef __cplusplus
}
#endif

#endif
