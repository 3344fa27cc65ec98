/*
 * dobfs.h -- direction-optimized breadth-first search on one AMD Instinct
 * MI355X (gfx950), whole graph resident in device memory.
 *
 * The problem (Section 4, "Methodology"): given an undirected graph stored
 * as CSR with every undirected edge as two directed entries, and a root,
 * compute the BFS parent tree and each vertex's depth (hop distance).  The
 * traversal is level-synchronous (Section 2.2): each level expands the
 * current frontier either top-down (every frontier vertex claims its
 * unvisited neighbours, Algorithm 1 top-down branch) or bottom-up (every
 * unvisited vertex looks for a neighbour in the frontier and stops at the
 * first, Algorithm 1 bottom-up branch), and a switching rule picks the
 * direction per level (Section 3.3).
 *
 * Conventions for every entry point:
 *   - Return value: DOBFS_OK (0) or a negative DOBFS_E* status.  Nothing
 *     throws or aborts across this interface.  dobfs_last_error() gives a
 *     text for the calling thread's most recent failure (HIP's own text for
 *     DOBFS_EDEVICE).
 *   - Vertex IDs are the caller's: int32 in [0, n), n <= 2^31 - 1.  Any
 *     internal relabelling is undone before results are written.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *   - Output buffers are caller-allocated device memory; the library writes
 *     them asynchronously on `stream` and they are valid once the stream has
 *     been synchronised.
 *   - The library allocates device memory only in dobfs_graph_upload,
 *     dobfs_pack_upload and the first dobfs_run / dobfs_batch_submit on a
 *     graph handle (workspaces, reused afterwards); dobfs_run_noalloc never
 *     allocates.
 */
#ifndef DOBFS_H
#define DOBFS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------ */
#define DOBFS_OK 0
#define DOBFS_EINVAL (-1)   /* null pointer, bad size, bad flag, bad CSR       */
#define DOBFS_ERANGE (-2)   /* a root outside [0, n)                           */
#define DOBFS_ENOMEM (-3)   /* device allocation failed; nothing leaked        */
#define DOBFS_EDEVICE (-4)  /* HIP launch or runtime failure                   */
#define DOBFS_EBUSY (-5)    /* graph still in use (free with runs in flight)   */
#define DOBFS_ENOTSUP (-6)  /* valid request this build does not support       */

typedef struct dobfs_graph_s* dobfs_graph_t; /* opaque, library-owned */

/* ---- upload flags -------------------------------------------------------- */
#define DOBFS_SRC_DEVICE 0x1u      /* offsets/indices are device pointers      */
#define DOBFS_VALIDATE 0x2u        /* check offsets monotone, offsets[0] = 0,
                                      offsets[n] = m, 0 <= indices < n        */
#define DOBFS_VALIDATE_SYMMETRY 0x4u /* also check every (u,v) has (v,u);
                                      rows must then be sorted ascending      */
#define DOBFS_REINDEX_DEGREE 0x8u  /* relabel internally by degree (highest
                                      first, ties by ID) and order every
                                      adjacency list highest-degree neighbour
                                      first (Section 3.4)                     */
#define DOBFS_BORROW 0x10u         /* with DOBFS_SRC_DEVICE: use the caller's
                                      arrays in place, no copy; the caller
                                      keeps them alive and unchanged until
                                      dobfs_graph_free                        */

/* ---- run flags (dobfs_params.flags) --------------------------------------- */
#define DOBFS_RUN_TIME_KERNELS 0x1u /* bracket every level-kernel launch with
                                      HIP events on `stream`; the summed
                                      durations per kernel are reported in
                                      dobfs_stats                           */
#define DOBFS_RUN_GRAPH 0x2u       /* run the traversal as one captured HIP
                                      graph: init, 2 * chunk_levels level
                                      slots and the finalize, recorded once
                                      per workspace and replayed while the
                                      arguments (graph, outputs, roots,
                                      params) repeat; a traversal with more
                                      levels continues with ordinary
                                      launches.  The default of
                                      dobfs_batch_submit and dobfs_pack_run;
                                      for dobfs_run / dobfs_run_multi only on
                                      request.  Excludes the two flags below
                                      (EINVAL).                             */
#define DOBFS_RUN_EAGER 0x4u       /* never use a captured graph             */
#define DOBFS_RUN_HUB_DECIDES 0x8u /* hybrid runs with the PAPER policy only:
                                      the host (hub) partition's own next
                                      frontier decides the top-down ->
                                      bottom-up switch (Section 3.3); the
                                      other runs reject it (EINVAL)          */

/* ---- direction policies (Section 3.3) ------------------------------------ */
#define DOBFS_POLICY_EDGE 0      /* top-down -> bottom-up when the next
                                    frontier's edges times alpha exceed the
                                    unvisited vertices' edges; back when the
                                    frontier shrinks below n / beta          */
#define DOBFS_POLICY_PAPER 1     /* top-down -> bottom-up when paper_pct% of
                                    the frontier's edges (the estimated next
                                    frontier) exceeds n / paper_div; back to
                                    top-down after paper_bu_steps bottom-up
                                    levels, for the rest of the traversal    */
#define DOBFS_POLICY_FORCED_TD 2 /* every level top-down                      */
#define DOBFS_POLICY_FORCED_BU 3 /* every level bottom-up                     */
#define DOBFS_POLICY_RANDOM 4    /* direction of level L = bit of a hash of
                                    (seed, L); for testing invariance        */
#define DOBFS_POLICY_COST 5      /* top-down -> bottom-up when the next
                                    frontier's edges exceed kappa/1000 times
                                    the unvisited vertices of degree >= 1
                                    (the work each direction would do on a
                                    GPU, where bottom-up cost follows the
                                    vertices scanned); back to top-down as
                                    for EDGE                                */

typedef struct {
  int32_t policy;          /* DOBFS_POLICY_*                                */
  int32_t alpha;           /* EDGE, default 14                              */
  int32_t beta;            /* EDGE, default 24                              */
  int32_t paper_pct;       /* PAPER, default 10                             */
  int32_t paper_div;       /* PAPER, default 64                             */
  int32_t paper_bu_steps;  /* PAPER, default 3                              */
  int32_t td_wave_cut;     /* top-down: degree above which a whole wavefront
                              works on one vertex (default 16)              */
  int32_t td_huge_cut;     /* top-down: degree above which a vertex's edges
                              are split over many wavefronts (default 256,
                              at least 64)                                  */
  int32_t bu_heavy_cut;    /* bottom-up: most neighbours one vertex tests per
                              search round, at least 64 (default 256)       */
  int32_t chunk_levels;    /* levels enqueued per host check (default 8)    */
  uint32_t flags;          /* DOBFS_RUN_* (default 0)                       */
  int32_t kappa_x1000;     /* COST, default 500                             */
  uint64_t seed;           /* RANDOM policy                                 */
} dobfs_params;

/* One record per level, written on the device without host involvement. */
typedef struct {
  int32_t level;           /* L: the frontier holds the vertices of depth L */
  int32_t dir;             /* 0 top-down, 1 bottom-up                        */
  int64_t n_f;             /* frontier vertices                              */
  int64_t m_f;             /* summed degree of the frontier                  */
  int64_t m_u;             /* summed degree of unvisited vertices before L   */
  int64_t scanned;         /* bottom-up: unvisited vertices examined         */
  int64_t checked;         /* edges examined (bottom-up: up to first hit)    */
  int64_t found;           /* vertices of depth L+1                          */
  int64_t found_deg;       /* their summed degree                            */
  uint64_t t_end;          /* device wall clock (100 MHz) at level end       */
  float kernel_ms;         /* reserved, 0                                    */
  int32_t reserved;
} dobfs_level_rec;

typedef struct {
  int32_t levels;          /* levels expanded (deepest depth + 1)           */
  int32_t log_len;         /* records written to `log` (<= log_cap)         */
  int64_t reached;         /* vertices with depth >= 0                       */
  int64_t m_c;             /* undirected edges in the root's component:
                              half the summed degree of reached vertices   */
  int64_t checked;         /* edges examined, all levels                     */
  uint64_t t_begin;        /* device wall clock at init                      */
  dobfs_level_rec* log;    /* caller's host array, or NULL                   */
  int32_t log_cap;         /* its capacity in records                        */
  int32_t level_launches;  /* level slots enqueued: each launches the
                              top-down kernel, the bottom-up kernel and the
                              aux kernel (split rows, frontier conversion);
                              the ones not needed, or launched after the
                              traversal finished, return at once           */
  double level_kernel_ms;  /* summed duration of all those launches
                              (DOBFS_RUN_TIME_KERNELS, else 0)              */
  double td_kernel_ms;     /* ... of the top-down kernel's launches         */
  double bu_kernel_ms;     /* ... of the bottom-up kernel's launches        */
  double aux_kernel_ms;    /* ... of the aux kernel's launches              */
} dobfs_stats;

typedef struct {
  int64_t n, m;            /* vertices, directed CSR entries                 */
  int64_t n_nonisolated;   /* vertices of degree >= 1                        */
  int64_t max_degree;
  int64_t device_bytes;    /* graph arrays resident on the device            */
  uint32_t flags;          /* upload flags kept (DOBFS_REINDEX_DEGREE)       */
  int32_t reserved;
} dobfs_graph_info_t;

/* Fills `p` with the defaults listed above. */
void dobfs_default_params(dobfs_params* p);

/* Makes the graph resident on the current device.
   offsets: int64[n+1], indices: int32[m], host memory unless
   DOBFS_SRC_DEVICE (then copied on the device, or adopted without a copy
   with DOBFS_BORROW); the CSR must be symmetric (bottom-up steps read the
   reverse edges) and free of self-loops; rows need not be sorted unless
   DOBFS_VALIDATE_SYMMETRY is given.  Unless borrowed, the arrays are
   copied and the caller may free them when the call returns.  Offsets and
   neighbour IDs are always range-checked.  The call is synchronous.
   Errors: EINVAL (null pointers, n < 1, n > 2^31-1, m < 0, unknown flag,
   validation failure), ENOMEM, EDEVICE. */
int dobfs_graph_upload(const int64_t* offsets, const int32_t* indices, int64_t n, int64_t m,
                       uint32_t flags, void* stream, dobfs_graph_t* out);

/* Releases a graph and its workspaces after waiting for its runs to end.
   NULL is accepted.  Errors: EBUSY (a session of the graph is open; nothing
   is released), EDEVICE. */
int dobfs_graph_free(dobfs_graph_t g);

int dobfs_graph_info(dobfs_graph_t g, dobfs_graph_info_t* info);

/* Single-source direction-optimized BFS from `root`.
   depth:  device int32[n], out: hop distance from root, -1 if unreachable.
   parent: device int32[n] or NULL, out: a neighbour one level closer to the
           root (root: itself; unreachable: -1).  Any such neighbour is a
           correct answer; which one is picked may vary between runs.
   p:      NULL for defaults.
   stats:  NULL, or filled before return (the call then waits for the
           stream to finish the traversal).
   The level loop runs on the device; the host only checks, once per
   `chunk_levels` levels, whether the traversal has ended, so the call
   returns once the last level is known to be enqueued.
   Errors: EINVAL, ERANGE (root), ENOMEM (first-run workspace), EDEVICE. */
int dobfs_run(dobfs_graph_t g, int64_t root, int32_t* depth, int32_t* parent, const dobfs_params* p,
              dobfs_stats* stats, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
   capture, tight serving loops, harnesses that forbid hipMalloc): the
   single-source traversal of dobfs_run with its whole workspace in one
   fixed device array of 64 MiB per device, which holds the graph's traversal
   state for up to about 2.5M vertices (bitmaps, queues, control block, level
   log, and 8 bytes per vertex of packed labels on relabelled graphs or 4 of
   parents when `parent` is NULL).  The call allocates nothing: no device,
   pinned or library allocation and no events.  It checks for the end of the
   traversal after each chunk of levels with a stream synchronisation and
   returns once depth/parent are complete.  Arguments and results as for
   dobfs_run, except that DOBFS_RUN_TIME_KERNELS and DOBFS_RUN_GRAPH are
   refused (EINVAL) and a
   relabelled graph uses its caller-ID column only if an earlier dobfs_run
   built it.  The array is shared by every call on the device and keeps the
   last call's contents (each call clears what it reads first); calls that
   overlap on one device race and give wrong results.
   Errors: as dobfs_run, plus EINVAL (the graph lives on another device) and
   ENOTSUP (the graph needs more scratch than the array holds). */
int dobfs_run_noalloc(dobfs_graph_t g, int64_t root, int32_t* depth, int32_t* parent, const dobfs_params* p,
                      dobfs_stats* stats, void* stream);

/* One traversal seeded from several roots at once (host int64[nroots],
   caller IDs; duplicates allowed): depth = hop distance to the nearest root,
   parent as for dobfs_run with every root its own parent.  Errors as for
   dobfs_run, plus EINVAL when nroots < 1. */
int dobfs_run_multi(dobfs_graph_t g, const int64_t* roots, int32_t nroots, int32_t* depth, int32_t* parent,
                    const dobfs_params* p, dobfs_stats* stats, void* stream);

/* Many small graphs resident as one pack and traversed in one pass, one root
   per graph.  Graph i keeps its own vertex IDs 0..n[i]-1; in the pack it
   occupies IDs bases[i] .. bases[i+1]-1 (bases[0] = 0, bases[count] = total
   vertices).  The graphs are disjoint, so one multi-root traversal gives
   every graph its own single-source result.
   dobfs_pack_upload: arrays of count pointers to each graph's CSR (host
     memory, or device with DOBFS_SRC_DEVICE); flags as for upload except
     DOBFS_BORROW.  The pack's vertex count must stay below 2^31.
   dobfs_pack_bases: bases[0..count] into a host array of count+1.
   dobfs_pack_run: roots: host int64[count], graph-local IDs.
     depth: device int32[bases[count]], each graph's depths in its slice.
     parent: device int32[bases[count]] or NULL, pack IDs (bases[i] + local).
   Errors: EINVAL, ERANGE (a root outside its graph), ENOMEM, EDEVICE. */
int dobfs_pack_upload(int32_t count, const int64_t* const* offsets, const int32_t* const* indices, const int64_t* n,
                      const int64_t* m, uint32_t flags, void* stream, dobfs_graph_t* out);
int dobfs_pack_bases(dobfs_graph_t pack, int64_t* bases);
int dobfs_pack_run(dobfs_graph_t pack, const int64_t* roots, int32_t* depth, int32_t* parent, const dobfs_params* p,
                   dobfs_stats* stats, void* stream);

/* Up to 64 single-source traversals of one graph in one pass: slot b of a
   64-bit mask per vertex follows root b (the same level-synchronous step of
   Algorithm 1 applied to all slots at once; push or pull chosen per level
   like dobfs_run).
   roots:  host int64[k], caller IDs, duplicates allowed; 1 <= k <= 64.
   depth:  device int32[k * n], root-major: depth[b*n + v] = hop distance of
           v from roots[b], -1 if unreachable.  Parents are not produced.
   stats:  NULL, or filled (totals over the k slots: reached, m_c).
   Device memory: 32 bytes per vertex, plus 4*k per vertex of degree >= 1 on
   relabelled graphs, allocated on the first batch and kept.
   Errors: EINVAL (k, NULL), ERANGE (a root), ENOMEM, EDEVICE. */
int dobfs_batch_submit(dobfs_graph_t g, const int64_t* roots, int32_t k, int32_t* depth, const dobfs_params* p,
                       dobfs_stats* stats, void* stream);

/* Continuous batching: a session keeps the 64 slots of the batched
   traversal running and lets queries join and leave between level chunks.
   A query joins at the session's current level with its root as its only
   frontier vertex and counts its depths from there, so its result is the
   same as a dobfs_run of that root alone, whatever else shares the session.
   A slot is free again once its query's frontier is empty; its bit is
   cleared from every vertex before the next query takes it.
   The direction of each level is shared by all slots: it compares the
   frontier (popcount-weighted) with the vertices the active slots could
   still reach, using alpha and beta of the params.
   A session holds one workspace of the graph (32 bytes per vertex) until
   closed; several sessions on one graph are allowed.  All calls of one
   session come from one thread and run on the session's stream.

   dobfs_session_open: p NULL for defaults; stream as for dobfs_run.
   dobfs_session_admit: queues a query; root in caller IDs; depth: device
     int32[n] owned by the caller and not touched by it until the query is
     reported done; it is set to -1 and then filled like dobfs_run's depth.
     tag: the caller's name for the query, returned by dobfs_session_step.
     Errors: ERANGE (root), EBUSY (64 queries admitted and not yet done).
   dobfs_session_step: lets pending queries join, runs one chunk of
     chunk_levels levels and waits for it; done_tags (host int64[cap])
     receives the tags of the queries that ended (their depth arrays are
     complete when the call returns), *n_done their number; queries beyond
     cap are reported by the next calls.  Returns at once, with *n_done 0,
     when nothing is admitted.
   dobfs_session_counts: *active = queries holding a slot, *pending =
     admitted but not yet joined, *levels = levels run so far.
   dobfs_session_levels: the per-level records of the last step's chunk
     (at most cap into recs, *n of them); dir is 0 push, 1 pull, 2 mixed;
     kernel_ms is 0.
   dobfs_session_close: waits for the stream, forgets queries not reported
     done and releases the workspace.  NULL is accepted.
   Errors: EINVAL (NULL arguments), ERANGE, EBUSY, ENOMEM, EDEVICE. */
typedef struct dobfs_session_s* dobfs_session_t;

int dobfs_session_open(dobfs_graph_t g, const dobfs_params* p, void* stream, dobfs_session_t* out);
int dobfs_session_admit(dobfs_session_t s, int64_t root, int32_t* depth, int64_t tag);
int dobfs_session_step(dobfs_session_t s, int64_t* done_tags, int32_t cap, int32_t* n_done);
int dobfs_session_counts(dobfs_session_t s, int32_t* active, int32_t* pending, int64_t* levels);
int dobfs_session_levels(dobfs_session_t s, dobfs_level_rec* recs, int32_t cap, int32_t* n);
int dobfs_session_close(dobfs_session_t s);

/* ---- Hybrid host + GPU traversal: graphs larger than device memory ----
   The specialized partitioning of Section 3.2 with level-synchronous
   processing on both processors (Section 3.1, Algorithms 2 and 3) and the
   direction switching of Section 3.3 taken on both partitions' counts.

   dobfs_hybrid_upload: takes a host CSR (same layout and symmetry
     requirements as dobfs_graph_upload; host pointers, read during the call
     only), relabels it by degree class (highest first, ties by caller ID)
     and splits the internal IDs at h, the smallest multiple of 64 whose
     GPU share fits gpu_budget_bytes of device memory: rows of [h, n) go to
     the device with all per-vertex state, rows of [0, h) (the hubs) stay in
     host memory and are traversed by `threads` host threads.  (Beyond the
     budget the device also holds 4 bytes per device row longer than 2,048
     entries, a list for their top-down expansion.)  A budget at
     or above the whole graph's share puts every row on the GPU (h = 0); a
     budget that holds the per-vertex state only puts every row on the host.
     The library owns *out; the stream orders the uploads.
   dobfs_hybrid_info: *split = host-owned vertices (min(h, n)),
     *host_entries / *gpu_entries = CSR entries each side holds,
     *gpu_bytes = device bytes the graph holds.  NULL outputs are skipped.
   dobfs_hybrid_run: a traversal from `root` (caller ID) on the stream.
     depth (device int32[n]) and parent (device int32[n], nullable) are in
     caller IDs with the meaning of dobfs_run's; the call returns when they
     are written.  Policies EDGE, PAPER, COST and the forced ones are taken
     (RANDOM: ENOTSUP).  flags: DOBFS_RUN_HUB_DECIDES is taken (PAPER
     only, else EINVAL); without it the rule sees both partitions' summed
     counts.  DOBFS_RUN_TIME_KERNELS fills td/bu_kernel_ms with the GPU
     partition's level kernels and aux_kernel_ms with its mark-apply and
     parent kernels; the other run flags and the kernel-shape parameters are
     ignored.  stats (nullable) gets levels, reached, m_c, checked and, when
     log_cap > 0, one record per level with both partitions' counts summed;
     in these records t_end is host nanoseconds since the run began, at the
     level's end (exchanges included), and kernel_ms the host partition's
     time in the level.  Runs of one hybrid graph are serialised.
     Host resources held by the graph: the host rows, `threads - 1` worker
     threads and 24 ceil(n/64) + 8 min(h, n) + 64 bytes of pinned memory.
   dobfs_hybrid_free: releases the graph's device and host memory; NULL is
     accepted.  The caller ensures no run of the graph is in flight.
   Errors: EINVAL (NULL pointers, bad CSR, threads outside [1, 1024], a
     budget below the per-vertex state: 8(n+1) + 16n + 40 ceil(n/64) +
     64 bytes), ERANGE (root), ENOMEM (device or pinned host allocation),
     ENOTSUP (policy), EDEVICE. */
typedef struct dobfs_hybrid_s* dobfs_hybrid_t;

int dobfs_hybrid_upload(const int64_t* offsets, const int32_t* indices, int64_t n, int64_t m,
                        int64_t gpu_budget_bytes, int32_t threads, void* stream, dobfs_hybrid_t* out);
int dobfs_hybrid_info(dobfs_hybrid_t h, int64_t* split, int64_t* host_entries, int64_t* gpu_entries,
                      int64_t* gpu_bytes);
int dobfs_hybrid_run(dobfs_hybrid_t h, int64_t root, int32_t* depth, int32_t* parent, const dobfs_params* p,
                     dobfs_stats* stats, void* stream);
int dobfs_hybrid_free(dobfs_hybrid_t h);

/* Strings for a status; valid forever. */
const char* dobfs_strerror(int status);
/* Text of the calling thread's most recent failure ("" if none). */
const char* dobfs_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* DOBFS_H */
