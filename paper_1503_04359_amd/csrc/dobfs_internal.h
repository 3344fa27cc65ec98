/*
 * Internal declarations of the direction-optimized BFS library.
 *
 * Device-memory layout of one resident graph (all device arrays):
 *   off      int64[n+1]   CSR row offsets (both directions of every edge)
 *   idx      int32[m]     neighbour IDs, each row in the order bottom-up
 *                         steps scan it
 *   iso      uint64[W]    W = ceil(n/64) words; bit v set when deg(v) = 0 or
 *                         v >= n.  It is the visited bitmap's initial state:
 *                         such vertices can never be reached through an edge,
 *                         so marking them visited lets bottom-up steps skip
 *                         them without reading their offsets.
 *   new2old / old2new int32[n]   only for degree-relabelled graphs.
 *
 * Workspace of one traversal (reused by later traversals of the graph):
 *   vis      uint64[W]    visited set (bit per vertex)
 *   fr[2]    uint64[W]    frontier bitmaps of levels L (even/odd)
 *   q        int32[n]     frontier queue of a top-down level (rebuilt from
 *                         the frontier bitmap before each such level)
 *   huge_u / huge_base    top-down vertices whose edges are split across
 *                         wavefronts, with the first chunk index of each
 *   ctl                   level state and counters (below)
 *   log                   one dobfs_level_rec per level
 */
#ifndef DOBFS_INTERNAL_H
#define DOBFS_INTERNAL_H

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "dobfs.h"

namespace dobfs {

constexpr int kBlock = 256;          /* threads per workgroup (4 wavefronts) */
constexpr int kWave = 64;
constexpr int kHugeChunk = 512;      /* edges per wavefront task for split vertices */
constexpr int kHugeBatch = 8;        /* a split task's entries a lane claims at a time */
constexpr int kMinHugeCut = 64;      /* lower bound of td_huge_cut */
constexpr int kDirTD = 0;
constexpr int kDirBU = 1;
constexpr int kAuxNone = 0;
constexpr int kAuxHuge = 1;          /* split top-down vertices still to expand */
constexpr int kAuxToQueue = 2;       /* next level top-down: bitmap to queue */
constexpr int kAuxMsUpdate = 3;      /* batched level: fold nxt into the frontier     */
constexpr int kAuxMsSplit = 4;       /* batched level: chunks of split vertices left  */
constexpr int kMsPushSplit = 256;    /* batched push: degree above which a vertex is split */
constexpr int kMsPullSplit = 2048;   /* batched pull: degree above which a vertex may be split */
constexpr int kMsPullProbe = 512;    /* batched pull: entries such a vertex scans before it is split */
constexpr int kMsTake = 256;         /* batched push: entries per row and round */

constexpr int kGroups = 64;
constexpr int kBuWords = 4;          /* 64-vertex words a bottom-up wavefront takes at a time */
constexpr int kBuBlock = 1024;       /* threads per bottom-up workgroup (two per CU) */
constexpr int kBuHot32 = 16384;      /* 32-bit frontier words a bottom-up workgroup keeps in LDS (64 KB) */
constexpr int kDirectCap = 1 << 16;  /* entries of a direct queue; a top-down level whose
                                        frontier has at most this many edges appends its
                                        claims to the next level's queue itself */
constexpr int kXcds = 8;             /* dies (XCDs) of an MI355X; workgroups are dealt round-robin */
constexpr int kMaxSeg = 72;          /* degree classes of int64 degrees, plus one */
constexpr int kFinBlock = 4096;      /* minimum caller IDs per finalize workgroup */
constexpr int kFinGrid = 1024;       /* finalize workgroups (4 per CU) */          /* completion groups per kernel (see finish_block) */

struct GroupSlot {
  int64_t sum[4];
  unsigned long long bits; /* OR of the batched slots that found vertices */
  uint32_t ticket;
  uint32_t pad[21];     /* one 128-byte cache line per group */
};

/* Level state, advanced on the device by the last workgroup of each level. */
/* Per-slot counters of a batched traversal, for the per-slot switching
   rule.  Frontier edges are estimated: each wavefront credits a slot with
   its count of new vertices times their mean degree. */
struct SlotStat {
  int64_t nf;                    /* frontier vertices of the slot, level L  */
  int64_t mf;                    /* estimated frontier edges                */
  int64_t mu;                    /* estimated edges not yet explored        */
  unsigned long long nf_next;    /* accumulators of the level in progress   */
  unsigned long long mf_next;
  int64_t pad[3];
};

struct Ctl {
  int32_t level;        /* L: frontier = vertices of depth L              */
  int32_t dir;          /* direction of level L                           */
  int32_t done;         /* set when a level finds no new vertex           */
  int32_t pad2;
  int32_t aux;          /* kAux*: work for the aux kernel of this level   */
  int32_t bu_run;       /* consecutive bottom-up levels just completed    */
  int32_t bu_phases;    /* bottom-up phases started so far                */
  int32_t levels;       /* final level count                              */
  int32_t log_len;
  int32_t pad0;
  int64_t n_f, m_f, m_u;
  /* accumulators of the level in progress */
  int64_t nf_next;
  int64_t mf_next;
  int64_t checked;
  int64_t scanned;
  unsigned long long huge_pack; /* (entries << 32) | chunks               */
  int64_t q_fill;       /* bitmap->queue append cursor                    */
  uint32_t ticket;      /* workgroups finished in the current kernel      */
  uint32_t pad1;
  /* totals */
  int64_t reached, reached_deg, checked_total;
  uint64_t t_begin;
  /* batched sessions */
  unsigned long long live_next; /* slots that found vertices in this level   */
  unsigned long long live;      /* ... in the last completed level           */
  int32_t active_slots;         /* slots being served                        */
  int32_t pad3;
  unsigned long long pull_mask; /* batched: slots pulled (bottom-up) in level L */
  /* small top-down levels hand their queue on directly */
  int32_t q_append;     /* top-down level L appends its claims to the next queue */
  int32_t q_direct;     /* level L's queue is a direct buffer, not q0            */
  unsigned long long qd_fill; /* append cursor of the next queue               */
  GroupSlot grp[kGroups]; /* zero between kernels */
  SlotStat slot[64];      /* batched: per-slot counters                      */
};

struct KParams {
  int32_t policy, alpha, beta, paper_pct, paper_div, paper_bu_steps;
  int32_t td_wave_cut, td_huge_cut, bu_heavy_cut;
  int32_t kappa_x1000;
  uint64_t seed;
};

struct GView {
  const int64_t* off;
  const int32_t* idx;
  const uint64_t* iso;
  const int32_t* first;    /* first neighbour of each vertex (-1: degree 0): the
                              bottom-up round 0 reads it as one coalesced column */
  const int32_t* first_caller; /* relabelled graphs: caller ID of first[v]   */
  const int32_t* old2new;  /* relabelled graphs: caller ID -> internal ID  */
  const int32_t* new2old;  /* relabelled graphs: internal ID -> caller ID  */
  const int64_t* seg_lo;   /* relabelled graphs: internal start of each degree
                              class, ascending, seg_lo[nseg] = n           */
  int32_t nseg;
  int32_t pad_seg;
  int64_t n, m;
  int64_t n_nonisolated;
  int64_t words;         /* ceil(n/64)                                     */
  int64_t words_active;  /* words that may hold an unvisited vertex        */
};

struct WView {
  uint64_t* vis;
  uint64_t* fr0;
  uint64_t* fr1;
  int32_t* q0;          /* frontier queue of a top-down level            */
  int32_t* qd0;         /* direct queues (kDirectCap entries), level parity */
  int32_t* qd1;
  int32_t* huge_u;
  uint32_t* huge_base;
  int32_t* depth;         /* caller's outputs (caller labels)              */
  int32_t* parent;
  int64_t* packed;        /* relabelled graphs: internal (parent, depth)   */
  Ctl* ctl;
  dobfs_level_rec* log;
  int32_t log_cap;
  int32_t pad;
};

/* Batched traversal state (msbfs.hip): bit b of each mask = root slot b. */
struct MsView {
  uint64_t* visit;
  uint64_t* cur0;
  uint64_t* cur1;
  uint64_t* nxt;
  int32_t* out;         /* caller's depths, root-major [k][n], caller IDs      */
  int32_t* internal;    /* relabelled graphs: [k][n_nonisolated], internal IDs */
  int32_t k;
  int32_t pad;
  uint64_t full;        /* the k low bits                                     */
  Ctl* ctl;
  dobfs_level_rec* log;
  int32_t log_cap;
  int32_t session;      /* 1: per-slot outputs below, slots join and leave */
  int32_t** slot_out;   /* session: device table, depth array of each slot  */
  int32_t* slot_start;  /* session: device table, level each slot joined at */
  int32_t* split_u;     /* split vertices of the running level (list entries) */
  uint32_t* split_base; /* first chunk number of each entry, increasing      */
};

struct MsRoots {
  int32_t r[64];        /* caller IDs */
};

hipError_t launch_ms_init(const GView& g, const MsView& m, const MsRoots& r, int first_pull, int grid, hipStream_t s);
hipError_t launch_ms_level(const GView& g, const MsView& m, const KParams& kp, int grid, hipStream_t s);
hipError_t launch_ms_finalize(const GView& g, const MsView& m, const MsRoots& r, int grid, hipStream_t s);
/* Output array of each slot of a session admission or finalize. */
struct SlotOuts {
  int32_t* p[64];
};

/* Session: empty masks and an idle control block. */
hipError_t launch_ms_session_start(const GView& g, const MsView& m, int grid, hipStream_t s);
/* Session admission: forget the slots in clear_bits, then seed the slots in
   new_bits with roots r.r[b] (caller IDs) and outputs outs.p[b]. */
hipError_t launch_ms_session_admit(const GView& g, const MsView& m, unsigned long long clear_bits, const MsRoots& r,
                                   const SlotOuts& outs, unsigned long long new_bits, int first_pull, int grid,
                                   hipStream_t s);
/* Session, relabelled graphs: caller-order depths of the slots in `ended`
   (roots r.r[b], outputs outs.p[b]) from their internal rows. */
hipError_t launch_ms_session_finalize(const GView& g, const MsView& m, const MsRoots& r, const SlotOuts& outs,
                                      unsigned long long ended, int grid, hipStream_t s);

/* Kernel launchers (bfs_kernels.hip). */
hipError_t launch_init(const GView& g, const WView& w, const int32_t* roots, int32_t nroots, int64_t root0,
                       int32_t first_dir, int grid, hipStream_t s);
hipError_t launch_fix_roots(const WView& w, const int32_t* roots, int32_t nroots, hipStream_t s);
hipError_t launch_level(const GView& g, const WView& w, const KParams& kp, int grid, hipStream_t s);
/* the two halves of launch_level, for timing each kernel on its own */
hipError_t launch_level_td(const GView& g, const WView& w, const KParams& kp, int grid, hipStream_t s);
hipError_t launch_level_bu(const GView& g, const WView& w, const KParams& kp, int grid, hipStream_t s);
hipError_t launch_aux(const GView& g, const WView& w, const KParams& kp, int grid, hipStream_t s);
hipError_t launch_finalize(const GView& g, const WView& w, int64_t root, int grid, hipStream_t s);
hipError_t level_grid(int* grid);

/* Sets the text dobfs_last_error() returns on this thread (api.hip); the
   HIP error's name is appended when e is not hipSuccess. */
void set_last_error(const char* what, hipError_t e);

/* Degree relabelling (reindex.hip): builds the internal CSR of a graph whose
   vertices are renumbered by degree, highest first (ties by caller ID),
   every row sorted by internal ID, i.e. highest-degree neighbour first. */
int build_reindexed(const int64_t* off, const int32_t* idx, int64_t n, int64_t m, int grid, hipStream_t s,
                    int64_t** off_new, int32_t** idx_new, int32_t** new2old, int32_t** old2new,
                    int64_t** seg_lo, int32_t* nseg, std::string* err);

/* Graph preparation launchers (graph_kernels.hip). */
hipError_t launch_first_caller(const int32_t* first, const int32_t* new2old, int64_t n, int32_t* out, int grid,
                               hipStream_t s);
hipError_t launch_first_column(const int64_t* off, const int32_t* idx, int64_t n, int32_t* first, int grid,
                               hipStream_t s);
hipError_t launch_graph_scan(const int64_t* off, int64_t n, uint64_t* iso, int64_t* counters,
                             int grid, hipStream_t s);
hipError_t launch_pack_copy(const int64_t* off, const int32_t* idx, int64_t n, int64_t m, int64_t nbase, int64_t mbase,
                            bool src_device, int64_t* uoff, int32_t* uidx, hipStream_t s);
hipError_t launch_validate(const int64_t* off, const int32_t* idx, int64_t n, int64_t m, int symmetry,
                           int32_t* bad, int grid, hipStream_t s);

}  // namespace dobfs

#endif
