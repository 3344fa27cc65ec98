/*
 * ORACLE for breadth-first search over an undirected graph stored as a
 * symmetric CSR (offsets int64[n+1], neighbour IDs int32[m]; every undirected
 * edge appears as two directed entries, Section 4 "Methodology").
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow, obviously correct
 * statement of what the traversal computes.  It shares no code with the
 * device library and must never be reached from the product path: only the
 * test suite, the smoke check and the benchmark's CPU-baseline leg use it.
 *
 * Contents
 *   oracle_bfs            serial FIFO-queue BFS: hop distance and a parent
 *                         (the definition of level-synchronous BFS, Section
 *                         2.2: the next frontier is the set of not-yet-visited
 *                         vertices adjacent to the current one; top-down step
 *                         of Algorithm 1).
 *   oracle_check_tree     the BFS-tree properties that fix every depth uniquely
 *                         and accept any valid parent choice (parents are
 *                         required by the Graph500 methodology, Section 4).
 *   oracle_traversed_edges  undirected edges of the root's component (the TEPS
 *                         numerator, Section 4 "Methodology").
 *   oracle_replay         exact work counts of a direction schedule: frontier
 *                         sizes and edge counts of top-down steps, and
 *                         vertices scanned / edges checked with first-hit exit
 *                         by bottom-up steps (Algorithm 1, bottom-up branch).
 *
 * Pins (tests): closed forms (path, cycle, star, complete, bipartite, grid,
 * hypercube, binary tree, disjoint unions), boolean reachability powers on
 * tiny random graphs, scipy's unweighted shortest paths, planted faults for
 * the checker and a pure-Python recount for the replay.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORACLE_EINVAL (-1)
#define ORACLE_ENOMEM (-3)

/* Serial queue BFS from `root`.  depth[v] = hop distance or -1; parent[v] =
   the vertex whose adjacency list first reached v (root: itself; unreached:
   -1).  `queue` is caller scratch of n int32 (may be NULL: allocated here). */
int oracle_bfs(int64_t n, const int64_t* off, const int32_t* idx, int64_t root, int32_t* depth,
               int32_t* parent, int32_t* queue) {
  if (n < 1 || !off || !depth || !parent || root < 0 || root >= n) return ORACLE_EINVAL;
  int32_t* q = queue;
  if (!q) {
    q = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
    if (!q) return ORACLE_ENOMEM;
  }
  for (int64_t v = 0; v < n; ++v) {
    depth[v] = -1;
    parent[v] = -1;
  }
  depth[root] = 0;
  parent[root] = (int32_t)root;
  int64_t head = 0, tail = 0;
  q[tail++] = (int32_t)root;
  while (head < tail) {
    const int32_t u = q[head++];
    for (int64_t e = off[u]; e < off[u + 1]; ++e) {
      const int32_t v = idx[e];
      if (depth[v] < 0) {
        depth[v] = depth[u] + 1;
        parent[v] = u;
        q[tail++] = v;
      }
    }
  }
  if (!queue) free(q);
  return 0;
}

/* Failure codes of oracle_check_tree. */
enum {
  CHECK_OK = 0,
  CHECK_ROOT = 1,            /* depth[root] != 0 or parent[root] != root   */
  CHECK_RANGE = 2,           /* depth < -1, or parent outside [-1, n)      */
  CHECK_UNREACHED = 3,       /* depth == -1 but parent != -1 (or reverse)  */
  CHECK_PARENT_NOT_EDGE = 4, /* (parent[v], v) is not an edge              */
  CHECK_PARENT_DEPTH = 5,    /* depth[parent[v]] != depth[v] - 1           */
  CHECK_EDGE_SPAN = 6,       /* an edge joins reached and unreached, or
                                endpoint depths differ by more than one    */
};

/* Checks, for the traversal from `root`:
     root:      depth[root] = 0, parent[root] = root;
     unreached: depth[v] = -1 exactly when parent[v] = -1;
     tree:      for every reached v != root (depth 0 included), (parent[v], v)
                is an edge and depth[parent[v]] = depth[v] - 1, so depth[v] >= 1;
     edges:     for every edge (u, v) both ends are reached or both are not,
                and |depth[u] - depth[v]| <= 1.
   The tree property bounds each depth from above by the hop distance's walk
   and the edge property bounds it from below along a shortest path, so
   together they fix depth = hop distance and the reached set = the root's
   component, while accepting any valid parent.  Returns CHECK_OK or a code,
   with the smallest offending vertex in *bad.  Vertices are checked in
   parallel (each vertex's checks read only its own row). */
int oracle_check_tree(int64_t n, const int64_t* off, const int32_t* idx, int64_t root,
                      const int32_t* depth, const int32_t* parent, int64_t* bad) {
  if (n < 1 || root < 0 || root >= n || !bad) return ORACLE_EINVAL;
  *bad = -1;
  if (depth[root] != 0 || parent[root] != (int32_t)root) {
    *bad = root;
    return CHECK_ROOT;
  }
  int64_t first_bad = n;
  int first_code = CHECK_OK;
#pragma omp parallel for schedule(dynamic, 1024) reduction(min : first_bad)
  for (int64_t v = 0; v < n; ++v) {
    const int32_t dv = depth[v], pv = parent[v];
    int code = CHECK_OK;
    if (dv < -1 || pv < -1 || (int64_t)pv >= n) {
      code = CHECK_RANGE;
    } else if ((dv == -1) != (pv == -1)) {
      code = CHECK_UNREACHED;
    } else {
      if (dv >= 0 && v != root) {
        /* I2 holds for every reached vertex other than the root; a second
           vertex of depth 0 has no parent one level up. */
        int found = 0;
        for (int64_t e = off[v]; e < off[v + 1] && !found; ++e) found = (idx[e] == pv);
        if (!found) code = CHECK_PARENT_NOT_EDGE;
        else if (dv == 0 || depth[pv] != dv - 1) code = CHECK_PARENT_DEPTH;
      }
      for (int64_t e = off[v]; e < off[v + 1] && code == CHECK_OK; ++e) {
        const int32_t du = depth[idx[e]];
        if ((du == -1) != (dv == -1)) code = CHECK_EDGE_SPAN;
        else if (dv >= 0 && (du - dv > 1 || dv - du > 1)) code = CHECK_EDGE_SPAN;
      }
    }
    if (code != CHECK_OK && v < first_bad) first_bad = v;
  }
  if (first_bad == n) return CHECK_OK;
  /* Re-derive the code of the smallest offending vertex serially. */
  {
    const int64_t v = first_bad;
    const int32_t dv = depth[v], pv = parent[v];
    if (dv < -1 || pv < -1 || (int64_t)pv >= n) first_code = CHECK_RANGE;
    else if ((dv == -1) != (pv == -1)) first_code = CHECK_UNREACHED;
    else {
      if (dv >= 0 && v != root) {
        int found = 0;
        for (int64_t e = off[v]; e < off[v + 1] && !found; ++e) found = (idx[e] == pv);
        if (!found) first_code = CHECK_PARENT_NOT_EDGE;
        else if (dv == 0 || depth[pv] != dv - 1) first_code = CHECK_PARENT_DEPTH;
      }
      if (first_code == CHECK_OK) first_code = CHECK_EDGE_SPAN;
    }
  }
  *bad = first_bad;
  return first_code;
}

/* Undirected edges traversed from the root: half the summed degree of the
   reached vertices (each undirected edge of the component is stored twice). */
int64_t oracle_traversed_edges(int64_t n, const int64_t* off, const int32_t* depth) {
  int64_t s = 0;
  for (int64_t v = 0; v < n; ++v)
    if (depth[v] >= 0) s += off[v + 1] - off[v];
  return s / 2;
}

/* Work of a level-synchronous traversal that takes direction dirs[L]
   (0 = top-down, 1 = bottom-up) at level L = 0 .. nlev-1, given the exact
   depths.  Per level, out[L*8 + k] receives
     k=0  n_f       vertices in the level-L frontier (depth == L)
     k=1  m_f       summed degree of the frontier
     k=2  scanned   bottom-up: vertices not yet visited (depth == -1 or
                    depth > L) of degree >= 1; top-down: 0
     k=3  checked   top-down: m_f (every edge of the frontier is examined);
                    bottom-up: for each scanned vertex, the 1-based position
                    in its adjacency list of the first neighbour of depth L,
                    else its degree
     k=4  found     vertices of depth L+1
     k=5  found_deg summed degree of those vertices
     k=6  unvisited_deg  summed degree of vertices with depth > L or -1
                    after the level (depth == -1 or depth > L+1)
     k=7  0 (reserved)
   Only depths and adjacency order matter, so these counts are exact for any
   correct implementation that follows the same direction schedule. */
int oracle_replay(int64_t n, const int64_t* off, const int32_t* idx, const int32_t* depth,
                  int32_t nlev, const int8_t* dirs, int64_t* out) {
  if (n < 1 || nlev < 0 || !out) return ORACLE_EINVAL;
  memset(out, 0, sizeof(int64_t) * 8 * (size_t)nlev);
  for (int32_t L = 0; L < nlev; ++L) {
    int64_t* o = out + 8 * (size_t)L;
    for (int64_t v = 0; v < n; ++v) {
      const int32_t dv = depth[v];
      const int64_t deg = off[v + 1] - off[v];
      if (dv == L) {
        o[0] += 1;
        o[1] += deg;
      }
      if (dv == L + 1) {
        o[4] += 1;
        o[5] += deg;
      }
      if (dv == -1 || dv > L + 1) o[6] += deg;
      if (dirs[L] == 1 && (dv == -1 || dv > L) && deg > 0) {
        o[2] += 1;
        int64_t pos = deg;
        for (int64_t e = off[v]; e < off[v + 1]; ++e) {
          if (depth[idx[e]] == L) {
            pos = e - off[v] + 1;
            break;
          }
        }
        o[3] += pos;
      }
    }
    if (dirs[L] == 0) o[3] = o[1];
  }
  return 0;
}
