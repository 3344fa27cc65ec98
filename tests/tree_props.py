"""BFS-tree properties checked with plain torch tensor operations, on any
device, at any size (test infrastructure; independent of the HIP path).

For a symmetric CSR, a root and candidate (depth, parent) arrays, these
hold exactly when depth is the hop distance from the root (-1 where
unreachable) and parent is a BFS tree (Section 4's validation of a
traversal):

1. depth[root] == 0 and parent[root] == root;
2. depth[v] == -1 exactly when parent[v] == -1;
3. for every reached v != root: depth[parent[v]] == depth[v] - 1;
4. for every edge (u, v): u and v are both reached or both unreached, and
   |depth[u] - depth[v]| <= 1;
5. for every reached v != root: (v, parent[v]) is an edge.

(3) and (5) give every reached vertex a path of depth[v] edges to the root,
so depth is at least the distance; (4) along a shortest path gives at most
the distance, and confines reached vertices to the root's component.
"""
from __future__ import annotations


def bfs_tree_violations(off, idx, depth, parent, root: int, chunk: int = 1 << 27) -> list[str]:
    """off int64[n+1], idx int32/int64[m], depth/parent int32[n] torch
    tensors on one device.  Returns the names of violated properties."""
    import torch
    dev = depth.device
    n = depth.numel()
    bad: list[str] = []
    d = depth.long()
    p = parent.long()
    if int(d[root]) != 0 or int(p[root]) != root:
        bad.append("root")
    if bool(((d < 0) != (p < 0)).any()):
        bad.append("unreached-parent")
    reached = d >= 0
    nonroot = reached.clone()
    nonroot[root] = False
    pv = p[nonroot]
    if pv.numel():
        if bool(((pv < 0) | (pv >= n)).any()):
            bad.append("parent-range")
            pv = pv.clamp(0, n - 1)
        if bool((d[pv] != d[nonroot] - 1).any()):
            bad.append("parent-depth")
    hit = torch.zeros(n, dtype=torch.bool, device=dev)
    off_c = off.to(dev).long()
    r0 = 0
    while r0 < n:
        e0 = int(off_c[r0])
        # largest r1 with off[r1] - e0 <= chunk (at least one row)
        r1 = int(torch.searchsorted(off_c, torch.tensor([e0 + chunk], device=dev), right=True)) - 1
        r1 = max(r0 + 1, min(r1, n))
        e1 = int(off_c[r1])
        if e1 > e0:
            cnt = off_c[r0 + 1:r1 + 1] - off_c[r0:r1]
            src = torch.repeat_interleave(torch.arange(r0, r1, device=dev), cnt)
            dst = idx[e0:e1].to(dev).long()
            ds, dd = d[src], d[dst]
            if bool(((ds >= 0) != (dd >= 0)).any()):
                bad.append("edge-reach")
            if bool((((ds - dd).abs() > 1) & (ds >= 0)).any()):
                bad.append("edge-span")
            on_tree = p[src] == dst
            hit[src[on_tree]] = True
            del src, dst, ds, dd, on_tree
        r0 = r1
    if bool((nonroot & ~hit).any()):
        bad.append("parent-edge")
    return sorted(set(bad))


def bfs_depth_violations(off, idx, depth, root: int, chunk: int = 1 << 27) -> list[str]:
    """Depth labels alone (batched outputs carry no parents).  These hold
    exactly when depth is the hop distance from the root (-1 where
    unreachable):

    1. depth[root] == 0;
    2. for every edge (u, v): u and v are both reached or both unreached,
       and |depth[u] - depth[v]| <= 1;
    3. every reached v != root has a neighbour of depth depth[v] - 1.

    (3) gives every reached vertex a walk of depth[v] edges to a depth-0
    vertex, which by (3) again can only be the root, so depth is at least
    the distance; (2) along a shortest path gives at most the distance.
    Returns the names of violated properties."""
    import torch
    dev = depth.device
    n = depth.numel()
    bad: list[str] = []
    d = depth.long()
    if int(d[root]) != 0:
        bad.append("root")
    big = 1 << 40
    # smallest reached-neighbour depth of every vertex
    low = torch.full((n,), big, dtype=torch.long, device=dev)
    off_c = off.to(dev).long()
    r0 = 0
    while r0 < n:
        e0 = int(off_c[r0])
        r1 = int(torch.searchsorted(off_c, torch.tensor([e0 + chunk], device=dev), right=True)) - 1
        r1 = max(r0 + 1, min(r1, n))
        e1 = int(off_c[r1])
        if e1 > e0:
            cnt = off_c[r0 + 1:r1 + 1] - off_c[r0:r1]
            src = torch.repeat_interleave(torch.arange(r0, r1, device=dev), cnt)
            dst = idx[e0:e1].to(dev).long()
            ds, dd = d[src], d[dst]
            if bool(((ds >= 0) != (dd >= 0)).any()):
                bad.append("edge-reach")
            if bool((((ds - dd).abs() > 1) & (ds >= 0)).any()):
                bad.append("edge-span")
            low.scatter_reduce_(0, src, torch.where(dd >= 0, dd, torch.full_like(dd, big)), reduce="amin")
            del src, dst, ds, dd
        r0 = r1
    nonroot = d >= 0
    nonroot[root] = False
    if bool((low[nonroot] != d[nonroot] - 1).any()):
        bad.append("no-parent")
    return sorted(set(bad))
