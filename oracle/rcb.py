"""Nested element aggregates by recursive coordinate bisection (oracle side).

The paper forms the hierarchy top-down: the coarsest level is a split of the
mesh graph into 2^d connected parts of about equal size, each aggregate is split
again into 2^d parts, and so on until singletons (Section 4.1; Algorithm 5,
first step).  It uses METIS for the splits.  Here each 2^d-way split is ``b``
successive bisections of a recursive coordinate bisection (RCB) tree:

* a node with m >= 2 elements is split along the axis of largest centroid
  extent (max - min; ties go to the lowest axis);
* its elements are sorted by (coordinate, element id); the left child takes the
  first ceil(m/2), the right child the rest; nodes of size 1 are leaves;
* with D = ceil(log2 n_elem), the level-k aggregates (k >= 1) are the tree nodes
  at depth D - k*b, and a leaf above that depth is its own aggregate; level 0 is
  the singletons.  Aggregate ids follow the depth-first (left-to-right) order.

Reading: counting levels from the leaves (rather than strictly from the root as
the paper's top-down description does) keeps the level-1 aggregates at about
2^b elements whatever n_elem is; connectivity of the parts is not enforced.

The tree is built one depth at a time: at every depth all nodes are contiguous
segments of one permutation, sorted together by (segment, coordinate, id).
"""
import math

import numpy as np


def tree_depth(n_elem):
    return math.ceil(math.log2(n_elem)) if n_elem > 1 else 0


def rcb_segments(centroids, max_depth=None):
    """Yields (depth, perm, seg_start) for depth = 0..D: at each depth the tree
    nodes (leaves that stopped earlier included) are perm[seg_start[i]:seg_start[i+1]]."""
    cent = np.asarray(centroids, dtype=np.float64)
    ne, dim = cent.shape
    D = tree_depth(ne) if max_depth is None else max_depth
    perm = np.arange(ne, dtype=np.int64)
    start = np.array([0, ne], dtype=np.int64)
    for depth in range(D + 1):
        yield depth, perm, start
        if depth == D:
            break
        sizes = np.diff(start)
        seg = np.repeat(np.arange(len(sizes)), sizes)
        c = cent[perm]
        ext = np.maximum.reduceat(c, start[:-1], axis=0) - np.minimum.reduceat(c, start[:-1], axis=0)
        axis = np.argmax(ext, axis=1)  # first maximum -> lowest axis on ties
        key = c[np.arange(ne), axis[seg]]
        perm = perm[np.lexsort((perm, key, seg))]
        left = (sizes + 1) // 2
        right = sizes - left
        new_sizes = np.stack([left, right], axis=1).ravel()
        new_sizes = new_sizes[new_sizes > 0]
        start = np.concatenate([[0], np.cumsum(new_sizes)])


def rcb_hierarchy(centroids, n_levels, bisections):
    """Returns (aggs, leaf_order).

    aggs[k-1] for k = 1..n_levels-1 is an int32 array mapping each level-(k-1)
    unit (an element for k = 1, a level-(k-1) aggregate otherwise) to its
    level-k aggregate id.  leaf_order lists the elements in depth-first leaf
    order.
    """
    cent = np.asarray(centroids, dtype=np.float64)
    ne = len(cent)
    D = tree_depth(ne)
    want = {D - k * bisections: k for k in range(1, n_levels)}
    if n_levels > 1 and min(want) < 0:
        raise ValueError("too many levels for this mesh")
    elem_agg = {}
    leaf_order = None
    for depth, perm, start in rcb_segments(cent):
        if depth in want:
            a = np.empty(ne, dtype=np.int64)
            a[perm] = np.repeat(np.arange(len(start) - 1), np.diff(start))
            elem_agg[want[depth]] = a
        if depth == D:
            leaf_order = perm.copy()
    aggs = []
    prev = np.arange(ne)
    for k in range(1, n_levels):
        cur = elem_agg[k]
        m = np.empty(prev.max() + 1, dtype=np.int64)
        m[prev] = cur
        aggs.append(m.astype(np.int32))
        prev = cur
    return aggs, leaf_order


def agg_of_elem_levels(aggs):
    """Compose the per-level maps into element -> level-k aggregate maps."""
    out = []
    cur = np.arange(len(aggs[0]))
    for a in aggs:
        cur = a[cur]
        out.append(cur.astype(np.int32))
    return out


def replicate_top(aggs, leaf_order):
    """Algorithm 5's intra-element coarsening at the top level: level 0 is
    replicated, so the first coarse level's aggregates are the single elements
    (an h*-step, eq:sik).  They are numbered by depth-first leaf position, which
    keeps the children of every geometric aggregate consecutive; the geometric
    maps follow, the first one re-indexed by that position."""
    ne = len(leaf_order)
    pos = np.empty(ne, dtype=np.int32)
    pos[leaf_order] = np.arange(ne, dtype=np.int32)
    out = [pos]
    if aggs:
        out.append(np.asarray(aggs[0])[leaf_order].astype(np.int32))
        out.extend(aggs[1:])
    return out
