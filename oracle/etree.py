"""Elimination-tree utilities (oracle).

Test infrastructure only (see ``oracle/__init__``).

Paper, Sect. 3.2.1: the symbolic factorisation yields the pattern of the
factor and the elimination tree, whose root is the variable eliminated last;
ancestors of v are the vertices on the path from v to the root, the parent is
the first ancestor, children/leaves/descendants follow.  Sect. 3.2.2: the
factorisation visits the tree in a postorder (a topological order in which
every subtree is visited contiguously).  Sect. 3.3.1: computing the inverse
entry (i, j) only visits the path from j to the root (forward solve with the
sparse right-hand side e_j) and the path from the root to i (backward solve
restricted to component i) -- "pruning" the tree.

The parent of column j is the row index of the first off-diagonal non-zero
of column j of L (the standard definition, Liu 1990).  Indices are 0-based.
"""
from __future__ import annotations


def symbolic_cholesky(n, edges):
    """Pattern of L for a symmetric pattern, by plain elimination.

    ``edges`` holds off-diagonal pairs (i, j), i != j (either orientation).
    Returns ``struct[j]`` = sorted row indices i > j with L_ij != 0.
    Eliminating j connects all of its not-yet-eliminated neighbours.
    """
    adj = [set() for _ in range(n)]
    for i, j in edges:
        if i != j:
            adj[i].add(j)
            adj[j].add(i)
    struct = []
    for j in range(n):
        later = sorted(k for k in adj[j] if k > j)
        struct.append(later)
        for a in later:
            for c in later:
                if a != c:
                    adj[a].add(c)
    return struct


def etree_from_struct(struct):
    """parent[j] = min{i > j : L_ij != 0}, or -1 for a root."""
    return [s[0] if s else -1 for s in struct]


def children(parent):
    ch = [[] for _ in parent]
    for v, p in enumerate(parent):
        if p >= 0:
            ch[p].append(v)
    return ch


def roots(parent):
    return [v for v, p in enumerate(parent) if p < 0]


def leaves(parent):
    ch = children(parent)
    return [v for v in range(len(parent)) if not ch[v]]


def ancestors(parent, v):
    """Vertices on the path from v (exclusive) to the root (inclusive)."""
    out = []
    p = parent[v]
    while p >= 0:
        out.append(p)
        p = parent[p]
    return out


def descendants(parent, v):
    ch = children(parent)
    out, stack = [], list(ch[v])
    while stack:
        u = stack.pop()
        out.append(u)
        stack.extend(ch[u])
    return sorted(out)


def postorder(parent):
    """A postorder: children (by increasing index) before their parent,
    every subtree contiguous."""
    ch = children(parent)
    order = []

    def visit(v):
        for c in ch[v]:
            visit(c)
        order.append(v)

    for r in roots(parent):
        visit(r)
    return order


def is_postorder(order, parent):
    """True iff ``order`` is topological and visits each subtree contiguously."""
    n = len(parent)
    if sorted(order) != list(range(n)):
        return False
    pos = {v: k for k, v in enumerate(order)}
    for v, p in enumerate(parent):
        if p >= 0 and pos[p] < pos[v]:
            return False
    for v in range(n):
        sub = [v] + descendants(parent, v)
        ks = sorted(pos[u] for u in sub)
        if ks[-1] - ks[0] + 1 != len(ks) or ks[-1] != pos[v]:
            return False
    return True

