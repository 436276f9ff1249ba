"""Independent reference computations used to pin the oracle.

None of these share code with the oracle: they are textbook dynamic programs,
exhaustive enumeration and a synchronous (Jacobi) message schedule written
with numpy broadcasting and the O(L^2) min-plus definition of a message.
"""
from __future__ import annotations

import itertools

import numpy as np


def vpair(lam, tau, L):
    """Pairwise cost matrix V[f, g] = lam * min(|f - g|, tau)."""
    f = np.arange(L)
    return lam * np.minimum(np.abs(f[:, None] - f[None, :]), tau)


def edges_of(W, H, mask=None):
    """Undirected edges ((x, y), (x2, y2)) of a 4-connected grid, optionally masked."""
    out = []
    for y in range(H):
        for x in range(W):
            if x + 1 < W and (mask is None or mask[y, x] & 1):
                out.append(((x, y), (x + 1, y)))
            if y + 1 < H and (mask is None or mask[y, x] & 2):
                out.append(((x, y), (x, y + 1)))
    return out


def energy(labels, cost, edges, V):
    """Sum of data terms plus pairwise terms of a labelling labels[y, x]."""
    L, H, W = cost.shape
    e = sum(cost[labels[y, x], y, x] for y in range(H) for x in range(W))
    for (a, b) in edges:
        e += V[labels[a[1], a[0]], labels[b[1], b[0]]]
    return e


def enumerate_min_marginals(cost, edges, V):
    """Exact min-marginals mm[f, y, x] by exhaustive enumeration (tiny grids)."""
    L, H, W = cost.shape
    n = H * W
    mm = np.full((L, H, W), np.inf)
    best_e, best_lab = np.inf, None
    for lab in itertools.product(range(L), repeat=n):
        labels = np.array(lab).reshape(H, W)
        e = energy(labels, cost, edges, V)
        if e < best_e:
            best_e, best_lab = e, labels
        for y in range(H):
            for x in range(W):
                f = labels[y, x]
                if e < mm[f, y, x]:
                    mm[f, y, x] = e
    return mm, best_e, best_lab


def chain_min_marginals(unary, V):
    """Forward-backward Viterbi on a chain: unary [N][L] -> min-marginals [N][L]."""
    N, L = unary.shape
    fwd = np.zeros((N, L))
    bwd = np.zeros((N, L))
    for i in range(1, N):
        fwd[i] = np.min((fwd[i - 1] + unary[i - 1])[:, None] + V, axis=0)
    for i in range(N - 2, -1, -1):
        bwd[i] = np.min((bwd[i + 1] + unary[i + 1])[:, None] + V, axis=0)
    return unary + fwd + bwd


def tree_min_marginals(cost, edges, V):
    """Min-marginals on a tree (any edge set without cycles) by two-pass DP."""
    L, H, W = cost.shape
    nodes = [(x, y) for y in range(H) for x in range(W)]
    adj = {p: [] for p in nodes}
    for a, b in edges:
        adj[a].append(b)
        adj[b].append(a)
    msg = {}

    def unary(p):
        return cost[:, p[1], p[0]]

    # Root every component, collect messages leaves-to-root then root-to-leaves.
    seen = set()
    for root in nodes:
        if root in seen:
            continue
        order, parent = [], {root: None}
        stack = [root]
        while stack:
            p = stack.pop()
            seen.add(p)
            order.append(p)
            for q in adj[p]:
                if q not in parent:
                    parent[q] = p
                    stack.append(q)
        for p in reversed(order):
            par = parent[p]
            if par is None:
                continue
            inc = sum((msg[(c, p)] for c in adj[p] if c != par), np.zeros(L))
            msg[(p, par)] = np.min((unary(p) + inc)[:, None] + V, axis=0)
        for p in order:
            for c in adj[p]:
                if parent.get(c) != p:
                    continue
                inc = sum((msg[(o, p)] for o in adj[p] if o != c), np.zeros(L))
                msg[(p, c)] = np.min((unary(p) + inc)[:, None] + V, axis=0)
    mm = np.empty((L, H, W))
    for p in nodes:
        mm[:, p[1], p[0]] = unary(p) + sum((msg[(q, p)] for q in adj[p]), np.zeros(L))
    return mm


def synchronous_bp(cost, lam, tau, iters):
    """Jacobi-schedule min-sum BP on the full 4-connected grid.

    Every pixel sends to every neighbour at every iteration, using the
    messages of the previous iteration; messages are normalised to minimum 0.
    Returns a list M[s] (s = 0..iters) of arrays [4][L][H][W] holding the
    message each pixel received from its neighbour on side k (0 left,
    1 right, 2 up, 3 down).
    """
    L, H, W = cost.shape
    V = vpair(lam, tau, L)
    M = [np.zeros((4, L, H, W))]
    for _ in range(iters):
        prev = M[-1]
        total = cost + prev.sum(axis=0)
        new = np.zeros_like(prev)
        # Message sent to the right neighbour: excludes what came from the right.
        for k_recv, k_excl, sl_src, sl_dst in (
            (0, 1, (slice(None), slice(0, W - 1)), (slice(None), slice(1, W))),   # to right
            (1, 0, (slice(None), slice(1, W)), (slice(None), slice(0, W - 1))),   # to left
            (2, 3, (slice(0, H - 1), slice(None)), (slice(1, H), slice(None))),   # to down
            (3, 2, (slice(1, H), slice(None)), (slice(0, H - 1), slice(None))),   # to up
        ):
            h = (total - prev[k_excl])[:, sl_src[0], sl_src[1]]          # [L][h][w]
            m = np.min(h[:, None, :, :] + V[:, :, None, None], axis=0)   # min over g -> [f][h][w]
            m = m - m.min(axis=0, keepdims=True)
            new[k_recv][:, sl_dst[0], sl_dst[1]] = m
        M.append(new)
    return M
