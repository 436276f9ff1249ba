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


def round_f16(a):
    """Nearest binary16 value of each FP64 entry (numpy converts double to
    half directly, ties to even)."""
    return np.asarray(a, np.float64).astype(np.float16).astype(np.float64)


def round_bf16(a):
    """Nearest bfloat16 value of each FP64 entry, ties to even.

    torch converts double to bfloat16 through float32, which can round twice.
    Going to float32 with round-to-odd first (truncate toward zero, then set
    the last bit when the value was inexact) keeps the final round-to-nearest
    correct, because float32 carries more than two bits beyond bfloat16's.
    """
    import torch
    a = np.asarray(a, np.float64)
    f = a.astype(np.float32)
    over = np.abs(f.astype(np.float64)) > np.abs(a)
    f = np.where(over, np.nextafter(f, np.float32(0)), f).astype(np.float32)
    inexact = f.astype(np.float64) != a
    f = (f.view(np.uint32) | inexact.astype(np.uint32)).view(np.float32)
    return torch.from_numpy(np.ascontiguousarray(f)).to(torch.bfloat16).to(torch.float64).numpy().reshape(a.shape)


def _has_nb(H, W):
    yy, xx = np.mgrid[0:H, 0:W]
    return [xx > 0, xx < W - 1, yy > 0, yy < H - 1], yy, xx


def checkerboard_bp(cost, lam, tau, iters, init=None, rnd=None):
    """Checkerboard min-sum BP with messages by the O(L^2) min-plus definition.

    Half-sweep t updates the pixels with (x + y + t) even; each sends to every
    in-grid neighbour q the message min_g h(g) + lam*min(|f-g|, tau), minus its
    minimum, where h is the cost plus the incoming messages except q's (added
    in slot order).  `rnd`, if given, is applied to every sent message as it
    is stored.  Returns the message array [4][L][H][W] (slot k = received from
    side k: left, right, up, down).
    """
    L, H, W = cost.shape
    V = vpair(lam, tau, L)
    m = np.zeros((4, L, H, W)) if init is None else np.array(init, dtype=np.float64)
    inb, yy, xx = _has_nb(H, W)
    step = ((0, -1, 0), (1, 1, 0), (2, 0, -1), (3, 0, 1))   # (side, dx, dy)
    for t in range(iters):
        act = (xx + yy + t) % 2 == 0
        for q, dx, dy in step:
            ys, xs = np.nonzero(act & inb[q])
            if ys.size == 0:
                continue
            h = cost[:, ys, xs].copy()
            for k in range(4):
                if k != q:
                    h = h + np.where(inb[k][ys, xs], m[k][:, ys, xs], 0.0)
            msg = np.min(h[None, :, :] + V[:, :, None], axis=1)
            msg = msg - msg.min(axis=0, keepdims=True)
            if rnd is not None:
                msg = rnd(msg)
            m[q ^ 1][:, ys + dy, xs + dx] = msg
    return m


def hierarchical_bp(cost, levels, iters, lam, tau, rnd=None):
    """Coarse-to-fine checkerboard BP.  Level costs are sums of the existing
    children; the coarsest level starts from zero and keeps full precision;
    every finer level starts from its parent's final messages at (x/2, y/2),
    stored through `rnd`, and stores every sent message through `rnd`.
    Returns the finest level's messages with out-of-grid slots zeroed."""
    costs = [np.asarray(cost, np.float64)]
    for _ in range(1, levels):
        c = costs[-1]
        L, H, W = c.shape
        pad = np.zeros((L, H + H % 2, W + W % 2))
        pad[:, :H, :W] = c
        costs.append(pad.reshape(L, (H + 1) // 2, 2, (W + 1) // 2, 2).sum(axis=(2, 4)))
    m = None
    for lev in range(levels - 1, -1, -1):
        L, H, W = costs[lev].shape
        r = None if lev == levels - 1 else rnd
        init = None
        if m is not None:
            init = m[:, :, np.arange(H)[:, None] // 2, np.arange(W)[None, :] // 2]
            if r is not None:
                init = r(init)
        m = checkerboard_bp(costs[lev], lam, tau, iters, init, r)
    inb, _, _ = _has_nb(*costs[0].shape[1:])
    for k in range(4):
        m[k][:, ~inb[k]] = 0.0
    return m


def autograd_soft_bp(cost, lam, tau, iters, temperature):
    """Single-level checkerboard BP with a soft-argmin readout, written with
    torch FP64 operations so that autograd gives its derivative.

    The two-pass transform is spelled out with torch.where so that every
    comparison takes the documented branch on ties: the forward pass keeps
    h(f) when h(f) <= a(f-1) + lam, the backward pass takes a(f+1) + lam only
    when strictly smaller, truncation applies only when strictly smaller, and
    the normaliser is h at its lowest minimiser.  Arguments are torch tensors
    (cost [L][H][W], scalar lam and tau).  Returns the soft disparity [H][W].
    """
    import torch
    L, H, W = cost.shape
    yy, xx = torch.meshgrid(torch.arange(H), torch.arange(W), indexing="ij")
    inb = [xx > 0, xx < W - 1, yy > 0, yy < H - 1]
    m = torch.zeros((4, L, H, W), dtype=torch.float64)
    step = ((0, -1, 0), (1, 1, 0), (2, 0, -1), (3, 0, 1))
    for t in range(iters):
        act = (xx + yy + t) % 2 == 0
        new = m.clone()
        for q, dx, dy in step:
            ys, xs = torch.nonzero(act & inb[q], as_tuple=True)
            if ys.numel() == 0:
                continue
            h = cost[:, ys, xs]
            for k in range(4):
                if k != q:
                    h = h + torch.where(inb[k][ys, xs], m[k][:, ys, xs], torch.zeros((), dtype=torch.float64))
            a = [h[0]]
            for f in range(1, L):
                v = a[-1] + lam
                a.append(torch.where(h[f] <= v, h[f], v))
            b = [None] * L
            b[L - 1] = a[L - 1]
            for f in range(L - 2, -1, -1):
                v = b[f + 1] + lam
                b[f] = torch.where(v < a[f], v, a[f])
            b = torch.stack(b)
            gmin = torch.argmin(h, dim=0)        # first minimiser on ties
            hmin = torch.gather(h, 0, gmin[None])[0]
            cap = hmin + lam * tau
            msg = torch.where(cap < b, cap, b) - hmin
            new[q ^ 1][:, ys + dy, xs + dx] = msg
        m = new
    zero = torch.zeros((), dtype=torch.float64)
    bel = cost + sum(torch.where(inb[k], m[k], zero) for k in range(4))
    p = torch.softmax(-bel / temperature, dim=0)
    return (torch.arange(L, dtype=torch.float64)[:, None, None] * p).sum(dim=0)
