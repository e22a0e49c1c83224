"""Brute-force contraction-path optimum (oracle, test infrastructure).

Supplement, "Heuristic algorithm to search for the optimal tensor contraction
path": a linear path i_1 -> ... -> i_N contracts C^{i_1} with C^{i_2}, the
result with C^{i_3}, and so on.  Its score is S_{i_1} = 0 and
S_{i_1..i_{m+1}} = S_{i_1..i_m} + Cost(C^{i_1..i_m}, C^{i_{m+1}}), and the
optimal score is the minimum of S over all N! orders.

The paper leaves Cost undefined; the reading used throughout is the number of
complex multiply-adds of the pairwise contraction, i.e. the product of the
dimensions of every bond carried by either operand (the union of their legs).
The open legs of the contracted set are the bonds with exactly one endpoint in
the set.
"""

import itertools
import math


def _legs(n, edges):
    legs = [[] for _ in range(n)]
    for e, (u, v) in enumerate(edges):
        legs[u].append(e)
        legs[v].append(e)
    return legs


def cost(open_set, site_legs, dims):
    return math.prod(dims[e] for e in (set(open_set) | set(site_legs)))


def score(order, n, edges, dims):
    """(score, largest intermediate size) of a linear path."""
    legs = _legs(n, edges)
    cur = set(legs[order[0]])
    total, biggest = 0, math.prod(dims[e] for e in cur)
    for j in order[1:]:
        total += cost(cur, legs[j], dims)
        cur = cur ^ set(legs[j])
        biggest = max(biggest, math.prod(dims[e] for e in cur))
    return total, biggest


def brute_force(n, edges, dims):
    """Minimum score over all N! linear orders, and one order reaching it."""
    if n > 9:
        raise ValueError("brute force is limited to N <= 9")
    best, arg = None, None
    for order in itertools.permutations(range(n)):
        s, _ = score(order, n, edges, dims)
        if best is None or s < best:
            best, arg = s, order
    return best, list(arg)


def subset_dp(n, edges, dims):
    """The same optimum through the optimal-substructure recursion of the
    supplement's Eq. (optscore): S*(set) = min over the last element j of
    S*(set - j) + Cost(C^{set - j}, C^j), with S*({i}) = 0."""
    if n > 18:
        raise ValueError("subset DP is limited to N <= 18")
    legs = _legs(n, edges)
    full = (1 << n) - 1
    open_of = {}

    def open_legs(mask):
        if mask not in open_of:
            cnt = {}
            for q in range(n):
                if mask >> q & 1:
                    for e in legs[q]:
                        cnt[e] = cnt.get(e, 0) + 1
            open_of[mask] = frozenset(e for e, c in cnt.items() if c == 1)
        return open_of[mask]

    best = {1 << q: 0 for q in range(n)}
    for size in range(2, n + 1):
        for combo in itertools.combinations(range(n), size):
            mask = sum(1 << q for q in combo)
            val = None
            for j in combo:
                prev = mask & ~(1 << j)
                c = best[prev] + cost(open_legs(prev), legs[j], dims)
                if val is None or c < val:
                    val = c
            best[mask] = val
    return best[full]


def tree_score(order, windows, n, edges, dims):
    """(score, largest main-path intermediate, largest branch tensor) of a
    linear order relaxed into a main path with side branches ("several main
    paths", which the supplement leaves open beside its single main path).

    Each window (a, b) of positions of ``order`` (a >= 1, windows disjoint)
    is contracted by its own linear path in the order's sequence; the main
    path takes the remaining positions in sequence and absorbs a branch's
    tensor whole just before it reaches a position >= b (branches whose
    window reaches the end are absorbed after the last main site, by
    increasing b).  Every pairwise step costs Cost() above."""
    legs = _legs(n, edges)
    size = lambda s: math.prod(dims[e] for e in s)
    inwin = {}
    for w, (a, b) in enumerate(windows):
        for i in range(a, b):
            inwin[i] = w
    total, biggest, branch_biggest = 0, 0, 0

    def branch(w):
        nonlocal total, branch_biggest
        a, b = windows[w]
        t = set(legs[order[a]])
        branch_biggest = max(branch_biggest, size(t))
        for i in range(a + 1, b):
            total += cost(t, legs[order[i]], dims)
            t = t ^ set(legs[order[i]])
            branch_biggest = max(branch_biggest, size(t))
        return t

    pending = sorted(range(len(windows)), key=lambda w: windows[w][1])
    cur = None
    for i, q in enumerate(order):
        if i in inwin:
            continue
        while cur is not None and pending and windows[pending[0]][1] <= i:
            x = branch(pending.pop(0))
            total += cost(cur, x, dims)
            cur = cur ^ x
            biggest = max(biggest, size(cur))
        if cur is None:
            cur = set(legs[q])
            biggest = size(cur)
        else:
            total += cost(cur, legs[q], dims)
            cur = cur ^ set(legs[q])
            biggest = max(biggest, size(cur))
    while pending:
        x = branch(pending.pop(0))
        total += cost(cur, x, dims)
        cur = cur ^ x
        biggest = max(biggest, size(cur))
    return total, biggest, branch_biggest


def tree_optimum(n, edges, dims):
    """Least summed Cost over every binary contraction tree (any pairing of
    any two disjoint groups at each step), by recursion over subsets: the
    cost of a group is the best split into two non-empty parts plus the
    Cost of contracting their two tensors.  A lower bound for linear paths
    and for main paths with branches alike."""
    if n > 12:
        raise ValueError("tree optimum is limited to N <= 12")
    legs = _legs(n, edges)
    open_of = {}

    def open_legs(mask):
        if mask not in open_of:
            cnt = {}
            for q in range(n):
                if mask >> q & 1:
                    for e in legs[q]:
                        cnt[e] = cnt.get(e, 0) + 1
            open_of[mask] = frozenset(e for e, c in cnt.items() if c == 1)
        return open_of[mask]

    best = {1 << q: 0 for q in range(n)}
    for size_ in range(2, n + 1):
        for combo in itertools.combinations(range(n), size_):
            mask = sum(1 << q for q in combo)
            val = None
            sub = (mask - 1) & mask
            while sub:
                rest = mask ^ sub
                if sub < rest:   # each unordered split once
                    c = best[sub] + best[rest] + cost(open_legs(sub), open_legs(rest), dims)
                    if val is None or c < val:
                        val = c
                sub = (sub - 1) & mask
            best[mask] = val
    return best[(1 << n) - 1]


def brute_force_bounded(n, edges, dims, max_size):
    """Minimum score over the linear orders whose every intermediate (the
    first tensor included) has at most ``max_size`` elements, and one order
    reaching it; (None, None) when no order fits.  The size-aware bound that
    can accompany the supplement's rank bound on intermediates."""
    if n > 9:
        raise ValueError("brute force is limited to N <= 9")
    best, arg = None, None
    for order in itertools.permutations(range(n)):
        s, big = score(order, n, edges, dims)
        if big <= max_size and (best is None or s < best):
            best, arg = s, order
    return best, (list(arg) if arg is not None else None)
