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
