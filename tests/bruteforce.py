"""Brute-force structural clustering for tiny graphs, written directly from
GPUSCAN++ Section 2.1 (Defs 2.1-2.7).  Independent of the oracle: it uses
Python sets, a 60-digit decimal square root for sigma (Eq. 1) instead of the
oracle's squared integer comparison, explicit reachability closures
(Def 2.5) and an explicit check of the two cluster conditions (Def 2.6).
"""
from __future__ import annotations

from decimal import Decimal, localcontext
from itertools import combinations

UNCLASSIFIED, CORE, BORDER = 0, 1, 2


def closed_sets(n, edges):
    nbr = [set() for _ in range(n)]
    for u, v in edges:
        nbr[u].add(v)
        nbr[v].add(u)
    return [nbr[v] | {v} for v in range(n)], nbr


def sigma_at_least(Nu, Nv, p, q):
    """sigma(u, v) >= p/q with sigma = |N[u]&N[v]| / sqrt(|N[u]||N[v]|) (Eq. 1).

    Equality is only possible when |N[u]||N[v]| is a perfect square; then the
    decimal square root is exact and both sides are the same correctly rounded
    quotient.  Otherwise the two sides differ by far more than 1e-50."""
    with localcontext() as ctx:
        ctx.prec = 60
        c = Decimal(len(Nu & Nv))
        s = c / (Decimal(len(Nu)) * Decimal(len(Nv))).sqrt()
        return s >= Decimal(p) / Decimal(q)


def brute_scan(n, edges, p, q, mu, literal_subsets=False):
    """Returns (labels, roles, clusters, hub) with clusters as a sorted list of
    frozensets; labels are the minimum core id of the cluster, borders take the
    minimum label among the clusters that contain them."""
    N, nbr = closed_sets(n, edges)
    # Def 2.3: N_eps[u] = {v in N[u] : sigma(u, v) >= eps}; u itself is in it.
    Neps = [{v for v in N[u] if sigma_at_least(N[u], N[v], p, q)} for u in range(n)]
    for u in range(n):
        assert u in Neps[u]
    # Def 2.4
    core = [len(Neps[u]) >= mu for u in range(n)]

    # Def 2.5: v is reachable from u when a chain u = v1, ..., vl = v has cores
    # v1..v_{l-1} and v_{i+1} in N_eps[v_i].
    def reach(u):
        seen = {u}
        stack = [u]
        while stack:
            x = stack.pop()
            if not core[x]:
                continue
            for y in Neps[x]:
                if y not in seen:
                    seen.add(y)
                    stack.append(y)
        return seen

    R = [reach(u) for u in range(n)]

    def connected(C):
        return all(any(a in R[w] and b in R[w] for w in C) for a in C for b in C)

    def maximal(C):
        return all(R[w] <= C for w in C if core[w])

    # Def 2.6, read with the usual requirement that a cluster holds a core
    # (otherwise every single non-core vertex would satisfy it on its own).
    cands = {frozenset(R[u]) for u in range(n) if core[u]}
    for C in cands:
        assert connected(C) and maximal(C)
    if literal_subsets:
        found = set()
        for k in range(1, n + 1):
            for S in combinations(range(n), k):
                C = frozenset(S)
                if any(core[w] for w in C) and connected(C) and maximal(C):
                    found.add(C)
        assert found == cands, (found, cands)
    clusters = sorted(cands, key=lambda C: min(w for w in C if core[w]))
    label_of = {C: min(w for w in C if core[w]) for C in clusters}
    labels, roles = [-1] * n, [UNCLASSIFIED] * n
    for v in range(n):
        holding = [label_of[C] for C in clusters if v in C]
        if core[v]:
            assert len(holding) == 1  # cores belong to exactly one cluster
            roles[v], labels[v] = CORE, holding[0]
        elif holding:
            roles[v], labels[v] = BORDER, min(holding)
    # Def 2.7: an unclustered vertex is a hub if its neighbours lie in two or
    # more clusters (membership over all clusters, borders may be in several).
    hub = [False] * n
    for u in range(n):
        if roles[u] == UNCLASSIFIED:
            cl = {label_of[C] for C in clusters for w in nbr[u] if w in C}
            hub[u] = len(cl) >= 2
    return labels, roles, clusters, hub


def closed_count(n, edges, u, v):
    N, _ = closed_sets(n, edges)
    return len(N[u] & N[v])
