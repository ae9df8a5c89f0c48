"""Brute-force restatement of each step with explicit Python sets.

Test infrastructure: every function here works on tiny hypergraphs only and is
written directly from the definitions (Sec. II-A, Eq. 1-3, Sec. III-A, IV-A/B)
without the algebraic shortcuts of the oracle (inclusion-exclusion unions,
loss split over indicators, local connectivity deltas, recursive matching).

A level is given as a list of hedges, each a dict {pin: is_dst}, a weight list
and a node-size list.
"""
from __future__ import annotations

import itertools


class Lvl:
    def __init__(self, n, hedges, w, size):
        self.n = n
        self.hedges = hedges  # list of {pin: bool is_dst}
        self.w = list(w)
        self.size = list(size)

    def I(self, v):
        return {e for e, h in enumerate(self.hedges) if v in h}

    def inb(self, v):
        return {e for e, h in enumerate(self.hedges) if h.get(v, False)}


def level_from_input(g, role=0):
    """role: the pins whose hedges count toward Delta — 0 destinations
    (inbound), 1 sources (outbound), 2 every pin (incident)."""
    hedges = []
    for e in range(g.n_hedges):
        b, en = int(g.hedge_off[e]), int(g.hedge_off[e + 1])
        ns = int(g.n_src[e])
        h = {}
        for j in range(b, en):
            dst = (j - b) >= ns
            h[int(g.pins[j])] = dst if role == 0 else (not dst if role == 1 else True)
        hedges.append(h)
    return Lvl(g.n_nodes, hedges, [int(x) for x in g.hedge_w], [int(x) for x in g.node_w])


def level_from_trace(hoff, hpin, size, w):
    hedges = []
    for e in range(len(hoff) - 1):
        h = {}
        for j in range(int(hoff[e]), int(hoff[e + 1])):
            x = int(hpin[j]) & 0xFFFFFFFF
            h[x & 0x7FFFFFFF] = bool(x >> 31)
        hedges.append(h)
    return Lvl(len(size), hedges, w, [int(s) for s in size])


def conn(L: Lvl, rho) -> int:
    """Eq. 1 (a hedge without pins contributes nothing)."""
    tot = 0
    for e, h in enumerate(L.hedges):
        parts = {rho[v] for v in h}
        if parts:
            tot += L.w[e] * (len(parts) - 1)
    return tot


def rate_select(L: Lvl, omega, delta):
    """pair/score of Sec. III-A with Eq. 2 and a literal union for Delta."""
    pair, score = [-1] * L.n, [0] * L.n
    for n in range(L.n):
        In = L.I(n)
        nbrs = set()
        for e in In:
            nbrs |= set(L.hedges[e])
        nbrs.discard(n)
        best, bh = -1, None
        for m in sorted(nbrs):
            hist = sum(L.w[e] for e in In if m in L.hedges[e])
            ok = L.size[n] + L.size[m] <= omega and len(L.inb(n) | L.inb(m)) <= delta
            if ok and (bh is None or hist > bh or (hist == bh and m > best)):
                best, bh = m, hist
        pair[n] = best
        score[n] = bh if best >= 0 else 0
    return pair, score


def match_procedural(pair, score):
    """The two traversals of Sec. III-B, simulated sequentially.

    1) every proposing node places (score, id) on its candidate with a max
       (a free candidate takes any proposal);
    2) two-cycles are roots and match each other;
    3) walking from the roots towards the leaves, a node locks
       match(n) = pair(n) iff it still sees match(pair(n)) = n.
    """
    N = len(pair)
    match = list(range(N))
    for n in range(N):
        p = pair[n]
        if p < 0:
            continue
        cur = match[p]
        if cur == p or (score[n], n) > (score[cur], cur):
            match[p] = n
    roots = []
    for n in range(N):
        p = pair[n]
        if p < 0:
            roots.append(n)
        elif pair[p] == n:
            roots.append(n)
            match[n] = p
    children = {v: [] for v in range(N)}
    for n in range(N):
        p = pair[n]
        if p >= 0 and pair[p] != n:
            children[p].append(n)
    order = []
    frontier = list(roots)
    seen = set(frontier)
    while frontier:
        nxt = []
        for v in frontier:
            for c in children[v]:
                if c not in seen:
                    seen.add(c)
                    order.append(c)
                    nxt.append(c)
        frontier = nxt
    assert len(seen) == N, "pairing graph must be a pseudo-forest with 2-cycles"
    for n in order:
        p = pair[n]
        if match[p] == n:
            match[n] = p
    return match


def contract(L: Lvl, match):
    """Coarse level: clusters {n, match(n)}, numbered by smaller member."""
    reps = sorted({min(n, match[n]) for n in range(L.n)})
    idx = {r: i for i, r in enumerate(reps)}
    gamma = [idx[min(n, match[n])] for n in range(L.n)]
    size = [0] * len(reps)
    for v in range(L.n):
        size[gamma[v]] += L.size[v]
    hedges = []
    for h in L.hedges:
        c = {}
        for v, d in h.items():
            c[gamma[v]] = c.get(gamma[v], False) or d
        hedges.append(c)
    return gamma, Lvl(len(reps), hedges, L.w, size)


def pins(L: Lvl, rho, p, e):
    return sum(1 for v in L.hedges[e] if rho[v] == p)


def part_valid_all(L: Lvl, rho, n_parts, omega, delta):
    """Number of parts violating size <= Omega or |U in(n)| <= Delta."""
    bad = 0
    for p in range(n_parts):
        members = [v for v in range(L.n) if rho[v] == p]
        sz = sum(L.size[v] for v in members)
        inb = set()
        for v in members:
            inb |= L.inb(v)
        if sz > omega or len(inb) > delta:
            bad += 1
    return bad


def propose(L: Lvl, rho, n_parts, omega):
    """Eq. 3 over every part p != rho(n) that can take n; gain > 0 kept."""
    psize = [0] * n_parts
    for v in range(L.n):
        psize[rho[v]] += L.size[v]
    dest, gain = [-1] * L.n, [0] * L.n
    for n in range(L.n):
        ps = rho[n]
        In = L.I(n)
        saving = sum(L.w[e] for e in In if pins(L, rho, ps, e) == 1)
        bp, bg = -1, None
        for p in range(n_parts):
            if p == ps or psize[p] + L.size[n] > omega:
                continue
            loss = sum(L.w[e] for e in In if pins(L, rho, p, e) == 0)
            g = saving - loss
            if bg is None or g > bg or (g == bg and p > bp):
                bp, bg = p, g
        if bp >= 0 and bg > 0:
            dest[n], gain[n] = bp, bg
    return dest, gain


def refine_round(L: Lvl, rho, n_parts, omega, delta):
    """One round of Sec. IV-A with from-scratch Conn and validity per prefix."""
    dest, gain = propose(L, rho, n_parts, omega)
    seq = sorted([n for n in range(L.n) if dest[n] >= 0], key=lambda n: (gain[n], n), reverse=True)
    state = list(rho)
    c0 = conn(L, state)
    gp, G, viol = [0], [0], [part_valid_all(L, state, n_parts, omega, delta)]
    prev = c0
    for n in seq:
        state[n] = dest[n]
        c = conn(L, state)
        gp.append(prev - c)
        G.append(c0 - c)
        viol.append(part_valid_all(L, state, n_parts, omega, delta))
        prev = c
    istar = None
    for i in range(len(seq) + 1):
        if viol[i] == 0 and (istar is None or G[i] >= G[istar]):
            istar = i
    applied = istar is not None and G[istar] > 0
    out = list(rho)
    if applied:
        for n in seq[:istar]:
            out[n] = dest[n]
    return dict(dest=dest, gain=gain, seq=seq, gp=gp, G=G, viol=viol, istar=istar, applied=applied, rho=out)


def set_partitions(items):
    """All set partitions of a list (Bell-number many)."""
    if not items:
        yield []
        return
    first, rest = items[0], items[1:]
    for sub in set_partitions(rest):
        for i in range(len(sub)):
            yield sub[:i] + [[first] + sub[i]] + sub[i + 1:]
        yield [[first]] + sub


def exhaustive_optimum(L: Lvl, omega, delta):
    """Minimum Eq. 1 over every valid partition (tiny n only)."""
    best = None
    for parts in set_partitions(list(range(L.n))):
        rho = [0] * L.n
        ok = True
        for i, p in enumerate(parts):
            sz = 0
            inb = set()
            for v in p:
                rho[v] = i
                sz += L.size[v]
                inb |= L.inb(v)
            if sz > omega or len(inb) > delta:
                ok = False
                break
        if not ok:
            continue
        c = conn(L, rho)
        if best is None or c < best:
            best = c
    return best


def random_tiny(rng, n, n_hedges, max_pins, wmax=5, node_wmax=1):
    """A small random directed hypergraph as (n, [(src, dst)], w, node_w)."""
    hedges = []
    for _ in range(n_hedges):
        k = rng.randint(1, min(max_pins, n))
        pins = rng.sample(range(n), k)
        ns = rng.randint(0, k)
        hedges.append((pins[:ns], pins[ns:]))
    w = [rng.randint(1, wmax) for _ in range(n_hedges)]
    nw = [rng.randint(1, node_wmax) for _ in range(n)]
    return hedges, w, nw


def combos(n):
    return itertools.combinations(range(n), 2)


# ---------------------------------------------------------------------------
# learned merge proposal (extension; the definitions are those of the oracle
# header), restated with explicit sets
# ---------------------------------------------------------------------------
def qlog_closed(f: int) -> int:
    """8 floor(log2(f+1)) + floor(8 (v / 2^e - 1)), v = f+1, e = floor(log2 v), capped at 255."""
    v = f + 1
    e = v.bit_length() - 1
    return min(255, 8 * e + ((v - (1 << e)) * 8) // (1 << e))


def candidates(L: Lvl, omega, delta, K):
    """topK(n) by (hist, id) among valid m, and the symmetric sets
    C(n) = topK(n) u {m : n in topK(m)} as {m: (hist, c)}."""
    top = []
    for n in range(L.n):
        In = L.I(n)
        nbrs = set()
        for e in In:
            nbrs |= set(L.hedges[e])
        nbrs.discard(n)
        valid = []
        for m in nbrs:
            hist = sum(L.w[e] for e in In if m in L.hedges[e])
            c = len(L.inb(n) & L.inb(m))
            if L.size[n] + L.size[m] <= omega and len(L.inb(n) | L.inb(m)) <= delta:
                valid.append((hist, m, c))
        valid.sort(key=lambda t: (t[0], t[1]), reverse=True)
        top.append(valid[:K])
    C = [dict() for _ in range(L.n)]
    for n in range(L.n):
        for hist, m, c in top[n]:
            C[n][m] = (hist, c)
            C[m][n] = (hist, c)
    return top, C


def pair_features(L: Lvl, level, omega, delta, n, m, hist, c):
    a, b = min(n, m), max(n, m)
    uni = len(L.inb(a) | L.inb(b))
    f = [hist, c, L.size[a], L.size[b], uni, len(L.I(a)), len(L.I(b)), level, omega - L.size[a] - L.size[b],
         delta - uni]
    return [qlog_closed(x) for x in f] + [0] * 6


def pairing_edges(pair, score):
    """The edges {n, pair(n)} of a pairing pseudo-forest with their weight
    score(n) (a 2-cycle gives one edge)."""
    edges = {}
    for n, p in enumerate(pair):
        if p >= 0:
            key = (min(n, p), max(n, p))
            edges[key] = int(score[n])
    return edges


def max_weight_matching(pair, score):
    """Weight of a maximum-weight matching over the pairing edges, by trying
    every subset of edges (tiny inputs only)."""
    edges = list(pairing_edges(pair, score).items())
    best = 0
    for r in range(len(edges) + 1):
        for sub in itertools.combinations(edges, r):
            used = set()
            ok = True
            for (a, b), _ in sub:
                if a in used or b in used:
                    ok = False
                    break
                used.add(a)
                used.add(b)
            if ok:
                best = max(best, sum(x for _, x in sub))
    return best


def matching_weight(pair, score, match):
    """Total weight of a matching given as match[n] (n if unmatched); checks it
    is an involution over pairing edges."""
    edges = pairing_edges(pair, score)
    tot = 0
    for n, m in enumerate(match):
        m = int(m)
        assert int(match[m]) == n, "matching is not an involution"
        if m > n:
            assert (n, m) in edges, "matched pair is not a pairing edge"
            tot += edges[(n, m)]
    return tot
