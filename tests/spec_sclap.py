"""Executable specification of SCLaP and the multilevel partitioner, for tiny
graphs (n up to a few hundred).

A second, independent coding of the method, written from the readings of the
paper listed in the design notes (Section 3.1 label propagation with size
constraints and its refinement rule, Section 4.3 contraction, Section 4.4
iterated V-cycles, Section 4.5 the overall multilevel loop) in plain Python
with dictionaries and sorted lists.  It imports neither the oracle nor the GPU
library; the tests compare all three.  Test infrastructure only.

Graphs are dicts as produced by ``synth`` (``n``, ``xadj``, ``adjncy``,
optional ``adjwgt`` / ``vwgt``).
"""
import math

M64 = (1 << 64) - 1
CLUSTER, REFINE, INITIAL = 0, 1, 2
BIG = 1 << 30


def mix(z):
    """SplitMix64 output function of z + golden gamma (Steele, Lea, Flood 2014)."""
    z = (z + 0x9E3779B97F4A7C15) & M64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & M64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & M64
    return z ^ (z >> 31)


def H(*words):
    h = mix(words[0] & M64)
    for w in words[1:]:
        h = mix(h ^ (w & M64))
    return h


def adjacency(g):
    """Row v as a list of (neighbour, edge weight) and the node weights."""
    n, xa, adj = g["n"], g["xadj"], g["adjncy"]
    ew, nw = g.get("adjwgt"), g.get("vwgt")
    rows = [[(int(adj[i]), 1 if ew is None else int(ew[i])) for i in range(int(xa[v]), int(xa[v + 1]))]
            for v in range(n)]
    c = [1 if nw is None else int(nw[v]) for v in range(n)]
    return rows, c


def lmax(cV, k, eps):
    T = -(-cV // k)
    ppm = int(math.floor(eps * 1e6 + 0.5))
    return T + T * ppm // 10 ** 6


def degree_colors(rows, nsub, block=None):
    """Nodes with neighbours (same-block ones with a block array) ranked by
    (degree, id) and cut into nsub equal consecutive groups; others in 0."""
    deg = [sum(1 for u, _ in r if block is None or block[u] == block[v]) for v, r in enumerate(rows)]
    ranked = sorted((d, v) for v, d in enumerate(deg) if d > 0)
    col = [0] * len(rows)
    for r, (_, v) in enumerate(ranked):
        col[v] = r * nsub // len(ranked)
    return col


def run(rows, c, label, w, phase, level, seed, bound, rounds, nsub, colors=None, block=None):
    """Label propagation rounds in place; returns (rounds run, slots visited)."""
    n = len(rows)
    col = colors if colors is not None else [H(seed, 1, level, phase, v) % nsub for v in range(n)]
    visits = 0
    for r in range(rounds):
        moved = 0
        for s in range(nsub):
            cands = []  # (target, -gain, node, old label)
            for v in range(n):
                if col[v] != s:
                    continue
                conn = {}
                for u, wt in rows[v]:
                    if block is not None and block[u] != block[v]:
                        continue
                    visits += 1
                    conn[label[u]] = conn.get(label[u], 0) + wt
                a = label[v]
                own = conn.get(a, 0)
                over = phase != CLUSTER and w[a] > bound
                ok = [x for x in conn if x != a and w[x] + c[v] <= bound]
                if not ok:
                    continue
                t = min(ok, key=lambda x: (-conn[x], H(seed, 2, level, phase, r, x), x))
                gain = conn[t] - own
                if over or gain > 0:
                    cands.append((t, -gain, v, a))
            cands.sort()
            start = dict(w)  # departures in this sub-round are not credited
            i = 0
            while i < len(cands):  # each target takes its longest prefix within the bound
                t = cands[i][0]
                room, full = bound - start[t], False
                while i < len(cands) and cands[i][0] == t:
                    _, _, v, a = cands[i]
                    if not full and c[v] <= room:
                        room -= c[v]
                        label[v] = t
                        w[t] += c[v]
                        w[a] -= c[v]
                        moved += 1
                    else:
                        full = True
                    i += 1
        if moved == 0:
            return r + 1, visits
    return rounds, visits


def cluster(g, U, rounds=10, seed=1, level=0, nsub=4, colors=None, block=None):
    rows, c = adjacency(g)
    label = list(range(g["n"]))
    w = dict(enumerate(c))
    rr, visits = run(rows, c, label, w, CLUSTER, level, seed, U, rounds, nsub, colors, block)
    return label, rr, visits


def refine(g, k, Lmax, part, rounds=10, seed=1, level=0, nsub=4, colors=None):
    rows, c = adjacency(g)
    label = list(part)
    w = {b: 0 for b in range(k)}
    for v, b in enumerate(label):
        w[b] += c[v]
    rr, visits = run(rows, c, label, w, REFINE, level, seed, Lmax, rounds, nsub, colors)
    return label, rr, visits


def contract(g, label):
    """Coarse id = rank of the label among used labels; coarse rows sorted."""
    rows, c = adjacency(g)
    rank = {x: i for i, x in enumerate(sorted(set(label)))}
    C = [rank[label[v]] for v in range(g["n"])]
    nc = len(rank)
    cw = [0] * nc
    edges = [dict() for _ in range(nc)]
    for v, r in enumerate(rows):
        cw[C[v]] += c[v]
        for u, wt in r:
            if C[u] != C[v]:
                edges[C[v]][C[u]] = edges[C[v]].get(C[u], 0) + wt
    xadj, adj, ew = [0], [], []
    for i in range(nc):
        for j in sorted(edges[i]):
            adj.append(j)
            ew.append(edges[i][j])
        xadj.append(len(adj))
    return C, {"n": nc, "xadj": xadj, "adjncy": adj, "adjwgt": ew, "vwgt": cw}


def cut(g, part, k):
    rows, c = adjacency(g)
    bw = [0] * k
    s = 0
    for v, r in enumerate(rows):
        bw[part[v]] += c[v]
        s += sum(wt for u, wt in r if part[u] != part[v])
    return s // 2, bw


def initial_partition(g, k, T):
    """Greedy growth of blocks 0..k-2 by breadth-first search, then the rest
    to the lightest block."""
    rows, c = adjacency(g)
    n = g["n"]
    part = [-1] * n
    wb = [0] * k
    for b in range(k - 1):
        for s in range(n):
            if part[s] >= 0 or not rows[s] or wb[b] + c[s] > T:
                continue
            part[s] = b
            wb[b] += c[s]
            queue = [s]
            while queue:
                u = queue.pop(0)
                for x in sorted(x for x, _ in rows[u]):
                    if part[x] < 0 and wb[b] + c[x] <= T:
                        part[x] = b
                        wb[b] += c[x]
                        queue.append(x)
    for v in range(n):
        if part[v] < 0:
            b = min(range(k), key=lambda j: (wb[j], j))
            part[v] = b
            wb[b] += c[v]
    return part


def initial_partition_lp(g, k, T, Lmax, seed=1, level=0, rounds=10, nsub=4):
    """Seeds of smallest H(seed,5,level,v) open blocks; the rest start in an
    always-overloaded pool label k; refinement rounds with phase 2; the pool
    left over fills the blocks' remaining room in id and block order."""
    rows, c = adjacency(g)
    n = g["n"]
    ranked = sorted((H(seed, 5, level, v), v) for v in range(n) if rows[v])
    part = [k] * n
    for i, (_, v) in enumerate(ranked[:k]):
        part[v] = i
    w = {b: 0 for b in range(k + 1)}
    for v in range(n):
        w[part[v]] += c[v]
    w[k] += BIG
    rr, visits = run(rows, c, part, w, INITIAL, level, seed, Lmax, rounds, nsub)
    room = [max(0, T - w[b]) for b in range(k)]
    cum = [sum(room[:b + 1]) for b in range(k)]
    P = 0
    for v in range(n):
        if part[v] == k:
            part[v] = next((b for b in range(k) if cum[b] > P), k - 1)
            P += c[v]
    return part, rr, visits


def partition(g, k, eps=0.03, seed=1, coarsen_rounds=10, refine_rounds=10, subrounds=4, cluster_divisor=18,
              coarsest_nodes=10000, max_levels=64, vcycles=1, degree_order=0, initial=0):
    """The multilevel loop of Section 4.5 with iterated V-cycles (Section 4.4)."""
    n = g["n"]
    c0 = adjacency(g)[1]
    cV = sum(c0)
    L = lmax(cV, k, eps)
    W = cV // (cluster_divisor * k)
    T = -(-cV // k)
    prev, visits = None, 0
    for cyc in range(vcycles):
        sd = seed if cyc == 0 else H(seed, 4, cyc)
        graphs, maps, blocks = [g], [], [prev]
        while graphs[-1]["n"] > coarsest_nodes and len(maps) < max_levels:
            G, blk = graphs[-1], blocks[-1]
            U = max(max(adjacency(G)[1]), W)
            lev = len(maps)
            col = degree_colors(adjacency(G)[0], subrounds, blk) if degree_order else None
            lab, _, vis = cluster(G, U, coarsen_rounds, sd, lev, subrounds, col, blk)
            visits += vis
            C, cg = contract(G, lab)
            if cg["n"] >= G["n"]:
                break
            maps.append(C)
            graphs.append(cg)
            if blk is not None:
                cb = [0] * cg["n"]
                for v in range(G["n"]):
                    cb[C[v]] = blk[v]
                blocks.append(cb)
            else:
                blocks.append(None)
            if 20 * cg["n"] > 19 * G["n"]:
                break
        top = len(maps)
        if blocks[top] is not None:
            part = list(blocks[top])
        elif initial == 1:
            part, _, vis = initial_partition_lp(graphs[top], k, T, L, sd, top, refine_rounds, subrounds)
            visits += vis
        else:
            part = initial_partition(graphs[top], k, T)
        for lev in range(top, -1, -1):
            if lev < top:
                part = [part[maps[lev][v]] for v in range(graphs[lev]["n"])]
            part, _, vis = refine(graphs[lev], k, L, part, refine_rounds, sd, lev, subrounds)
            visits += vis
        prev = part
    cu, bw = cut(g, prev, k)
    return {"part": prev, "cut": cu, "block_weights": bw, "status": 1 if max(bw) > L else 0, "visits": visits}
