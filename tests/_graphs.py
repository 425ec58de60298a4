"""Small graph helpers shared by the tests (inputs only)."""
import itertools

import numpy as np

from paper_2411_02268_amd import synth


def clique_edges(vs):
    return [(a, b) for a, b in itertools.combinations(vs, 2)]


def disjoint_cliques(r, s):
    edges = []
    for c in range(r):
        edges += clique_edges(range(c * s, (c + 1) * s))
    return synth.from_edges(r * s, edges)


def to_nx(g):
    import networkx as nx
    G = nx.Graph()
    G.add_nodes_from(range(g.n))
    for i in range(g.n):
        for e in range(g.offsets[i], g.offsets[i + 1]):
            j = int(g.indices[e])
            if j >= i:
                G.add_edge(i, j, weight=int(g.weights[e]))
    return G


def nx_modularity(g, C):
    import networkx as nx
    groups = {}
    for v, c in enumerate(C):
        groups.setdefault(int(c), set()).add(v)
    return nx.community.modularity(to_nx(g), list(groups.values()), weight="weight")


def set_partitions(items):
    if not items:
        yield []
        return
    first, rest = items[0], items[1:]
    for p in set_partitions(rest):
        for i in range(len(p)):
            yield p[:i] + [[first] + p[i]] + p[i + 1:]
        yield [[first]] + p


def partition_labels(n, parts):
    C = np.zeros(n, dtype=np.int32)
    for c, part in enumerate(parts):
        for v in part:
            C[v] = c
    return C
