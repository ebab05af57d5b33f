"""Nested-dissection ordering and symbolic factorization of the interior
block (pd_nd_analyse, the host half of the interior_order = 1 factor; no GPU
work).  Checked against definitions, not against the library's own code:
the order is a permutation of x1 whose supernodes form an elimination tree
(every edge joins a supernode to itself or an ancestor), and each boundary
set is the row set of the supernode's dense front, found by the elimination
game on the graph of K11 with the region nodes kept to the end and each
supernode eliminated as one block; it holds the row structure of the
Cholesky factor's columns below the supernode (Sec. 4.3: the partial
factorization of A11), and equals it for single-node supernodes."""
import numpy as np
import pytest

import pd_inputs as P


def _lib():
    from paper_2008_01541_amd import nd_analyse
    return nd_analyse


def free_graph(sc):
    """Adjacency sets of the free nodes (K's sparsity without the diagonal)."""
    n = sc.n_nodes
    free = ~sc.dirichlet
    adj = [set() for _ in range(n)]
    for e in range(sc.n_tets):
        vs = [int(v) for v in sc.tets[:, e] if free[v]]
        for a in vs:
            for b in vs:
                if a != b:
                    adj[a].add(b)
    return adj


def keyed_graph(sc, elim):
    """Graph of the free nodes on keys: elimination position, or n1 + r for
    the region node r."""
    n1 = len(elim)
    rid = sc.region_ids()
    key = {int(v): p for p, v in enumerate(elim)}
    key.update({int(v): n1 + r for r, v in enumerate(rid)})
    adj = free_graph(sc)
    return {key[v]: {key[w] for w in adj[v]} for v in key}


def structure_by_elimination(sc, elim):
    """Row structure (later keys) of every column of the Cholesky factor for
    the order elim followed by the region nodes: eliminate each interior node
    in turn and join its later neighbours pairwise (the elimination game)."""
    g = keyed_graph(sc, elim)
    cols = []
    for p in range(len(elim)):
        later = {k for k in g[p] if k > p}
        cols.append(later)
        for a in later:
            g[a] |= later - {a}
    return cols


def structure_by_block_elimination(sc, elim, first):
    """The same game with every supernode eliminated as one block: the later
    neighbours of the block (the rows of its dense front below it) are
    joined pairwise."""
    g = keyed_graph(sc, elim)
    out = []
    for s in range(len(first) - 1):
        f0, f1 = first[s], first[s + 1]
        later = set()
        for p in range(f0, f1):
            later |= {k for k in g[p] if k >= f1}
        out.append(later)
        for a in later:
            g[a] |= later - {a}
    return out


SCENES = {
    "cube8": lambda: P.scene_cube8(),
    "g9x7x6": lambda: P.scene_small(9, 7, 6, h=0.5, region_top_layers=2, seed=4),
    "irregular": lambda: P.scene_irregular(),
    "irregular_small": lambda: P.scene_irregular(6, 5, 4, seed=1),
    "allregion": lambda: P.scene_small(3, 3, 3, h=1.0, region_top_layers=4, seed=6),
}


@pytest.mark.parametrize("name", list(SCENES))
@pytest.mark.parametrize("leaf", [1, 7, 40, 256])
def test_nd_order_is_an_elimination_tree(name, leaf):
    sc = SCENES[name]()
    r = _lib()(sc.rest, sc.tets, sc.region, sc.dirichlet, leaf)
    interior = np.nonzero(~sc.dirichlet & ~sc.region)[0]
    elim, first, parent = r["elim"], r["first"], r["parent"]
    assert r["n1"] == interior.size
    assert np.array_equal(np.sort(elim), interior)
    ns = parent.size
    assert first[0] == 0 and first[-1] == interior.size and np.all(np.diff(first) > 0)
    assert np.all((parent == -1) | (parent > np.arange(ns)))     # children first
    sn = np.repeat(np.arange(ns), np.diff(first))                # supernode of each position
    # leaves (supernodes without children) hold at most `leaf` nodes, each
    # one connected piece of the graph
    has_child = np.zeros(ns, bool)
    has_child[parent[parent >= 0]] = True
    assert np.all(np.diff(first)[~has_child] <= leaf)
    adj0 = free_graph(sc)
    for s in np.nonzero(~has_child)[0]:
        nodes = set(elim[first[s]:first[s + 1]].tolist())
        seen, todo = set(), [next(iter(nodes))]
        while todo:
            v = todo.pop()
            if v in seen:
                continue
            seen.add(v)
            todo += [w for w in adj0[v] if w in nodes]
        assert seen == nodes

    def ancestors(s):
        out = []
        while s >= 0:
            out.append(s)
            s = parent[s]
        return out

    anc = [set(ancestors(s)) for s in range(ns)]
    pos = np.full(sc.n_nodes, -1)
    pos[elim] = np.arange(elim.size)
    adj = free_graph(sc)
    for u in interior:
        for w in adj[u]:
            if pos[w] > pos[u]:
                assert sn[pos[w]] in anc[sn[pos[u]]], (u, w)


@pytest.mark.parametrize("name", list(SCENES))
@pytest.mark.parametrize("leaf", [1, 7, 40])
def test_nd_boundaries_match_elimination_game(name, leaf):
    """Each boundary is the row set of its supernode's dense front (block
    elimination game), contains the factor's true column structure below the
    supernode (so no fill is dropped), and equals it for single-node
    supernodes."""
    sc = SCENES[name]()
    r = _lib()(sc.rest, sc.tets, sc.region, sc.dirichlet, leaf)
    elim, first, parent, bptr, bkey = r["elim"], r["first"], r["parent"], r["bptr"], r["bkey"]
    cols = structure_by_elimination(sc, elim)
    blocks = structure_by_block_elimination(sc, elim, first)
    n1 = r["n1"]
    for s in range(first.size - 1):
        f0, f1 = first[s], first[s + 1]
        got = bkey[bptr[s]:bptr[s + 1]]
        assert np.all(np.diff(got) > 0)
        assert set(got.tolist()) == blocks[s], s
        below = set()
        for p in range(f0, f1):
            below |= {k for k in cols[p] if k >= f1}
        assert below <= set(got.tolist())
        if f1 - f0 == 1:
            assert below == set(got.tolist())
        # the parent holds the first boundary key (elimination tree)
        if got.size and got[0] < n1:
            assert first[parent[s]] <= got[0] < first[parent[s] + 1]
        else:
            assert parent[s] == -1


def test_nd_separators_are_small_on_a_grid():
    """On a 16 x 15 x 8 grid with the top two layers as region, the
    bisection cuts along grid planes: every separator is at most one plane
    of the part it splits, and the tree is a few levels deep."""
    sc = P.scene_small(16, 15, 8, h=1.0, region_top_layers=2, seed=5)
    r = _lib()(sc.rest, sc.tets, sc.region, sc.dirichlet, 64)
    first, parent = r["first"], r["parent"]
    sizes = np.diff(first)
    has_child = np.zeros(parent.size, bool)
    has_child[parent[parent >= 0]] = True
    # the largest plane of the 17 x 16 x 7 interior block: 17 x 16 nodes
    assert sizes[has_child].max() <= 17 * 16
    depth = 0
    for s in range(parent.size):
        d, q = 0, s
        while parent[q] >= 0:
            q, d = parent[q], d + 1
        depth = max(depth, d)
    assert depth <= 8


def test_nd_analyse_rejects_bad_arguments():
    import ctypes as C
    from paper_2008_01541_amd import load_library
    from paper_2008_01541_amd._lib import pd_mesh
    lib = load_library()
    sc = P.scene_cube8()
    rest = np.ascontiguousarray(sc.rest)
    tets = np.ascontiguousarray(sc.tets, dtype=np.int32)
    reg = np.ascontiguousarray(sc.region, dtype=np.uint8)
    dr = np.ascontiguousarray(sc.dirichlet, dtype=np.uint8)
    mesh = pd_mesh(rest.shape[1], tets.shape[1], rest.ctypes.data, tets.ctypes.data,
                   reg.ctypes.data, dr.ctypes.data, 1.0, 0.0, 0.0, 0.0, 0.0, 0.0, 1, 0)
    sizes = np.zeros(3, np.int64)
    assert lib.pd_nd_analyse(C.byref(mesh), 0, sizes.ctypes.data, None, None, None, None,
                             None) == -1
    assert lib.pd_nd_analyse(C.byref(mesh), 8, None, None, None, None, None, None) == -1
    bad = tets.copy()
    bad[0, 0] = rest.shape[1]
    mesh.tets = bad.ctypes.data
    assert lib.pd_nd_analyse(C.byref(mesh), 8, sizes.ctypes.data, None, None, None, None,
                             None) == -1
