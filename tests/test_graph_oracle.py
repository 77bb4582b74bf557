"""Pins of the graph-construction oracle (Alg. 1 with Euclidean distance)
against a hand-worked example, brute force and independent routines."""
import math

import numpy as np
import pytest

from oracle import graph_oracle as G
from paper_2206_03410_amd import synth


def test_line_example_by_hand():
    """Five points on the x axis at spacing 0.5 with R = 1: the greedy pass
    (in x order) takes x = 0, then x = 1 (its distance 1 to the first node is
    not < R), then x = 2.  Weights by Eq. (3): equal distances give equal
    weights; a node's own point is weighted by itself alone."""
    V = np.array([[0.0, 0, 0], [0.5, 0, 0], [1.0, 0, 0], [1.5, 0, 0], [2.0, 0, 0]])
    g = G.build_graph(V, 1.0, 4)
    assert g["node_idx"].tolist() == [0, 2, 4]
    assert g["infl_idx"][:, :2].tolist() == [[0, -1], [0, 1], [1, -1], [1, 2], [2, -1]]
    assert np.all(g["infl_idx"][:, 2:] == -1)
    assert g["infl_w"][1, :2].tolist() == [0.5, 0.5]
    assert g["infl_w"][0, 0] == 1.0 and g["infl_w"][2, 0] == 1.0
    assert g["edges"].tolist() == [[0, 1], [1, 2]]
    # reversed input order: the axis sign convention keeps the x order
    g2 = G.build_graph(V[::-1].copy(), 1.0, 4)
    assert sorted(g2["node_idx"].tolist()) == [0, 2, 4]


def test_principal_axis_matches_svd():
    rng = np.random.default_rng(3)
    Q, _ = np.linalg.qr(rng.normal(size=(3, 3)))
    V = rng.normal(size=(500, 3)) * np.array([3.0, 1.0, 0.3]) @ Q
    m, a = G.principal_axis(V)
    _, _, Vt = np.linalg.svd(V - V.mean(0), full_matrices=False)
    b = Vt[0] * np.sign(Vt[0][np.argmax(np.abs(Vt[0]))])
    assert np.abs(a - b).max() < 1e-10
    assert np.allclose(m, V.mean(0), atol=1e-15)


@pytest.fixture(scope="module")
def cloud():
    pair = synth.torus_pair(1000, n_src=700, n_tgt=10, n_nodes=20, k=4, e=6)
    return pair.src


def test_greedy_nodes_are_the_first_maximal_independent_set(cloud):
    """Brute force over the full distance matrix: a point is a node iff no
    node earlier in the PCA order lies within R; hence nodes are pairwise at
    least R apart and every point lies within R of a node."""
    V = cloud
    R = 5 * G.mean_edge_length(V)
    g = G.build_graph(V, R, 8)
    D2 = G.d2_rows(V[:, None, :], V[None, :, :])
    order = G.pca_order(V)
    rank = np.empty(len(V), np.int64)
    rank[order] = np.arange(len(V))
    is_node = np.zeros(len(V), bool)
    is_node[g["node_idx"]] = True
    for i in range(len(V)):
        earlier_nodes = is_node & (rank < rank[i]) & (D2[i] < R * R)
        assert is_node[i] == (not earlier_nodes.any()), i
    nd = g["node_idx"]
    Dn = D2[np.ix_(nd, nd)]
    assert np.all(Dn[~np.eye(len(nd), dtype=bool)] >= R * R)
    assert np.all((D2[:, nd] < R * R).any(1))
    # node ids follow insertion (PCA) order
    assert np.all(np.diff(rank[nd]) > 0)


def test_influence_sets_weights_and_edges_by_brute_force(cloud):
    V = cloud
    R = 5 * G.mean_edge_length(V)
    k = 3
    g = G.build_graph(V, R, k)
    nd = g["node_idx"]
    D2 = G.d2_rows(V[:, None, :], V[nd][None, :, :])
    pairs = set()
    capped = 0
    for i in range(len(V)):
        inside = np.flatnonzero(D2[i] < R * R)
        capped += len(inside) > k
        srt = sorted(inside.tolist(), key=lambda j: (D2[i, j], j))[:k]
        got = [j for j in g["infl_idx"][i] if j >= 0]
        assert got == srt, i
        w = np.array([(1 - D2[i, j] / (R * R)) ** 3 for j in srt])
        w /= w.sum()
        assert np.allclose(g["infl_w"][i, :len(srt)], w, rtol=1e-14, atol=0)
        assert math.isclose(g["infl_w"][i].sum(), 1.0, rel_tol=1e-14)
        for a in range(len(srt)):
            for b in range(a + 1, len(srt)):
                pairs.add((min(srt[a], srt[b]), max(srt[a], srt[b])))
    assert g["edges"].tolist() == sorted([list(p) for p in pairs])
    assert g["n_capped"] == capped
    assert capped > 0


def test_mean_edge_length_by_brute_force():
    rng = np.random.default_rng(5)
    V = rng.random((300, 3))
    D2 = G.d2_rows(V[:, None, :], V[None, :, :])
    np.fill_diagonal(D2, np.inf)
    e = set()
    for i in range(len(V)):
        for j in np.argsort(D2[i], kind="stable")[:6]:
            e.add((min(i, j), max(i, j)))
    want = np.mean([math.sqrt(D2[i, j]) for i, j in e])
    assert G.mean_edge_length(V) == pytest.approx(want, rel=1e-13)
