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


# ---------------------------------------------------------------- geodesic (Eq. 1)

def _floyd_warshall(W):
    """All-pairs shortest paths of a dense matrix of edge lengths (inf = no
    edge), plain loops over the intermediate point."""
    D = W.copy()
    np.fill_diagonal(D, 0.0)
    for m in range(D.shape[0]):
        D = np.minimum(D, D[:, m:m + 1] + D[m:m + 1, :])
    return D


def test_geodesic_ball_against_floyd_warshall():
    """The bounded shortest-path search equals brute-force all-pairs shortest
    paths over the same edge graph: the same points within R (away from the
    boundary) at the same distances; geodesic >= Euclidean distance."""
    rng = np.random.default_rng(11)
    V = rng.uniform(-1, 1, size=(70, 3)) * np.array([1.0, 1.0, 0.2])
    i, j, L = G.knn_edges(V, 6)
    W = np.full((70, 70), np.inf)
    W[i, j] = L
    W[j, i] = L
    FW = _floyd_warshall(W)
    Gm = G.geodesic_graph(V, 6)
    R = 0.7
    for src in range(70):
        q, d = G.geodesic_ball(Gm, src, R)
        far = np.abs(FW[src] - R) > 1e-9
        assert set(q.tolist()) == set(np.nonzero((FW[src] < R) & far)[0].tolist()) | set(
            x for x in q.tolist() if not far[x])
        assert np.allclose(d, FW[src, q], rtol=0, atol=1e-12)
        assert np.all(d >= np.sqrt(G.d2_rows(V[q], V[src][None, :])) - 1e-12)


def test_knn_edges_by_brute_force():
    """Each point's 6 nearest other points by the full distance matrix (ties to
    the lower index), symmetrized and deduplicated."""
    rng = np.random.default_rng(12)
    V = np.round(rng.uniform(-1, 1, size=(40, 3)) * 4) / 4     # many exact ties
    n = len(V)
    pairs = set()
    for q in range(n):
        d2 = G.d2_rows(V, V[q][None, :])
        c = [x for x in np.lexsort((np.arange(n), d2)) if x != q][:6]
        pairs |= {(min(q, x), max(q, x)) for x in c}
    i, j, L = G.knn_edges(V, 6)
    assert sorted(pairs) == list(zip(i.tolist(), j.tolist()))
    assert np.array_equal(L, np.sqrt(G.d2_rows(V[i], V[j])))


def test_geodesic_graph_on_a_line_equals_euclidean():
    """Evenly spaced points on a line at dyadic positions, each joined to its
    two nearest (its neighbours on both sides): every path sum is exact and
    equals the Euclidean distance, so the geodesic build equals the
    Euclidean one bitwise."""
    rng = np.random.default_rng(13)
    x = np.arange(120) / 64.0
    V = np.stack([x, np.zeros_like(x), np.zeros_like(x)], 1)
    V = V[rng.permutation(len(V))]
    a = G.build_graph(V, 0.4, 4)
    b = G.build_graph_geodesic(V, 0.4, 4, k_edges=2)
    for key in ("node_idx", "infl_idx", "edges"):
        assert np.array_equal(a[key], b[key])
    assert np.array_equal(a["infl_w"], b["infl_w"])


def _folded_strip(n_per_arm=300, gap=0.1, seed=14):
    """A U-shaped strip: two parallel arms `gap` apart along x in [0, 1],
    joined by a half circle at x = 1 (one arm at y = 0, the other at
    y = gap), width 0.05 in z."""
    rng = np.random.default_rng(seed)
    t = rng.uniform(0, 1, n_per_arm)
    z = rng.uniform(0, 0.05, n_per_arm)
    arm0 = np.stack([t, np.zeros_like(t), z], 1)
    t = rng.uniform(0, 1, n_per_arm)
    z = rng.uniform(0, 0.05, n_per_arm)
    arm1 = np.stack([t, np.full_like(t, gap), z], 1)
    th = rng.uniform(-np.pi / 2, np.pi / 2, n_per_arm // 6)
    z = rng.uniform(0, 0.05, len(th))
    bend = np.stack([1 + 0.5 * gap * np.cos(th), 0.5 * gap + 0.5 * gap * np.sin(th), z], 1)
    V = np.concatenate([arm0, arm1, bend])
    arm = np.concatenate([np.zeros(n_per_arm), np.ones(n_per_arm), np.full(len(th), 2)])
    return V, arm


def test_geodesic_influence_stays_on_its_arm():
    """Folded strip with R larger than the gap between the arms: with
    Euclidean distance, points of one arm take nodes of the other; with the
    geodesic distance, a point more than R (along the strip) from the fold
    is influenced only by nodes of its own arm, and the nodes of each arm
    cover it on their own (so there are more nodes)."""
    V, arm = _folded_strip()
    R = 0.25
    e = G.build_graph(V, R, 6)
    g = G.build_graph_geodesic(V, R, 6)
    far = V[:, 0] < 1 - R - 0.05
    def crossings(res):
        na = arm[res["node_idx"]]
        n = 0
        for q in np.nonzero(far & (arm < 2))[0]:
            js = res["infl_idx"][q]
            js = js[js >= 0]
            n += int(np.any(na[js] != arm[q]))
        return n
    assert crossings(e) > 0
    assert crossings(g) == 0
    assert len(g["node_idx"]) > len(e["node_idx"])
    # every point keeps at least one influencing node; weights sum to 1
    assert np.all(g["infl_idx"][:, 0] >= 0)
    assert np.allclose(g["infl_w"].sum(1), 1.0)


def test_geodesic_greedy_invariants_by_brute_force():
    """Against all-pairs shortest paths: nodes are pairwise at geodesic
    distance >= R, every point is within R of a node, node j is the first
    point in axis order not within R of nodes 0..j-1, and each point's kept
    nodes are its nearest by geodesic distance with Eq. (3) weights."""
    rng = np.random.default_rng(15)
    th = rng.uniform(0, 2 * np.pi, 150)
    V = np.stack([np.cos(th), np.sin(th), rng.uniform(0, 0.3, 150)], 1)
    R, k = 0.6, 4
    g = G.build_graph_geodesic(V, R, k)
    i, j, L = G.knn_edges(V, 6)
    W = np.full((150, 150), np.inf)
    W[i, j] = L
    W[j, i] = L
    FW = _floyd_warshall(W)
    nodes = g["node_idx"]
    sub = FW[np.ix_(nodes, nodes)]
    assert np.all(sub[~np.eye(len(nodes), dtype=bool)] >= R - 1e-12)
    assert np.all(FW[nodes].min(0) < R)
    order = G.pca_order(V)
    rank = np.empty(150, np.int64)
    rank[order] = np.arange(150)
    assert np.all(np.diff(rank[nodes]) > 0)
    for q in range(150):
        js = g["infl_idx"][q]
        js = js[js >= 0]
        D = FW[nodes[js], q]
        within = np.nonzero(FW[nodes, q] < R)[0]
        best = within[np.lexsort((within, FW[nodes[within], q]))][:k]
        assert np.array_equal(js, best)
        w = (1 - D * D / (R * R)) ** 3
        assert np.allclose(g["infl_w"][q, :len(js)], w / w.sum(), rtol=1e-12)
