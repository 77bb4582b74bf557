"""FP64 CPU oracle for the deformation-graph construction of Sec. 3.1
(Alg. 1), with Euclidean distance in place of the geodesic one
(build_graph) and with the geodesic distance of Eq. (1) on a point cloud
(build_graph_geodesic).

TEST INFRASTRUCTURE ONLY.  This module is the plain, slow reference the HIP
graph builder is checked against.  Only the test-suite and the benchmark's
CPU leg may import it; the library never calls it and shares no code with it.

The steps, in the paper's order:

* principal axis of the source points (largest eigenvalue of their
  covariance) and the order of the points along it ......... Alg. 1, PCA
* greedy node insertion in that order: a point becomes a node when no
  earlier node lies within R of it; every point within R of a new node
  gains it as an influencing node ............................ Alg. 1, Eq. (1)
* influence weights ......................................... Eq. (3)
* edges between nodes that influence a common point ......... Alg. 1, edges
* the mean edge length of the source point cloud ............ Sec. 3.3.3

Readings (the paper is silent on them):
* Distance is Euclidean (the geodesic version needs a mesh and an exact
  geodesic method); "within R" is the strict D < R of Alg. 1, evaluated as
  ((dx*dx + dy*dy) + dz*dz) < R*R in float64.
* The sign of the principal axis is fixed so that its component of largest
  magnitude is positive (the first such component on a tie); points with
  equal projections keep their index order.
* The influence sets feed a solver with k slots per point: a point keeps
  its k nearest influencing nodes (ties to the lower node id), the weights of
  Eq. (3) are normalized over the kept ones, and the unused slots are -1.
  Edges join nodes that influence a common point through kept slots.
* Node ids follow the order of insertion.
* The mean edge length is that of the symmetrized, deduplicated 6-nearest-
  neighbour graph of the source points (the paper's point clouds have no
  mesh edges).
* Geodesic distance on a point cloud (Sec. 3 builds the edge set of a point
  cloud from each point's nearest neighbours): the length of the shortest
  path over the symmetrized, deduplicated 6-nearest-neighbour graph (ties to
  the lower index), each edge as long as its Euclidean length sqrt(((dx*dx +
  dy*dy) + dz*dz)).  Alg. 1's breadth-first neighbourhood and exact geodesic
  step become one shortest-path search from the new node, bounded by R: a
  path shorter than R never leaves the Euclidean ball of radius R, so the
  bound loses nothing.  Eq. (3) takes D^2 = D * D of that distance.
"""
from __future__ import annotations

import numpy as np
from scipy.sparse import csr_matrix
from scipy.sparse.csgraph import dijkstra
from scipy.spatial import cKDTree


def d2_rows(a: np.ndarray, b: np.ndarray) -> np.ndarray:
    """((dx*dx + dy*dy) + dz*dz) of the rows of a - b, left to right."""
    d = a - b
    return (d[..., 0] * d[..., 0] + d[..., 1] * d[..., 1]) + d[..., 2] * d[..., 2]


def principal_axis(V: np.ndarray):
    """Mean and unit eigenvector of the largest eigenvalue of the covariance
    of V (Alg. 1's PCA), sign fixed as stated in the module header."""
    m = V.mean(0)
    D = V - m
    C = D.T @ D / V.shape[0]
    w, U = np.linalg.eigh(C)
    a = U[:, int(np.argmax(w))].copy()
    c = int(np.argmax(np.abs(a)))
    if a[c] < 0:
        a = -a
    return m, a


def pca_order(V: np.ndarray) -> np.ndarray:
    """Points sorted by their projection onto the principal axis."""
    m, a = principal_axis(V)
    t = (V - m) @ a
    return np.argsort(t, kind="stable")


def build_graph(V: np.ndarray, R: float, k: int):
    """Alg. 1 with Euclidean distance.  Returns a dict with node_idx (source
    index of node 0, 1, ...), infl_idx [N][k] (-1 = unused), infl_w [N][k],
    edges [E][2] (sorted, i < j), the number of points that had more than k
    influencing nodes, and the largest such number."""
    V = np.asarray(V, np.float64)
    N = V.shape[0]
    R2 = R * R
    tree = cKDTree(V)
    order = pca_order(V)
    nodes = []
    infl = [[] for _ in range(N)]          # influencing node ids, in insertion order
    for i in order:
        if not nodes or not infl[i]:
            j = len(nodes)
            nodes.append(int(i))
            # candidates from the tree's closed ball, then the strict test
            cand = np.asarray(tree.query_ball_point(V[i], R * (1 + 1e-9)), np.int64)
            inside = cand[d2_rows(V[cand], V[i][None, :]) < R2]
            for q in inside:
                infl[q].append(j)
    node_idx = np.asarray(nodes, np.int64)
    infl_idx = np.full((N, k), -1, np.int64)
    infl_w = np.zeros((N, k))
    n_capped = 0
    max_infl = 0
    pairs = set()
    for q in range(N):
        js = np.asarray(infl[q], np.int64)
        d2 = d2_rows(V[node_idx[js]], V[q][None, :])
        max_infl = max(max_infl, len(js))
        if len(js) > k:
            n_capped += 1
        keep = np.lexsort((js, d2))[:k]     # nearest first, ties to the lower node id
        js, d2 = js[keep], d2[keep]
        w = (1.0 - d2 / R2) ** 3            # Eq. (3), numerator
        infl_idx[q, :len(js)] = js
        infl_w[q, :len(js)] = w / w.sum()
        for a in range(len(js)):
            for b in range(a + 1, len(js)):
                pairs.add((min(js[a], js[b]), max(js[a], js[b])))
    edges = np.asarray(sorted(pairs), np.int64).reshape(-1, 2)
    return dict(node_idx=node_idx, infl_idx=infl_idx, infl_w=infl_w, edges=edges,
                n_capped=n_capped, max_influences=max_infl)


def mean_edge_length(V: np.ndarray, k: int = 6) -> float:
    """Mean length of the symmetrized, deduplicated k-nearest-neighbour graph
    of V (each point's k nearest other points)."""
    V = np.asarray(V, np.float64)
    n = V.shape[0]
    kk = min(k + 1, n)
    _, nb = cKDTree(V).query(V, kk)
    nb = nb.reshape(n, kk)
    rows = []
    for q in range(n):
        others = [int(x) for x in nb[q] if x != q][:kk - 1]   # self dropped (else the farthest)
        rows.append(others)
    a = np.concatenate([np.full(len(r), q) for q, r in enumerate(rows)]).astype(np.int64)
    b = np.concatenate([np.asarray(r, np.int64) for r in rows])
    key = np.unique(np.minimum(a, b) * n + np.maximum(a, b))
    i, j = key // n, key % n
    return float(np.mean(np.sqrt(d2_rows(V[i], V[j]))))


def knn_edges(V: np.ndarray, k: int = 6):
    """The symmetrized, deduplicated k-nearest-neighbour graph of V: each
    point's k nearest other points (ties to the lower index) give undirected
    edges (i, j), i < j, sorted, with their Euclidean lengths."""
    V = np.asarray(V, np.float64)
    n = V.shape[0]
    kk = min(k + 5, n)
    _, nb = cKDTree(V).query(V, kk)
    nb = np.asarray(nb, np.int64).reshape(n, kk)
    a, b = [], []
    for q in range(n):
        c = nb[q][nb[q] != q]
        d2 = d2_rows(V[c], V[q][None, :])
        keep = c[np.lexsort((c, d2))][:min(k, n - 1)]
        a.extend([q] * len(keep))
        b.extend(keep.tolist())
    a, b = np.asarray(a, np.int64), np.asarray(b, np.int64)
    key = np.unique(np.minimum(a, b) * n + np.maximum(a, b))
    i, j = key // n, key % n
    return i, j, np.sqrt(d2_rows(V[i], V[j]))


def geodesic_graph(V: np.ndarray, k: int = 6):
    """The point cloud's edge graph as a symmetric sparse matrix of edge
    lengths."""
    n = np.asarray(V).shape[0]
    i, j, L = knn_edges(V, k)
    return csr_matrix((np.concatenate([L, L]), (np.concatenate([i, j]), np.concatenate([j, i]))), shape=(n, n))


def geodesic_ball(Gm, src: int, R: float):
    """Points at geodesic distance < R from point `src` and those distances
    (shortest paths over the edge graph, searched up to R)."""
    d = dijkstra(Gm, directed=False, indices=int(src), limit=R)
    q = np.nonzero(d < R)[0]
    return q, d[q]


def build_graph_geodesic(V: np.ndarray, R: float, k: int, k_edges: int = 6):
    """Alg. 1 with the geodesic distance of Eq. (1) on the point cloud's
    edge graph.  Same outputs as build_graph."""
    V = np.asarray(V, np.float64)
    N = V.shape[0]
    R2 = R * R
    Gm = geodesic_graph(V, k_edges)
    order = pca_order(V)
    nodes = []
    infl = [[] for _ in range(N)]          # (node id, geodesic distance), in insertion order
    for i in order:
        if not nodes or not infl[i]:
            j = len(nodes)
            nodes.append(int(i))
            q, d = geodesic_ball(Gm, i, R)
            for qq, dd in zip(q, d):
                infl[qq].append((j, float(dd)))
    node_idx = np.asarray(nodes, np.int64)
    infl_idx = np.full((N, k), -1, np.int64)
    infl_w = np.zeros((N, k))
    n_capped = 0
    max_infl = 0
    pairs = set()
    for q in range(N):
        js = np.asarray([e[0] for e in infl[q]], np.int64)
        D = np.asarray([e[1] for e in infl[q]], np.float64)
        max_infl = max(max_infl, len(js))
        if len(js) > k:
            n_capped += 1
        keep = np.lexsort((js, D))[:k]      # nearest first, ties to the lower node id
        js, D = js[keep], D[keep]
        w = (1.0 - (D * D) / R2) ** 3       # Eq. (3), numerator
        infl_idx[q, :len(js)] = js
        infl_w[q, :len(js)] = w / w.sum()
        for a in range(len(js)):
            for b in range(a + 1, len(js)):
                pairs.add((min(js[a], js[b]), max(js[a], js[b])))
    edges = np.asarray(sorted(pairs), np.int64).reshape(-1, 2)
    return dict(node_idx=node_idx, infl_idx=infl_idx, infl_w=infl_w, edges=edges,
                n_capped=n_capped, max_influences=max_infl)
