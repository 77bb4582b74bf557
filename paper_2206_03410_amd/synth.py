"""Seeded synthetic registration pairs and their deformation graphs.

This module produces the *inputs* of the registration hot path: source and
target point sets (with normals where they are cheap to get), a ground-truth
warp of every source point, and the embedded deformation graph (nodes,
per-point influence sets with their weights, node edges).  It holds none of
the majorization-minimization solver's arithmetic; both the HIP library and
the FP64 oracle receive exactly the arrays built here.

Workload recipes (the paper's datasets are replaced by synthetic scans that
keep their structure: noise, sparse outliers, a removed region for partial
overlap, articulated motion -- Sec. 4.3 of the paper):

* ``torus_pair``      -- torus (R=1, r=0.3) warped by Gaussian RBF bumps along
                         the surface normal, 5% outliers.
* ``sh_pair``         -- star-shaped surface r(d) = 1 + sum c_lm Y_lm(d) with
                         an articulated warp (two rigid halves blended by a
                         sigmoid across a plane), Gaussian noise, uniform
                         outliers and a spherical-cap cut.

Every pair is pre-scaled as in Sec. 4.1: one similarity for both point sets
that maps the joint bounding box to unit diagonal.

Deformation graph (stand-in for Alg. 1, whose geodesic distances need a
mesh): farthest-point sampled nodes (the alternative of the Remark in
Sec. 3.1), each point influenced by its k nearest nodes with the weights of
Eq. (3) using Euclidean distance and a per-point radius equal to the
distance of the (k+1)-th nearest node, and node edges from the symmetrized
e-nearest-neighbour graph, repaired to be connected.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np
from scipy import sparse
from scipy.sparse import csgraph
from scipy.spatial import cKDTree

# sub-stream offsets of a pair's base seed
_S_SRC, _S_TGT, _S_WARP, _S_NOISE, _S_OUT, _S_CUT = range(6)


@dataclasses.dataclass
class Pair:
    """One registration problem, already scaled to unit bounding-box diagonal."""

    src: np.ndarray            # (N, 3) float64 source points V
    tgt: np.ndarray            # (M, 3) float64 target points U
    gt: np.ndarray             # (N, 3) float64 ground-truth position of every source point
    node_idx: np.ndarray       # (n,) int32, graph nodes as indices into src
    infl_idx: np.ndarray       # (N, k) int32 node ids influencing each point
    infl_w: np.ndarray         # (N, k) float64 weights of Eq. (3), rows sum to 1
    edges: np.ndarray          # (E, 2) int32 undirected node edges, i < j, sorted
    mean_edge_len: float       # average edge length of the source (6-NN graph)
    scale: float               # original units per scaled unit (bbox diagonal)
    src_nrm: Optional[np.ndarray] = None
    tgt_nrm: Optional[np.ndarray] = None
    name: str = ""

    @property
    def n_src(self) -> int:
        return int(self.src.shape[0])

    @property
    def n_tgt(self) -> int:
        return int(self.tgt.shape[0])

    @property
    def n_nodes(self) -> int:
        return int(self.node_idx.shape[0])

    @property
    def k(self) -> int:
        return int(self.infl_idx.shape[1])

    @property
    def n_edges(self) -> int:
        return int(self.edges.shape[0])


def _rng(base: int, sub: int) -> np.random.Generator:
    return np.random.default_rng(base + sub)


# --------------------------------------------------------------------------
# surfaces
# --------------------------------------------------------------------------

def torus_points(n: int, rng: np.random.Generator, R: float = 1.0, r: float = 0.3):
    """Area-uniform torus samples: theta uniform, phi by rejection with
    acceptance (R + r cos phi)/(R + r).  Returns points and unit normals."""
    th = np.empty(0)
    ph = np.empty(0)
    while th.size < n:
        m = 2 * (n - th.size) + 16
        t = rng.uniform(0.0, 2.0 * np.pi, m)
        p = rng.uniform(0.0, 2.0 * np.pi, m)
        acc = rng.uniform(0.0, 1.0, m) < (R + r * np.cos(p)) / (R + r)
        th = np.concatenate([th, t[acc]])
        ph = np.concatenate([ph, p[acc]])
    th, ph = th[:n], ph[:n]
    ring = R + r * np.cos(ph)
    pts = np.stack([ring * np.cos(th), ring * np.sin(th), r * np.sin(ph)], 1)
    nrm = np.stack([np.cos(ph) * np.cos(th), np.cos(ph) * np.sin(th), np.sin(ph)], 1)
    return pts, nrm


def _real_sh_basis(dirs: np.ndarray, lmax: int) -> np.ndarray:
    """Real orthonormal spherical harmonics up to degree lmax at unit dirs,
    from the fully normalized associated Legendre recurrence (columns ordered
    l = 0..lmax, m = -l..l).  Returns (len(dirs), (lmax+1)^2)."""
    z = np.clip(dirs[:, 2], -1.0, 1.0)
    st = np.sqrt(np.maximum(0.0, 1.0 - z * z))
    phi = np.arctan2(dirs[:, 1], dirs[:, 0])
    n = dirs.shape[0]
    P = {}                                   # normalized P_l^m(z), m >= 0
    pmm = np.full(n, math.sqrt(1.0 / (4.0 * math.pi)))
    for m in range(lmax + 1):
        if m > 0:
            pmm = -math.sqrt((2 * m + 1) / (2.0 * m)) * st * pmm
        P[(m, m)] = pmm
        if m + 1 <= lmax:
            P[(m + 1, m)] = math.sqrt(2 * m + 3) * z * pmm
        for l in range(m + 2, lmax + 1):
            a = math.sqrt((4.0 * l * l - 1.0) / (l * l - m * m))
            b = math.sqrt(((l - 1.0) ** 2 - m * m) / (4.0 * (l - 1.0) ** 2 - 1.0))
            P[(l, m)] = a * (z * P[(l - 1, m)] - b * P[(l - 2, m)])
    cols = []
    cosm = [np.cos(m * phi) for m in range(lmax + 1)]
    sinm = [np.sin(m * phi) for m in range(lmax + 1)]
    for l in range(lmax + 1):
        for m in range(-l, l + 1):
            if m < 0:
                cols.append(math.sqrt(2.0) * P[(l, -m)] * sinm[-m])
            elif m == 0:
                cols.append(P[(l, 0)])
            else:
                cols.append(math.sqrt(2.0) * P[(l, m)] * cosm[m])
    return np.stack(cols, 1)


class SHSurface:
    """Star-shaped closed surface r(d) = 1 + sum_{l<=lmax} c_lm Y_lm(d)."""

    def __init__(self, lmax: int, rng: np.random.Generator, coef_std: float = 0.02):
        self.lmax = lmax
        self.coef = rng.normal(0.0, coef_std, (lmax + 1) ** 2)

    def radius(self, dirs: np.ndarray) -> np.ndarray:
        out = np.empty(dirs.shape[0])
        for s in range(0, dirs.shape[0], 65536):
            out[s:s + 65536] = 1.0 + _real_sh_basis(dirs[s:s + 65536], self.lmax) @ self.coef
        if np.any(out <= 0.2):
            raise ValueError("spherical-harmonic radius dropped below 0.2")
        return out

    def points(self, dirs: np.ndarray, normals: bool = False):
        r = self.radius(dirs)
        pts = r[:, None] * dirs
        if not normals:
            return pts, None
        # normal = cross of the two tangent derivatives (central differences)
        h = 1e-5
        a = np.where(np.abs(dirs[:, :1]) < 0.9, np.array([[1.0, 0, 0]]), np.array([[0, 1.0, 0]]))
        e1 = np.cross(dirs, a)
        e1 /= np.linalg.norm(e1, axis=1, keepdims=True)
        e2 = np.cross(dirs, e1)

        def at(d):
            d = d / np.linalg.norm(d, axis=1, keepdims=True)
            return self.radius(d)[:, None] * d

        t1 = at(dirs + h * e1) - at(dirs - h * e1)
        t2 = at(dirs + h * e2) - at(dirs - h * e2)
        nrm = np.cross(t1, t2)
        nrm /= np.linalg.norm(nrm, axis=1, keepdims=True)
        flip = np.sum(nrm * dirs, 1) < 0
        nrm[flip] *= -1.0
        return pts, nrm


def uniform_dirs(n: int, rng: np.random.Generator) -> np.ndarray:
    d = rng.normal(size=(n, 3))
    return d / np.linalg.norm(d, axis=1, keepdims=True)


# --------------------------------------------------------------------------
# warps (ground-truth deformations)
# --------------------------------------------------------------------------

class BumpWarp:
    """x + sum_b amp * exp(-|x - c_b|^2 / (2 sigma^2)) * n_b."""

    def __init__(self, centers, normals, sigma=0.3, amp=0.1):
        self.c = np.asarray(centers, float)
        self.n = np.asarray(normals, float)
        self.sigma, self.amp = sigma, amp

    def __call__(self, x):
        out = x.copy()
        for c, n in zip(self.c, self.n):
            g = np.exp(-np.sum((x - c) ** 2, 1) / (2.0 * self.sigma ** 2))
            out += self.amp * g[:, None] * n[None, :]
        return out


def _axis_rotation(axis, angle):
    axis = np.asarray(axis, float) / np.linalg.norm(axis)
    K = np.array([[0, -axis[2], axis[1]], [axis[2], 0, -axis[0]], [-axis[1], axis[0], 0]])
    return np.eye(3) + math.sin(angle) * K + (1.0 - math.cos(angle)) * (K @ K)


class ArticulatedWarp:
    """Two rigid halves joined by a smooth blend: x' = (1-s) x + s R x with
    s(x) = sigmoid((a . x) / width), R a rotation about an axis normal to a."""

    def __init__(self, rng: np.random.Generator, angle_deg=15.0, width=0.15):
        a = uniform_dirs(1, rng)[0]
        t = rng.normal(size=3)
        t -= a * np.dot(a, t)
        t /= np.linalg.norm(t)
        self.a, self.axis, self.width = a, t, width
        self.angle_deg = angle_deg
        self.R = _axis_rotation(t, math.radians(angle_deg))

    def __call__(self, x):
        s = 1.0 / (1.0 + np.exp(-(x @ self.a) / self.width))
        return (1.0 - s)[:, None] * x + s[:, None] * (x @ self.R.T)


# --------------------------------------------------------------------------
# deformation graph
# --------------------------------------------------------------------------

def farthest_point_sampling(pts: np.ndarray, n: int, start: int = 0) -> np.ndarray:
    """Euclidean FPS starting at `start`; ties go to the lowest index.  Each
    new node can only lower the distance of points within the current
    largest distance, so only that ball (found with a kd-tree) is updated."""
    N = pts.shape[0]
    n = min(n, N)
    idx = np.empty(n, np.int64)
    d = np.full(N, np.inf)
    tree = cKDTree(pts)
    cur = start
    for s in range(n):
        idx[s] = cur
        dmax = float(np.max(d))
        if np.isfinite(dmax):
            near = np.asarray(tree.query_ball_point(pts[cur], math.sqrt(dmax) * (1 + 1e-9) + 1e-300))
        else:
            near = np.arange(N)
        if near.size:
            diff = pts[near] - pts[cur]
            d[near] = np.minimum(d[near], np.einsum("ij,ij->i", diff, diff))
        cur = int(np.argmax(d))
    return idx


def influence(pts: np.ndarray, nodes: np.ndarray, k: int):
    """k nearest nodes per point and the normalized weights of Eq. (3) with
    Euclidean distance and radius = distance to the (k+1)-th nearest node."""
    n = nodes.shape[0]
    if n < k:
        raise ValueError("fewer graph nodes than influences per point")
    tree = cKDTree(nodes)
    kk = min(k + 1, n)
    dist, idx = tree.query(pts, kk)
    dist = dist.reshape(pts.shape[0], kk)
    idx = idx.reshape(pts.shape[0], kk)
    if kk > k:
        rad = dist[:, k]
    else:
        rad = 2.0 * dist[:, k - 1]
    d = dist[:, :k]
    rad = np.where(rad > 0, rad, 1.0)
    base = np.clip(1.0 - (d / rad[:, None]) ** 2, 0.0, None) ** 3
    tot = base.sum(1, keepdims=True)
    w = np.where(tot > 0, base / np.where(tot > 0, tot, 1.0), 1.0 / k)
    return idx[:, :k].astype(np.int32), w


def node_edges(nodes: np.ndarray, e: int) -> np.ndarray:
    """Symmetrized e-NN edges among nodes, made connected by adding the
    shortest edge from the component of node 0 to the rest, repeatedly."""
    n = nodes.shape[0]
    if n < 2:
        return np.zeros((0, 2), np.int32)
    ee = min(e + 1, n)
    _, nb = cKDTree(nodes).query(nodes, ee)
    nb = nb.reshape(n, ee)
    a = np.repeat(np.arange(n), ee - 1)
    b = nb[:, 1:].reshape(-1)
    i, j = np.minimum(a, b), np.maximum(a, b)
    keep = i != j
    pairs = set(zip(i[keep].tolist(), j[keep].tolist()))
    while True:
        E = np.array(sorted(pairs), np.int64).reshape(-1, 2)
        g = sparse.coo_matrix((np.ones(len(E)), (E[:, 0], E[:, 1])), shape=(n, n))
        ncomp, lab = csgraph.connected_components(g, directed=False)
        if ncomp == 1:
            break
        in0 = np.flatnonzero(lab == lab[0])
        out = np.flatnonzero(lab != lab[0])
        d, j2 = cKDTree(nodes[out]).query(nodes[in0], 1)
        s = int(np.argmin(d))
        u, v = int(in0[s]), int(out[j2[s]])
        pairs.add((min(u, v), max(u, v)))
    return E.astype(np.int32)


def mean_knn_edge_length(pts: np.ndarray, k: int = 6) -> float:
    """Average length of the deduplicated symmetrized k-NN graph of pts."""
    n = pts.shape[0]
    kk = min(k + 1, n)
    _, nb = cKDTree(pts).query(pts, kk)
    nb = nb.reshape(n, kk)
    a = np.repeat(np.arange(n), kk - 1)
    b = nb[:, 1:].reshape(-1)
    key = np.unique(np.minimum(a, b).astype(np.int64) * n + np.maximum(a, b))
    i, j = key // n, key % n
    keep = i != j
    return float(np.mean(np.linalg.norm(pts[i[keep]] - pts[j[keep]], axis=1)))


def build_graph(src: np.ndarray, n_nodes: int, k: int, e: int):
    node_idx = farthest_point_sampling(src, n_nodes).astype(np.int32)
    nodes = src[node_idx]
    infl_idx, infl_w = influence(src, nodes, k)
    edges = node_edges(nodes, e)
    return node_idx, infl_idx, infl_w, edges


def _scale_pair(src, tgt, gt):
    allp = np.concatenate([src, tgt], 0)
    lo, hi = allp.min(0), allp.max(0)
    c = 0.5 * (lo + hi)
    diag = float(np.linalg.norm(hi - lo))
    s = 1.0 / diag
    return (src - c) * s, (tgt - c) * s, (gt - c) * s, diag


def _finish(name, src, tgt, gt, n_nodes, k, e, src_nrm=None, tgt_nrm=None) -> Pair:
    src, tgt, gt, diag = _scale_pair(src, tgt, gt)
    node_idx, infl_idx, infl_w, edges = build_graph(src, n_nodes, k, e)
    return Pair(src=src, tgt=tgt, gt=gt, node_idx=node_idx, infl_idx=infl_idx,
                infl_w=infl_w, edges=edges, mean_edge_len=mean_knn_edge_length(src),
                scale=diag, src_nrm=src_nrm, tgt_nrm=tgt_nrm, name=name)


# --------------------------------------------------------------------------
# pair recipes
# --------------------------------------------------------------------------

def torus_pair(seed: int, n_src=2000, n_tgt=2000, outlier_frac=0.05, noise=0.002,
               n_bumps=8, n_nodes=80, k=4, e=6) -> Pair:
    src, src_n = torus_points(n_src, _rng(seed, _S_SRC))
    c, cn = torus_points(n_bumps, _rng(seed, _S_WARP))
    warp = BumpWarp(c, cn, sigma=0.3, amp=0.1)
    t0, tn = torus_points(n_tgt, _rng(seed, _S_TGT))
    tgt = warp(t0) + _rng(seed, _S_NOISE).normal(0.0, noise, t0.shape)
    n_out = int(round(outlier_frac * n_tgt))
    lo, hi = tgt.min(0), tgt.max(0)
    outl = _rng(seed, _S_OUT).uniform(lo, hi, (n_out, 3))
    tgt_all = np.concatenate([tgt, outl], 0)
    tgt_nrm = np.concatenate([tn, np.zeros((n_out, 3))], 0)
    return _finish(f"torus{n_src}", src, tgt_all, warp(src), n_nodes, k, e, src_n, tgt_nrm)


def sh_pair(seed: int, n_src: int, n_tgt: Optional[int] = None, lmax=8, outlier_frac=0.10,
            cut_frac=0.20, noise=0.003, n_nodes=1000, k=4, e=8, angle_deg=15.0,
            normals=False) -> Pair:
    """Spherical-harmonic surface pair with articulated warp, noise, outliers
    and a removed spherical cap of area fraction `cut_frac` on the target."""
    if n_tgt is None:
        n_tgt = n_src
    surf = SHSurface(lmax, _rng(seed, _S_SRC))
    srng = _rng(seed, _S_SRC + 100)
    src, src_n = surf.points(uniform_dirs(n_src, srng), normals)
    warp = ArticulatedWarp(_rng(seed, _S_WARP), angle_deg=angle_deg)
    cap = uniform_dirs(1, _rng(seed, _S_CUT))[0]
    cos_c = 1.0 - 2.0 * cut_frac
    n_in = n_tgt - int(round(outlier_frac * n_tgt))
    trng = _rng(seed, _S_TGT)
    dirs = np.zeros((0, 3))
    while dirs.shape[0] < n_in:
        d = uniform_dirs(2 * (n_in - dirs.shape[0]) + 64, trng)
        dirs = np.concatenate([dirs, d[d @ cap < cos_c]], 0)
    dirs = dirs[:n_in]
    t0, tn = surf.points(dirs, normals)
    tgt = warp(t0) + _rng(seed, _S_NOISE).normal(0.0, noise, t0.shape)
    lo, hi = tgt.min(0), tgt.max(0)
    outl = _rng(seed, _S_OUT).uniform(lo, hi, (n_tgt - n_in, 3))
    tgt_all = np.concatenate([tgt, outl], 0)
    tgt_nrm = None
    if normals:
        tgt_nrm = np.concatenate([tn, np.zeros((n_tgt - n_in, 3))], 0)
    return _finish(f"sh{n_src}", src, tgt_all, warp(src), n_nodes, k, e, src_n, tgt_nrm)


@dataclasses.dataclass
class Sequence:
    """A template (frame 0's source points and deformation graph) and target
    frames of the same surface bent ever further, all in one scaling."""
    template: Pair                  # template.tgt = the first target frame
    frames: List[np.ndarray]        # target points of frames step, 2 step, ...
    gts: List[np.ndarray]           # ground truth: the template warped to each frame
    frame_ids: List[int]


def sh_sequence(seed: int, n_src: int, n_frames: int = 8, step: int = 2, lmax=8, deg_per_frame=2.5,
                outlier_frac=0.05, noise=0.003, n_nodes=1000, k=4, e=8) -> Sequence:
    """Sequence-tracking workload (the paper's frame i -> i + 2 protocol,
    Sec. 4): one spherical-harmonic surface under an articulated warp whose
    angle grows by `deg_per_frame` per frame; target frames step, 2 step, ...
    are resampled independently with noise and uniform outliers; the
    template is frame 0's surface sampled at n_src points."""
    surf = SHSurface(lmax, _rng(seed, _S_SRC))
    src, _ = surf.points(uniform_dirs(n_src, _rng(seed, _S_SRC + 100)), False)
    wrng = _rng(seed, _S_WARP)
    base = ArticulatedWarp(wrng, angle_deg=0.0)
    ids = [step * (f + 1) for f in range(n_frames)]
    frames, gts = [], []
    for f, t in enumerate(ids):
        w = ArticulatedWarp(_rng(seed, _S_WARP), angle_deg=deg_per_frame * t)
        assert np.allclose(w.a, base.a) and np.allclose(w.axis, base.axis)
        n_in = n_src - int(round(outlier_frac * n_src))
        dirs = uniform_dirs(n_in, _rng(seed + 7 * t, _S_TGT))
        pts, _ = surf.points(dirs, False)
        tgt = w(pts) + _rng(seed + 7 * t, _S_NOISE).normal(0.0, noise, pts.shape)
        lo, hi = tgt.min(0), tgt.max(0)
        outl = _rng(seed + 7 * t, _S_OUT).uniform(lo, hi, (n_src - n_in, 3))
        frames.append(np.concatenate([tgt, outl], 0))
        gts.append(w(src))
    allp = np.concatenate([src] + frames, 0)
    lo, hi = allp.min(0), allp.max(0)
    c = 0.5 * (lo + hi)
    sc = 1.0 / float(np.linalg.norm(hi - lo))
    src = (src - c) * sc
    frames = [(fr - c) * sc for fr in frames]
    gts = [(g - c) * sc for g in gts]
    node_idx, infl_idx, infl_w, edges = build_graph(src, n_nodes, k, e)
    tpl = Pair(src=src, tgt=frames[0], gt=gts[0], node_idx=node_idx, infl_idx=infl_idx, infl_w=infl_w,
               edges=edges, mean_edge_len=mean_knn_edge_length(src), scale=1.0 / sc, name=f"seq{n_src}")
    return Sequence(tpl, frames, gts, ids)


# The five workloads (sizes, graph shape and iteration budgets).
WORKLOADS = {
    "torus2k": dict(kind="torus", seed=1000, n_src=2000, n_nodes=80, k=4, e=6,
                    max_total_iters=30, aa_m=5),
    "sh50k": dict(kind="sh", seed=2000, n_src=50000, lmax=8, outlier_frac=0.10, cut_frac=0.20,
                  noise=0.003, n_nodes=1000, k=4, e=8, max_total_iters=0, aa_m=5),
    "sh200k": dict(kind="sh", seed=3000, n_src=200000, lmax=16, outlier_frac=0.15,
                   cut_frac=0.30, noise=0.003, n_nodes=4000, k=6, e=10, max_total_iters=50,
                   aa_m=6),
    "grad100k": dict(kind="sh", seed=5000, n_src=100000, lmax=8, outlier_frac=0.10,
                     cut_frac=0.20, noise=0.003, n_nodes=2000, k=4, e=8, max_total_iters=0,
                     aa_m=5),
}


def make_workload(name: str, **override) -> Pair:
    cfg = dict(WORKLOADS[name])
    cfg.update(override)
    kind = cfg.pop("kind")
    cfg.pop("max_total_iters", None)
    cfg.pop("aa_m", None)
    if kind == "torus":
        seed = cfg.pop("seed")
        n = cfg.pop("n_src")
        return torus_pair(seed, n_src=n, n_tgt=n, **cfg)
    seed = cfg.pop("seed")
    n = cfg.pop("n_src")
    return sh_pair(seed, n, **cfg)


def batch_sizes(n_pairs=64, lo=5000, hi=60000, seed=4000):
    rng = np.random.default_rng(seed)
    return rng.integers(lo, hi + 1, n_pairs)


def batch_pairs(n_pairs=64, lo=5000, hi=60000, per_node=50, k=4, e=8, seed=4000):
    """Uneven batch: point counts uniform in [lo, hi], nodes ~ points/per_node,
    each pair generated like the 50k workload with its own seed."""
    sizes = batch_sizes(n_pairs, lo, hi, seed)
    pairs = []
    for b, nb in enumerate(sizes):
        pairs.append(sh_pair(40000 + 100 * b, int(nb), lmax=8, outlier_frac=0.10,
                             cut_frac=0.20, noise=0.003,
                             n_nodes=max(k + 1, int(round(nb / per_node))), k=k, e=e))
    return pairs


def perturbed_transforms(n_nodes: int, seed: int, sd_a=0.01, sd_t=0.001) -> np.ndarray:
    """X = identity + delta, layout [n][4][3] (rows A^T, then t^T)."""
    rng = np.random.default_rng(seed)
    X = identity_transforms(n_nodes)
    X[:, :3, :] += rng.normal(0.0, sd_a, (n_nodes, 3, 3))
    X[:, 3, :] += rng.normal(0.0, sd_t, (n_nodes, 3))
    return X


def identity_transforms(n_nodes: int) -> np.ndarray:
    X = np.zeros((n_nodes, 4, 3))
    X[:, 0, 0] = X[:, 1, 1] = X[:, 2, 2] = 1.0
    return X


def identical_pair(base: Pair) -> Pair:
    """Target = source (same samples): the registration fixed point is X = I."""
    return dataclasses.replace(base, tgt=base.src.copy(), gt=base.src.copy(),
                               tgt_nrm=None if base.src_nrm is None else base.src_nrm.copy(),
                               name=base.name + "-identical")


def rigid_pair(base: Pair, seed: int, angle_deg=5.0, shift=0.01) -> Pair:
    """Target = R V + t with the same samples (no noise, no outliers)."""
    rng = np.random.default_rng(seed)
    axis = uniform_dirs(1, rng)[0]
    R = _axis_rotation(axis, math.radians(angle_deg))
    t = uniform_dirs(1, rng)[0] * shift
    moved = base.src @ R.T + t
    p = dataclasses.replace(base, tgt=moved, gt=moved.copy(), tgt_nrm=None,
                            name=base.name + "-rigid")
    p.rigid_R, p.rigid_t = R, t  # type: ignore[attr-defined]
    return p
