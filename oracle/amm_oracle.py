"""FP64 CPU oracle for robust non-rigid registration by accelerated
majorization-minimization (Yao, Deng, Xu, Zhang, arXiv 2206.03410).

TEST INFRASTRUCTURE ONLY.  This module is the plain, slow, obviously correct
reference the HIP library is checked against.  Only the test-suite, the smoke
check and the CPU-baseline leg of the benchmark may import it; the library
never calls it and shares no code with it.

Everything is float64 numpy/scipy, written step by step from the paper:

* deformation warp ............................ Sec. 3, Eq. (2)
* closest-point correspondence ................ Sec. 3.2 (alignment term)
* Welsch function ............................. Eq. (6)
* alignment / regularization / rotation terms . Eqs. (4), (5), (7)-(9)
* edge normalization weights r_ij ............. Eq. (8)
* projection onto SO(3) ....................... Sec. 3.2 (rotation term)
* quadratic surrogate, matrix form, normal
  equations K X = B ........................... Sec. 3.3.1-3.3.2, Eqs. (13)-(21)
* nu continuation ............................. Sec. 3.3.3
* Anderson acceleration + energy fallback ..... Sec. 3.3.4, Eqs. (22)-(23), Alg. 2
* weight rule for alpha, beta ................. Eq. (26)
* squared-norm and fixed-nu variants .......... Sec. 4.1 (effect of the Welsch
  function and of the nu update)

Readings taken where the paper is silent or garbled are listed with the
functions that take them (search for "Reading").  The gradient of the energy
(``energy_grad``) is not in the paper; it is the derivative of Eq. (4) with
the closest points held fixed, pinned by finite differences.

Layouts: transforms X are (n, 4, 3) with rows A_j^T (three rows) then t_j^T,
which is the block X_j of the paper's stacked variable X in R^{4n x 3}.
"""
from __future__ import annotations

import dataclasses
import math
import os
from concurrent.futures import ThreadPoolExecutor
from typing import List, Optional

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla


# --------------------------------------------------------------------------
# problem
# --------------------------------------------------------------------------

@dataclasses.dataclass
class Problem:
    """Inputs of one registration problem (Sec. 3): source points V, target
    points U, deformation graph nodes p_j (a subset of V), influence sets
    I(v_i) with weights w_ij (Eq. 3), undirected node edges E_G."""

    src: np.ndarray
    tgt: np.ndarray
    node_idx: np.ndarray
    infl_idx: np.ndarray
    infl_w: np.ndarray
    edges: np.ndarray
    mean_edge_len: float

    def __post_init__(self):
        self.src = np.asarray(self.src, np.float64)
        self.tgt = np.asarray(self.tgt, np.float64)
        self.node_idx = np.asarray(self.node_idx, np.int64)
        self.infl_idx = np.asarray(self.infl_idx, np.int64)
        self.infl_w = np.asarray(self.infl_w, np.float64)
        # A point with fewer influencing nodes than slots marks the rest -1
        # (weight 0).  Such a slot is absent from Eq. (2)'s sum; it is
        # pointed at the row's first node so that every gather stays valid,
        # and its zero weight removes it from every sum and matrix entry.
        pad = self.infl_idx < 0
        if pad.any():
            assert np.all(self.infl_w[pad] == 0.0)
            first = self.infl_idx[np.arange(self.infl_idx.shape[0]), np.argmax(~pad, 1)]
            self.infl_idx = np.where(pad, first[:, None], self.infl_idx)
        self.edges = np.asarray(self.edges, np.int64).reshape(-1, 2)
        self.nodes = self.src[self.node_idx]
        self.dir_edges = directed_edges(self.edges)
        self.r = edge_weights(self.nodes, self.dir_edges)

    @property
    def n_src(self):
        return self.src.shape[0]

    @property
    def n_nodes(self):
        return self.nodes.shape[0]

    @property
    def n_undirected(self):
        return self.edges.shape[0]


def from_pair(pair) -> Problem:
    return Problem(pair.src, pair.tgt, pair.node_idx, pair.infl_idx, pair.infl_w,
                   pair.edges, pair.mean_edge_len)


def identity(n: int) -> np.ndarray:
    X = np.zeros((n, 4, 3))
    X[:, 0, 0] = X[:, 1, 1] = X[:, 2, 2] = 1.0
    return X


# --------------------------------------------------------------------------
# influence weights and graph weights
# --------------------------------------------------------------------------

def influence_weights(dist: np.ndarray, radius: np.ndarray) -> np.ndarray:
    """Eq. (3): w_ij = (1 - D^2/R^2)^3 / sum_k (1 - D^2/R^2)^3 over the
    influence set of point i.  dist is (N, k), radius (N,)."""
    b = (1.0 - (dist / radius[:, None]) ** 2) ** 3
    return b / b.sum(1, keepdims=True)


def directed_edges(edges: np.ndarray) -> np.ndarray:
    """Each undirected edge {i, j} yields the two ordered pairs (i, j) and
    (j, i): the regularization sum of Eq. (9) runs over every node i and every
    neighbour j in N(p_i), i.e. over both orders."""
    e = np.asarray(edges, np.int64).reshape(-1, 2)
    return np.concatenate([e, e[:, ::-1]], 0)


def edge_weights(nodes: np.ndarray, dir_edges: np.ndarray) -> np.ndarray:
    """Eq. (8): r_ij = 2|E_G| |p_i - p_j|^-1 / sum over ordered neighbour
    pairs of |p_i - p_j|^-1.  |E_G| counts undirected edges, so the mean of
    r over the 2|E_G| ordered pairs is exactly 1."""
    inv = 1.0 / np.linalg.norm(nodes[dir_edges[:, 0]] - nodes[dir_edges[:, 1]], axis=1)
    return dir_edges.shape[0] * inv / math.fsum(inv)


# --------------------------------------------------------------------------
# Welsch function and its quadratic surrogate
# --------------------------------------------------------------------------

def welsch(x2, nu):
    """Eq. (6) as a function of the squared argument: psi = 1 - exp(-x^2/(2 nu^2)),
    evaluated as -expm1(.) so that small arguments keep full precision."""
    return -np.expm1(-np.asarray(x2, np.float64) / (2.0 * nu * nu))


def welsch_weight(y2, nu):
    """Coefficient of x^2 in the surrogate of Eq. (13) at y:
    (1 - psi(y)) / (2 nu^2) = exp(-y^2/(2 nu^2)) / (2 nu^2).  These are the
    squared entries of W_a and W_r in Sec. 3.3.2."""
    return np.exp(-np.asarray(y2, np.float64) / (2.0 * nu * nu)) / (2.0 * nu * nu)


# Robust-term variants of Sec. 4.1.  "welsch" is the method itself; "l2"
# replaces both Welsch functions by squared norms with unit weights
# ("l2-norm"); "l2r" keeps unit weights only for alignment residuals shorter
# than 3 nu_a and zero otherwise, with squared norms on the regularization
# ("l2-norm-r").
ROBUST = ("welsch", "l2", "l2r")


def align_penalty(x2, nu, robust="welsch"):
    """Per-point alignment term as a function of the squared distance.
    Reading for "l2r": the 0/1 weight rule is the MM weight of the truncated
    quadratic min(x^2, (3 nu)^2) (a constant majorizes it where the residual
    is at least 3 nu, x^2 elsewhere), which is the energy that this variant
    decreases."""
    x2 = np.asarray(x2, np.float64)
    if robust == "welsch":
        return welsch(x2, nu)
    if robust == "l2":
        return x2.copy()
    if robust == "l2r":
        return np.minimum(x2, 9.0 * nu * nu)
    raise ValueError(robust)


def align_weight(y2, nu, robust="welsch"):
    """Coefficient of x^2 in the alignment surrogate at y (squared entries of
    W_a): the Welsch weight of Eq. (13), 1 for "l2", and for "l2r" 1 where
    |y| < 3 nu and 0 elsewhere."""
    y2 = np.asarray(y2, np.float64)
    if robust == "welsch":
        return welsch_weight(y2, nu)
    if robust == "l2":
        return np.ones_like(y2)
    if robust == "l2r":
        return (y2 < 9.0 * nu * nu).astype(np.float64)
    raise ValueError(robust)


def reg_penalty(x2, nu, robust="welsch"):
    """Regularization term per directed edge: Eq. (9)'s Welsch value, or the
    squared norm in both squared-norm variants."""
    return welsch(x2, nu) if robust == "welsch" else np.asarray(x2, np.float64).copy()


def reg_weight(y2, nu, robust="welsch"):
    """Squared entries of W_r: Eq. (14)'s Welsch weight, or 1."""
    y2 = np.asarray(y2, np.float64)
    return welsch_weight(y2, nu) if robust == "welsch" else np.ones_like(y2)


def welsch_surrogate(x, y, nu):
    """Eq. (13): psi(x|y) = psi(y) + (1 - psi(y))/(2 nu^2) (x^2 - y^2)."""
    x = np.asarray(x, np.float64)
    y = np.asarray(y, np.float64)
    return welsch(y * y, nu) + welsch_weight(y * y, nu) * (x * x - y * y)


# --------------------------------------------------------------------------
# warp, closest points, residuals
# --------------------------------------------------------------------------

def warp(prob: Problem, X: np.ndarray, src: Optional[np.ndarray] = None) -> np.ndarray:
    """Eq. (2): v_hat_i = sum_j w_ij (A_j (v_i - p_j) + p_j + t_j)."""
    V = prob.src if src is None else np.asarray(src, np.float64)
    out = np.zeros_like(V)
    for s in range(prob.infl_idx.shape[1]):
        j = prob.infl_idx[:, s]
        w = prob.infl_w[:, s]
        d = V - prob.nodes[j]
        A = X[j, :3, :]            # rows are A^T, so d @ A^T-rows = (A d)^T
        t = X[j, 3, :]
        out += w[:, None] * (np.einsum("ni,nij->nj", d, A) + prob.nodes[j] + t)
    return out


def nearest(query: np.ndarray, tgt: np.ndarray, chunk: int = 64, threads: Optional[int] = None):
    """Closest target point of every query by brute force (Sec. 3.2, the
    definition of u_rho(i)).  Distances in difference form sum_c (u_c - q_c)^2;
    ties go to the lowest target index.  Returns (rho, d2, d2_second) where
    d2_second is the second smallest squared distance (inf if M == 1)."""
    q = np.asarray(query, np.float64)
    u = np.asarray(tgt, np.float64)
    n = q.shape[0]
    rho = np.empty(n, np.int64)
    d1 = np.empty(n)
    d2 = np.empty(n)

    def work(s):
        e = min(n, s + chunk)
        dd = ((u[None, :, :] - q[s:e, None, :]) ** 2).sum(-1)   # (c, M)
        a = np.argmin(dd, 1)                                   # first minimum = lowest index
        rho[s:e] = a
        best = dd[np.arange(e - s), a]
        d1[s:e] = best
        if u.shape[0] > 1:
            dd[np.arange(e - s), a] = np.inf
            d2[s:e] = dd.min(1)
        else:
            d2[s:e] = np.inf

    starts = range(0, n, chunk)
    nt = threads or min(16, os.cpu_count() or 1)
    if nt > 1 and n > chunk:
        with ThreadPoolExecutor(nt) as ex:
            list(ex.map(work, starts))
    else:
        for s in starts:
            work(s)
    return rho, d1, d2


def reg_residuals(prob: Problem, X: np.ndarray) -> np.ndarray:
    """Eq. (7) for every ordered neighbour pair (i, j):
    D_ij = r_ij (A_j (p_i - p_j) + p_j + t_j - (p_i + t_i))."""
    i = prob.dir_edges[:, 0]
    j = prob.dir_edges[:, 1]
    d = prob.nodes[i] - prob.nodes[j]
    Aj = X[j, :3, :]
    val = np.einsum("ni,nij->nj", d, Aj) + prob.nodes[j] + X[j, 3, :] - prob.nodes[i] - X[i, 3, :]
    return prob.r[:, None] * val


def proj_rotation(A: np.ndarray):
    """Closest rotation to each 3x3 matrix in Frobenius norm (rotation term
    of Sec. 3.2): with A = U S V^T, R = U diag(1, 1, det(U V^T)) V^T.
    Returns R (n,3,3) and the per-node term |A - R|_F^2."""
    U, S, Vt = np.linalg.svd(A)
    d = np.sign(np.linalg.det(U @ Vt))
    d[d == 0] = 1.0
    D = np.ones((A.shape[0], 3))
    D[:, 2] = d
    R = np.einsum("nij,nj,njk->nik", U, D, Vt)
    e = ((A - R) ** 2).sum((1, 2))
    return R, e


# --------------------------------------------------------------------------
# energy (Eq. 4)
# --------------------------------------------------------------------------

@dataclasses.dataclass
class Eval:
    X: np.ndarray
    vhat: np.ndarray
    rho: np.ndarray
    d2: np.ndarray
    d2_second: np.ndarray
    D: np.ndarray
    R: np.ndarray
    e_rot: np.ndarray
    E_align: float
    E_reg: float
    E_rot: float
    E: float


def evaluate(prob: Problem, X: np.ndarray, nu_a: float, nu_r: float, alpha: float,
             beta: float, src: Optional[np.ndarray] = None, nn=None, robust="welsch") -> Eval:
    """E(X) = E_align + alpha E_reg + beta E_rot (Eq. 4) with Eqs. (5), (9)
    and the rotation term; the closest points are recomputed at X.  Other
    `robust` variants swap the per-term functions (Sec. 4.1)."""
    vhat = warp(prob, X, src)
    rho, d2, d2s = (nn or nearest)(vhat, prob.tgt)
    D = reg_residuals(prob, X)
    R, e_rot = proj_rotation(X[:, :3, :].transpose(0, 2, 1))
    Ea = math.fsum(align_penalty(d2, nu_a, robust))
    Er = math.fsum(reg_penalty((D ** 2).sum(1), nu_r, robust))
    Eo = math.fsum(e_rot)
    return Eval(X, vhat, rho, d2, d2s, D, R, e_rot, Ea, Er, Eo, Ea + alpha * Er + beta * Eo)


def rescore(prob: Problem, ev: Eval, nu_a, nu_r, alpha, beta, robust="welsch") -> Eval:
    """Energy of the same X at other (nu, alpha, beta): closest points and
    rotations do not depend on them."""
    Ea = math.fsum(align_penalty(ev.d2, nu_a, robust))
    Er = math.fsum(reg_penalty((ev.D ** 2).sum(1), nu_r, robust))
    return dataclasses.replace(ev, E_align=Ea, E_reg=Er, E=Ea + alpha * Er + beta * ev.E_rot)


# --------------------------------------------------------------------------
# surrogate in matrix form and its minimizer (Sec. 3.3.2, Eq. 21)
# --------------------------------------------------------------------------

def matrices(prob: Problem, ev: Eval, nu_a: float, nu_r: float, robust="welsch"):
    """Build F, Q, W_a^2 (as a vector), H, Y, W_r^2, J, Z of Sec. 3.3.2 at the
    evaluation point ev (its closest points u^k, residuals D^k, rotations)."""
    N, n, k = prob.n_src, prob.n_nodes, prob.infl_idx.shape[1]
    rows = np.repeat(np.arange(N), 4 * k)
    cols = (4 * prob.infl_idx[:, :, None] + np.arange(4)[None, None, :]).reshape(-1)
    d = prob.src[:, None, :] - prob.nodes[prob.infl_idx]                 # (N, k, 3)
    blk = np.concatenate([d, np.ones((N, k, 1))], 2) * prob.infl_w[:, :, None]
    F = sp.csr_matrix((blk.reshape(-1), (rows, cols)), shape=(N, 4 * n))
    Q = prob.tgt[ev.rho] - np.einsum("nk,nkc->nc", prob.infl_w, prob.nodes[prob.infl_idx])
    wa = align_weight(ev.d2, nu_a, robust)

    i = prob.dir_edges[:, 0]
    j = prob.dir_edges[:, 1]
    h = prob.dir_edges.shape[0]
    dp = prob.nodes[i] - prob.nodes[j]
    r = prob.r
    hr = np.repeat(np.arange(h), 5)
    hc = np.concatenate([4 * j[:, None] + np.arange(4)[None, :], 4 * i[:, None] + 3], 1).reshape(-1)
    hv = np.concatenate([r[:, None] * dp, r[:, None], -r[:, None]], 1).reshape(-1)
    H = sp.csr_matrix((hv, (hr, hc)), shape=(h, 4 * n))
    Y = r[:, None] * dp
    wr = reg_weight((ev.D ** 2).sum(1), nu_r, robust)

    jd = np.tile(np.array([1.0, 1.0, 1.0, 0.0]), n)
    J = sp.diags(jd)
    Z = np.zeros((n, 4, 3))
    Z[:, :3, :] = ev.R.transpose(0, 2, 1)
    return F, Q, wa, H, Y, wr, J, Z.reshape(4 * n, 3)


def normal_equations(prob: Problem, ev: Eval, nu_a, nu_r, alpha, beta, robust="welsch"):
    """Eq. (21): K = F^T W_a^2 F + alpha H^T W_r^2 H + beta J^T J,
    B = F^T W_a^2 Q + alpha H^T W_r^2 Y + beta J^T J Z."""
    F, Q, wa, H, Y, wr, J, Z = matrices(prob, ev, nu_a, nu_r, robust)
    Wa = sp.diags(wa)
    Wr = sp.diags(wr)
    K = (F.T @ Wa @ F + alpha * (H.T @ Wr @ H) + beta * (J.T @ J)).tocsc()
    B = F.T @ (wa[:, None] * Q) + alpha * (H.T @ (wr[:, None] * Y)) + beta * (J.T @ (J @ Z))
    return K, np.asarray(B)


def mm_update(prob: Problem, ev: Eval, nu_a, nu_r, alpha, beta, robust="welsch"):
    """Minimizer of the quadratic surrogate: solve K X = B (Eq. 21) with one
    sparse LU factorization and three right-hand sides."""
    K, B = normal_equations(prob, ev, nu_a, nu_r, alpha, beta, robust)
    lu = spla.splu(K)
    Xn = lu.solve(B)
    return Xn.reshape(prob.n_nodes, 4, 3), K, B


def surrogate_value(prob: Problem, X: np.ndarray, ev: Eval, nu_a, nu_r, alpha, beta,
                    src: Optional[np.ndarray] = None, robust="welsch") -> float:
    """Full surrogate E(X | X^k) with the constants of Eq. (13) kept, so that
    it equals E at X^k: alignment with fixed u^k (Eqs. 13, 15-16),
    regularization (Eq. 14) and rotation with fixed proj(A^k)."""
    vhat = warp(prob, X, src)
    u = prob.tgt[ev.rho]
    x2 = ((vhat - u) ** 2).sum(1)
    Sa = math.fsum(align_penalty(ev.d2, nu_a, robust) + align_weight(ev.d2, nu_a, robust) * (x2 - ev.d2))
    D = reg_residuals(prob, X)
    y2 = (ev.D ** 2).sum(1)
    Sr = math.fsum(reg_penalty(y2, nu_r, robust) + reg_weight(y2, nu_r, robust) * ((D ** 2).sum(1) - y2))
    A = X[:, :3, :].transpose(0, 2, 1)
    So = math.fsum(((A - ev.R) ** 2).sum((1, 2)))
    return Sa + alpha * Sr + beta * So


# --------------------------------------------------------------------------
# Anderson acceleration (Sec. 3.3.4)
# --------------------------------------------------------------------------

def _cholesky_solve(G: np.ndarray, b: np.ndarray, rel_pivot: float = 1e-14):
    """Cholesky of the small Gram matrix.  Reading: the paper leaves a
    rank-deficient least-squares problem open; if any pivot (the value under
    the square root) is <= rel_pivot * max diag, return None (the caller then
    uses theta = 0, i.e. the plain MM step)."""
    m = G.shape[0]
    L = np.zeros_like(G)
    tol = rel_pivot * max(float(np.max(np.diag(G))), 0.0)
    for j in range(m):
        piv = G[j, j] - sum(L[j, q] * L[j, q] for q in range(j))
        if not piv > tol:
            return None
        L[j, j] = math.sqrt(piv)
        for i in range(j + 1, m):
            L[i, j] = (G[i, j] - sum(L[i, q] * L[j, q] for q in range(j))) / L[j, j]
    y = np.zeros(m)
    for i in range(m):
        y[i] = (b[i] - sum(L[i, q] * y[q] for q in range(i))) / L[i, i]
    x = np.zeros(m)
    for i in reversed(range(m)):
        x[i] = (y[i] - sum(L[q, i] * x[q] for q in range(i + 1, m))) / L[i, i]
    return x


def anderson(hist_G: List[np.ndarray], hist_F: List[np.ndarray], m: int):
    """Eqs. (22)-(23), standard type-II Anderson acceleration over the last
    m_k + 1 entries of the history (G^(k) = G(X^(k)), F^(k) = G^(k) - X^(k)):
    theta = argmin |F^k - sum_j theta_j (F^(k-j+1) - F^(k-j))|^2, then
    X_AA = G^k - sum_j theta_j (G^(k-j+1) - G^(k-j)).

    Reading: m_k = min(len(history) - 1, m), so the first iteration of every
    stage has m_k = 0 and returns G^k.  Returns (X_AA, theta, m_k, used),
    used = False when m_k = 0 or the Gram solve fell back to theta = 0."""
    mk = min(len(hist_G) - 1, m)
    Gk = hist_G[-1]
    if mk == 0:
        return Gk.copy(), np.zeros(0), 0, False
    dF = np.stack([hist_F[-j] - hist_F[-j - 1] for j in range(1, mk + 1)], 1)
    dG = np.stack([hist_G[-j] - hist_G[-j - 1] for j in range(1, mk + 1)], 1)
    Fk = hist_F[-1]
    gram = dF.T @ dF
    rhs = dF.T @ Fk
    theta = _cholesky_solve(gram, rhs)
    if theta is None:
        return Gk.copy(), np.zeros(mk), mk, False
    return Gk - dG @ theta, theta, mk, True


# --------------------------------------------------------------------------
# parameters (Sec. 3.3.3, Eq. 26)
# --------------------------------------------------------------------------

@dataclasses.dataclass
class Params:
    k_alpha: float = 100.0
    k_beta: float = 1.0
    eps: float = 1e-5          # convergence threshold on max displacement (Sec. 4.1)
    imax: int = 100            # iteration cap per nu stage (Sec. 4.1)
    max_total_iters: int = 0   # 0 = no cap on the number of surrogate solves
    aa_m: int = 5
    nu_a0: float = 0.0         # <= 0: median closest-point distance at X = I
    nu_a_min: float = 0.0      # <= 0: mean edge length / sqrt(3)
    nu_r0: float = 0.0         # <= 0: 3 * mean edge length
    robust: str = "welsch"     # one of ROBUST (Sec. 4.1 variants)
    nu_mode: str = "dynamic"   # "dynamic" or the fixed "max", "min", "med" (Sec. 4.1)


def term_weights(prob: Problem, p: Params, nu_a: float, nu_r: float):
    """Eq. (26): alpha = k_alpha |V|/|E_G| nu_r^2/nu_a^2,
    beta = k_beta |V|/|V_G| / (2 nu_a^2).  Reading: recomputed at every nu
    stage.

    Reading for the squared-norm variants (Sec. 4.1 names no weights): the
    Welsch energy scaled by 2 nu_a^2 tends, for small residuals, to
    sum |e|^2 + k_alpha |V|/|E_G| sum |D|^2 + k_beta |V|/|V_G| E_rot, so
    alpha = k_alpha |V|/|E_G| and beta = k_beta |V|/|V_G| there."""
    N, n, E = prob.n_src, prob.n_nodes, prob.n_undirected
    if p.robust != "welsch":
        return p.k_alpha * (N / E), p.k_beta * (N / n)
    alpha = p.k_alpha * (N / E) * (nu_r * nu_r) / (nu_a * nu_a)
    beta = p.k_beta * (N / n) / (2.0 * nu_a * nu_a)
    return alpha, beta


def initial_nu(prob: Problem, p: Params, d2_at_identity: np.ndarray):
    """Sec. 3.3.3: nu_a starts at the median closest-point distance and stops
    at l/sqrt(3); nu_r starts at 3 l (l = mean source edge length).
    Reading: the start is clamped to be >= the lower bound (an identical pair
    has median distance 0)."""
    lbar = prob.mean_edge_len
    nu_min = p.nu_a_min if p.nu_a_min > 0 else lbar / math.sqrt(3.0)
    nu_a = p.nu_a0 if p.nu_a0 > 0 else float(np.median(np.sqrt(d2_at_identity)))
    nu_a = max(nu_a, nu_min)
    nu_r = p.nu_r0 if p.nu_r0 > 0 else 3.0 * lbar
    return nu_a, nu_min, nu_r


def nu_schedule(nu_a, nu_min, nu_r):
    """The (nu_a, nu_r) of every stage of the dynamic update (Sec. 3.3.3):
    nu_a halves down to its bound, nu_r halves with it."""
    out = [(nu_a, nu_r)]
    while nu_a != nu_min:
        nu_a = max(nu_a / 2.0, nu_min)
        nu_r = nu_r / 2.0
        out.append((nu_a, nu_r))
    return out


def fixed_nu(nu_a, nu_min, nu_r, mode):
    """Sec. 4.1's fixed-parameter variants: both parameters held at the
    largest ("max"), smallest ("min") or midway ("med") values that the
    dynamic update would reach from this start."""
    sch = nu_schedule(nu_a, nu_min, nu_r)
    (a_hi, r_hi), (a_lo, r_lo) = sch[0], sch[-1]
    if mode == "max":
        return a_hi, r_hi
    if mode == "min":
        return a_lo, r_lo
    if mode == "med":
        return 0.5 * (a_hi + a_lo), 0.5 * (r_hi + r_lo)
    raise ValueError(mode)


# --------------------------------------------------------------------------
# the solver (Alg. 2)
# --------------------------------------------------------------------------

def solve(prob: Problem, p: Params, X0: Optional[np.ndarray] = None, nn=None,
          force: Optional[List[Optional[bool]]] = None, log_evals: bool = False,
          force_stage_end: Optional[List[Optional[bool]]] = None, step_noise=None):
    """Alg. 2: nu continuation around MM iterations accelerated by Anderson
    acceleration with the energy-decrease safeguard.

    Readings:
    * an "MM iteration" is one surrogate solve; `max_total_iters` caps the
      number of solves over all stages (0 = no cap);
    * at the first iteration of a stage (m_k = 0), or when the Gram solve
      falls back to theta = 0, the candidate is G(X^k) itself and is accepted
      without a test (MM never increases E);
    * otherwise X_AA is accepted iff E(X_AA) < E(X^k) (the displayed rule of
      Sec. 3.3.4); on rejection X^{k+1} = G(X^k) is taken without a second
      test, and the history is kept;
    * a stage ends when max_i |v_hat^{k+1} - v_hat^k| < eps or after imax
      solves in the stage; the whole solve ends after the stage whose nu_a
      equals its lower bound, or when the solve budget is used up;
    * at every new stage nu_a = max(nu_a/2, lower bound), nu_r = nu_r/2,
      alpha and beta follow Eq. (26), the history is cleared;
    * Sec. 4.1 variants: a fixed nu_mode holds (nu_a, nu_r) at fixed_nu's
      values for one stage; "l2" has no parameter to update and runs one
      stage; "l2r" follows the dynamic update of nu_a like the method.
    `force[t]` overrides the accept/reject decision of solve t and
    `force_stage_end[t]` whether a stage ends after it (replay).
    `step_noise` = (seed, sigma) adds seeded N(0, sigma^2) noise to every
    surrogate minimizer, to measure how the trajectory responds to an
    inexact step (a sensitivity probe for the tests, not part of Alg. 2)."""
    rb = p.robust
    X = identity(prob.n_nodes) if X0 is None else np.array(X0, np.float64)
    ev0 = evaluate(prob, X, 1.0, 1.0, 0.0, 0.0, nn=nn)
    nu_a, nu_min, nu_r = initial_nu(prob, p, ev0.d2)
    if p.nu_mode != "dynamic":
        nu_a, nu_r = fixed_nu(nu_a, nu_min, nu_r, p.nu_mode)
        nu_min = nu_a
    if rb == "l2":
        nu_min = nu_a
    alpha, beta = term_weights(prob, p, nu_a, nu_r)
    ev = rescore(prob, ev0, nu_a, nu_r, alpha, beta, rb)
    log = []
    total = 0
    stage = 0
    noise_rng = np.random.default_rng(step_noise[0]) if step_noise is not None else None
    while True:
        hist_G: List[np.ndarray] = []
        hist_F: List[np.ndarray] = []
        it = 0
        while True:
            Xn, _, _ = mm_update(prob, ev, nu_a, nu_r, alpha, beta, rb)
            if noise_rng is not None:
                Xn = Xn + step_noise[1] * noise_rng.standard_normal(Xn.shape)
            hist_G.append(Xn.reshape(-1).copy())
            hist_F.append((Xn - X).reshape(-1))
            if len(hist_G) > p.aa_m + 1:
                hist_G.pop(0)
                hist_F.pop(0)
            xaa, theta, mk, used = anderson(hist_G, hist_F, p.aa_m)
            E_before = ev.E
            E_cand = None
            if used:
                ev_c = evaluate(prob, xaa.reshape(X.shape), nu_a, nu_r, alpha, beta, nn=nn, robust=rb)
                E_cand = ev_c.E
                acc = ev_c.E < ev.E
                if force is not None and total < len(force) and force[total] is not None:
                    acc = bool(force[total])
                if acc:
                    ev_n = ev_c
                else:
                    ev_n = evaluate(prob, Xn, nu_a, nu_r, alpha, beta, nn=nn, robust=rb)
            else:
                acc = True
                ev_n = evaluate(prob, Xn, nu_a, nu_r, alpha, beta, nn=nn, robust=rb)
            disp = float(np.sqrt(((ev_n.vhat - ev.vhat) ** 2).sum(1).max()))
            entry = dict(total=total, stage=stage, it=it, nu_a=nu_a, nu_r=nu_r, alpha=alpha,
                         beta=beta, E_before=E_before, E_cand=E_cand, aa_used=used,
                         accepted=bool(acc) if used else None, m_k=mk, theta=theta,
                         E_after=ev_n.E, maxdisp=disp)
            if log_evals:
                entry["X"] = ev_n.X.copy()
            log.append(entry)
            X, ev = ev_n.X, ev_n
            it += 1
            total += 1
            budget = p.max_total_iters > 0 and total >= p.max_total_iters
            end = disp < p.eps or it >= p.imax
            if force_stage_end is not None and total - 1 < len(force_stage_end) \
                    and force_stage_end[total - 1] is not None:
                end = bool(force_stage_end[total - 1])
            if end or budget:
                break
        if nu_a == nu_min or (p.max_total_iters > 0 and total >= p.max_total_iters):
            break
        stage += 1
        nu_a = max(nu_a / 2.0, nu_min)
        nu_r = nu_r / 2.0
        alpha, beta = term_weights(prob, p, nu_a, nu_r)
        ev = rescore(prob, ev, nu_a, nu_r, alpha, beta, rb)
    return dict(X=X, vhat=ev.vhat, E=ev.E, log=log, total=total, stages=stage + 1,
                nu_a=nu_a, nu_r=nu_r, eval=ev)


# --------------------------------------------------------------------------
# gradient of E (differentiable form)
# --------------------------------------------------------------------------

def energy_grad(prob: Problem, X: np.ndarray, nu_a, nu_r, alpha, beta,
                src: Optional[np.ndarray] = None, ev: Optional[Eval] = None):
    """Gradient of E (Eq. 4) with respect to X (n,4,3) and the source points
    (N,3).  The closest points are held fixed (E is piecewise smooth in them
    and the minimum over targets has the gradient of its active piece); the
    graph (p_j, w_ij, r_ij) is frozen, so only the explicit v_i of Eq. (2)
    moves with the source.

    d psi_nu(|e|)/d e = exp(-|e|^2/(2 nu^2)) e / nu^2;
    d |A - proj(A)|_F^2 / dA = 2 (A - proj(A))."""
    V = prob.src if src is None else np.asarray(src, np.float64)
    if ev is None:
        ev = evaluate(prob, X, nu_a, nu_r, alpha, beta, src=V)
    e = ev.vhat - prob.tgt[ev.rho]
    g = np.exp(-ev.d2 / (2 * nu_a * nu_a))[:, None] * e / (nu_a * nu_a)      # dE/dv_hat
    gX = np.zeros((prob.n_nodes, 4, 3))
    gV = np.zeros_like(V)
    for s in range(prob.infl_idx.shape[1]):
        j = prob.infl_idx[:, s]
        w = prob.infl_w[:, s]
        d = V - prob.nodes[j]
        aff = np.concatenate([d, np.ones((d.shape[0], 1))], 1)               # [v_i - p_j; 1]
        np.add.at(gX, j, w[:, None, None] * aff[:, :, None] * g[:, None, :])
        A = X[j, :3, :].transpose(0, 2, 1)
        gV += w[:, None] * np.einsum("nij,ni->nj", A, g)                       # A^T g
    D = ev.D
    h = np.exp(-(D ** 2).sum(1) / (2 * nu_r * nu_r))[:, None] * D / (nu_r * nu_r)
    i = prob.dir_edges[:, 0]
    j = prob.dir_edges[:, 1]
    dp = prob.nodes[i] - prob.nodes[j]
    aff = np.concatenate([dp, np.ones((dp.shape[0], 1))], 1) * prob.r[:, None]
    np.add.at(gX, j, alpha * aff[:, :, None] * h[:, None, :])
    np.add.at(gX[:, 3, :], i, -alpha * prob.r[:, None] * h)
    A = X[:, :3, :].transpose(0, 2, 1)
    gX[:, :3, :] += 2.0 * beta * (A - ev.R).transpose(0, 2, 1)
    return gX, gV, ev
