"""The coarse level of the CG preconditioner at its largest order: 2,000
graph nodes give 32 aggregates, a coarse matrix of order 128, whose inverse
is the largest one the matrix-core Gauss-Jordan kernel forms.  One float64
MM step (Eq. 21) with each preconditioner: both must reach the same
minimizer, and the two-level one in far fewer CG iterations (a wrong or
inaccurate coarse inverse still converges, only slower, so the iteration
count is what exposes it)."""
import sys

import numpy as np
import pytest

from paper_2206_03410_amd import amm, synth
from tests.helpers import Session

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _scalars(pair):
    """Sec. 3.3.3 start values of nu and the Eq. 26 weights, from scipy's
    exact closest points at the undeformed sources."""
    from scipy.spatial import cKDTree
    d = cKDTree(pair.tgt).query(pair.src)[0]
    lbar = pair.mean_edge_len
    nu_a = max(float(np.median(d)), lbar / np.sqrt(3.0))
    nu_r = 3.0 * lbar
    prm = amm.amm_params_default()
    alpha = prm.k_alpha * pair.n_src / pair.n_edges * (nu_r / nu_a) ** 2
    beta = prm.k_beta * pair.n_src / pair.n_nodes / (2.0 * nu_a * nu_a)
    return nu_a, nu_r, alpha, beta


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_two_level_matches_block_jacobi_at_order_128(dtype):
    print(f"[gpu-test] test_two_level_matches_block_jacobi_at_order_128 {dtype}", file=sys.stderr, flush=True)
    pair = synth.sh_pair(6100, n_src=20000, n_nodes=2000, k=4, e=8)
    assert pair.n_nodes == 2000
    nu_a, nu_r, alpha, beta = _scalars(pair)
    X = synth.perturbed_transforms(pair.n_nodes, 6101, 0.01, 0.001)
    t_dt = torch.float64 if dtype == "f64" else torch.float32
    prec = amm.AMM_FP64_PLAIN if dtype == "f64" else amm.AMM_FP32_REFINE
    res = {}
    with Session(pair, t_dt) as s:
        Xt = torch.tensor(X, dtype=t_dt, device="cuda:0")
        for name, pc in (("two_level", amm.AMM_PRECOND_TWO_LEVEL), ("block_jacobi", amm.AMM_PRECOND_BLOCK_JACOBI)):
            Xn = torch.empty_like(Xt)
            out = amm.amm_step(s.h, Xt, nu_a, nu_r, alpha, beta, prec, cg_precond=pc, X_next=Xn)
            torch.cuda.synchronize()
            res[name] = (out, Xn.cpu().numpy().astype(np.float64))
    (o2, x2), (oj, xj) = res["two_level"], res["block_jacobi"]
    print(f"order 128 coarse level ({dtype}): CG iterations two-level {o2['cg_iters']}, block Jacobi "
          f"{oj['cg_iters']}; rel residuals {o2['rel_residual']:.2e}, {oj['rel_residual']:.2e}", file=sys.stderr)
    assert o2["rel_residual"] <= 1e-10 and oj["rel_residual"] <= 1e-10
    # both solve the same system to the requested relative residual 1e-10
    assert np.abs(x2 - xj).max() <= 1e-6 * max(1.0, np.abs(xj).max())
    assert o2["cg_iters"] <= 0.6 * oj["cg_iters"]
