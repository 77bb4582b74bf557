"""Parity on a pair whose node rows of K are wide: every point is influenced
by three nodes drawn at random (not the nearest ones), so a solver tile's
rows reach hundreds of distinct column nodes and up to ~90 column blocks
per row.  This takes the CG step's per-block path (a tile with more column
nodes than its shared table holds) and the loop over column blocks past
each lane's first two."""
import dataclasses
import math
import sys

import numpy as np
import pytest

from oracle import amm_oracle as O
from paper_2206_03410_amd import amm, synth
from tests.helpers import Session

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _announce(name):
    print(f"[gpu-test] {name}", file=sys.stderr, flush=True)


def _wide_pair():
    base = synth.torus_pair(1000, n_src=3000, n_tgt=3000, n_nodes=300, k=3, e=6)
    rng = np.random.default_rng(77)
    idx = np.stack([rng.choice(base.n_nodes, 3, replace=False) for _ in range(base.n_src)]).astype(np.int32)
    return dataclasses.replace(base, infl_idx=idx, infl_w=np.full((base.n_src, 3), 1.0 / 3.0))


def _replay(log):
    fa = [e["accepted"] if e["aa_used"] else None for e in log]
    fs = [1 if (b is None or b["stage"] != a["stage"]) else 0 for a, b in zip(log, log[1:] + [None])]
    return fa, fs


def test_wide_rows_follow_the_oracle():
    """Float64, 8 MM iterations with the oracle's decisions replayed: final
    energy within 1e-5 relative, deformed points within 1e-5 RMS."""
    _announce("test_wide_rows_follow_the_oracle")
    pair = _wide_pair()
    prob = O.from_pair(pair)
    res = O.solve(prob, O.Params(aa_m=5, max_total_iters=8))
    fa, fs = _replay(res["log"])
    with Session(pair, torch.float64) as s:
        v = torch.empty(prob.n_src, 3, dtype=torch.float64, device="cuda:0")
        prm = amm.amm_params_default(aa_m=5, max_total_iters=8, precision=amm.AMM_FP64_PLAIN)
        st = amm.amm_solve(s.h, prm, None, v, force_accept=fa, force_stage_end=fs)[0]
        torch.cuda.synchronize()
        v = v.cpu().numpy()
    rms = math.sqrt(((v - res["vhat"]) ** 2).sum(1).mean())
    print(f"wide rows: E {st['energy']:.10e} vs {res['E']:.10e}, rms {rms:.3e}, cg {st['cg_iters']}",
          file=sys.stderr)
    assert st["iters"] == res["total"]
    assert st["energy"] == pytest.approx(res["E"], rel=1e-5)
    assert rms < 1e-5


def test_wide_rows_fp32_step_matches_oracle_step():
    """One float32 + refinement step at X = I + delta against the oracle's
    sparse-LU step at the same X: deformed points of the surrogate
    minimizer within 1e-5 RMS, relative residual at most 1e-10."""
    _announce("test_wide_rows_fp32_step_matches_oracle_step")
    pair = _wide_pair()
    pr = dataclasses.replace(pair, src=pair.src.astype(np.float32).astype(np.float64),
                             tgt=pair.tgt.astype(np.float32).astype(np.float64),
                             infl_w=pair.infl_w.astype(np.float32).astype(np.float64))
    prob = O.from_pair(pr)
    p = O.Params()
    ev0 = O.evaluate(prob, O.identity(prob.n_nodes), 1.0, 1.0, 0.0, 0.0)
    nu_a, _, nu_r = O.initial_nu(prob, p, ev0.d2)
    alpha, beta = O.term_weights(prob, p, nu_a, nu_r)
    X = synth.perturbed_transforms(prob.n_nodes, 78, 0.01, 0.001).astype(np.float32).astype(np.float64)
    with Session(pr, torch.float32) as s:
        Xt = torch.tensor(X, dtype=torch.float32, device="cuda:0")
        Xn = torch.empty_like(Xt)
        out = amm.amm_step(s.h, Xt, nu_a, nu_r, alpha, beta, amm.AMM_FP32_REFINE, X_next=Xn)
        torch.cuda.synchronize()
        Xn = Xn.cpu().numpy().astype(np.float64)
    ev = O.evaluate(prob, X, nu_a, nu_r, alpha, beta)
    Xo = np.asarray(O.mm_update(prob, ev, nu_a, nu_r, alpha, beta)[0])
    rms = math.sqrt(((O.warp(prob, Xo) - O.warp(prob, Xn)) ** 2).sum(1).mean())
    print(f"wide rows fp32 step: rms {rms:.3e}, rel residual {out['rel_residual']:.3e}", file=sys.stderr)
    assert out["rel_residual"] <= 1e-10
    assert rms < 1e-5
