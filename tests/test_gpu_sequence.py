"""Sequence tracking: new targets for a set-up template, warm-started
solves along the frames, and resuming a solve from its returned state,
against fresh uploads and the FP64 oracle."""
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


@pytest.fixture(scope="module")
def seq():
    return synth.sh_sequence(6000, 3000, n_frames=4, n_nodes=100, k=4, e=8)


def _frame_pair(seq, f):
    return dataclasses.replace(seq.template, tgt=seq.frames[f], gt=seq.gts[f])


def _replay(log):
    fa = [e["accepted"] if e["aa_used"] else None for e in log]
    fs = [1 if (b is None or b["stage"] != a["stage"]) else 0 for a, b in zip(log, log[1:] + [None])]
    return fa, fs


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_set_targets_equals_fresh_upload(seq, prec):
    """Swapping a pair's targets gives bitwise the solve of a new upload
    with those targets."""
    _announce(f"test_set_targets_equals_fresh_upload {prec}")
    dt = torch.float64 if prec == "f64" else torch.float32
    p = amm.AMM_FP64_PLAIN if prec == "f64" else amm.AMM_FP32_REFINE
    n = seq.template.n_nodes
    res = []
    for swap in (False, True):
        with Session(_frame_pair(seq, 0 if swap else 2), dt) as s:
            if swap:
                amm.amm_set_targets(s.h, 0, torch.tensor(seq.frames[2], dtype=dt, device="cuda:0"))
            X = torch.empty(n, 4, 3, dtype=dt, device="cuda:0")
            st = amm.amm_solve(s.h, amm.amm_params_default(aa_m=5, max_total_iters=10, precision=p), X)[0]
            torch.cuda.synchronize()
            res.append((X.cpu().numpy(), st))
    assert np.array_equal(res[0][0], res[1][0])
    assert res[0][1]["energy"] == res[1][1]["energy"]
    assert res[0][1]["iters"] == res[1][1]["iters"]


def test_warm_started_chain_matches_oracle(seq):
    """Frame 2 from X = I, then frame 4 from frame 2's result on the same
    handle (targets swapped), float64 with decisions replayed, against the
    oracle doing the same."""
    _announce("test_warm_started_chain_matches_oracle")
    iters = 12
    p = O.Params(aa_m=5, max_total_iters=iters)
    pa, pb = O.from_pair(_frame_pair(seq, 0)), O.from_pair(_frame_pair(seq, 1))
    ra = O.solve(pa, p)
    rb = O.solve(pb, p, X0=ra["X"])
    n = seq.template.n_nodes
    with Session(_frame_pair(seq, 0), torch.float64) as s:
        X = torch.empty(n, 4, 3, dtype=torch.float64, device="cuda:0")
        fa, fs = _replay(ra["log"])
        prm = amm.amm_params_default(aa_m=5, max_total_iters=iters, precision=amm.AMM_FP64_PLAIN)
        sa = amm.amm_solve(s.h, prm, X, force_accept=fa, force_stage_end=fs)[0]
        amm.amm_set_targets(s.h, 0, torch.tensor(seq.frames[1], device="cuda:0"))
        v = torch.empty(seq.template.n_src, 3, dtype=torch.float64, device="cuda:0")
        fa, fs = _replay(rb["log"])
        prm = amm.amm_params_default(aa_m=5, max_total_iters=iters, precision=amm.AMM_FP64_PLAIN,
                                     init_identity=0)
        sb = amm.amm_solve(s.h, prm, X, v, force_accept=fa, force_stage_end=fs)[0]
        torch.cuda.synchronize()
        v = v.cpu().numpy()
    assert sa["iters"] == ra["total"] and sb["iters"] == rb["total"]
    assert sb["energy"] == pytest.approx(rb["E"], rel=1e-5)
    assert math.sqrt(((v - rb["vhat"]) ** 2).sum(1).mean()) < 1e-5


def test_resume_from_returned_state_matches_oracle(seq):
    """A solve cut at its budget resumes from its returned X with nu set to
    the returned nu (the checkpoint is X and nu); both parts follow the
    oracle doing the same."""
    _announce("test_resume_from_returned_state_matches_oracle")
    pr = _frame_pair(seq, 2)
    prob = O.from_pair(pr)
    r1 = O.solve(prob, O.Params(aa_m=5, max_total_iters=8))
    p2 = O.Params(aa_m=5, max_total_iters=8, nu_a0=r1["nu_a"], nu_r0=r1["nu_r"])
    r2 = O.solve(prob, p2, X0=r1["X"])
    with Session(pr, torch.float64) as s:
        X = torch.empty(pr.n_nodes, 4, 3, dtype=torch.float64, device="cuda:0")
        fa, fs = _replay(r1["log"])
        prm = amm.amm_params_default(aa_m=5, max_total_iters=8, precision=amm.AMM_FP64_PLAIN)
        s1 = amm.amm_solve(s.h, prm, X, force_accept=fa, force_stage_end=fs)[0]
        assert s1["nu_a"] == pytest.approx(r1["nu_a"], rel=1e-12)
        fa, fs = _replay(r2["log"])
        prm = amm.amm_params_default(aa_m=5, max_total_iters=8, precision=amm.AMM_FP64_PLAIN, init_identity=0,
                                     nu_a0=s1["nu_a"], nu_r0=s1["nu_r"])
        s2 = amm.amm_solve(s.h, prm, X, force_accept=fa, force_stage_end=fs)[0]
        torch.cuda.synchronize()
    assert s2["iters"] == r2["total"]
    assert s2["nu_a"] == pytest.approx(r2["nu_a"], rel=1e-12)
    assert s2["energy"] == pytest.approx(r2["E"], rel=1e-5)


def test_set_targets_arguments_are_validated(seq):
    _announce("test_set_targets_arguments_are_validated")
    with Session(_frame_pair(seq, 0), torch.float64) as s:
        t = torch.tensor(seq.frames[1], device="cuda:0")
        for args, code in (((1, t), amm.AMM_ERR_INVALID_ARG), ((0, t[:-1]), amm.AMM_ERR_INVALID_ARG)):
            with pytest.raises(amm.AmmError) as ei:
                amm.amm_set_targets(s.h, *args)
            assert ei.value.status == code
        bad = t.clone()
        bad[3, 2] = float("inf")
        with pytest.raises(amm.AmmError) as ei:
            amm.amm_set_targets(s.h, 0, bad)
        assert ei.value.status == amm.AMM_ERR_NONFINITE
    h = amm.amm_create(0, torch.cuda.current_stream().cuda_stream)
    try:
        with pytest.raises(amm.AmmError) as ei:
            amm.amm_set_targets(h, 0, t)
        assert ei.value.status == amm.AMM_ERR_STATE
    finally:
        amm.amm_destroy(h)


def test_set_targets_from_host_float32(seq):
    """New targets given as float32 coordinates in host memory: the solve
    equals, bitwise, that of a new upload of the same (float32-valued)
    coordinates."""
    _announce("test_set_targets_from_host_float32")
    t32 = np.ascontiguousarray(seq.frames[3], np.float32)
    n = seq.template.n_nodes
    res = []
    for swap in (False, True):
        pair = _frame_pair(seq, 0) if swap else dataclasses.replace(_frame_pair(seq, 3), tgt=t32.astype(np.float64))
        with Session(pair, torch.float64) as s:
            if swap:
                amm.amm_set_targets(s.h, 0, t32)
            X = torch.empty(n, 4, 3, dtype=torch.float64, device="cuda:0")
            st = amm.amm_solve(s.h, amm.amm_params_default(aa_m=5, max_total_iters=8,
                                                           precision=amm.AMM_FP64_PLAIN), X)[0]
            torch.cuda.synchronize()
            res.append((X.cpu().numpy(), st))
    assert np.array_equal(res[0][0], res[1][0])
    assert res[0][1]["energy"] == res[1][1]["energy"]


def test_set_targets_permuted_200k():
    """The 200,000 targets of the large pair handed back in a shuffled
    order (a new Morton sort and new octree tables, built on the device):
    every closest distance equals the set-up structure's bitwise, and the
    closest target is the same point wherever the best and second-best
    distances differ by more than 1e-6 relative."""
    _announce("test_set_targets_permuted_200k")
    from scipy.spatial import cKDTree
    from tests.helpers import margin_ok, rounded
    pair = rounded(synth.make_workload("sh200k"), np.float32)
    N, n = pair.n_src, pair.n_nodes
    X = torch.tensor(synth.perturbed_transforms(n, 7111, 0.01, 0.001).astype(np.float32), device="cuda:0")
    perm = np.random.default_rng(7112).permutation(pair.n_tgt)
    out = []
    with Session(pair, torch.float32) as s:
        for swap in (False, True):
            if swap:
                amm.amm_set_targets(s.h, 0, torch.tensor(pair.tgt[perm], dtype=torch.float32, device="cuda:0"))
            rho = torch.empty(N, dtype=torch.int32, device="cuda:0")
            d2 = torch.empty(N, dtype=torch.float32, device="cuda:0")
            vh = torch.empty(N, 3, dtype=torch.float32, device="cuda:0")
            amm.amm_step(s.h, X, 0.02, 0.05, 10.0, 100.0, amm.AMM_FP32_REFINE, rho=rho, d2=d2, v_hat=vh)
            torch.cuda.synchronize()
            out.append((rho.cpu().numpy(), d2.cpu().numpy(), vh.cpu().numpy().astype(np.float64)))
    (r0, d0, v0), (r1, d1, v1) = out
    assert np.array_equal(v0, v1)
    assert np.array_equal(d0, d1)
    dk, _ = cKDTree(pair.tgt).query(v0, k=2)
    ok = margin_ok(dk[:, 0] ** 2, dk[:, 1] ** 2)
    print(f"sh200k permuted targets: {ok.sum()} of {N} above the margin, "
          f"{int((perm[r1][ok] != r0[ok]).sum())} differ", file=sys.stderr)
    assert ok.mean() > 0.99
    assert np.array_equal(perm[r1][ok], r0[ok])
