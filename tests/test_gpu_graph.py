"""Parity of the device graph builder (Alg. 1 with Euclidean distance)
with the graph oracle, and a registration run on a graph it built."""
import math
import sys

import numpy as np
import pytest

from oracle import amm_oracle as O
from oracle import graph_oracle as G
from paper_2206_03410_amd import amm, synth
from tests.helpers import Session

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _announce(name):
    print(f"[gpu-test] {name}", file=sys.stderr, flush=True)


def _handle():
    return amm.amm_create(0, torch.cuda.current_stream().cuda_stream)


def _axis_margin(V):
    """Smallest gap between consecutive projections, relative to their
    spread: the order is a decision both sides take in float64."""
    m, a = G.principal_axis(V)
    t = np.sort((V - m) @ a)
    return np.diff(t).min() / (t[-1] - t[0])


def _check_against_oracle(V, k, got, radius=None, w_tol=1e-12):
    info, node, idx, w, edges = got
    lbar = G.mean_edge_length(V)
    R = radius if radius else 5.0 * lbar
    ref = G.build_graph(V, R, k)
    assert info["mean_edge_len"] == pytest.approx(lbar, rel=1e-12)
    assert info["radius"] == pytest.approx(R, rel=1e-12)
    assert np.array_equal(node.cpu().numpy(), ref["node_idx"])
    assert np.array_equal(idx.cpu().numpy(), ref["infl_idx"])
    assert np.abs(w.cpu().numpy().astype(np.float64) - ref["infl_w"]).max() <= w_tol
    assert np.array_equal(edges.cpu().numpy(), ref["edges"])
    assert info["n_capped"] == ref["n_capped"]
    assert info["max_influences"] == ref["max_influences"]
    return ref


@pytest.mark.parametrize("case", ["torus700_k4", "torus2k_k3", "sh50k_k6"])
def test_graph_matches_oracle(case):
    """Nodes, influence indices and edges bit-exact, weights within 1e-12,
    mean edge length and R = 5 l within 1e-12 relative."""
    _announce(f"test_graph_matches_oracle {case}")
    if case == "torus700_k4":
        V, k = synth.torus_pair(1000, n_src=700, n_tgt=10, n_nodes=20, k=4, e=6).src, 4
    elif case == "torus2k_k3":
        V, k = synth.make_workload("torus2k").src, 3
    else:
        V, k = synth.make_workload("sh50k").src, 6
    assert _axis_margin(V) > 1e-12
    h = _handle()
    try:
        got = amm.build_graph(h, torch.tensor(V, device="cuda:0"), k)
        torch.cuda.synchronize()
    finally:
        amm.amm_destroy(h)
    print(f"{case}: {got[0]}", file=sys.stderr)
    ref = _check_against_oracle(V, k, got)
    if case == "torus2k_k3":
        assert ref["n_capped"] > 0          # the k cap is exercised


def test_graph_float32_input_and_explicit_radius():
    """float32 points (the oracle sees the same rounded values) and a given
    R: same integers, float32 weights within float32 rounding."""
    _announce("test_graph_float32_input_and_explicit_radius")
    V = synth.make_workload("torus2k").src.astype(np.float32)
    R = 0.05
    h = _handle()
    try:
        got = amm.build_graph(h, torch.tensor(V, device="cuda:0"), 4, radius=R)
        torch.cuda.synchronize()
    finally:
        amm.amm_destroy(h)
    _check_against_oracle(V.astype(np.float64), 4, got, radius=R, w_tol=1e-6)


def test_graph_arguments_are_validated():
    _announce("test_graph_arguments_are_validated")
    V = torch.tensor(synth.make_workload("torus2k").src[:100], device="cuda:0")
    h = _handle()
    try:
        for kw in (dict(k=0), dict(k=9)):
            with pytest.raises(amm.AmmError) as ei:
                amm.amm_build_graph(h, V, **kw)
            assert ei.value.status == amm.AMM_ERR_INVALID_ARG
        with pytest.raises(amm.AmmError) as ei:
            amm.amm_build_graph(h, V[:1], 4)
        assert ei.value.status == amm.AMM_ERR_INVALID_ARG
        bad = V.clone()
        bad[5, 1] = float("nan")
        with pytest.raises(amm.AmmError) as ei:
            amm.amm_build_graph(h, bad, 4)
        assert ei.value.status == amm.AMM_ERR_NONFINITE
        with pytest.raises(amm.AmmError) as ei:
            amm.amm_graph_copy(h)
        assert ei.value.status == amm.AMM_ERR_STATE
    finally:
        amm.amm_destroy(h)


def test_registration_on_a_built_graph():
    """The graph built on the device, with unused influence slots, drives
    Alg. 2 (float64, 15 MM iterations, decisions replayed) to the oracle's
    trajectory on the same graph."""
    _announce("test_registration_on_a_built_graph")
    import dataclasses
    base = synth.make_workload("torus2k")
    k = 4
    h = _handle()
    try:
        info, node, idx, w, edges = amm.build_graph(h, torch.tensor(base.src, device="cuda:0"), k)
        torch.cuda.synchronize()
    finally:
        amm.amm_destroy(h)
    pair = dataclasses.replace(base, node_idx=node.cpu().numpy(), infl_idx=idx.cpu().numpy(),
                               infl_w=w.cpu().numpy(), edges=edges.cpu().numpy(),
                               mean_edge_len=info["mean_edge_len"])
    assert (pair.infl_idx < 0).any()        # unused slots are exercised
    prob = O.from_pair(pair)
    p = O.Params(aa_m=5, max_total_iters=15)
    res = O.solve(prob, p)
    fa = [e["accepted"] if e["aa_used"] else None for e in res["log"]]
    fs = [1 if (b is None or b["stage"] != a["stage"]) else 0
          for a, b in zip(res["log"], res["log"][1:] + [None])]
    with Session(pair, torch.float64) as s:
        v = torch.empty(prob.n_src, 3, dtype=torch.float64, device="cuda:0")
        prm = amm.amm_params_default(aa_m=5, max_total_iters=15, precision=amm.AMM_FP64_PLAIN)
        st = amm.amm_solve(s.h, prm, None, v, force_accept=fa, force_stage_end=fs)[0]
        torch.cuda.synchronize()
        v = v.cpu().numpy()
    assert st["iters"] == res["total"]
    assert st["energy"] == pytest.approx(res["E"], rel=1e-5)
    assert math.sqrt(((v - res["vhat"]) ** 2).sum(1).mean()) < 1e-5


def test_graphs_of_many_sets_in_one_build_equal_single_builds():
    """Several point sets of different sizes and densities built in one
    pass give, set by set, exactly the single-set builds."""
    _announce("test_graphs_of_many_sets_in_one_build_equal_single_builds")
    sets = [synth.torus_pair(1000 + 11 * b, n_src=n, n_tgt=10, n_nodes=20, k=4, e=6).src * sc
            for b, (n, sc) in enumerate(((700, 1.0), (1500, 0.5), (2600, 2.0), (300, 1.0)))]
    srcs = [torch.tensor(V, device="cuda:0") for V in sets]
    h = _handle()
    try:
        many = amm.build_graphs(h, srcs, 4)
        torch.cuda.synchronize()
        single = [amm.build_graph(h, sp, 4) for sp in srcs]
        torch.cuda.synchronize()
    finally:
        amm.amm_destroy(h)
    for (im, *tm), (is_, *ts) in zip(many, single):
        for key in ("n_nodes", "n_edges", "radius", "mean_edge_len", "n_capped", "max_influences"):
            assert im[key] == is_[key], key
        for a, b in zip(tm, ts):
            assert torch.equal(a, b)
    # and set 2 against the oracle
    _check_against_oracle(sets[2], 4, many[2])


def _check_geodesic_against_oracle(V, k, got, radius):
    info, node, idx, w, edges = got
    ref = G.build_graph_geodesic(V, radius, k)
    assert info["radius"] == pytest.approx(radius, rel=1e-15)
    assert np.array_equal(node.cpu().numpy(), ref["node_idx"])
    assert np.array_equal(idx.cpu().numpy(), ref["infl_idx"])
    assert np.abs(w.cpu().numpy().astype(np.float64) - ref["infl_w"]).max() <= 1e-12
    assert np.array_equal(edges.cpu().numpy(), ref["edges"])
    assert info["n_capped"] == ref["n_capped"]
    assert info["max_influences"] == ref["max_influences"]
    return ref


@pytest.mark.parametrize("case", ["torus700_k4", "strip_k6", "sh50k_k4"])
def test_geodesic_graph_matches_oracle(case):
    """Alg. 1 with the geodesic distance of Eq. (1) over the symmetrized 6-NN
    edge graph: nodes, influence indices and edges bit-exact against the
    oracle's shortest-path build, weights within 1e-12; on the folded strip
    the influence sets of points away from the fold stay on their own arm."""
    _announce(f"test_geodesic_graph_matches_oracle {case}")
    arm = None
    if case == "torus700_k4":
        V, k = synth.torus_pair(1000, n_src=700, n_tgt=10, n_nodes=20, k=4, e=6).src, 4
        R = 5.0 * G.mean_edge_length(V)
    elif case == "strip_k6":
        rng = np.random.default_rng(21)
        n, gap = 800, 0.1                   # at most ~800 points within R of a point
        t0, t1 = rng.uniform(0, 1, n), rng.uniform(0, 1, n)
        th = rng.uniform(-np.pi / 2, np.pi / 2, n // 6)
        V = np.concatenate([np.stack([t0, np.zeros(n), rng.uniform(0, 0.05, n)], 1),
                            np.stack([t1, np.full(n, gap), rng.uniform(0, 0.05, n)], 1),
                            np.stack([1 + 0.5 * gap * np.cos(th), 0.5 * gap + 0.5 * gap * np.sin(th),
                                      rng.uniform(0, 0.05, len(th))], 1)])
        arm = np.concatenate([np.zeros(n), np.ones(n), np.full(len(th), 2)])
        k, R = 6, 0.25
    else:
        V, k = synth.make_workload("sh50k").src, 4
        R = 5.0 * G.mean_edge_length(V)
    assert _axis_margin(V) > 1e-12
    h = _handle()
    try:
        got = amm.build_graph(h, torch.tensor(V, device="cuda:0"), k, radius=R, geodesic=True)
        torch.cuda.synchronize()
    finally:
        amm.amm_destroy(h)
    print(f"{case} geodesic: {got[0]}", file=sys.stderr)
    ref = _check_geodesic_against_oracle(V, k, got, R)
    if arm is not None:
        na = arm[ref["node_idx"]]
        far = (V[:, 0] < 1 - R - 0.05) & (arm < 2)
        idx = got[2].cpu().numpy()
        for q in np.nonzero(far)[0]:
            js = idx[q][idx[q] >= 0]
            assert np.all(na[js] == arm[q])


def test_geodesic_graph_registration():
    """A registration run on a graph built with the geodesic distance: the
    50,000-point pair's graph from the device build feeds amm_problem and
    Alg. 2 converges, with a registration error close to the Euclidean
    graph's (Eq. 25, both against the generator's ground truth)."""
    _announce("test_geodesic_graph_registration")
    pair = synth.make_workload("sh50k")
    dev = "cuda:0"
    rm = {}
    for geo in (False, True):
        h = _handle()
        try:
            info, node, idx, w, edges = amm.build_graph(h, torch.tensor(pair.src, device=dev), 4, geodesic=geo)
            t = lambda a, dt: torch.as_tensor(np.ascontiguousarray(a), dtype=dt, device=dev)
            prob = amm.make_problem(t(pair.src, torch.float32), t(pair.tgt, torch.float32), node, idx,
                                    w.to(torch.float32), edges, info["mean_edge_len"])
            amm.amm_set_problem(h, prob)
            v = torch.empty(pair.n_src, 3, dtype=torch.float32, device=dev)
            st = amm.amm_solve(h, amm.amm_params_default(aa_m=5), None, v)[0]
            torch.cuda.synchronize()
            rm[geo] = math.sqrt(((v.cpu().numpy().astype(np.float64) - pair.gt) ** 2).sum(1).mean())
            print(f"geodesic={geo}: {info['n_nodes']} nodes, {st['iters']} MM iterations, rmse {rm[geo]:.4e}",
                  file=sys.stderr)
            assert st["iters"] > 0 and math.isfinite(st["energy"])
        finally:
            amm.amm_destroy(h)
    assert rm[True] < 1.5 * rm[False]
