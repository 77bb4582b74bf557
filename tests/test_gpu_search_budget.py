"""The closest-point search's step budget (Sec. 3.2's rho(i)): searches past
the budget are finished by the wave-wide search, which must give the same
exact answer.  Energies, closest points and squared distances are bitwise
equal for every budget (the tile sums keep one order), cold and seeded,
in float32 and float64, and the closest points equal scipy's exact k-d
tree's wherever the best and second-best distances differ by more than
1e-6 relative.  A budget of 1 sends nearly every point to the wave-wide
search, and cold searches from the octree's root there overflow its
frontier and take the one-lane fallback."""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2206_03410_amd import amm, synth
from tests.helpers import Session, margin_ok, rounded

pytestmark = pytest.mark.gpu


def _announce(name):
    print(f"[gpu-test] {name}", file=sys.stderr, flush=True)


def _energy(s, X, n_src, dt, scal):
    rho = torch.empty(n_src, dtype=torch.int32, device="cuda:0")
    d2 = torch.empty(n_src, dtype=dt, device="cuda:0")
    e = amm.amm_energy(s.h, X, None, *scal, rho=rho, d2=d2)
    torch.cuda.synchronize()
    return e, rho.cpu().numpy(), d2.cpu().numpy()


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_budget_does_not_change_results(prec):
    _announce(f"test_budget_does_not_change_results {prec}")
    from scipy.spatial import cKDTree
    dt = torch.float32 if prec == "f32" else torch.float64
    np_dt = np.float32 if prec == "f32" else np.float64
    pair = rounded(synth.make_workload("sh50k"), np_dt)
    X = torch.tensor(synth.perturbed_transforms(pair.n_nodes, 8101, 0.01, 0.001).astype(np_dt), device="cuda:0")
    scal = (0.02, 0.05, 10.0, 100.0)
    ref = None
    with Session(pair, dt) as s:
        for budget in (0, 1, 8, 64, 1000000):
            for seeded in (False, True):
                amm.amm_set_search_budget(s.h, budget)
                if not seeded:
                    # a new upload forgets the previous closest points: a cold search
                    amm.amm_set_problems(s.h, s.problems)
                got = _energy(s, X, pair.n_src, dt, scal)
                if ref is None:
                    ref = got
                    continue
                print(f"{prec} budget {budget} seeded {seeded}: energy {got[0][0]!r}", file=sys.stderr)
                assert got[0] == ref[0]
                assert np.array_equal(got[1], ref[1])
                assert np.array_equal(got[2], ref[2])
        # the warped points of X against the exact k-d tree
        vh = torch.empty(pair.n_src, 3, dtype=dt, device="cuda:0")
        amm.amm_set_search_budget(s.h, 1)
        amm.amm_step(s.h, X, *scal, amm.AMM_FP32_REFINE if prec == "f32" else amm.AMM_FP64_PLAIN, v_hat=vh)
        torch.cuda.synchronize()
        vh = vh.cpu().numpy().astype(np.float64)
    dk, ik = cKDTree(pair.tgt).query(vh, k=2)
    ok = margin_ok(dk[:, 0] ** 2, dk[:, 1] ** 2)
    assert ok.mean() > 0.99
    assert np.array_equal(ref[1][ok], ik[ok, 0])


def test_budget_on_the_200k_pair_and_a_batch():
    """The 200,000-point pair (float32) at budgets 0, 1 and 64, and three
    pairs of the batch together at budgets 0 and 4: bitwise equal."""
    _announce("test_budget_on_the_200k_pair_and_a_batch")
    pair = rounded(synth.make_workload("sh200k"), np.float32)
    X = torch.tensor(synth.perturbed_transforms(pair.n_nodes, 8102, 0.01, 0.001).astype(np.float32),
                     device="cuda:0")
    scal = (0.02, 0.05, 10.0, 100.0)
    with Session(pair, torch.float32) as s:
        outs = []
        for budget in (0, 1, 64):
            amm.amm_set_search_budget(s.h, budget)
            amm.amm_set_problems(s.h, s.problems)
            outs.append(_energy(s, X, pair.n_src, torch.float32, scal))
        for o in outs[1:]:
            assert o[0] == outs[0][0]
            assert np.array_equal(o[1], outs[0][1]) and np.array_equal(o[2], outs[0][2])
    pairs = synth.batch_pairs(n_pairs=64)
    sel = [rounded(pairs[b], np.float32) for b in (3, 17, 40)]
    n = sum(p.n_nodes for p in sel)
    X = torch.tensor(synth.perturbed_transforms(n, 8103, 0.01, 0.001).astype(np.float32), device="cuda:0")
    with Session(sel, torch.float32) as s:
        res = []
        for budget in (0, 4):
            amm.amm_set_search_budget(s.h, budget)
            v = torch.empty(sum(p.n_src for p in sel), 3, dtype=torch.float32, device="cuda:0")
            st = amm.amm_solve(s.h, amm.amm_params_default(aa_m=5, max_total_iters=6), X.clone(), v)
            torch.cuda.synchronize()
            res.append(([x["energy"] for x in st], v.cpu().numpy()))
        assert res[0][0] == res[1][0]
        assert np.array_equal(res[0][1], res[1][1])
