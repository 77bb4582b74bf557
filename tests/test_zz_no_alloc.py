"""The allocation-free energy entry point against amm_energy through the C
ABI: energies (all four terms), closest points and squared distances equal
bitwise, in float32 and float64, on two calls in a row on one GPU, the
second with a smaller problem (the static scratch keeps the first call's
contents), with and without a source-position override."""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2206_03410_amd import amm, synth
from tests.helpers import Session, rounded

pytestmark = pytest.mark.gpu


def _announce(name):
    print(f"[gpu-test] {name}", file=sys.stderr, flush=True)


def _both(s, pair, X, src, dt, scal):
    dev = "cuda:0"
    out = []
    for fn in (amm.amm_energy, amm.amm_energy_noalloc):
        rho = torch.empty(pair.n_src, dtype=torch.int32, device=dev)
        d2 = torch.empty(pair.n_src, dtype=dt, device=dev)
        e = fn(s.h, X, src, *scal, rho=rho, d2=d2)
        torch.cuda.synchronize()
        out.append((e, rho.cpu().numpy(), d2.cpu().numpy()))
    return out


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_energy_noalloc_equals_energy(prec):
    _announce(f"test_energy_noalloc_equals_energy {prec}")
    dt = torch.float32 if prec == "f32" else torch.float64
    np_dt = np.float32 if prec == "f32" else np.float64
    big = rounded(synth.make_workload("sh50k"), np_dt)
    small = rounded(synth.torus_pair(1000, n_src=600, n_tgt=650, n_nodes=40, k=4, e=6), np_dt)
    scal = (0.02, 0.05, 10.0, 100.0)
    dev = "cuda:0"
    for pair, seed, with_src in ((big, 11, False), (small, 12, True)):
        X = torch.tensor(synth.perturbed_transforms(pair.n_nodes, seed, 0.01, 0.001), dtype=dt, device=dev)
        src = None
        if with_src:
            rng = np.random.default_rng(seed)
            src = torch.tensor(pair.src + rng.normal(0, 1e-3, pair.src.shape), dtype=dt, device=dev)
        with Session(pair, dt) as s:
            (e0, r0, d0), (e1, r1, d1) = _both(s, pair, X, src, dt, scal)
        print(f"{prec} {pair.n_src} points: E {e0[0]:.12e} / {e1[0]:.12e}", file=sys.stderr)
        assert e1 == e0
        assert np.array_equal(r1, r0)
        assert np.array_equal(d1, d0)


def test_energy_noalloc_refuses_batches():
    _announce("test_energy_noalloc_refuses_batches")
    pairs = [synth.torus_pair(1000 + b, n_src=300, n_tgt=320, n_nodes=20, k=4, e=6) for b in range(2)]
    with Session(pairs, torch.float64) as s:
        X = torch.zeros(sum(p.n_nodes for p in pairs), 4, 3, dtype=torch.float64, device="cuda:0")
        with pytest.raises(amm.AmmError):
            amm.amm_energy_noalloc(s.h, X, None, 0.02, 0.05, 10.0, 100.0)
