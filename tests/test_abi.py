"""Host-side checks of the C ABI (no GPU needed): the shared library loads,
exports every function include/amm.h declares, and its problem validation
turns malformed inputs into the documented status codes."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_2206_03410_amd import amm

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "amm.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^[A-Za-z_][\w \*]*?\b(amm_\w+)\s*\(", text, flags=re.M)
    return sorted(set(names))


def test_header_declares_the_binding_names():
    assert set(declared_functions()) == set(amm.EXPORTED)


def test_binding_structs_match_the_header_layout(tmp_path):
    """Every ctypes structure of the binding has the size and field offsets
    that a C compiler gives the header's typedef of the same name."""
    import shutil
    import subprocess
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    structs = [getattr(amm, n) for n in ("amm_problem", "amm_params", "amm_stats", "amm_iter_record",
                                         "amm_step_in", "amm_step_out", "amm_graph_in", "amm_graph_info")]
    lines = ["#include <stddef.h>", "#include <stdio.h>", '#include "amm.h"', "int main(void) {"]
    for st in structs:
        lines.append(f'printf("{st.__name__} size %zu\\n", sizeof({st.__name__}));')
        for f in st._fields_:
            lines.append(f'printf("{st.__name__} {f[0]} %zu\\n", offsetof({st.__name__}, {f[0]}));')
    lines += ["return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run([cc, "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = {}
    for line in subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.splitlines():
        name, field, val = line.split()
        got[(name, field)] = int(val)
    for st in structs:
        assert got[(st.__name__, "size")] == C.sizeof(st), st.__name__
        for f in st._fields_:
            assert got[(st.__name__, f[0])] == getattr(st, f[0]).offset, (st.__name__, f[0])


def test_library_exports_every_declared_symbol():
    L = C.CDLL(amm._LIB_PATH)
    missing = [n for n in declared_functions() if not hasattr(L, n)]
    assert not missing, missing


def test_status_strings_and_version():
    for s in range(8):
        txt = amm.lib().amm_status_string(s)
        assert txt and len(txt) >= 2
    assert amm.lib().amm_version().decode().startswith("amm-gfx950")


def test_params_default_are_the_paper_values():
    p = amm.amm_params_default()
    assert p.eps == 1e-5 and p.imax == 100           # Sec. 4.1
    assert p.k_alpha == 100.0 and p.k_beta == 1.0     # Eq. (26) scales
    assert p.nu_a0 <= 0 and p.nu_a_min <= 0 and p.nu_r0 <= 0   # Sec. 3.3.3 rules
    assert p.cg_rtol == 1e-10
    assert p.precision == amm.AMM_FP32_REFINE


def _arrays(pair, dt=np.float64):
    return dict(src=np.ascontiguousarray(pair.src, dt), tgt=np.ascontiguousarray(pair.tgt, dt),
                node_idx=np.ascontiguousarray(pair.node_idx, np.int32),
                infl_idx=np.ascontiguousarray(pair.infl_idx, np.int32),
                infl_w=np.ascontiguousarray(pair.infl_w, dt),
                edges=np.ascontiguousarray(pair.edges, np.int32), mean_edge_len=pair.mean_edge_len)


def _check(a):
    return amm.amm_check_problem(amm.make_problem(**a))


@pytest.mark.parametrize("dt", [np.float64, np.float32])
def test_check_accepts_generated_problem(small_pair, dt):
    assert _check(_arrays(small_pair, dt)) == amm.AMM_OK


def _mutated(small_pair, fn):
    a = _arrays(small_pair)
    a = {k: (v.copy() if isinstance(v, np.ndarray) else v) for k, v in a.items()}
    fn(a)
    return _check(a)


def test_check_nonfinite(small_pair):
    def nan_src(a):
        a["src"][7, 1] = np.nan

    def inf_tgt(a):
        a["tgt"][3, 0] = np.inf

    def nan_w(a):
        a["infl_w"][5, 0] = np.nan
    for fn in (nan_src, inf_tgt, nan_w):
        assert _mutated(small_pair, fn) == amm.AMM_ERR_NONFINITE


def test_check_partition_of_unity(small_pair):
    def off(a):
        a["infl_w"][11, 0] += 1e-3

    def just_inside(a):
        a["infl_w"][11, 0] += 5e-6
    assert _mutated(small_pair, off) == amm.AMM_ERR_GRAPH
    assert _mutated(small_pair, just_inside) == amm.AMM_OK


def test_check_index_ranges(small_pair):
    n = small_pair.node_idx.shape[0]

    def infl_oob(a):
        a["infl_idx"][2, 1] = n

    def infl_neg(a):
        a["infl_idx"][2, 1] = -1

    def node_oob(a):
        a["node_idx"][0] = a["src"].shape[0]

    def edge_oob(a):
        a["edges"][0, 1] = n

    def lbar(a):
        a["mean_edge_len"] = 0.0
    for fn in (infl_oob, infl_neg, node_oob, edge_oob, lbar):
        assert _mutated(small_pair, fn) == amm.AMM_ERR_INVALID_ARG, fn.__name__


def test_check_unused_influence_slots(small_pair):
    """-1 marks an unused slot: accepted with weight 0, rejected with a
    nonzero weight or below -1, and a point needs one used slot."""
    def pad_ok(a):
        w = a["infl_w"][2]
        a["infl_idx"][2, 3] = -1
        w[3] = 0.0
        w /= w.sum()

    def pad_weight(a):
        a["infl_idx"][2, 3] = -1

    def minus_two(a):
        a["infl_idx"][2, 3] = -2
        a["infl_w"][2, 3] = 0.0

    def all_unused(a):
        a["infl_idx"][2, :] = -1
        a["infl_w"][2, :] = 0.0
    assert _mutated(small_pair, pad_ok) == amm.AMM_OK
    assert _mutated(small_pair, pad_weight) == amm.AMM_ERR_INVALID_ARG
    assert _mutated(small_pair, minus_two) == amm.AMM_ERR_INVALID_ARG
    assert _mutated(small_pair, all_unused) == amm.AMM_ERR_GRAPH


def test_check_graph_structure(small_pair):
    def infl_dup(a):
        a["infl_idx"][2, 1] = a["infl_idx"][2, 0]

    def node_dup(a):
        a["node_idx"][1] = a["node_idx"][0]

    def negative_weight(a):
        a["infl_w"][4, 0] += 2.0
        a["infl_w"][4, 1] -= 2.0

    def self_loop(a):
        a["edges"][0, 1] = a["edges"][0, 0]

    def duplicate(a):
        a["edges"][1] = a["edges"][0]

    def reversed_duplicate(a):
        a["edges"][1] = a["edges"][0][::-1]

    def disconnected(a):
        # cut node 0 off from the rest
        e = a["edges"]
        keep = (e[:, 0] != 0) & (e[:, 1] != 0)
        a["edges"] = np.ascontiguousarray(e[keep])
    for fn in (infl_dup, node_dup, negative_weight, self_loop, duplicate, reversed_duplicate,
               disconnected):
        assert _mutated(small_pair, fn) == amm.AMM_ERR_GRAPH, fn.__name__


def test_check_sizes(small_pair):
    a = _arrays(small_pair)
    p = amm.make_problem(**a)
    p.k = 0
    assert amm.amm_check_problem(p) == amm.AMM_ERR_INVALID_ARG
    p = amm.make_problem(**a)
    p.k = 9
    assert amm.amm_check_problem(p) == amm.AMM_ERR_INVALID_ARG
    p = amm.make_problem(**a)
    p.n_src = 0
    assert amm.amm_check_problem(p) == amm.AMM_ERR_INVALID_ARG
    p = amm.make_problem(**a)
    p.n_tgt = 0
    assert amm.amm_check_problem(p) == amm.AMM_ERR_INVALID_ARG
    p = amm.make_problem(**a)
    p.src_xyz = None
    assert amm.amm_check_problem(p) == amm.AMM_ERR_INVALID_ARG
    assert amm.lib().amm_check_problem(None) == amm.AMM_ERR_INVALID_ARG


def test_create_without_device_reports_hip_error():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a HIP device is present")
    h = C.c_void_p()
    st = amm.lib().amm_create(C.byref(h), 0, None)
    assert st == amm.AMM_ERR_HIP
    assert not h.value
    assert amm.amm_last_error(None)


def test_null_handle_calls_are_rejected():
    L = amm.lib()
    n = C.c_int64()
    assert L.amm_k_nnzb(None, C.byref(n)) == amm.AMM_ERR_INVALID_ARG
    p = amm.amm_params_default()
    assert L.amm_solve(None, C.byref(p), None, None, None) == amm.AMM_ERR_INVALID_ARG


def test_size_query_needs_a_handle():
    L = amm.lib()
    P, k = C.c_int32(), C.c_int32()
    N, n, M = C.c_int64(), C.c_int64(), C.c_int64()
    assert L.amm_get_sizes(None, C.byref(P), C.byref(N), C.byref(n), C.byref(M), C.byref(k)) == \
        amm.AMM_ERR_INVALID_ARG


def test_binding_rejects_mismatched_device_buffers():
    """Raw pointers reach the library only for GPU tensors of the element
    type and count the call uses: a host array, a CPU tensor, a wrong dtype,
    a wrong size or a non-contiguous view raise before any call."""
    import torch
    with pytest.raises(TypeError):
        amm._device_buffer("X", np.zeros(12, np.float32), amm.AMM_F32, 12)
    with pytest.raises(TypeError):
        amm._device_buffer("X", torch.zeros(12, dtype=torch.float32), amm.AMM_F32, 12)
    amm._device_buffer("X", None, amm.AMM_F32, 12)   # optional buffers pass

    class FakeCuda:
        is_cuda = True

        def __init__(self, dtype, n, contiguous=True):
            self.dtype, self.n, self.c = dtype, n, contiguous

        def is_contiguous(self):
            return self.c

        def numel(self):
            return self.n
    amm._device_buffer("X", FakeCuda(torch.float32, 12), amm.AMM_F32, 12)
    with pytest.raises(TypeError):
        amm._device_buffer("X", FakeCuda(torch.float64, 12), amm.AMM_F32, 12)
    with pytest.raises(ValueError):
        amm._device_buffer("X", FakeCuda(torch.float32, 24), amm.AMM_F32, 12)
    with pytest.raises(ValueError):
        amm._device_buffer("X", FakeCuda(torch.float32, 12, contiguous=False), amm.AMM_F32, 12)
    with pytest.raises(TypeError):
        amm._device_buffer("rho", FakeCuda(torch.int64, 5), "int32", 5)
