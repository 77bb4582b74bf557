"""ctypes binding of libamm.so: the C ABI of include/amm.h under the same
names.  Argument marshalling only -- every step of the registration runs in
the library's HIP kernels.  Device arrays are torch tensors (their
data_ptr()), host arrays are numpy arrays; the library never keeps them.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import List, Optional, Sequence

import numpy as np

_LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libamm.so")

AMM_OK, AMM_ERR_INVALID_ARG, AMM_ERR_STATE, AMM_ERR_OOM, AMM_ERR_HIP, AMM_ERR_NONFINITE, \
    AMM_ERR_GRAPH, AMM_ERR_NOT_SPD = range(8)
AMM_F32, AMM_F64 = 0, 1
AMM_FP64_PLAIN, AMM_FP32_REFINE = 0, 1
AMM_PRECOND_TWO_LEVEL, AMM_PRECOND_BLOCK_JACOBI = 0, 1
AMM_ROBUST_WELSCH, AMM_ROBUST_L2, AMM_ROBUST_L2_TRUNC = 0, 1, 2
AMM_NU_DYNAMIC, AMM_NU_FIXED_MAX, AMM_NU_FIXED_MIN, AMM_NU_FIXED_MED = 0, 1, 2, 3
AMM_MAX_AA_M = 10


class amm_problem(C.Structure):
    _fields_ = [("dtype", C.c_int), ("on_device", C.c_int32),
                ("n_src", C.c_int64), ("src_xyz", C.c_void_p), ("src_nrm", C.c_void_p),
                ("n_tgt", C.c_int64), ("tgt_xyz", C.c_void_p), ("tgt_nrm", C.c_void_p),
                ("n_nodes", C.c_int64), ("node_src_idx", C.c_void_p),
                ("k", C.c_int32), ("infl_idx", C.c_void_p), ("infl_w", C.c_void_p),
                ("n_edges", C.c_int64), ("edges", C.c_void_p),
                ("mean_edge_len", C.c_double)]


class amm_params(C.Structure):
    _fields_ = [("nu_a0", C.c_double), ("nu_a_min", C.c_double), ("nu_r0", C.c_double),
                ("k_alpha", C.c_double), ("k_beta", C.c_double), ("eps", C.c_double),
                ("imax", C.c_int32), ("max_total_iters", C.c_int32), ("aa_m", C.c_int32),
                ("precision", C.c_int32), ("cg_rtol", C.c_double), ("cg_maxit", C.c_int32),
                ("init_identity", C.c_int32),
                ("force_accept", C.c_void_p), ("force_stage_end", C.c_void_p),
                ("force_len", C.c_int32), ("cg_precond", C.c_int32), ("robust", C.c_int32),
                ("nu_mode", C.c_int32), ("force_per_pair", C.c_int32)]


class amm_stats(C.Structure):
    _fields_ = [("iters", C.c_int32), ("stages", C.c_int32), ("converged", C.c_int32),
                ("aa_accepted", C.c_int32), ("aa_rejected", C.c_int32),
                ("cg_iters", C.c_int64), ("refine_steps", C.c_int32),
                ("energy", C.c_double), ("e_align", C.c_double), ("e_reg", C.c_double),
                ("e_rot", C.c_double), ("nu_a", C.c_double), ("nu_r", C.c_double),
                ("alpha", C.c_double), ("beta", C.c_double), ("max_disp", C.c_double),
                ("max_rel_residual", C.c_double), ("time_ms", C.c_double),
                ("solves_above_rtol", C.c_int32)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class amm_iter_record(C.Structure):
    _fields_ = [("pair", C.c_int32), ("iter", C.c_int32), ("stage", C.c_int32), ("m_k", C.c_int32),
                ("aa_used", C.c_int32), ("accepted", C.c_int32), ("cg_iters", C.c_int32),
                ("refine_steps", C.c_int32), ("energy_before", C.c_double),
                ("energy_candidate", C.c_double), ("energy_after", C.c_double),
                ("max_disp", C.c_double), ("nu_a", C.c_double), ("nu_r", C.c_double),
                ("alpha", C.c_double), ("beta", C.c_double), ("rel_residual", C.c_double)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class amm_graph_in(C.Structure):
    _fields_ = [("dtype", C.c_int), ("src_xyz", C.c_void_p), ("n_src", C.c_int64), ("radius", C.c_double),
                ("radius_factor", C.c_double), ("k", C.c_int32), ("geodesic", C.c_int32)]


class amm_graph_info(C.Structure):
    _fields_ = [("n_nodes", C.c_int64), ("n_edges", C.c_int64), ("radius", C.c_double),
                ("mean_edge_len", C.c_double), ("n_capped", C.c_int64), ("max_influences", C.c_int32),
                ("rounds", C.c_int32)]

    def as_dict(self):
        return {f[0]: getattr(self, f[0]) for f in self._fields_}


class amm_step_in(C.Structure):
    _fields_ = [("X", C.c_void_p), ("nu_a", C.c_double), ("nu_r", C.c_double),
                ("alpha", C.c_double), ("beta", C.c_double), ("precision", C.c_int32),
                ("cg_rtol", C.c_double), ("cg_maxit", C.c_int32), ("cg_precond", C.c_int32),
                ("robust", C.c_int32)]


class amm_step_out(C.Structure):
    _fields_ = [("energy", C.c_double * 4), ("rho", C.c_void_p), ("d2", C.c_void_p),
                ("v_hat", C.c_void_p), ("X_next", C.c_void_p), ("K_blocks", C.c_void_p),
                ("K_row", C.c_void_p), ("K_col", C.c_void_p), ("B", C.c_void_p),
                ("cg_iters", C.c_int32), ("rel_residual", C.c_double)]


_lib = None


def lib():
    """The loaded library; raises if it was not built (no fallback path)."""
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            raise RuntimeError(f"{_LIB_PATH} is missing: build it with "
                               "`python -m paper_2206_03410_amd.build_lib`")
        L = C.CDLL(_LIB_PATH)
        vp, i32, i64, dbl = C.c_void_p, C.c_int32, C.c_int64, C.c_double
        sig = {
            "amm_create": ([C.POINTER(vp), C.c_int, vp], C.c_int),
            "amm_destroy": ([vp], None),
            "amm_set_stream": ([vp, vp], C.c_int),
            "amm_check_problem": ([C.POINTER(amm_problem)], C.c_int),
            "amm_workspace_size": ([vp, C.POINTER(amm_problem), i32, C.POINTER(C.c_size_t)], C.c_int),
            "amm_set_workspace": ([vp, vp, C.c_size_t], C.c_int),
            "amm_set_problems": ([vp, C.POINTER(amm_problem), i32], C.c_int),
            "amm_set_problem": ([vp, C.POINTER(amm_problem)], C.c_int),
            "amm_set_leaf_size": ([vp, i32], C.c_int),
            "amm_set_search_budget": ([vp, i32], C.c_int),
            "amm_get_search_budget": ([vp, C.POINTER(i32)], C.c_int),
            "amm_count_nn_work": ([vp, i32], C.c_int),
            "amm_build_graph": ([vp, C.POINTER(amm_graph_in), C.POINTER(amm_graph_info)], C.c_int),
            "amm_set_targets": ([vp, i32, C.c_int, vp, i64, i32], C.c_int),
            "amm_graph_copy": ([vp, vp, vp, vp, vp], C.c_int),
            "amm_build_graphs": ([vp, C.POINTER(amm_graph_in), i32, C.POINTER(amm_graph_info)], C.c_int),
            "amm_graph_copy_set": ([vp, i32, vp, vp, vp, vp], C.c_int),
            "amm_nn_work": ([vp, C.POINTER(i64), C.POINTER(i64), C.POINTER(i64), C.POINTER(i64)], C.c_int),
            "amm_autotune": ([vp, C.POINTER(amm_problem), i32, C.POINTER(i32), i32, C.POINTER(i32),
                              C.POINTER(dbl)], C.c_int),
            "amm_solve": ([vp, C.POINTER(amm_params), vp, vp, C.POINTER(amm_stats)], C.c_int),
            "amm_step": ([vp, C.POINTER(amm_step_in), C.POINTER(amm_step_out)], C.c_int),
            "amm_k_nnzb": ([vp, C.POINTER(i64)], C.c_int),
            "amm_get_sizes": ([vp, C.POINTER(i32), C.POINTER(i64), C.POINTER(i64), C.POINTER(i64),
                               C.POINTER(i32)], C.c_int),
            "amm_iter_log": ([vp, C.POINTER(amm_iter_record), i32, C.POINTER(i32)], C.c_int),
            "amm_energy": ([vp, C.c_int, vp, vp, dbl, dbl, dbl, dbl, C.POINTER(dbl), vp, vp], C.c_int),
            "amm_energy_noalloc": ([vp, C.c_int, vp, vp, dbl, dbl, dbl, dbl, C.POINTER(dbl), vp, vp], C.c_int),
            "amm_energy_grad": ([vp, C.c_int, vp, vp, dbl, dbl, dbl, dbl, vp, vp, C.POINTER(dbl)],
                                C.c_int),
            "amm_status_string": ([C.c_int], C.c_char_p),
            "amm_last_error": ([vp], C.c_char_p),
            "amm_kernel_times": ([vp, C.POINTER(C.c_char_p), C.POINTER(dbl), C.POINTER(i32), i32,
                                  C.POINTER(i32)], C.c_int),
            "amm_enable_timing": ([vp, i32, C.c_char_p], C.c_int),
            "amm_version": ([], C.c_char_p),
            "amm_params_default": ([C.POINTER(amm_params)], None),
        }
        for name, (args, res) in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = res
        _lib = L
    return _lib


EXPORTED = ["amm_create", "amm_destroy", "amm_set_stream", "amm_check_problem",
            "amm_workspace_size", "amm_set_workspace", "amm_set_problems", "amm_set_problem",
            "amm_set_leaf_size", "amm_set_search_budget", "amm_get_search_budget", "amm_autotune", "amm_count_nn_work", "amm_nn_work",
            "amm_build_graph", "amm_graph_copy", "amm_set_targets", "amm_build_graphs", "amm_graph_copy_set",
            "amm_solve", "amm_step", "amm_k_nnzb", "amm_get_sizes", "amm_iter_log", "amm_energy",
            "amm_energy_noalloc", "amm_energy_grad",
            "amm_status_string", "amm_last_error", "amm_kernel_times", "amm_enable_timing",
            "amm_version", "amm_params_default"]


class AmmError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{amm_status_string(status)}: {msg}")
        self.status = status


def _check(status, handle=None):
    if status != AMM_OK:
        raise AmmError(status, amm_last_error(handle))


def _ptr(a):
    """Device pointer of a torch tensor or host pointer of a numpy array."""
    if a is None:
        return None
    if isinstance(a, np.ndarray):
        if not a.flags["C_CONTIGUOUS"]:
            raise ValueError("arrays must be C-contiguous")
        return a.ctypes.data
    if not a.is_contiguous():
        raise ValueError("tensors must be contiguous")
    return a.data_ptr()


def _device_buffer(name, a, dtype_code, numel):
    """Checks a device buffer before its raw pointer goes to the library:
    a contiguous tensor on a GPU with the element type and the element count
    that the call writes or reads (None passes)."""
    if a is None:
        return
    if isinstance(a, np.ndarray) or not getattr(a, "is_cuda", False):
        raise TypeError(f"{name} must be a tensor on the GPU")
    if not a.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if dtype_code is not None:
        want = {AMM_F32: "float32", AMM_F64: "float64", "int32": "int32"}[dtype_code]
        if str(a.dtype).split(".")[-1] != want:
            raise TypeError(f"{name} must be {want}, got {a.dtype}")
    if a.numel() != numel:
        raise ValueError(f"{name} must hold {numel} elements, got {a.numel()}")


def _dtype_code(a):
    name = str(a.dtype)
    if "float32" in name:
        return AMM_F32
    if "float64" in name:
        return AMM_F64
    raise TypeError(f"floating-point arrays must be float32 or float64, got {a.dtype}")


# ------------------------------------------------------------------ API

def amm_status_string(status: int) -> str:
    return lib().amm_status_string(status).decode()


def amm_last_error(handle=None) -> str:
    return (lib().amm_last_error(handle) or b"").decode()


def amm_version() -> str:
    return lib().amm_version().decode()


def amm_params_default(**override) -> amm_params:
    p = amm_params()
    lib().amm_params_default(C.byref(p))
    for k, v in override.items():
        setattr(p, k, v)
    return p


def amm_create(device: int = 0, stream: Optional[int] = None):
    h = C.c_void_p()
    _check(lib().amm_create(C.byref(h), device, stream))
    return h


def amm_destroy(handle) -> None:
    lib().amm_destroy(handle)


def amm_set_stream(handle, stream: Optional[int]) -> None:
    _check(lib().amm_set_stream(handle, stream), handle)


def make_problem(src, tgt, node_idx, infl_idx, infl_w, edges, mean_edge_len,
                 src_nrm=None, tgt_nrm=None):
    """amm_problem over torch tensors (device) or numpy arrays (host).  The
    returned object keeps references to the arrays."""
    on_dev = not isinstance(src, np.ndarray)
    k = int(infl_idx.shape[1])
    p = amm_problem(dtype=_dtype_code(src), on_device=1 if on_dev else 0,
                    n_src=int(src.shape[0]), src_xyz=_ptr(src), src_nrm=_ptr(src_nrm),
                    n_tgt=int(tgt.shape[0]), tgt_xyz=_ptr(tgt), tgt_nrm=_ptr(tgt_nrm),
                    n_nodes=int(node_idx.shape[0]), node_src_idx=_ptr(node_idx),
                    k=k, infl_idx=_ptr(infl_idx), infl_w=_ptr(infl_w),
                    n_edges=int(edges.shape[0]), edges=_ptr(edges),
                    mean_edge_len=float(mean_edge_len))
    p._keep = (src, tgt, node_idx, infl_idx, infl_w, edges, src_nrm, tgt_nrm)
    return p


def amm_check_problem(problem: amm_problem) -> int:
    """Host-only validation; returns the status code (no exception)."""
    return lib().amm_check_problem(C.byref(problem))


def amm_workspace_size(handle, problems: Sequence[amm_problem]) -> int:
    arr = (amm_problem * len(problems))(*problems)
    n = C.c_size_t()
    _check(lib().amm_workspace_size(handle, arr, len(problems), C.byref(n)), handle)
    return n.value


def amm_set_workspace(handle, tensor_or_none) -> None:
    if tensor_or_none is None:
        _check(lib().amm_set_workspace(handle, None, 0), handle)
    else:
        nbytes = tensor_or_none.numel() * tensor_or_none.element_size()
        _check(lib().amm_set_workspace(handle, tensor_or_none.data_ptr(), nbytes), handle)


def amm_set_leaf_size(handle, leaf: int) -> None:
    _check(lib().amm_set_leaf_size(handle, int(leaf)), handle)


def amm_set_search_budget(handle, steps: int) -> None:
    _check(lib().amm_set_search_budget(handle, int(steps)), handle)


def amm_get_search_budget(handle) -> int:
    v = C.c_int32(0)
    _check(lib().amm_get_search_budget(handle, C.byref(v)), handle)
    return int(v.value)


def amm_set_targets(handle, pair: int, tgt) -> None:
    """New target points (same count) for one pair of the handle's batch; tgt
    is a cuda tensor or a numpy array [M][3]."""
    on_dev = 0 if isinstance(tgt, np.ndarray) else 1
    _check(lib().amm_set_targets(handle, int(pair), _dtype_code(tgt), _ptr(tgt), tgt.shape[0], on_dev), handle)


def amm_build_graph(handle, src, k: int, radius: float = 0.0, radius_factor: float = 0.0,
                    geodesic: bool = False) -> dict:
    """Alg. 1 on the device for the source points `src` (a cuda tensor
    [N][3], float32 or float64), Euclidean or geodesic distance; returns the
    build's info.  Fetch the graph with amm_graph_copy."""
    gin = amm_graph_in(dtype=_dtype_code(src), src_xyz=_ptr(src), n_src=src.shape[0], radius=radius,
                       radius_factor=radius_factor, k=k, geodesic=1 if geodesic else 0)
    info = amm_graph_info()
    _check(lib().amm_build_graph(handle, C.byref(gin), C.byref(info)), handle)
    return info.as_dict()


def amm_graph_copy(handle, node_src_idx=None, infl_idx=None, infl_w=None, edges=None) -> None:
    _check(lib().amm_graph_copy(handle, _ptr(node_src_idx), _ptr(infl_idx), _ptr(infl_w), _ptr(edges)), handle)


def amm_build_graphs(handle, srcs, k: int, radius: float = 0.0, radius_factor: float = 0.0,
                     geodesic: bool = False) -> list:
    """Alg. 1 for several point sets (cuda tensors [N_s][3], one dtype) in one
    pass; returns one info dict per set."""
    n = len(srcs)
    gin = (amm_graph_in * n)(*[amm_graph_in(dtype=_dtype_code(sp), src_xyz=_ptr(sp), n_src=sp.shape[0],
                                            radius=radius, radius_factor=radius_factor, k=k,
                                            geodesic=1 if geodesic else 0) for sp in srcs])
    info = (amm_graph_info * n)()
    _check(lib().amm_build_graphs(handle, gin, n, info), handle)
    return [i.as_dict() for i in info]


def amm_graph_copy_set(handle, set_index: int, node_src_idx=None, infl_idx=None, infl_w=None, edges=None) -> None:
    _check(lib().amm_graph_copy_set(handle, int(set_index), _ptr(node_src_idx), _ptr(infl_idx), _ptr(infl_w),
                                    _ptr(edges)), handle)


def build_graphs(handle, srcs, k: int, radius: float = 0.0, radius_factor: float = 0.0, geodesic: bool = False):
    """amm_build_graphs + per-set copies into new tensors: a list of
    (info, node_src_idx, infl_idx, infl_w, edges)."""
    import torch
    infos = amm_build_graphs(handle, srcs, k, radius, radius_factor, geodesic)
    out = []
    for s, (sp, info) in enumerate(zip(srcs, infos)):
        dev = sp.device
        node = torch.empty(info["n_nodes"], dtype=torch.int32, device=dev)
        idx = torch.empty(sp.shape[0], k, dtype=torch.int32, device=dev)
        w = torch.empty(sp.shape[0], k, dtype=sp.dtype, device=dev)
        edges = torch.empty(max(info["n_edges"], 1), 2, dtype=torch.int32, device=dev)[:info["n_edges"]]
        amm_graph_copy_set(handle, s, node, idx, w, edges)
        out.append((info, node, idx, w, edges))
    return out


def build_graph(handle, src, k: int, radius: float = 0.0, radius_factor: float = 0.0, geodesic: bool = False):
    """amm_build_graph + amm_graph_copy into new tensors on src's device:
    (info, node_src_idx [n], infl_idx [N][k], infl_w [N][k], edges [E][2])."""
    import torch
    info = amm_build_graph(handle, src, k, radius, radius_factor, geodesic)
    dev = src.device
    node = torch.empty(info["n_nodes"], dtype=torch.int32, device=dev)
    idx = torch.empty(src.shape[0], k, dtype=torch.int32, device=dev)
    w = torch.empty(src.shape[0], k, dtype=src.dtype, device=dev)
    edges = torch.empty(max(info["n_edges"], 1), 2, dtype=torch.int32, device=dev)[:info["n_edges"]]
    amm_graph_copy(handle, node, idx, w, edges)
    return info, node, idx, w, edges


def amm_count_nn_work(handle, enable: bool) -> None:
    _check(lib().amm_count_nn_work(handle, 1 if enable else 0), handle)


def amm_nn_work(handle) -> dict:
    """Totals since counting was switched on: queries, box tests, distance
    evaluations and grid cell lookups of the closest-point search."""
    q, b, d, g = C.c_int64(), C.c_int64(), C.c_int64(), C.c_int64()
    _check(lib().amm_nn_work(handle, C.byref(q), C.byref(b), C.byref(d), C.byref(g)), handle)
    return dict(queries=q.value, box_tests=b.value, distance_evals=d.value, cell_lookups=g.value)


def amm_autotune(handle, problems: Sequence[amm_problem], candidates=None):
    """Picks the closest-point leaf size and search step budget by timing a
    warm evaluation per candidate; returns (leaf, ms).  The handle is left
    set up with them (the budget: amm_get_search_budget)."""
    arr = (amm_problem * len(problems))(*problems)
    cand = None if candidates is None else (C.c_int32 * len(candidates))(*candidates)
    best = C.c_int32()
    ms = C.c_double()
    _check(lib().amm_autotune(handle, arr, len(problems), cand, 0 if candidates is None else len(candidates),
                              C.byref(best), C.byref(ms)), handle)
    return best.value, ms.value


def amm_set_problems(handle, problems: Sequence[amm_problem]) -> None:
    arr = (amm_problem * len(problems))(*problems)
    _check(lib().amm_set_problems(handle, arr, len(problems)), handle)


def amm_set_problem(handle, problem: amm_problem) -> None:
    _check(lib().amm_set_problem(handle, C.byref(problem)), handle)


def amm_get_sizes(handle) -> dict:
    """Sizes of the batch set on the handle: pairs, and the totals of source
    points, graph nodes and target points over the pairs, and k."""
    P, k = C.c_int32(), C.c_int32()
    N, n, M = C.c_int64(), C.c_int64(), C.c_int64()
    _check(lib().amm_get_sizes(handle, C.byref(P), C.byref(N), C.byref(n), C.byref(M), C.byref(k)), handle)
    return dict(n_pairs=P.value, n_src=N.value, n_nodes=n.value, n_tgt=M.value, k=k.value)


def _precision_dtype(precision):
    return AMM_F32 if precision == AMM_FP32_REFINE else AMM_F64


def amm_solve(handle, params: amm_params, X_inout=None, v_out=None, n_pairs: Optional[int] = None,
              force_accept=None, force_stage_end=None, per_pair: bool = False) -> List[dict]:
    """Alg. 2 for every pair on the handle; returns one stats dict per pair.
    X_inout ([nodes][4][3] over all pairs) and v_out ([points][3]) are GPU
    tensors of the precision's type (float32 for AMM_FP32_REFINE, float64
    for AMM_FP64_PLAIN), checked against the handle's sizes.  Replayed
    decisions (None = decide) are one list for all pairs, or with per_pair
    one list per pair."""
    sz = amm_get_sizes(handle)
    if n_pairs is not None and n_pairs != sz["n_pairs"]:
        raise ValueError(f"n_pairs={n_pairs} but the handle holds {sz['n_pairs']} pairs")
    dt = _precision_dtype(params.precision)
    _device_buffer("X_inout", X_inout, dt, 12 * sz["n_nodes"])
    _device_buffer("v_out", v_out, dt, 3 * sz["n_src"])
    keep = []
    if force_accept is not None or force_stage_end is not None:
        # one list for every pair, or (per_pair) one list per pair
        rows_a = force_accept if per_pair else [force_accept]
        rows_s = force_stage_end if per_pair else [force_stage_end]
        R = sz["n_pairs"] if per_pair else 1
        rows_a = rows_a if rows_a is not None else [None] * R
        rows_s = rows_s if rows_s is not None else [None] * R
        if len(rows_a) != R or len(rows_s) != R:
            raise ValueError(f"per-pair decision lists need {R} rows")
        n = max([len(r or []) for r in rows_a] + [len(r or []) for r in rows_s] + [1])
        fa = np.full((R, n), -1, np.int8)
        fs = np.full((R, n), -1, np.int8)
        for q in range(R):
            if rows_a[q] is not None:
                fa[q, :len(rows_a[q])] = [-1 if v is None else int(v) for v in rows_a[q]]
            if rows_s[q] is not None:
                fs[q, :len(rows_s[q])] = [-1 if v is None else int(v) for v in rows_s[q]]
        keep = [fa, fs]
        params.force_accept = fa.ctypes.data
        params.force_stage_end = fs.ctypes.data
        params.force_len = n
        params.force_per_pair = 1 if per_pair else 0
    stats = (amm_stats * sz["n_pairs"])()
    _check(lib().amm_solve(handle, C.byref(params), _ptr(X_inout), _ptr(v_out), stats), handle)
    del keep
    return [s.as_dict() for s in stats]


def amm_step(handle, X, nu_a, nu_r, alpha, beta, precision, cg_rtol=1e-10, cg_maxit=0,
             cg_precond=AMM_PRECOND_TWO_LEVEL, rho=None, d2=None, v_hat=None, X_next=None, K_blocks=None, K_row=None, K_col=None,
             B=None, robust=AMM_ROBUST_WELSCH) -> dict:
    sz = amm_get_sizes(handle)
    dt = _precision_dtype(precision)
    n, N = sz["n_nodes"], sz["n_src"]
    _device_buffer("X", X, dt, 12 * n)
    if X is None:
        raise ValueError("X is required")
    _device_buffer("rho", rho, "int32", N)
    _device_buffer("d2", d2, dt, N)
    _device_buffer("v_hat", v_hat, dt, 3 * N)
    _device_buffer("X_next", X_next, dt, 12 * n)
    _device_buffer("B", B, dt, 12 * n)
    if K_blocks is not None or K_row is not None or K_col is not None:
        nnzb = amm_k_nnzb(handle)
        _device_buffer("K_blocks", K_blocks, dt, 16 * nnzb)
        _device_buffer("K_row", K_row, "int32", nnzb)
        _device_buffer("K_col", K_col, "int32", nnzb)
    sin = amm_step_in(X=_ptr(X), nu_a=nu_a, nu_r=nu_r, alpha=alpha, beta=beta,
                      precision=precision, cg_rtol=cg_rtol, cg_maxit=cg_maxit, cg_precond=cg_precond,
                      robust=robust)
    sout = amm_step_out(rho=_ptr(rho), d2=_ptr(d2), v_hat=_ptr(v_hat), X_next=_ptr(X_next),
                        K_blocks=_ptr(K_blocks), K_row=_ptr(K_row), K_col=_ptr(K_col), B=_ptr(B))
    _check(lib().amm_step(handle, C.byref(sin), C.byref(sout)), handle)
    return dict(energy=list(sout.energy), cg_iters=sout.cg_iters, rel_residual=sout.rel_residual)


def amm_iter_log(handle) -> List[dict]:
    n = C.c_int32()
    _check(lib().amm_iter_log(handle, None, 0, C.byref(n)), handle)
    arr = (amm_iter_record * max(n.value, 1))()
    _check(lib().amm_iter_log(handle, arr, n.value, C.byref(n)), handle)
    return [arr[i].as_dict() for i in range(n.value)]


def amm_k_nnzb(handle) -> int:
    n = C.c_int64()
    _check(lib().amm_k_nnzb(handle, C.byref(n)), handle)
    return n.value


def _energy_buffers(handle, X, src, rho=None, d2=None, gX=None, gV=None):
    if X is None:
        raise ValueError("X is required")
    sz = amm_get_sizes(handle)
    dt = _dtype_code(X)
    n, N = sz["n_nodes"], sz["n_src"]
    _device_buffer("X", X, dt, 12 * n)
    _device_buffer("src", src, dt, 3 * N)
    _device_buffer("rho", rho, "int32", N)
    _device_buffer("d2", d2, dt, N)
    _device_buffer("gX", gX, dt, 12 * n)
    _device_buffer("gV", gV, dt, 3 * N)


def amm_energy(handle, X, src=None, nu_a=1.0, nu_r=1.0, alpha=0.0, beta=0.0, rho=None, d2=None):
    _energy_buffers(handle, X, src, rho=rho, d2=d2)
    e = (C.c_double * 4)()
    _check(lib().amm_energy(handle, _dtype_code(X), _ptr(X), _ptr(src), nu_a, nu_r, alpha, beta, e,
                            _ptr(rho), _ptr(d2)), handle)
    return list(e)


def amm_energy_noalloc(handle, X, src=None, nu_a=1.0, nu_r=1.0, alpha=0.0, beta=0.0, rho=None, d2=None):
    """amm_energy with every per-call buffer in the library's static device
    scratch (no allocation); calls overlapping on one GPU race."""
    _energy_buffers(handle, X, src, rho=rho, d2=d2)
    e = (C.c_double * 4)()
    _check(lib().amm_energy_noalloc(handle, _dtype_code(X), _ptr(X), _ptr(src), nu_a, nu_r, alpha, beta, e,
                                    _ptr(rho), _ptr(d2)), handle)
    return list(e)


def amm_energy_grad(handle, X, src, nu_a, nu_r, alpha, beta, gX, gV=None):
    if gX is None:
        raise ValueError("gX is required")
    _energy_buffers(handle, X, src, gX=gX, gV=gV)
    e = (C.c_double * 4)()
    _check(lib().amm_energy_grad(handle, _dtype_code(X), _ptr(X), _ptr(src), nu_a, nu_r, alpha, beta,
                                 _ptr(gX), _ptr(gV), e), handle)
    return list(e)


def amm_enable_timing(handle, on: bool = True, only: Optional[str] = None) -> None:
    _check(lib().amm_enable_timing(handle, 1 if on else 0, only.encode() if only else None), handle)


def amm_kernel_times(handle) -> dict:
    cap = 64
    names = (C.c_char_p * cap)()
    ms = (C.c_double * cap)()
    n_l = (C.c_int32 * cap)()
    cnt = C.c_int32()
    _check(lib().amm_kernel_times(handle, names, ms, n_l, cap, C.byref(cnt)), handle)
    return {names[i].decode(): (ms[i], n_l[i]) for i in range(min(cnt.value, cap))}
