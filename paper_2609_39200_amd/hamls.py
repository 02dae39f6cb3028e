"""ctypes binding of the C ABI in include/hamls.h (argument marshalling only).

Device buffers are torch tensors on the current HIP device (float64,
contiguous); streams default to torch's current stream.  Every step of the
path runs in libhamls.so; there is no fallback of any kind, and a missing or
unloadable library raises at import.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhamls.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(
        f"{LIB_PATH} is not built; run `python paper_2609_39200_amd/build.py` "
        "(there is no CPU fallback)")

_lib = C.CDLL(LIB_PATH)

HAMLS_OK = 0
STATUS = {0: "ok", -1: "invalid argument", -2: "unsupported", -3: "out of memory", -4: "device error",
          -5: "domain error", -6: "grid not exact"}
DOMAINS = {"s2": 0, "so3": 1, "t3": 2}
REGS = {"none": 0, "fixed": 1, "chi": 2}
PRECISIONS = {"fp64": 0, "mixed": 1}

ST_REGULARIZED = 1
ST_UNDERDETERMINED = 2
ST_EMPTY = 4
ST_HEMISPHERE = 8
ST_ILLCOND = 16


class hamls_params(C.Structure):
    _fields_ = [
        ("struct_size", C.c_int32),
        ("domain", C.c_int32),
        ("bandwidth", C.c_int32),
        ("degree", C.c_int32),
        ("support_radius", C.c_double),
        ("knn_count", C.c_int32),
        ("wendland", C.c_int32),
        ("knn_eps", C.c_double),
        ("reg", C.c_int32),
        ("precision", C.c_int32),
        ("tau_fixed", C.c_double),
        ("chi_target", C.c_double),
        ("chi_full", C.c_double),
        ("grid_shape", C.c_int32 * 3),
        ("smooth_aux", C.c_int32),
    ]


class hamls_plan_info(C.Structure):
    _fields_ = [
        ("domain", C.c_int32),
        ("bandwidth", C.c_int32),
        ("degree", C.c_int32),
        ("m", C.c_int32),
        ("grid_dims", C.c_int32 * 3),
        ("precision", C.c_int32),
        ("num_grid", C.c_int64),
        ("num_coeffs", C.c_int64),
        ("num_nodes", C.c_int64),
        ("node_capacity", C.c_int64),
        ("resident_bytes", C.c_int64),
        ("num_cells", C.c_int64),
    ]


class hamls_request(C.Structure):
    _fields_ = [
        ("struct_size", C.c_int32),
        ("F", C.c_int32),
        ("params", hamls_params),
        ("nodes", C.c_void_p),
        ("node_weights", C.c_void_p),
        ("M", C.c_int64),
        ("values", C.c_void_p),
        ("coeffs", C.c_void_p),
        ("tag", C.c_uint64),
    ]


class hamls_completion(C.Structure):
    _fields_ = [
        ("tag", C.c_uint64),
        ("status", C.c_int32),
        ("plan_reused", C.c_int32),
        ("t_submit", C.c_double),
        ("t_admit", C.c_double),
        ("t_done", C.c_double),
    ]


_vp = C.c_void_p
_i32, _i64 = C.c_int32, C.c_int64
_P = C.POINTER
_SIGS = {
    "hamls_params_init": [_P(hamls_params)],
    "hamls_plan": [_P(hamls_params), _vp, _i64, _vp, _vp, _P(_vp)],
    "hamls_plan_rebind": [_vp, _vp, _i64, _vp, _vp],
    "hamls_mls_to_grid": [_vp, _vp, _i32, _i64, _vp, _vp],
    "hamls_grid_to_coeffs": [_vp, _vp, _i32, _vp, _vp],
    "hamls_grid_to_coeffs_noalloc": [_vp, _vp, _i32, _vp, _vp],
    "hamls_eval": [_vp, _vp, _i32, _vp, _i64, _vp, _vp],
    "hamls_plan_voronoi_areas": [_vp, _vp, _vp],
    "hamls_plan_destroy": [_vp],
    "hamls_plan_info_get": [_vp, _P(hamls_plan_info)],
    "hamls_plan_grid": [_vp, _vp, _vp],
    "hamls_plan_neighbors": [_vp, _vp, _vp],
    "hamls_plan_radii": [_vp, _vp, _vp],
    "hamls_diagnostics": [_vp, _vp, _vp, _vp, _vp],
    "hamls_timing_enable": [_vp, _i32],
    "hamls_timing_phases": [_vp, C.c_uint32],
    "hamls_timing_read": [_vp, _i32, _vp, _vp],
    "hamls_plan_footprint": [_P(hamls_params), _i64, _i32, _P(_i64)],
    "hamls_plan_tune": [_vp, _vp, _P(_i32), _vp],
    "hamls_plan_routing": [_vp, _i32, _P(_i32), _vp],
    "hamls_plan_assembly_form": [_vp, _vp, _i32],
    "hamls_plan_cost_order": [_vp, _vp],
    "hamls_fit_capture": [_vp, _vp, _i32, _i64, _vp, _vp, _vp, _P(_vp)],
    "hamls_graph_launch": [_vp, _vp],
    "hamls_graph_destroy": [_vp],
    "hamls_gen_build": [_vp, _vp],
    "hamls_gen_apply": [_vp, _vp, _i32, _i64, _vp, _vp],
    "hamls_gen_get": [_vp, _vp, _vp, _vp],
    "hamls_server_create": [_i32, _i64, _P(_vp)],
    "hamls_server_submit": [_vp, _P(hamls_request)],
    "hamls_server_wait": [_vp, _P(hamls_completion), _i32, _P(_i32), C.c_double],
    "hamls_server_load": [_vp, _P(_i32), _P(_i64), _P(_i32)],
    "hamls_server_destroy": [_vp],
}
for _name, _args in _SIGS.items():
    _f = getattr(_lib, _name)
    _f.argtypes = _args
    _f.restype = C.c_int
_lib.hamls_status_string.argtypes = [C.c_int]
_lib.hamls_status_string.restype = C.c_char_p
_lib.hamls_server_clock.argtypes = []
_lib.hamls_server_clock.restype = C.c_double
_lib.hamls_last_error.argtypes = []
_lib.hamls_last_error.restype = C.c_char_p
_lib.hamls_noalloc_scratch_bytes.argtypes = []
_lib.hamls_noalloc_scratch_bytes.restype = C.c_size_t


class HamlsError(RuntimeError):
    def __init__(self, code: int, where: str):
        self.code = code
        msg = _lib.hamls_last_error().decode(errors="replace")
        super().__init__(f"{where}: {STATUS.get(code, code)}: {msg}")


def _check(code: int, where: str):
    if code != HAMLS_OK:
        raise HamlsError(code, where)


def _stream(stream):
    if stream is None:
        import torch

        return C.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return C.c_void_p(stream)
    return C.c_void_p(stream.cuda_stream)


def _dev(t, name, shape=None):
    import torch

    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a device tensor")
    if t.dtype != torch.float64 or not t.is_contiguous():
        raise TypeError(f"{name} must be contiguous float64")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")
    return C.c_void_p(t.data_ptr())


def hamls_params_init(**kw) -> hamls_params:
    """Defaults of the C library, then keyword overrides (domain/reg/precision
    may be given by name)."""
    p = hamls_params()
    _check(_lib.hamls_params_init(C.byref(p)), "hamls_params_init")
    for k, v in kw.items():
        if k == "domain" and isinstance(v, str):
            v = DOMAINS[v]
        elif k == "reg" and isinstance(v, str):
            v = REGS[v]
        elif k == "precision" and isinstance(v, str):
            v = PRECISIONS[v]
        if k == "grid_shape":
            gs = list(v) + [0] * (3 - len(v))
            for i in range(3):
                p.grid_shape[i] = int(gs[i])
            continue
        if not hasattr(p, k):
            raise KeyError(k)
        setattr(p, k, v)
    return p


def hamls_plan(params: hamls_params, nodes, node_weights=None, stream=None) -> int:
    h = C.c_void_p()
    w = None if node_weights is None else _dev(node_weights, "node_weights")
    _check(_lib.hamls_plan(C.byref(params), _dev(nodes, "nodes"), nodes.shape[0], w, _stream(stream),
                           C.byref(h)), "hamls_plan")
    return h.value


def hamls_plan_rebind(plan: int, nodes, node_weights=None, stream=None):
    w = None if node_weights is None else _dev(node_weights, "node_weights")
    _check(_lib.hamls_plan_rebind(C.c_void_p(plan), _dev(nodes, "nodes"), nodes.shape[0], w,
                                  _stream(stream)), "hamls_plan_rebind")


def hamls_mls_to_grid(plan: int, values, grid_values, stream=None):
    """values: (F, M) contiguous; grid_values: (F, M_Q)."""
    F = values.shape[0]
    _check(_lib.hamls_mls_to_grid(C.c_void_p(plan), _dev(values, "values"), F, values.shape[1],
                                  _dev(grid_values, "grid_values"), _stream(stream)), "hamls_mls_to_grid")


def hamls_grid_to_coeffs(plan: int, grid_values, coeffs, stream=None):
    """grid_values: (F, M_Q); coeffs: (F, n_coeff, 2)."""
    F = grid_values.shape[0]
    _check(_lib.hamls_grid_to_coeffs(C.c_void_p(plan), _dev(grid_values, "grid_values"), F,
                                     _dev(coeffs, "coeffs"), _stream(stream)), "hamls_grid_to_coeffs")


def hamls_grid_to_coeffs_noalloc(plan: int, grid_values, coeffs, stream=None):
    """As hamls_grid_to_coeffs, with the step-3 work memory in the library's
    static device array (no allocation)."""
    F = grid_values.shape[0]
    _check(_lib.hamls_grid_to_coeffs_noalloc(C.c_void_p(plan), _dev(grid_values, "grid_values"), F,
                                             _dev(coeffs, "coeffs"), _stream(stream)),
           "hamls_grid_to_coeffs_noalloc")


def hamls_noalloc_scratch_bytes() -> int:
    return int(_lib.hamls_noalloc_scratch_bytes())


def hamls_plan_voronoi_areas(plan: int, areas, stream=None):
    """areas: (M,) FP64 device tensor, the spherical Voronoi-cell area of every
    bound node (S2 plans)."""
    _check(_lib.hamls_plan_voronoi_areas(C.c_void_p(plan), _dev(areas, "areas"), _stream(stream)),
           "hamls_plan_voronoi_areas")


def hamls_eval(plan: int, coeffs, points, out, stream=None):
    F = coeffs.shape[0]
    _check(_lib.hamls_eval(C.c_void_p(plan), _dev(coeffs, "coeffs"), F, _dev(points, "points"),
                           points.shape[0], _dev(out, "out"), _stream(stream)), "hamls_eval")


def hamls_plan_destroy(plan: int):
    _check(_lib.hamls_plan_destroy(C.c_void_p(plan)), "hamls_plan_destroy")


def hamls_plan_info_get(plan: int) -> hamls_plan_info:
    o = hamls_plan_info()
    _check(_lib.hamls_plan_info_get(C.c_void_p(plan), C.byref(o)), "hamls_plan_info_get")
    return o


def _np_ptr(a):
    return a.ctypes.data_as(C.c_void_p)


def hamls_plan_grid(plan: int):
    info = hamls_plan_info_get(plan)
    dim = 4 if info.domain == 1 else 3
    pts = np.zeros((info.num_grid, dim))
    w = np.zeros(info.num_grid)
    _check(_lib.hamls_plan_grid(C.c_void_p(plan), _np_ptr(pts), _np_ptr(w)), "hamls_plan_grid")
    return pts, w


def hamls_plan_neighbors(plan: int):
    info = hamls_plan_info_get(plan)
    rp = np.zeros(info.num_grid + 1, dtype=np.int64)
    _check(_lib.hamls_plan_neighbors(C.c_void_p(plan), _np_ptr(rp), None), "hamls_plan_neighbors")
    idx = np.zeros(int(rp[-1]), dtype=np.int32)
    _check(_lib.hamls_plan_neighbors(C.c_void_p(plan), _np_ptr(rp), _np_ptr(idx)), "hamls_plan_neighbors")
    return rp, idx


def hamls_plan_radii(plan: int):
    info = hamls_plan_info_get(plan)
    d = np.zeros(info.num_grid)
    c = np.zeros(info.num_grid)
    _check(_lib.hamls_plan_radii(C.c_void_p(plan), _np_ptr(d), _np_ptr(c)), "hamls_plan_radii")
    return d, c


def hamls_diagnostics(plan: int):
    info = hamls_plan_info_get(plan)
    n = np.zeros(info.num_grid, dtype=np.int32)
    chi = np.zeros(info.num_grid)
    tau = np.zeros(info.num_grid)
    st = np.zeros(info.num_grid, dtype=np.uint8)
    _check(_lib.hamls_diagnostics(C.c_void_p(plan), _np_ptr(n), _np_ptr(chi), _np_ptr(tau), _np_ptr(st)),
           "hamls_diagnostics")
    return dict(n=n, chi=chi, tau=tau, status=st)


PHASES = {"binning": 0, "radius": 1, "assemble": 2, "solve": 3, "ring_dft": 4, "contract": 5, "gather": 6,
          "gen_apply": 7, "resolve": 8, "fold": 9}


def hamls_timing_enable(plan: int, enable: bool = True):
    _check(_lib.hamls_timing_enable(C.c_void_p(plan), int(bool(enable))), "hamls_timing_enable")


def hamls_timing_phases(plan: int, phases=None):
    """Time only the named phases (all when None)."""
    mask = 0xFFFFFFFF if phases is None else sum(1 << (PHASES[p] if isinstance(p, str) else int(p)) for p in phases)
    _check(_lib.hamls_timing_phases(C.c_void_p(plan), C.c_uint32(mask)), "hamls_timing_phases")


def hamls_timing_read(plan: int, phase) -> tuple:
    """(launches, total_ms) of one phase since the last read (synchronizes)."""
    ph = PHASES[phase] if isinstance(phase, str) else int(phase)
    n = C.c_int64()
    ms = C.c_double()
    _check(_lib.hamls_timing_read(C.c_void_p(plan), ph, C.byref(n), C.byref(ms)), "hamls_timing_read")
    return int(n.value), float(ms.value)


def hamls_status_string(code: int) -> str:
    return _lib.hamls_status_string(code).decode()


def hamls_last_error() -> str:
    return _lib.hamls_last_error().decode(errors="replace")


def params_from_workload(wp: dict, **over) -> hamls_params:
    """hamls_params from a workloads.Workload.params dict (plus overrides)."""
    kw = dict(domain=wp["domain"], bandwidth=wp["bandwidth"], degree=wp["degree"],
              support_radius=float(wp.get("support_radius", 0.0)), knn_count=int(wp.get("knn_count", 0)),
              knn_eps=float(wp.get("knn_eps", 0.05)), reg=wp.get("reg", "chi"),
              tau_fixed=float(wp.get("tau_fixed", 0.0)), chi_target=float(wp.get("chi_target", 10.0)),
              chi_full=float(wp.get("chi_full", 20.0)), grid_shape=tuple(wp.get("grid_shape", (0, 0, 0))),
              smooth_aux=int(wp.get("smooth_aux", 0)))
    kw.update(over)
    return hamls_params_init(**kw)


def hamls_plan_footprint(params: hamls_params, M: int, F: int = 1) -> int:
    out = C.c_int64(0)
    _check(_lib.hamls_plan_footprint(C.byref(params), int(M), int(F), C.byref(out)), "hamls_plan_footprint")
    return int(out.value)


def hamls_server_create(slots: int = 4, hbm_budget: int = 0) -> int:
    out = C.c_void_p()
    _check(_lib.hamls_server_create(int(slots), int(hbm_budget), C.byref(out)), "hamls_server_create")
    return out.value


def hamls_server_submit(server: int, params: hamls_params, nodes, values, coeffs, node_weights=None,
                        tag: int = 0):
    """Queue one fit; the tensors must stay alive and unchanged until its completion."""
    M = nodes.shape[0]
    F = values.shape[0] if values.dim() == 2 else 1
    r = hamls_request()
    r.struct_size = C.sizeof(hamls_request)
    r.F = F
    r.params = params
    r.nodes = _dev(nodes, "nodes").value
    r.node_weights = None if node_weights is None else _dev(node_weights, "node_weights", (M,)).value
    r.M = M
    r.values = _dev(values, "values").value
    r.coeffs = _dev(coeffs, "coeffs").value
    r.tag = int(tag)
    if values.numel() != F * M:
        raise ValueError("values must hold F x M entries")
    _check(_lib.hamls_server_submit(C.c_void_p(server), C.byref(r)), "hamls_server_submit")


def hamls_server_wait(server: int, max_count: int = 64, timeout_s: float = 1.0) -> list:
    """Completions as dicts (tag, status, plan_reused, t_submit, t_admit, t_done)."""
    buf = (hamls_completion * max_count)()
    n = C.c_int32(0)
    _check(_lib.hamls_server_wait(C.c_void_p(server), buf, int(max_count), C.byref(n), float(timeout_s)),
           "hamls_server_wait")
    return [dict(tag=int(c.tag), status=int(c.status), plan_reused=bool(c.plan_reused), t_submit=c.t_submit,
                 t_admit=c.t_admit, t_done=c.t_done) for c in buf[:n.value]]


def hamls_server_load(server: int) -> tuple:
    a, b, c = C.c_int32(0), C.c_int64(0), C.c_int32(0)
    _check(_lib.hamls_server_load(C.c_void_p(server), C.byref(a), C.byref(b), C.byref(c)), "hamls_server_load")
    return int(a.value), int(b.value), int(c.value)


def hamls_server_destroy(server: int):
    _check(_lib.hamls_server_destroy(C.c_void_p(server)), "hamls_server_destroy")


def hamls_server_clock() -> float:
    return float(_lib.hamls_server_clock())


def hamls_gen_build(plan: int, stream=None):
    _check(_lib.hamls_gen_build(C.c_void_p(plan), _stream(stream)), "hamls_gen_build")


def hamls_gen_apply(plan: int, values, grid_values, stream=None):
    """values: (F, M) contiguous; grid_values: (F, M_Q)."""
    F = values.shape[0]
    _check(_lib.hamls_gen_apply(C.c_void_p(plan), _dev(values, "values"), F, values.shape[1],
                                _dev(grid_values, "grid_values"), _stream(stream)), "hamls_gen_apply")


def hamls_gen_get(plan: int):
    """(row_ptr, idx, val) numpy arrays: the generating functions per grid node."""
    info = hamls_plan_info_get(plan)
    rp = np.zeros(info.num_grid + 1, dtype=np.int64)
    _check(_lib.hamls_gen_get(C.c_void_p(plan), _np_ptr(rp), None, None), "hamls_gen_get")
    idx = np.zeros(max(int(rp[-1]), 1), dtype=np.int32)
    val = np.zeros(max(int(rp[-1]), 1))
    _check(_lib.hamls_gen_get(C.c_void_p(plan), _np_ptr(rp), _np_ptr(idx), _np_ptr(val)), "hamls_gen_get")
    return rp, idx[: rp[-1]], val[: rp[-1]]


def hamls_fit_capture(plan: int, values, grid_values, coeffs, stream) -> int:
    """Capture step 2 + step 3 on `stream` (not the default stream); returns a graph handle."""
    out = C.c_void_p()
    F = values.shape[0]
    _check(_lib.hamls_fit_capture(C.c_void_p(plan), _dev(values, "values"), F, values.shape[1],
                                  _dev(grid_values, "grid_values"), _dev(coeffs, "coeffs"), _stream(stream),
                                  C.byref(out)), "hamls_fit_capture")
    return out.value


def hamls_graph_launch(graph: int, stream=None):
    _check(_lib.hamls_graph_launch(C.c_void_p(graph), _stream(stream)), "hamls_graph_launch")


def hamls_graph_destroy(graph: int):
    _check(_lib.hamls_graph_destroy(C.c_void_p(graph)), "hamls_graph_destroy")


def hamls_plan_tune(plan: int, stream=None) -> tuple:
    """(form, [grid order ms, cost-ordered dispatch ms, queue 8/CU ms, queue 12/CU ms]);
    form 0 = grid order, 1 = cost-ordered dispatch, else the queue's block count."""
    q = C.c_int32(0)
    t = (C.c_float * 4)()
    _check(_lib.hamls_plan_tune(C.c_void_p(plan), _stream(stream), C.byref(q), t), "hamls_plan_tune")
    return int(q.value), [float(v) for v in t]


def hamls_plan_routing(plan: int, set: int = -1) -> tuple:
    """(enabled, [step-2 ms without, with routing] from the tuner or -1);
    set: -1 query, 0 off, 1 on."""
    en = C.c_int32(0)
    t = (C.c_float * 2)()
    _check(_lib.hamls_plan_routing(C.c_void_p(plan), int(set), C.byref(en), t), "hamls_plan_routing")
    return bool(en.value), [float(v) for v in t]


def hamls_plan_assembly_form(plan: int, queue_blocks: int, stream=None):
    _check(_lib.hamls_plan_assembly_form(C.c_void_p(plan), _stream(stream), int(queue_blocks)),
           "hamls_plan_assembly_form")


def hamls_plan_cost_order(plan: int) -> np.ndarray:
    """The plan's cost order (grid node indices, int32 M_Q) behind forms >= 1."""
    info = hamls_plan_info_get(plan)
    out = np.empty(info.num_grid, dtype=np.int32)
    _check(_lib.hamls_plan_cost_order(C.c_void_p(plan), out.ctypes.data_as(C.c_void_p)), "hamls_plan_cost_order")
    return out
