"""Plain FP64 CPU oracle of the HAMLS hot path (TEST INFRASTRUCTURE ONLY).

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
import this package.  It shares no code with the GPU library: its arithmetic is
in hamls_oracle.c, which this module loads with ctypes and feeds numpy arrays.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

from . import build as _build

_DOMAINS = {"s2": 0, "so3": 1, "t3": 2}
_REGS = {"none": 0, "fixed": 1, "chi": 2}

ST_REGULARIZED = 1
ST_UNDERDETERMINED = 2
ST_EMPTY = 4
ST_HEMISPHERE = 8


class OrcParams(C.Structure):
    _fields_ = [
        ("domain", C.c_int32),
        ("bandwidth", C.c_int32),
        ("degree", C.c_int32),
        ("knn_count", C.c_int32),
        ("support_radius", C.c_double),
        ("knn_eps", C.c_double),
        ("wendland", C.c_int32),
        ("reg", C.c_int32),
        ("tau_fixed", C.c_double),
        ("chi_target", C.c_double),
        ("chi_full", C.c_double),
        ("grid_shape", C.c_int32 * 3),
        ("smooth_aux", C.c_int32),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        path = _build.LIB
        if not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(_build.SRC):
            _build.build()
        L = C.CDLL(path)
        P = C.POINTER
        d, i32, i64 = C.c_double, C.c_int32, C.c_int64
        vp = C.c_void_p
        L.orc_gauss_legendre.argtypes = [C.c_int, vp, vp]
        L.orc_grid_dims.argtypes = [P(OrcParams), vp]
        L.orc_grid_size.argtypes = [P(OrcParams)]
        L.orc_grid_size.restype = i64
        L.orc_grid.argtypes = [P(OrcParams), vp, vp]
        L.orc_neighbors.argtypes = [P(OrcParams), vp, i64, vp, i64, vp, i64, vp, vp, vp, vp]
        L.orc_neighbor_lists.argtypes = [P(OrcParams), vp, vp, i64, vp, i64, vp, vp, vp]
        L.orc_mls.argtypes = [P(OrcParams), vp, i64, vp, i64, vp, i64, vp, vp, i32, i64, vp, vp, vp, vp, vp]
        L.orc_fibonacci.argtypes = [C.c_int, vp]
        L.orc_fibonacci.restype = None
        L.orc_voronoi_areas.argtypes = [vp, i64, vp, i64, vp]
        L.orc_voronoi_areas.restype = i64
        L.orc_generating.argtypes = [P(OrcParams), vp, i64, vp, i64, vp, i64, vp, vp, vp, vp, vp, vp, vp]
        L.orc_alf.argtypes = [C.c_int, d, vp]
        L.orc_alf.restype = None
        L.orc_wigner_d.argtypes = [C.c_int, d, vp]
        L.orc_wigner_d.restype = None
        L.orc_num_coeffs.argtypes = [P(OrcParams)]
        L.orc_num_coeffs.restype = i64
        L.orc_coeffs.argtypes = [P(OrcParams), vp, i32, vp, C.c_int]
        L.orc_eval.argtypes = [P(OrcParams), vp, i32, vp, i64, vp]
        L.orc_num_monomials.argtypes = [C.c_int, C.c_int]
        L.orc_monomials.argtypes = [C.c_int, C.c_int, vp, vp]
        L.orc_monomials.restype = None
        L.orc_local_system.argtypes = [P(OrcParams), vp, d, vp, C.c_int, vp, vp, vp, i32, i64, vp, vp]
        _lib = L
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def params(domain="s2", bandwidth=16, degree=2, support_radius=0.0, knn_count=0, knn_eps=0.05,
           wendland=1, reg="chi", tau_fixed=0.0, chi_target=10.0, chi_full=20.0, grid_shape=(0, 0, 0),
           smooth_aux=0, **_ignored) -> OrcParams:
    p = OrcParams()
    p.domain = _DOMAINS[domain]
    p.bandwidth = int(bandwidth)
    p.degree = int(degree)
    p.knn_count = int(knn_count)
    p.support_radius = float(support_radius)
    p.knn_eps = float(knn_eps)
    p.wendland = int(wendland)
    p.reg = _REGS[reg]
    p.tau_fixed = float(tau_fixed)
    p.chi_target = float(chi_target)
    p.chi_full = float(chi_full)
    p.smooth_aux = int(smooth_aux)
    gs = list(grid_shape) + [0] * (3 - len(grid_shape))
    for k in range(3):
        p.grid_shape[k] = int(gs[k])
    return p


def _dimq(p: OrcParams) -> int:
    return 4 if p.domain == 1 else 3


def gauss_legendre(n: int):
    x = np.zeros(n)
    w = np.zeros(n)
    assert lib().orc_gauss_legendre(n, _ptr(x), _ptr(w)) == 0
    return x, w


def grid_dims(p: OrcParams):
    d = np.zeros(3, dtype=np.int32)
    rc = lib().orc_grid_dims(C.byref(p), _ptr(d))
    if rc:
        raise ValueError("invalid grid")
    return tuple(int(v) for v in d)


def grid(p: OrcParams):
    MQ = lib().orc_grid_size(C.byref(p))
    pts = np.zeros((MQ, _dimq(p)))
    w = np.zeros(MQ)
    assert lib().orc_grid(C.byref(p), _ptr(pts), _ptr(w)) == 0
    return pts, w


def _rows(rows):
    return None if rows is None else np.ascontiguousarray(rows, dtype=np.int64)


def neighbors(p: OrcParams, grid_pts, nodes, rows=None, lists=False):
    """Per centre: threshold, radius, count, status; optionally CSR lists."""
    grid_pts = np.ascontiguousarray(grid_pts, dtype=np.float64)
    nodes = np.ascontiguousarray(nodes, dtype=np.float64)
    rows = _rows(rows)
    R = grid_pts.shape[0] if rows is None else rows.shape[0]
    thr = np.zeros(R)
    dl = np.zeros(R)
    cnt = np.zeros(R, dtype=np.int32)
    st = np.zeros(R, dtype=np.uint8)
    rc = lib().orc_neighbors(C.byref(p), _ptr(grid_pts), grid_pts.shape[0], _ptr(rows), R, _ptr(nodes),
                             nodes.shape[0], _ptr(thr), _ptr(dl), _ptr(cnt), _ptr(st))
    if rc:
        raise ValueError("orc_neighbors failed")
    out = dict(threshold=thr, delta=dl, count=cnt, status=st)
    if lists:
        rp = np.zeros(R + 1, dtype=np.int64)
        rp[1:] = np.cumsum(cnt)
        idx = np.zeros(int(rp[-1]), dtype=np.int32)
        lib().orc_neighbor_lists(C.byref(p), _ptr(grid_pts), _ptr(rows), R, _ptr(nodes), nodes.shape[0],
                                 _ptr(thr), _ptr(rp), _ptr(idx))
        out["row_ptr"] = rp
        out["idx"] = idx
    return out


def mls(p: OrcParams, grid_pts, nodes, values, node_weights=None, rows=None):
    """Step 2 of Alg. 1 at the requested centres.  values: (F, M)."""
    grid_pts = np.ascontiguousarray(grid_pts, dtype=np.float64)
    nodes = np.ascontiguousarray(nodes, dtype=np.float64)
    values = np.ascontiguousarray(np.atleast_2d(values), dtype=np.float64)
    F, M = values.shape
    nu = None if node_weights is None else np.ascontiguousarray(node_weights, dtype=np.float64)
    rows = _rows(rows)
    R = grid_pts.shape[0] if rows is None else rows.shape[0]
    out = np.zeros((F, R))
    nj = np.zeros(R, dtype=np.int32)
    chi = np.zeros(R)
    tau = np.zeros(R)
    st = np.zeros(R, dtype=np.uint8)
    rc = lib().orc_mls(C.byref(p), _ptr(grid_pts), grid_pts.shape[0], _ptr(rows), R, _ptr(nodes), M,
                       _ptr(nu), _ptr(values), F, M, _ptr(out), _ptr(nj), _ptr(chi), _ptr(tau), _ptr(st))
    if rc:
        raise ValueError("orc_mls failed")
    return dict(values=out, n=nj, chi=chi, tau=tau, status=st)


def generating(p: OrcParams, grid_pts, nodes, node_weights=None, rows=None):
    """Generating functions of MLS at the requested centres (Rem. 2.5): CSR
    row_ptr / idx (ascending original index) / val with M_y(q_r) =
    sum_e val[e] y[idx[e]] over row r; plus chi, tau, status per centre."""
    grid_pts = np.ascontiguousarray(grid_pts, dtype=np.float64)
    nodes = np.ascontiguousarray(nodes, dtype=np.float64)
    nu = None if node_weights is None else np.ascontiguousarray(node_weights, dtype=np.float64)
    rows = _rows(rows)
    nb = neighbors(p, grid_pts, nodes, rows=rows)
    R = nb["count"].shape[0]
    rp = np.zeros(R + 1, dtype=np.int64)
    rp[1:] = np.cumsum(nb["count"])
    idx = np.zeros(max(int(rp[-1]), 1), dtype=np.int32)
    val = np.zeros(max(int(rp[-1]), 1))
    chi = np.zeros(R)
    tau = np.zeros(R)
    st = np.zeros(R, dtype=np.uint8)
    rc = lib().orc_generating(C.byref(p), _ptr(grid_pts), grid_pts.shape[0], _ptr(rows), R, _ptr(nodes),
                              nodes.shape[0], _ptr(nu), _ptr(rp), _ptr(idx), _ptr(val), _ptr(chi), _ptr(tau),
                              _ptr(st))
    if rc:
        raise ValueError("orc_generating failed")
    n = int(rp[-1])
    return dict(row_ptr=rp, idx=idx[:n], val=val[:n], chi=chi, tau=tau, status=st)


def voronoi_areas(nodes, rows=None):
    """Spherical Voronoi cell area of every node (S2 unit vectors, M x 3), or
    of the nodes `rows`, brute force over all nodes; NaN for a cell reaching
    ~90 degrees from its node."""
    x = np.ascontiguousarray(nodes, dtype=np.float64)
    if rows is None:
        a = np.zeros(x.shape[0])
        lib().orc_voronoi_areas(_ptr(x), x.shape[0], None, 0, _ptr(a))
    else:
        r = np.ascontiguousarray(rows, dtype=np.int64)
        a = np.zeros(r.shape[0])
        lib().orc_voronoi_areas(_ptr(x), x.shape[0], _ptr(r), r.shape[0], _ptr(a))
    return a


def fibonacci(n: int):
    """The auxiliary Fibonacci grid of the smoothed radius (n x 3)."""
    pts = np.zeros((n, 3))
    lib().orc_fibonacci(int(n), _ptr(pts))
    return pts


def num_coeffs(p: OrcParams) -> int:
    return int(lib().orc_num_coeffs(C.byref(p)))


def coeffs(p: OrcParams, grid_values, literal=False):
    gv = np.ascontiguousarray(np.atleast_2d(grid_values), dtype=np.float64)
    F = gv.shape[0]
    nc = num_coeffs(p)
    out = np.zeros((F, nc, 2))
    assert lib().orc_coeffs(C.byref(p), _ptr(gv), F, _ptr(out), int(bool(literal))) == 0
    return out[..., 0] + 1j * out[..., 1]


def evaluate(p: OrcParams, coef, pts):
    coef = np.atleast_2d(coef)
    F = coef.shape[0]
    c = np.ascontiguousarray(np.stack([coef.real, coef.imag], axis=-1), dtype=np.float64)
    pts = np.ascontiguousarray(pts, dtype=np.float64)
    out = np.zeros((F, pts.shape[0]))
    assert lib().orc_eval(C.byref(p), _ptr(c), F, _ptr(pts), pts.shape[0], _ptr(out)) == 0
    return out


def alf(N: int, x: float):
    P = np.zeros((N + 1) * (N + 2) // 2)
    lib().orc_alf(N, float(x), _ptr(P))
    return P


def wigner_d(N: int, beta: float):
    n = (N + 1) * (2 * N + 1) * (2 * N + 3) // 3
    d = np.zeros(n)
    lib().orc_wigner_d(N, float(beta), _ptr(d))
    return d


def monomials(domain: str, K: int):
    dom = _DOMAINS[domain]
    m = lib().orc_num_monomials(dom, K)
    e = np.zeros((m, 3), dtype=np.int32)
    g = np.zeros(m, dtype=np.int32)
    lib().orc_monomials(dom, K, _ptr(e), _ptr(g))
    return e, g


def local_system(p: OrcParams, q, delta, nb, nodes, values, node_weights=None):
    """B (n x m) and y_w (n x F) of one centre, as the oracle forms them."""
    q = np.ascontiguousarray(q, dtype=np.float64)
    nb = np.ascontiguousarray(nb, dtype=np.int32)
    nodes = np.ascontiguousarray(nodes, dtype=np.float64)
    values = np.ascontiguousarray(np.atleast_2d(values), dtype=np.float64)
    F, M = values.shape
    n = nb.shape[0]
    m = lib().orc_num_monomials(p.domain, p.degree)
    B = np.zeros((m, n))
    yw = np.zeros((F, n))
    nu = None if node_weights is None else np.ascontiguousarray(node_weights, dtype=np.float64)
    rc = lib().orc_local_system(C.byref(p), _ptr(q), float(delta), _ptr(nb), n, _ptr(nodes), _ptr(nu),
                                _ptr(values), F, M, _ptr(B), _ptr(yw))
    if rc:
        raise ValueError("local system failed")
    return B.T.copy(), yw.T.copy()
