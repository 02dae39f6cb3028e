"""Comparison helpers shared by the GPU parity tests (no arithmetic of the
method: norms, ulp distances, and the membership keys written out in numpy
with the same fixed association as the predicate of both sides)."""
import sys

import numpy as np


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def rell2(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.linalg.norm((a - b).ravel()) / max(np.linalg.norm(b.ravel()), 1e-300))


def maxrel(a, b):
    """max |a - b| / max |b| (the largest single deviation against the scale)."""
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def ulp_diff(a, b):
    """Number of representable doubles between a and b (elementwise)."""
    def ordered(x):
        i = np.asarray(x, dtype=np.float64).view(np.int64)
        return np.where(i < 0, np.int64(-(2 ** 63)) - i, i)

    return np.abs(ordered(a) - ordered(b))


def keys(domain, nodes, q):
    """Membership key of every node for centre q, in the predicate's fixed
    association without fused operations (numpy never contracts): S2 and SO3
    the dot product summed left to right (SO3 its absolute value), T3 the
    squared min-image distance."""
    x = np.asarray(nodes, dtype=np.float64)
    if domain == "s2":
        return (x[:, 0] * q[0] + x[:, 1] * q[1]) + x[:, 2] * q[2]
    if domain == "so3":
        return np.abs(((x[:, 0] * q[0] + x[:, 1] * q[1]) + x[:, 2] * q[2]) + x[:, 3] * q[3])
    s = np.zeros(x.shape[0])
    for d in range(3):
        dl = x[:, d] - q[d]
        dl = dl - np.rint(dl)
        s = s + dl * dl
    return s


def flip_count(domain, nodes, q, thr_a, thr_b):
    """Nodes whose membership differs between two thresholds of one centre:
    keys in the half-open interval between them (member iff key > c on S2 and
    SO3, key < c on T3)."""
    if thr_a == thr_b:
        return 0
    lo, hi = min(thr_a, thr_b), max(thr_a, thr_b)
    k = keys(domain, nodes, q)
    if domain == "t3":
        return int(np.count_nonzero((k >= lo) & (k < hi)))
    return int(np.count_nonzero((k > lo) & (k <= hi)))


def check_grids(gpts, gw, opts, ow):
    """The library and the oracle compute the quadrature grid by different
    methods; they agree to rounding.  Returns a summary string."""
    assert gpts.shape == opts.shape and gw.shape == ow.shape
    dp = np.abs(gpts - opts).max()
    # near the poles a one-ulp change of cos(theta) moves sin(theta) by
    # ~eps / sin(theta): the points agree to 1e-13, the weights to 1e-10
    assert dp < 1e-13, dp
    rw = np.abs(gw / ow - 1.0).max()
    assert rw < 1e-10, rw
    n_exact = int(np.sum(np.all(gpts == opts, axis=1)))
    return f"points max |diff| {dp:.1e} ({n_exact}/{gpts.shape[0]} bitwise), weights max rel {rw:.1e}"


def check_thresholds(domain, nodes, gpts, sel, thr_gpu, thr_orc, max_ulp=64):
    """Thresholds of the two sides (in the same convention) are compared in
    ulps, and for every centre where they differ no node key may lie between
    them, so that the neighbour sets are equal by construction."""
    d = ulp_diff(thr_gpu, thr_orc)
    n1 = int(np.count_nonzero(d == 1))
    n2 = int(np.count_nonzero(d > 1))
    flips = 0
    for r in np.nonzero(d)[0]:
        flips += flip_count(domain, nodes, gpts[sel[r]], float(thr_gpu[r]), float(thr_orc[r]))
    say(f"  thresholds: {d.size - n1 - n2} equal, {n1} differ by 1 ulp, {n2} by more "
        f"(max {int(d.max()) if d.size else 0}); node keys between them: {flips}")
    assert flips == 0
    assert d.size == 0 or int(d.max()) <= max_ulp
