"""Seeded synthetic workloads shaped like the paper's experiments.

This module only draws inputs: scattered nodes, values at the nodes and
evaluation points.  It holds none of the method's arithmetic (no grid, no
neighbour search, no local solve, no quadrature), so both the GPU path's tests
and the CPU oracle's tests may draw from it.

The paper's own data (the weather stations of Sec. 3.1 and the synthetic f0 of
Sec. 3.2) are not available; these generators stand in for them with the same
kind of structure: clusters, large holes and a uniform background on S2,
clustered rotations on SO(3) and clustered points on T3.

Band-limited test fields are built from zonal (S2), class (SO(3)) and separable
(T3) pieces, each of which is band-limited by construction, so that the whole
field lies in Pi_L without evaluating any harmonic basis of the method.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np


# --------------------------------------------------------------------- S2 nodes
def uniform_s2(M: int, rng: np.random.Generator) -> np.ndarray:
    """M points iid uniform on S2 (normalised Gaussians), shape (M, 3)."""
    x = rng.standard_normal((M, 3))
    return x / np.linalg.norm(x, axis=1, keepdims=True)


def vmf_s2(M: int, mu: np.ndarray, kappa: float, rng: np.random.Generator) -> np.ndarray:
    """von Mises-Fisher samples around the unit vector mu (Wood's method with
    the closed-form inverse for the cosine on S2)."""
    u = rng.random(M)
    w = 1.0 + np.log(u + (1.0 - u) * np.exp(-2.0 * kappa)) / kappa
    w = np.clip(w, -1.0, 1.0)
    # orthonormal frame around mu
    a = np.array([1.0, 0.0, 0.0]) if abs(mu[0]) < 0.9 else np.array([0.0, 1.0, 0.0])
    e1 = a - mu * (a @ mu)
    e1 /= np.linalg.norm(e1)
    e2 = np.cross(mu, e1)
    ang = 2.0 * math.pi * rng.random(M)
    s = np.sqrt(np.maximum(0.0, 1.0 - w * w))
    x = w[:, None] * mu[None, :] + s[:, None] * (np.cos(ang)[:, None] * e1 + np.sin(ang)[:, None] * e2)
    return x / np.linalg.norm(x, axis=1, keepdims=True)


def cluster_hole_s2(
    M: int,
    rng: np.random.Generator,
    n_clusters: int = 8,
    kappa: float = 20.0,
    frac_uniform: float = 0.2,
    caps: list | None = None,
) -> np.ndarray:
    """Mixture of von Mises-Fisher clusters plus a uniform fraction with
    spherical caps removed by rejection until exactly M nodes remain.
    caps: list of (centre unit vector, angular radius in rad)."""
    centres = uniform_s2(n_clusters, rng)
    caps = caps or []
    out = []
    have = 0
    while have < M:
        B = max(1024, int(1.3 * (M - have)))
        n_uni = rng.binomial(B, frac_uniform)
        parts = [uniform_s2(n_uni, rng)]
        which = rng.integers(0, n_clusters, B - n_uni)
        for c in range(n_clusters):
            k = int(np.sum(which == c))
            if k:
                parts.append(vmf_s2(k, centres[c], kappa, rng))
        x = np.concatenate(parts, axis=0)
        x = x[rng.permutation(x.shape[0])]
        keep = np.ones(x.shape[0], dtype=bool)
        for cen, rad in caps:
            keep &= (x @ cen) < math.cos(rad)
        x = x[keep]
        out.append(x)
        have += x.shape[0]
    return np.ascontiguousarray(np.concatenate(out, axis=0)[:M])


def random_caps(n: int, rmin_deg: float, rmax_deg: float, rng: np.random.Generator) -> list:
    cen = uniform_s2(n, rng)
    rad = np.deg2rad(rng.uniform(rmin_deg, rmax_deg, n))
    return [(cen[i], float(rad[i])) for i in range(n)]


# --------------------------------------------------------------------- S2 values
def _legendre_series(t: np.ndarray, coef: np.ndarray) -> np.ndarray:
    """sum_n coef[n] P_n(t) by the Clenshaw recurrence (textbook Legendre)."""
    L = coef.shape[0] - 1
    b1 = np.zeros_like(t)
    b2 = np.zeros_like(t)
    for n in range(L, -1, -1):
        # alpha_n(t) = (2n+1)/(n+1) t, beta_{n+1} = -(n+1)/(n+2)
        a = (2.0 * n + 1.0) / (n + 1.0)
        b = -(n + 1.0) / (n + 2.0)
        b0 = coef[n] + a * t * b1 + b * b2
        b2 = b1
        b1 = b0
    return b1


@dataclass
class ZonalField:
    """f(x) = sum_c sum_{n<=L} a_{c,n} P_n(x . mu_c) (+ optional smooth term),
    a band-limited field of degree <= L on S2.  Per-degree amplitudes decay
    like 1/(1+n)^2, the spectral shape the workloads ask for."""

    L: int
    mus: np.ndarray
    coef: np.ndarray  # (C, L+1)
    bump: float = 0.0  # weight of exp(-|x-x0|^2/0.1), not band-limited
    x0: np.ndarray = field(default_factory=lambda: np.ones(3) / math.sqrt(3.0))

    def __call__(self, x: np.ndarray) -> np.ndarray:
        x = np.asarray(x, dtype=np.float64)
        out = np.zeros(x.shape[0])
        chunk = 1 << 16
        for s in range(0, x.shape[0], chunk):
            xs = x[s : s + chunk]
            acc = np.zeros(xs.shape[0])
            for c in range(self.mus.shape[0]):
                acc += _legendre_series(np.clip(xs @ self.mus[c], -1.0, 1.0), self.coef[c])
            if self.bump:
                d2 = np.sum((xs - self.x0[None, :]) ** 2, axis=1)
                acc += self.bump * np.exp(-d2 / 0.1)
            out[s : s + chunk] = acc
        return out


def zonal_field(L: int, rng: np.random.Generator, n_centres: int = 6, bump: float = 0.0) -> ZonalField:
    mus = uniform_s2(n_centres, rng)
    n = np.arange(L + 1)
    amp = np.sqrt((2 * n + 1) / (4 * math.pi)) / (1.0 + n) ** 2 / math.sqrt(n_centres)
    coef = rng.standard_normal((n_centres, L + 1)) * amp[None, :]
    return ZonalField(L=L, mus=mus, coef=coef, bump=bump)


# --------------------------------------------------------------------- SO(3)
def haar_quaternions(M: int, rng: np.random.Generator) -> np.ndarray:
    q = rng.standard_normal((M, 4))
    return q / np.linalg.norm(q, axis=1, keepdims=True)


def _qmul(a: np.ndarray, b: np.ndarray) -> np.ndarray:
    w1, x1, y1, z1 = a[..., 0], a[..., 1], a[..., 2], a[..., 3]
    w2, x2, y2, z2 = b[..., 0], b[..., 1], b[..., 2], b[..., 3]
    return np.stack(
        [
            w1 * w2 - x1 * x2 - y1 * y2 - z1 * z2,
            w1 * x2 + x1 * w2 + y1 * z2 - z1 * y2,
            w1 * y2 - x1 * z2 + y1 * w2 + z1 * x2,
            w1 * z2 + x1 * y2 - y1 * x2 + z1 * w2,
        ],
        axis=-1,
    )


def clustered_rotations(M: int, rng: np.random.Generator, n_clusters: int = 4, sigma: float = 0.15,
                        frac_haar: float = 0.5) -> np.ndarray:
    """frac_haar Haar-uniform rotations plus clusters q_c exp(sigma xi),
    xi ~ N(0, I_3) (rotation vector), as unit quaternions (w, x, y, z)."""
    n_h = int(round(frac_haar * M))
    out = [haar_quaternions(n_h, rng)]
    cen = haar_quaternions(n_clusters, rng)
    which = rng.integers(0, n_clusters, M - n_h)
    v = sigma * rng.standard_normal((M - n_h, 3))
    ang = np.linalg.norm(v, axis=1)
    ax = v / np.maximum(ang, 1e-300)[:, None]
    dq = np.concatenate([np.cos(ang / 2)[:, None], np.sin(ang / 2)[:, None] * ax], axis=1)
    out.append(_qmul(cen[which], dq))
    q = np.concatenate(out, axis=0)
    q = q[rng.permutation(M)]
    return np.ascontiguousarray(q / np.linalg.norm(q, axis=1, keepdims=True))


@dataclass
class ClassField:
    """f(R) = sum_c sum_{n<=L} a_{c,n} chi_n(angle(R_c^{-1} R)) with the
    characters chi_n(w) = sin((2n+1)w/2)/sin(w/2): band-limited of degree <= L
    on SO(3)."""

    L: int
    cen: np.ndarray
    coef: np.ndarray

    def __call__(self, q: np.ndarray) -> np.ndarray:
        out = np.zeros(q.shape[0])
        for c in range(self.cen.shape[0]):
            t = np.clip(np.abs(q @ self.cen[c]), -1.0, 1.0)  # cos(w/2)
            # chi_n = U_{2n}(cos(w/2)), Chebyshev of the second kind
            u_prev = np.ones_like(t)  # U_0
            u = 2.0 * t  # U_1
            acc = self.coef[c, 0] * u_prev
            for k in range(2, 2 * self.L + 1):
                u_prev, u = u, 2.0 * t * u - u_prev
                if k % 2 == 0:
                    acc += self.coef[c, k // 2] * u
            out += acc
        return out


def class_field(L: int, rng: np.random.Generator, n_centres: int = 4) -> ClassField:
    n = np.arange(L + 1)
    coef = rng.standard_normal((n_centres, L + 1)) / (1.0 + n) ** 2 / n_centres
    return ClassField(L=L, cen=haar_quaternions(n_centres, rng), coef=coef)


# --------------------------------------------------------------------- T3
def clustered_torus(M: int, rng: np.random.Generator, n_clusters: int = 8, sigma: float = 0.05,
                    frac_uniform: float = 0.2, n_balls: int = 6, ball_r: float = 0.08) -> np.ndarray:
    """Periodic Gaussian clusters plus uniform points in [0,1)^3 with balls
    removed (min-image distance) by rejection until exactly M remain."""
    cen = rng.random((n_clusters, 3))
    balls = rng.random((n_balls, 3))
    out, have = [], 0
    while have < M:
        B = max(1024, int(1.3 * (M - have)))
        n_u = rng.binomial(B, frac_uniform)
        x_u = rng.random((n_u, 3))
        which = rng.integers(0, n_clusters, B - n_u)
        x_c = cen[which] + sigma * rng.standard_normal((B - n_u, 3))
        x = np.concatenate([x_u, x_c], axis=0) % 1.0
        keep = np.ones(x.shape[0], dtype=bool)
        for b in balls:
            d = x - b[None, :]
            d -= np.rint(d)
            keep &= np.sum(d * d, axis=1) >= ball_r * ball_r
        x = x[keep]
        out.append(x)
        have += x.shape[0]
    x = np.concatenate(out, axis=0)[:M]
    return np.ascontiguousarray(x[rng.permutation(M)])


@dataclass
class TorusField:
    """Sum of C products of real 1-D trigonometric polynomials with |k| < kmax:
    band-limited on T3 (inside [-kmax, kmax)^3), amplitude ~ 1/(1+|k|)^2 per
    axis."""

    kmax: int
    coef: np.ndarray  # (C, 3, 2*kmax-1, 2) complex as re/im

    def __call__(self, x: np.ndarray) -> np.ndarray:
        ks = np.arange(-self.kmax + 1, self.kmax)
        out = np.zeros(x.shape[0])
        chunk = 1 << 15
        for s in range(0, x.shape[0], chunk):
            xs = x[s : s + chunk]
            prod = np.ones((xs.shape[0], self.coef.shape[0]))
            for d in range(3):
                ph = 2.0 * math.pi * np.outer(xs[:, d], ks)
                # all terms of one axis share the trigonometric table
                prod *= np.cos(ph) @ self.coef[:, d, :, 0].T - np.sin(ph) @ self.coef[:, d, :, 1].T
            out[s : s + chunk] = prod.sum(axis=1)
        return out


def torus_field(kmax: int, rng: np.random.Generator, n_terms: int = 3) -> TorusField:
    ks = np.arange(-kmax + 1, kmax)
    amp = 1.0 / (1.0 + np.abs(ks)) ** 2
    coef = rng.standard_normal((n_terms, 3, 2 * kmax - 1, 2)) * amp[None, None, :, None]
    return TorusField(kmax=kmax, coef=coef)


# --------------------------------------------------------------------- configs
@dataclass
class Workload:
    name: str
    domain: str  # "s2" | "so3" | "t3"
    nodes: np.ndarray
    values: np.ndarray  # (F, M)
    params: dict
    truth: object = None


def s2_uniform_small(seed: int = 1000, M: int = 2000, N: int = 16, K: int = 2) -> Workload:
    """M nodes iid uniform on S2, band-limited field of degree <= 16 with
    N(0,1)/(1+n)^2 amplitudes plus iid noise of variance 1e-6; fixed support
    radius of three mean spacings, fixed ridge tau = 1e-8."""
    rng = np.random.default_rng(seed)
    x = uniform_s2(M, rng)
    f = zonal_field(16, rng)
    y = f(x) + 1e-3 * rng.standard_normal(M)
    h = math.sqrt(4 * math.pi / M)
    params = dict(domain="s2", bandwidth=N, degree=K, support_radius=3.0 * h, knn_count=0,
                  knn_eps=0.0, reg="fixed", tau_fixed=1e-8)
    return Workload("s2-uniform-M2000-N16-K2", "s2", x, y[None, :], params, truth=f)


def s2_clusters(seed: int = 2000, M: int = 200_000, N: int = 128, K: int = 3, n_caps: int = 5,
                cap_deg: tuple = (20.0, 20.0), field_degree: int = 160, knn: int | None = None,
                n_centres: int = 6) -> Workload:
    """Mixture of 8 von Mises-Fisher clusters (kappa = 20) plus 20 % uniform
    nodes with spherical-cap holes removed; field band-limited (degree <=
    field_degree) plus the smooth term exp(-|x-x0|^2/0.1)."""
    rng = np.random.default_rng(seed)
    caps = random_caps(n_caps, cap_deg[0], cap_deg[1], rng)
    x = cluster_hole_s2(M, rng, caps=caps)
    f = zonal_field(field_degree, rng, n_centres=n_centres, bump=1.0)
    y = f(x)
    m = (K + 1) * (K + 2) // 2
    params = dict(domain="s2", bandwidth=N, degree=K, support_radius=0.0,
                  knn_count=knn if knn is not None else 4 * m, knn_eps=0.05, reg="chi",
                  chi_target=10.0, chi_full=20.0)
    return Workload(f"s2-clusters-M{M}-N{N}-K{K}", "s2", x, y[None, :], params, truth=f)


def s2_clusters_fixed(seed: int = 2000, M: int = 200_000, N: int = 128, K: int = 3,
                      delta0: float = 0.1) -> Workload:
    """The S2 cluster + hole nodes under a fixed support radius delta0 (rad):
    no node in the holes, ~100 in the uniform part, ~2000 at the cluster
    modes -- the skewed neighbour counts of ill-distributed data."""
    wl = s2_clusters(seed=seed, M=M, N=N, K=K)
    wl.params = dict(wl.params, support_radius=float(delta0), knn_count=0)
    wl.name = f"s2-clusters-fixed{delta0:g}-M{M}-N{N}-K{K}"
    return wl


def s2_clusters_hybrid(seed: int = 2000, M: int = 200_000, N: int = 128, K: int = 3,
                       delta0: float = 0.16) -> Workload:
    """The S2 cluster + hole nodes under the hybrid radius max(delta0, (1 +
    eps) d_n) (both rules of eq. (12) and the fixed radius set, n = 4m): the
    fixed radius holds ~250 nodes in the uniform part and up to ~5000 at the
    cluster modes, while the adaptive one reaches across the holes."""
    wl = s2_clusters(seed=seed, M=M, N=N, K=K)
    wl.params = dict(wl.params, support_radius=float(delta0))
    wl.name = f"s2-clusters-hybrid{delta0:g}-M{M}-N{N}-K{K}"
    return wl


def s2_clusters_smooth(seed: int = 2000, M: int = 200_000, N: int = 128, K: int = 3,
                       smooth_aux: int = 65536) -> Workload:
    """The S2 cluster + hole workload with the smoothed adaptive radius: d_n
    on a Fibonacci grid of smooth_aux points, degree-zero MLS at the grid."""
    wl = s2_clusters(seed=seed, M=M, N=N, K=K)
    wl.params = dict(wl.params, smooth_aux=int(smooth_aux))
    wl.name = f"s2-clusters-smooth{smooth_aux}-M{M}-N{N}-K{K}"
    return wl


def s2_large(seed: int = 3000, M: int = 4_000_000, N: int = 512, K: int = 4) -> Workload:
    """The large S2 case: the cluster + hole generator with 12 caps of radius
    10-25 degrees, field band-limited to degree 640 plus the smooth bump,
    N = 512 (grid 513 x 1026), K = 4 (m = 15), kNN n = 60."""
    return s2_clusters(seed=seed, M=M, N=N, K=K, n_caps=12, cap_deg=(10.0, 25.0), field_degree=640,
                       knn=60)


def so3_clusters(seed: int = 5000, M: int = 1_000_000, N: int = 64, K: int = 2,
                 grid: tuple = (130, 130, 130), field_degree: int = 64) -> Workload:
    rng = np.random.default_rng(seed)
    q = clustered_rotations(M, rng)
    f = class_field(field_degree, rng)
    m = (K + 1) * (K + 2) * (K + 3) // 6
    params = dict(domain="so3", bandwidth=N, degree=K, support_radius=0.0, knn_count=4 * m,
                  knn_eps=0.05, reg="chi", chi_target=10.0, chi_full=20.0, grid_shape=grid)
    return Workload(f"so3-clusters-M{M}-N{N}-K{K}", "so3", q, f(q)[None, :], params, truth=f)


def t3_clusters(seed: int = 5100, M: int = 2_000_000, N: int = 64, K: int = 3,
                grid: int = 128, kmax: int = 64) -> Workload:
    rng = np.random.default_rng(seed)
    x = clustered_torus(M, rng)
    f = torus_field(kmax, rng)
    m = (K + 1) * (K + 2) * (K + 3) // 6
    params = dict(domain="t3", bandwidth=N, degree=K, support_radius=0.0, knn_count=4 * m,
                  knn_eps=0.05, reg="chi", chi_target=10.0, chi_full=20.0,
                  grid_shape=(grid, grid, grid))
    return Workload(f"t3-clusters-M{M}-N{N}-K{K}", "t3", x, f(x)[None, :], params, truth=f)


# ------------------------------------------------------------------- serving
@dataclass
class ServingTrace:
    """Requests of the serving workload: arrival times (s, Poisson process),
    per-request bandwidth N, degree K and node count M, and the node pool each
    request takes its first M nodes from (pools are cluster + hole node sets
    in random order, so every prefix is a sample of the same distribution)."""
    arrival: np.ndarray
    N: np.ndarray
    K: np.ndarray
    M: np.ndarray
    pool: np.ndarray
    pools: list  # node arrays (Mmax x 3)
    fields: list  # values on each pool (Mmax,)


def serving_trace(n: int = 512, rate: float = 200.0, seed: int = 7000, Ns=(32, 64, 128, 256),
                  Ks=(2, 3, 4), M_range=(1e4, 1e6), n_pools: int = 4) -> ServingTrace:
    """n requests arriving at `rate` per second; N uniform over Ns, K uniform
    over Ks, M log-uniform over M_range, nodes from the cluster + hole
    generator (8 vMF clusters, kappa = 20, 20 % uniform, 5 caps of 20 deg)."""
    rng = np.random.default_rng(seed)
    arrival = np.cumsum(rng.exponential(1.0 / rate, size=n))
    arrival -= arrival[0]
    N = rng.choice(np.asarray(Ns), size=n)
    K = rng.choice(np.asarray(Ks), size=n)
    lo, hi = np.log(M_range[0]), np.log(M_range[1])
    M = np.exp(rng.uniform(lo, hi, size=n)).astype(np.int64)
    pool = rng.integers(0, n_pools, size=n)
    Mmax = int(M.max())
    pools, fields = [], []
    for k in range(n_pools):
        prng = np.random.default_rng(seed + 1 + k)
        caps = random_caps(5, 20.0, 20.0, prng)
        x = cluster_hole_s2(Mmax, prng, caps=caps)
        x = x[prng.permutation(Mmax)]
        f = zonal_field(64, prng, n_centres=6, bump=1.0)
        pools.append(np.ascontiguousarray(x))
        fields.append(f(x))
    return ServingTrace(arrival, N, K, M, pool, pools, fields)


def serving_params(N: int, K: int) -> dict:
    """Parameters of one serving request: kNN radius n = 4m, eps = 0.05,
    chi-target regularization (chi_T = 10, chi_full = 20)."""
    m = (K + 1) * (K + 2) // 2
    return dict(domain="s2", bandwidth=int(N), degree=int(K), support_radius=0.0, knn_count=4 * m,
                knn_eps=0.05, reg="chi", chi_target=10.0, chi_full=20.0)
