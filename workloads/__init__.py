"""Seeded synthetic inputs shared by the HIP path, the oracle and the tests.

This module only *generates inputs*: boundary geometry, boundary-data and source
coefficients, evaluation-point candidates, and the closed-form solutions the
problems were manufactured from.  It holds none of the method's arithmetic (no
closest-point query, no walk, no Green's function, no boundary-integral sum), so
that the oracle and the HIP library can both consume it without sharing code.

The paper ships no assets; every scene here is a synthetic stand-in whose shape
follows the workloads of the paper's evaluation (2D polygons and 3D triangle
meshes with a Dirichlet boundary, optional Gaussian source term, dense grids of
evaluation points).  Seeds follow ``seed(k, p) = 1000*k + p`` with p = 1 geometry,
2 data coefficients, 3 cache sampling, 4 walks, 5 evaluation points, 6 sources,
7 observation noise.

Field kinds (the numeric values are an interface shared with the C headers):

=====  ===================  =====================================================
kind   name                 value at x
=====  ===================  =====================================================
0      ZERO                 0
1      CONST                param[0]
2      HARMONIC_2D          param[1]*Re((x+iy)^k) + param[2]*exp(x)cos(y), k=param[0]
3      GAUSS_SUM            sum_k A_k exp(-|x-c_k|^2/(2 s^2)), s=param[0];
                            coef = [A_0, c_0 (dim values), A_1, c_1, ...]
4      GAUSS_POTENTIAL_2D   sum_k A_k s^2/2 Ein(|x-c_k|^2/(2 s^2)) + HARMONIC_2D
                            part with (k, alpha, beta) = param[1:4]; s=param[0]
5      SOLID_HARMONICS_3D   sum_{l<=L, |m|<=l} coef[l*l+l+m] r^l Y_lm(x/r)
                            (orthonormal real spherical harmonics, no
                            Condon-Shortley phase), L = param[0]
6      FOURIER_2D           sum_m coef[m] phi_m(theta), theta=atan2(y-cy, x-cx),
                            (cx, cy) = param[0:2]; phi_0=1, phi_{2j-1}=cos(j theta),
                            phi_{2j}=sin(j theta), last basis cos(J theta) when the
                            count is even
7      POINT_SOURCE         2D: A ln|x-x0|; 3D: A/|x-x0|; A=param[0], x0=param[1:]
8      EXP_PLANE            A exp(a.x), A=param[0], a=param[1:1+dim]; solves
                            Lap u = |a|^2 u (screened Poisson, Eq. 1 with f = 0)
9      WEDGE_2D             A r^p cos(p phi), polar (r, phi in [0, 2 pi)) about
                            (param[2], param[3]); A=param[0], p=param[1]
=====  ===================  =====================================================
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Optional

import numpy as np

FIELD_ZERO = 0
FIELD_CONST = 1
FIELD_HARMONIC_2D = 2
FIELD_GAUSS_SUM = 3
FIELD_GAUSS_POTENTIAL_2D = 4
FIELD_SOLID_HARMONICS_3D = 5
FIELD_FOURIER_2D = 6
FIELD_POINT_SOURCE = 7
FIELD_EXP_PLANE = 8
FIELD_WEDGE_2D = 9
FIELD_QUADRATIC = 10


def seed(k: int, p: int) -> int:
    """Seed convention: config k, purpose p."""
    return 1000 * k + p


# --------------------------------------------------------------------------
# Field descriptors
# --------------------------------------------------------------------------
@dataclass
class Field:
    kind: int = FIELD_ZERO
    coef: np.ndarray = field(default_factory=lambda: np.zeros(0))
    param: np.ndarray = field(default_factory=lambda: np.zeros(8))

    def __post_init__(self):
        self.coef = np.ascontiguousarray(np.asarray(self.coef, dtype=np.float64))
        p = np.zeros(8)
        q = np.asarray(self.param, dtype=np.float64).ravel()
        p[: q.size] = q
        self.param = p

    @property
    def is_zero(self) -> bool:
        return self.kind == FIELD_ZERO


def harmonic_2d(k=3, alpha=1.0, beta=1.0) -> Field:
    return Field(FIELD_HARMONIC_2D, np.zeros(0), [k, alpha, beta])


def gauss_sum(amps, centers, sigma) -> Field:
    amps = np.asarray(amps, float)
    centers = np.asarray(centers, float)
    coef = np.concatenate([amps[:, None], centers], axis=1).ravel()
    return Field(FIELD_GAUSS_SUM, coef, [sigma])


def gauss_potential_2d(amps, centers, sigma, k=3, alpha=1.0, beta=1.0) -> Field:
    amps = np.asarray(amps, float)
    centers = np.asarray(centers, float)
    coef = np.concatenate([amps[:, None], centers], axis=1).ravel()
    return Field(FIELD_GAUSS_POTENTIAL_2D, coef, [sigma, k, alpha, beta])


def solid_harmonics_3d(coef, lmax) -> Field:
    coef = np.asarray(coef, float)
    assert coef.size == (lmax + 1) ** 2
    return Field(FIELD_SOLID_HARMONICS_3D, coef, [lmax])


def fourier_2d(coef, center=(0.0, 0.0)) -> Field:
    return Field(FIELD_FOURIER_2D, np.asarray(coef, float), [center[0], center[1]])


def point_source(amp, x0) -> Field:
    return Field(FIELD_POINT_SOURCE, np.zeros(0), [amp, *x0])


def exp_plane(amp, a) -> Field:
    return Field(FIELD_EXP_PLANE, np.zeros(0), [amp, *a])


def quadratic(A: float, B: float = 0.0, center=(0.0, 0.0, 0.0)) -> Field:
    """A |x - center|^2 + B (Lap = 2 dim A)."""
    return Field(FIELD_QUADRATIC, np.zeros(0), [A, B, *center])


def wedge_2d(amp, p, center=(0.0, 0.0)) -> Field:
    return Field(FIELD_WEDGE_2D, np.zeros(0), [amp, p, center[0], center[1]])


# --------------------------------------------------------------------------
# Closed forms used as ground truth (not the method)
# --------------------------------------------------------------------------
def ein(z):
    """Ein(z) = int_0^z (1 - e^-t)/t dt = E1(z) + ln z + gamma (z > 0)."""
    from scipy.special import exp1

    z = np.asarray(z, float)
    out = np.empty_like(z)
    small = z < 0.5
    zs = z[small]
    # power series sum_{k>=1} (-1)^{k+1} z^k / (k k!) for small arguments
    acc = np.zeros_like(zs)
    fact = 1.0
    for k in range(1, 40):
        fact *= k
        acc += (-1) ** (k + 1) * zs**k / (k * fact)
    out[small] = acc
    zl = z[~small]
    out[~small] = exp1(zl) + np.log(zl) + np.euler_gamma
    return out


def real_sph_harm(lmax: int, dirs: np.ndarray) -> np.ndarray:
    """Orthonormal real spherical harmonics, no Condon-Shortley phase.

    Returns (n, (lmax+1)^2) with column l*l+l+m.
    """
    from scipy.special import sph_harm_y

    dirs = np.asarray(dirs, float)
    r = np.linalg.norm(dirs, axis=1)
    theta = np.arccos(np.clip(dirs[:, 2] / np.where(r > 0, r, 1), -1, 1))
    phi = np.arctan2(dirs[:, 1], dirs[:, 0])
    out = np.zeros((dirs.shape[0], (lmax + 1) ** 2))
    for l in range(lmax + 1):
        for m in range(-l, l + 1):
            am = abs(m)
            y = sph_harm_y(l, am, theta, phi)  # includes (-1)^m
            y = y * (-1) ** am  # drop Condon-Shortley phase
            if m == 0:
                v = y.real
            elif m > 0:
                v = math.sqrt(2.0) * y.real
            else:
                v = math.sqrt(2.0) * y.imag
            out[:, l * l + l + m] = v
    return out


def field_value(fld: Field, x: np.ndarray) -> np.ndarray:
    """Closed-form value of a field descriptor at points x (n, dim)."""
    x = np.asarray(x, float)
    k = fld.kind
    p = fld.param
    if k == FIELD_ZERO:
        return np.zeros(x.shape[0])
    if k == FIELD_CONST:
        return np.full(x.shape[0], p[0])
    if k == FIELD_HARMONIC_2D:
        z = x[:, 0] + 1j * x[:, 1]
        return p[1] * (z ** int(p[0])).real + p[2] * np.exp(x[:, 0]) * np.cos(x[:, 1])
    if k == FIELD_GAUSS_SUM:
        d = x.shape[1]
        c = fld.coef.reshape(-1, 1 + d)
        s = p[0]
        r2 = ((x[:, None, :] - c[None, :, 1:]) ** 2).sum(-1)
        return (c[None, :, 0] * np.exp(-r2 / (2 * s * s))).sum(1)
    if k == FIELD_GAUSS_POTENTIAL_2D:
        c = fld.coef.reshape(-1, 3)
        s = p[0]
        r2 = ((x[:, None, :] - c[None, :, 1:]) ** 2).sum(-1)
        v = (c[None, :, 0] * s * s / 2 * ein(r2 / (2 * s * s))).sum(1)
        return v + field_value(harmonic_2d(p[1], p[2], p[3]), x)
    if k == FIELD_SOLID_HARMONICS_3D:
        lmax = int(p[0])
        r = np.linalg.norm(x, axis=1)
        Y = real_sph_harm(lmax, x)
        ls = np.array([l for l in range(lmax + 1) for _ in range(2 * l + 1)])
        return (Y * r[:, None] ** ls[None, :]) @ fld.coef
    if k == FIELD_FOURIER_2D:
        th = np.arctan2(x[:, 1] - p[1], x[:, 0] - p[0])
        return fourier_basis(th, fld.coef.size) @ fld.coef
    if k == FIELD_POINT_SOURCE:
        d = x.shape[1]
        r = np.linalg.norm(x - p[1 : 1 + d][None, :], axis=1)
        return p[0] * (np.log(r) if d == 2 else 1.0 / r)
    if k == FIELD_EXP_PLANE:
        d = x.shape[1]
        return p[0] * np.exp(x @ p[1 : 1 + d])
    if k == FIELD_QUADRATIC:
        d = x.shape[1]
        return p[0] * ((x - np.asarray(p[2 : 2 + d])[None, :]) ** 2).sum(1) + p[1]
    if k == FIELD_WEDGE_2D:
        dx, dy = x[:, 0] - p[2], x[:, 1] - p[3]
        phi = np.mod(np.arctan2(dy, dx), 2 * np.pi)
        return p[0] * np.hypot(dx, dy) ** p[1] * np.cos(p[1] * phi)
    raise ValueError(f"unknown field kind {k}")


def fourier_basis(theta: np.ndarray, n: int) -> np.ndarray:
    out = np.zeros((theta.size, n))
    out[:, 0] = 1.0
    for b in range(1, n):
        j = (b + 1) // 2
        out[:, b] = np.cos(j * theta) if b % 2 == 1 else np.sin(j * theta)
    return out


def field_grad_fd(fld: Field, x: np.ndarray, h=1e-5) -> np.ndarray:
    """Central finite-difference gradient of a closed form (used for truths)."""
    x = np.asarray(x, float)
    g = np.zeros_like(x)
    for a in range(x.shape[1]):
        e = np.zeros(x.shape[1])
        e[a] = h
        g[:, a] = (field_value(fld, x + e) - field_value(fld, x - e)) / (2 * h)
    return g


# --------------------------------------------------------------------------
# Geometry
# --------------------------------------------------------------------------
@dataclass
class Scene:
    dim: int
    verts: np.ndarray  # (nv, dim) float64
    prims: np.ndarray  # (np, dim) int32, CCW polylines / outward triangles
    name: str = ""

    def __post_init__(self):
        self.verts = np.ascontiguousarray(self.verts, dtype=np.float64)
        self.prims = np.ascontiguousarray(self.prims, dtype=np.int32)

    @property
    def bbox(self):
        return self.verts.min(0), self.verts.max(0)

    @property
    def diagonal(self) -> float:
        lo, hi = self.bbox
        return float(np.linalg.norm(hi - lo))


def circle_polygon(n: int = 128, radius: float = 1.0) -> Scene:
    th = 2 * np.pi * np.arange(n) / n
    v = radius * np.stack([np.cos(th), np.sin(th)], 1)
    p = np.stack([np.arange(n), (np.arange(n) + 1) % n], 1)
    return Scene(2, v, p, f"circle{n}")


def star_polygon(n: int = 4096, rng_seed: int = seed(2, 1), jitter: str = "isotropic",
                 sigma: float = 0.02, amp: float = 0.2, lobes: int = 7) -> Scene:
    """Star polygon r = 1 + amp*sin(lobes*theta) with Gaussian vertex jitter.

    ``isotropic`` jitters (x, y) independently (self-intersecting for the default
    sizes); ``radial`` jitters the radius only (a simple polygon).
    """
    rng = np.random.default_rng(rng_seed)
    th = 2 * np.pi * np.arange(n) / n
    r = 1 + amp * np.sin(lobes * th)
    if jitter == "radial":
        r = r + rng.normal(0, sigma, n)
        v = np.stack([r * np.cos(th), r * np.sin(th)], 1)
    elif jitter == "isotropic":
        v = np.stack([r * np.cos(th), r * np.sin(th)], 1) + rng.normal(0, sigma, (n, 2))
    elif jitter == "none":
        v = np.stack([r * np.cos(th), r * np.sin(th)], 1)
    else:
        raise ValueError(jitter)
    p = np.stack([np.arange(n), (np.arange(n) + 1) % n], 1)
    return Scene(2, v, p, f"star{n}-{jitter}")


def icosphere(level: int) -> Scene:
    t = (1 + 5**0.5) / 2
    v = np.array([[-1, t, 0], [1, t, 0], [-1, -t, 0], [1, -t, 0], [0, -1, t], [0, 1, t],
                  [0, -1, -t], [0, 1, -t], [t, 0, -1], [t, 0, 1], [-t, 0, -1], [-t, 0, 1]], float)
    f = np.array([[0, 11, 5], [0, 5, 1], [0, 1, 7], [0, 7, 10], [0, 10, 11], [1, 5, 9],
                  [5, 11, 4], [11, 10, 2], [10, 7, 6], [7, 1, 8], [3, 9, 4], [3, 4, 2],
                  [3, 2, 6], [3, 6, 8], [3, 8, 9], [4, 9, 5], [2, 4, 11], [6, 2, 10],
                  [8, 6, 7], [9, 8, 1]], np.int64)
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    for _ in range(level):
        e = np.concatenate([f[:, [0, 1]], f[:, [1, 2]], f[:, [2, 0]]], 0)
        key = np.sort(e, 1)
        uniq, inv = np.unique(key[:, 0] * (1 << 32) + key[:, 1], return_inverse=True)
        a = (uniq >> 32).astype(np.int64)
        b = (uniq & 0xFFFFFFFF).astype(np.int64)
        mid = v[a] + v[b]
        mid /= np.linalg.norm(mid, axis=1, keepdims=True)
        base = v.shape[0]
        v = np.concatenate([v, mid], 0)
        nf = f.shape[0]
        m01 = base + inv[:nf]
        m12 = base + inv[nf:2 * nf]
        m20 = base + inv[2 * nf:]
        f = np.concatenate([
            np.stack([f[:, 0], m01, m20], 1),
            np.stack([f[:, 1], m12, m01], 1),
            np.stack([f[:, 2], m20, m12], 1),
            np.stack([m01, m12, m20], 1)], 0)
    # orient outward (right-hand rule)
    a, b, c = v[f[:, 0]], v[f[:, 1]], v[f[:, 2]]
    nrm = np.cross(b - a, c - a)
    flip = (nrm * (a + b + c)).sum(1) < 0
    f[flip] = f[flip][:, [0, 2, 1]]
    return Scene(3, v, f.astype(np.int32), f"icosphere{level}")


def displaced_icosphere(level: int = 6, rng_seed: int = seed(3, 1), amp: float = 0.05,
                        lmax: int = 8, noise: str = "sh") -> Scene:
    """Icosphere radially displaced by r = 1 + amp*xi(v), max|xi| = 1.

    ``sh``: xi is a real spherical-harmonic series (degree <= lmax, N(0,1)
    coefficients).  ``iid``: xi ~ U(-1, 1) per vertex (stress variant).
    """
    s = icosphere(level)
    rng = np.random.default_rng(rng_seed)
    if noise == "sh":
        c = rng.normal(0, 1, (lmax + 1) ** 2)
        c[0] = 0.0
        xi = real_sph_harm(lmax, s.verts) @ c
        xi /= np.abs(xi).max()
    elif noise == "iid":
        xi = rng.uniform(-1, 1, s.verts.shape[0])
    else:
        raise ValueError(noise)
    v = s.verts * (1 + amp * xi)[:, None]
    return Scene(3, v, s.prims, f"dispsphere{level}")


def grid2d(n: int, lo, hi) -> np.ndarray:
    """Cell-centred n x n grid over the box [lo, hi] (row-major, y outer)."""
    lo = np.asarray(lo, float)
    hi = np.asarray(hi, float)
    xs = lo[0] + (np.arange(n) + 0.5) * (hi[0] - lo[0]) / n
    ys = lo[1] + (np.arange(n) + 0.5) * (hi[1] - lo[1]) / n
    X, Y = np.meshgrid(xs, ys)
    return np.stack([X.ravel(), Y.ravel()], 1)


def uniform_box(n: int, lo, hi, rng_seed: int) -> np.ndarray:
    rng = np.random.default_rng(rng_seed)
    lo = np.asarray(lo, float)
    hi = np.asarray(hi, float)
    return lo + rng.random((n, lo.size)) * (hi - lo)


# --------------------------------------------------------------------------
# Problem configurations
# --------------------------------------------------------------------------
@dataclass
class Problem:
    name: str
    scene: Scene
    g: Field
    f: Field
    n_cache: int           # cache candidates drawn per batch
    n_walks: int           # walks per cache point
    eps: float
    offset: float          # l
    n_sources: int         # source samples (0 when f == 0)
    eval_x: np.ndarray     # evaluation candidates (the method classifies them)
    truth: Field           # closed-form solution u*
    sides: int = 2         # 1: inward offsets only (simple closed boundary), 2: both sides
    precision: str = "f32"
    seed_walks: int = 0
    seed_cache: int = 0
    seed_sources: int = 0
    extra: dict = field(default_factory=dict)
    sigma: float = 0.0     # screening coefficient of Lap u - sigma u = f (Eq. 1)
    side_read: bool = False      # side rule of double-sided data (Appendix B)
    junction_drop: float = 0.0   # mixed cache: drop offset points within this * l of the Neumann part


def _harm_c1() -> Field:
    return harmonic_2d(3, 1.0, 1.0)


def problem_c1() -> Problem:
    """Unit-circle 128-gon, Laplace, g = Re(z^3) + e^x cos y, FP64."""
    sc = circle_polygon(128)
    g = _harm_c1()
    return Problem("c1_circle128_laplace", sc, g, Field(), 1024, 64, 1e-3, 1e-3, 0,
                   grid2d(64, (-1, -1), (1, 1)), g, sides=1, precision="f64",
                   seed_walks=seed(1, 4), seed_cache=seed(1, 3), seed_sources=seed(1, 6))


def _c2_source(k: int = 2, n_gauss: int = 8, sigma: float = 0.05):
    rng = np.random.default_rng(seed(k, 2))
    amps = rng.normal(0, 1, n_gauss)
    rr = 0.6 * np.sqrt(rng.random(n_gauss))
    tt = 2 * np.pi * rng.random(n_gauss)
    centers = np.stack([rr * np.cos(tt), rr * np.sin(tt)], 1)
    return amps, centers, sigma


def problem_c2(grid: int = 1024, jitter: str = "isotropic") -> Problem:
    """Jagged star (4096 segments), Poisson with 8 Gaussians, manufactured g."""
    sc = star_polygon(4096, seed(2, 1), jitter=jitter)
    amps, centers, sigma = _c2_source()
    f = gauss_sum(amps, centers, sigma)
    g = gauss_potential_2d(amps, centers, sigma, 3, 1.0, 1.0)
    eps = 1e-3 * sc.diagonal
    lo, hi = sc.bbox
    return Problem("c2_star4096_poisson", sc, g, f, 16384, 256, eps, 5 * eps, 16384,
                   grid2d(grid, lo, hi), g, sides=2, precision="f32",
                   seed_walks=seed(2, 4), seed_cache=seed(2, 3), seed_sources=seed(2, 6))


def slit_disk(n_circle: int = 256, n_slit: int = 64) -> Scene:
    """The unit disk cut along the segment [0, 1] x {0} (a double-sided
    boundary, Appendix B): one counter-clockwise polygon that runs round the
    circle from (1, 0), back along the lower side of the cut to the origin and
    out again along its upper side; the two sides are separate segments on
    the same line, so the cut adds nothing to winding numbers off it."""
    t = 2 * np.pi * np.arange(n_circle) / n_circle
    circle = np.stack([np.cos(t), np.sin(t)], 1)  # from (1, 0) round to just below it
    back = np.stack([1 - np.arange(0, n_slit + 1) / n_slit, np.zeros(n_slit + 1)], 1)  # (1, 0) to the origin
    out = np.stack([np.arange(1, n_slit) / n_slit, np.zeros(n_slit - 1)], 1)  # out again, closing at (1, 0)
    V = np.concatenate([circle, back, out])
    m = V.shape[0]
    P = np.array([[i, (i + 1) % m] for i in range(m)], dtype=np.int32)
    return Scene(2, V, P, f"slit_disk{n_circle}_{n_slit}")


def slit_field() -> Field:
    """u = r^(1/2) cos(phi/2), phi in [0, 2 pi): harmonic in the slit disk,
    sqrt(r) on the upper side of the cut and -sqrt(r) on the lower one."""
    return wedge_2d(1.0, 0.5)


def slit_disk_neumann(n_circle: int = 256, n_slit: int = 64):
    """The cut disk of slit_disk with a Neumann cut (both sides reflecting,
    Appendix B) and a Dirichlet circle: (whole boundary, Dirichlet segments,
    Neumann segments), each part with only the vertices it uses.  The field
    of slit_field has zero flux through both sides of the cut."""
    full = slit_disk(n_circle, n_slit)
    P = full.prims
    is_neu = np.arange(P.shape[0]) >= n_circle

    def part(mask, tag):
        Q = P[mask]
        used, inv = np.unique(Q.ravel(), return_inverse=True)
        return Scene(2, full.verts[used], inv.reshape(Q.shape).astype(np.int32), f"{full.name}_{tag}")

    return full, part(~is_neu, "dirichlet"), part(is_neu, "neumann")


def problem_slit_disk(grid: int = 256, n_cache: int = 16384, n_walks: int = 128) -> Problem:
    """Laplace in the slit disk with double-sided Dirichlet data on the cut."""
    sc = slit_disk()
    g = slit_field()
    eps = 1e-3 * sc.diagonal
    lo, hi = sc.bbox
    return Problem("slit_disk_double_sided", sc, g, Field(), n_cache, n_walks, eps, 5 * eps, 0,
                   grid2d(grid, lo, hi), g, sides=1, precision="f32",
                   seed_walks=seed(8, 4), seed_cache=seed(8, 3), seed_sources=seed(8, 6), side_read=True)


def mixed_polygon(verts, neumann, counts, name="mixed"):
    """A CCW polygon whose side i (vertex i to i + 1) is split into counts[i]
    equal segments and is Neumann where neumann[i]: returns the whole
    boundary and its Dirichlet and Neumann segment sets, each with only the
    vertices it uses."""
    V, F = [], []
    n = len(verts)
    for i in range(n):
        a, b = np.asarray(verts[i], float), np.asarray(verts[(i + 1) % n], float)
        for j in range(counts[i]):
            V.append(a + (b - a) * j / counts[i])
            F.append(bool(neumann[i]))
    V = np.array(V)
    m = len(V)
    segs = np.array([[i, (i + 1) % m] for i in range(m)], dtype=np.int32)
    F = np.array(F)

    def part(mask, tag):
        P = segs[mask]
        used, inv = np.unique(P.ravel(), return_inverse=True)
        return Scene(2, V[used], inv.reshape(P.shape).astype(np.int32), f"{name}_{tag}")

    return Scene(2, V, segs, name), part(~F, "dirichlet"), part(F, "neumann")


def mixed_box(lo, hi, neumann, m, name="box"):
    """The box [lo, hi] (3D) with each face split into an m x m grid of
    squares, two triangles each, outward by the right-hand rule; face f in
    (-x, +x, -y, +y, -z, +z) is Neumann where neumann[f].  Returns the whole
    boundary and its Dirichlet and Neumann triangle sets, each with only the
    vertices it uses."""
    lo = np.asarray(lo, float)
    hi = np.asarray(hi, float)
    verts, tris, flags, index = [], [], [], {}

    def vid(p):
        key = tuple(np.round(p, 12))
        if key not in index:
            index[key] = len(verts)
            verts.append(np.asarray(p, float))
        return index[key]

    for f in range(6):
        a, side = f // 2, f % 2       # normal axis, 0 = low face, 1 = high face
        b, c = (a + 1) % 3, (a + 2) % 3  # (b, c, a) is right-handed
        for i in range(m):
            for j in range(m):
                corners = []
                for di, dj in ((0, 0), (1, 0), (1, 1), (0, 1)):
                    p = np.empty(3)
                    p[a] = hi[a] if side else lo[a]
                    p[b] = lo[b] + (hi[b] - lo[b]) * (i + di) / m
                    p[c] = lo[c] + (hi[c] - lo[c]) * (j + dj) / m
                    corners.append(vid(p))
                q0, q1, q2, q3 = corners
                # counter-clockwise in (b, c) has normal +a: reversed on low faces
                for t in ((q0, q1, q2), (q0, q2, q3)):
                    tris.append(t if side else (t[0], t[2], t[1]))
                    flags.append(bool(neumann[f]))
    V = np.array(verts)
    P = np.array(tris, dtype=np.int32)
    F = np.array(flags)

    def part(mask, tag):
        Q = P[mask]
        used, inv = np.unique(Q.ravel(), return_inverse=True)
        return Scene(3, V[used], inv.reshape(Q.shape).astype(np.int32), f"{name}_{tag}")

    return Scene(3, V, P, name), part(~F, "dirichlet"), part(F, "neumann")


def problem_c2_mixed(grid: int = 1024, n_cache: int = 262144, n_walks: int = 256) -> Problem:
    """Channel [0, 6] x [0, pi] (4096 segments): Dirichlet ends, Neumann walls
    (h = 0), Laplace, u = x + 0.5 e^(x - 6) cos y (zero flux through y = 0
    and y = pi)."""
    full, dir_, neu = mixed_polygon([[0, 0], [6, 0], [6, np.pi], [0, np.pi]], [True, False, True, False],
                                    [1536, 512, 1536, 512], "c2_channel4096")
    g = harmonic_2d(1, 1.0, 0.5 * np.exp(-6.0))
    eps = 1e-3 * full.diagonal
    lo, hi = full.bbox
    return Problem("c2_channel4096_mixed", full, g, Field(), n_cache, n_walks, eps, 5 * eps, 0,
                   grid2d(grid, lo, hi), g, sides=1, precision="f32",
                   seed_walks=seed(7, 4), seed_cache=seed(7, 3), seed_sources=seed(7, 6),
                   extra=dict(dirichlet=dir_, neumann=neu), junction_drop=1e-2)


def problem_c3(n_eval_box: int = 2_320_000, slice_n: int = 256, level: int = 6) -> Problem:
    """Displaced icosphere (81,920 triangles), Laplace, solid-harmonic g."""
    sc = displaced_icosphere(level, seed(3, 1))
    rng = np.random.default_rng(seed(3, 2))
    coef = rng.normal(0, 1, 81)
    g = solid_harmonics_3d(coef, 8)
    eps = 1e-3 * sc.diagonal
    lo, hi = sc.bbox
    pts = uniform_box(n_eval_box, lo, hi, seed(3, 5)) if n_eval_box else np.zeros((0, 3))
    sl = grid2d(slice_n, (-1.05, -1.05), (1.05, 1.05)) if slice_n else np.zeros((0, 2))
    sl3 = np.concatenate([sl, np.zeros((sl.shape[0], 1))], 1)
    return Problem("c3_dispsphere_laplace", sc, g, Field(), 65536, 512, eps, 5 * eps, 0,
                   np.concatenate([pts, sl3], 0), g, sides=1, precision="f32",
                   seed_walks=seed(3, 4), seed_cache=seed(3, 3), seed_sources=seed(3, 6),
                   extra={"n_box": n_eval_box, "n_slice": sl3.shape[0]})


def exterior_of(sc: Scene, name: str = "") -> Scene:
    """The open domain outside a closed 3D mesh (Appendix B): the same
    triangles with their orientation reversed, so that normals point into
    the solid (out of the domain) and the pseudonormal inside test selects
    the exterior."""
    return Scene(sc.dim, sc.verts.copy(), sc.prims[:, [0, 2, 1]].copy(), name or sc.name + "_exterior")


def enclosing_sphere(sc: Scene, margin: float = 0.05):
    """Centre and radius of a sphere about the bounding-box centre that holds
    every vertex (hence every triangle) with a relative margin."""
    c = 0.5 * (sc.verts.min(0) + sc.verts.max(0))
    return c, float(np.linalg.norm(sc.verts - c, axis=1).max() * (1 + margin))


def problem_c3_open(n_eval_box: int = 2_320_000, level: int = 6) -> Problem:
    """The exterior of the displaced icosphere of the 3D Laplace workload: an
    open domain (Appendix B) with u -> 0 at infinity, Dirichlet data from the
    decaying potential u = 1/|x - q| of a point q inside the solid (the exact
    solution), evaluation points drawn uniformly in the box [-2, 2]^3 (those
    inside the solid are classified out)."""
    solid = displaced_icosphere(level, seed(3, 1))
    sc = exterior_of(solid, "c3o_dispsphere_exterior")
    g = point_source(1.0, (0.1, -0.05, 0.07))
    eps = 1e-3 * sc.diagonal
    pts = uniform_box(n_eval_box, (-2.0, -2.0, -2.0), (2.0, 2.0, 2.0), seed(3, 11)) if n_eval_box else np.zeros((0, 3))
    c, r = enclosing_sphere(sc)
    return Problem("c3o_dispsphere_exterior", sc, g, Field(), 65536, 512, eps, 5 * eps, 0, pts, g, sides=1,
                   precision="f32", seed_walks=seed(3, 12), seed_cache=seed(3, 13), seed_sources=seed(3, 14),
                   extra={"n_box": n_eval_box, "n_slice": 0, "open_sphere": (c, r)})


def problem_c3_screened(sigma: float = 4.0, n_eval_box: int = 2_320_000) -> Problem:
    """The displaced icosphere of the 3D Laplace workload with the screened
    equation Lap u = sigma u (Eq. 1, f = 0) and the plane wave u = exp(a.x),
    |a|^2 = sigma, as boundary data and closed-form solution."""
    p = problem_c3(n_eval_box=n_eval_box)
    rng = np.random.default_rng(seed(3, 8))
    a = rng.normal(0, 1, 3)
    a *= math.sqrt(sigma) / np.linalg.norm(a)
    g = exp_plane(1.0, a)
    return Problem("c3s_dispsphere_screened", p.scene, g, Field(), p.n_cache, p.n_walks, p.eps, p.offset, 0,
                   p.eval_x, g, sides=1, precision="f32", seed_walks=seed(3, 9), seed_cache=p.seed_cache,
                   seed_sources=p.seed_sources, extra=p.extra, sigma=sigma)


def problem_c2_screened(sigma: float = 4.0, grid: int = 1024) -> Problem:
    """The 4096-segment star of the 2D Poisson workload with the screened
    equation Lap u = sigma u (Eq. 1, f = 0) and the plane wave u = exp(a.x),
    |a|^2 = sigma, as boundary data and closed-form solution."""
    p = problem_c2(grid=grid)
    rng = np.random.default_rng(seed(2, 8))
    a = rng.normal(0, 1, 2)
    a *= math.sqrt(sigma) / np.linalg.norm(a)
    g = exp_plane(1.0, a)
    return Problem("c2s_star4096_screened", p.scene, g, Field(), p.n_cache, p.n_walks, p.eps, p.offset, 0,
                   p.eval_x, g, sides=p.sides, precision="f32", seed_walks=seed(2, 9), seed_cache=p.seed_cache,
                   seed_sources=p.seed_sources, extra=p.extra, sigma=sigma)


def c4_fields(n_fields: int = 64, lmax: int = 8) -> np.ndarray:
    """Coefficient matrix (n_fields, (lmax+1)^2) of the batched 3D workload."""
    rng = np.random.default_rng(seed(4, 2))
    return rng.normal(0, 1, (n_fields, (lmax + 1) ** 2))


def c4_scenes(n_scenes: int = 32):
    """Uneven 2D star scenes of the multi-scene workload: (scene, n_cache, n_eval)."""
    rng = np.random.default_rng(seed(4, 1))
    out = []
    for s in range(n_scenes):
        sc = star_polygon(4096, 4100 + s)
        nc = int(round(math.exp(rng.uniform(math.log(1024), math.log(65536)))))
        ne = int(round(math.exp(rng.uniform(math.log(4096), math.log(1 << 20)))))
        out.append((sc, nc, ne))
    return out


def problem_c5(n_coef: int = 256, n_obs_candidates: int = 16384):
    """Star domain, Laplace, g = Fourier series in theta with 256 coefficients."""
    sc = star_polygon(4096, seed(5, 1))
    rng = np.random.default_rng(seed(5, 2))
    m = np.arange(n_coef)
    theta_true = rng.normal(0, 1, n_coef) / (1.0 + m)
    eps = 1e-3 * sc.diagonal
    lo, hi = sc.bbox
    obs = uniform_box(n_obs_candidates, lo, hi, seed(5, 5))
    return dict(scene=sc, theta_true=theta_true, eps=eps, offset=5 * eps, n_cache=4096,
                n_walks=64, obs_candidates=obs, noise_sigma=1e-3,
                noise_seed=seed(5, 7), seed_walks=seed(5, 4), seed_cache=seed(5, 3))
