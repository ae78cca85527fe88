"""Pins of the offset rule for cache points (Section 3.2, "Boundary
Specification": l > eps, default l = 5 eps; Fig. "Ablations", top) and of the
rule that a cache walk takes its first ball before any termination test
(Section 3.1 with Eq. 7), on a flat wall, against facts independent of the
oracle's arithmetic.

Geometry: the strip [0, H] x [0, L] with H = 20 eps and L = 1, cache points
at distance l from the wall x = 0 (outward normal -e_x) and far from the
ends y = 0, L.  There the distance to the boundary is min(x, H - x), so a
walk's x coordinate is the scalar chain x <- x + R cos(theta),
R = min(x, H - x), stopped when R < eps, after a first ball of radius l; with
g = x the data read at the stop is 0 on the near wall and H on the far one.

- l = 0.1 eps: every first-ball point lies inside the epsilon shell, so every
  walk makes exactly one closest-point query and stops on the wall at the
  projection of x + l nu: the exit points spread along the wall with
  variance l^2 / 2 (a walk that stopped at its start would not move).  With
  g = x every sample U and D is exactly 0 although du/dn = -1; with
  g = e^x cos y the mean of D is 0 within its standard error although
  du/dn = -cos y: the cache's du/dn estimate collapses to zero, as the
  ablation figure reports.
- l = eps, 2 eps, 5 eps: the mean of the oracle's D matches the same mean
  from an independent simulation of the scalar chain (numpy) within four
  combined standard errors, and the bias against the large-offset value
  shrinks as l grows.  The first-order figure 1 + 2 E[nu_n (1 - nu_n);
  nu_n > 0] = 1.137 counts only the walks that stop in the first ball; the
  walks that continue read g at distance beta ~ 0.35 eps from where they
  stop, which pulls the ratio at l = eps below 1 (about 0.92).
"""
import numpy as np

import oracle as orc
import workloads as wl

EPS = 1e-3
H = 20 * EPS


def _strip():
    v = np.array([[0.0, 0.0], [H, 0.0], [H, 1.0], [0.0, 1.0]])
    p = np.array([[0, 1], [1, 2], [2, 3], [3, 0]], dtype=np.int32)
    return wl.Scene(2, v, p)


def _cache(l, n=64):
    y = np.linspace(0.35, 0.65, n)
    x = np.stack([np.full(n, l), y], 1)
    return dict(x=x, n=np.tile([-1.0, 0.0], (n, 1)), w=np.full(n, 1.0 / n), xbar=np.stack([np.zeros(n), y], 1),
                R0=np.full(n, l))


def _chain_mean(l, n, seed):
    """Mean and standard error of D = (2/l)(nu . n) W for g = x, from the
    scalar chain of the walk's x coordinate (the strip's distance function
    is min(x, H - x) away from its ends)."""
    rng = np.random.default_rng(seed)
    nx = np.cos(rng.uniform(0, 2 * np.pi, n))
    x = l + l * nx  # first ball: no termination test before it
    W = np.zeros(n)
    alive = np.ones(n, bool)
    for _ in range(1024):
        idx = np.nonzero(alive)[0]
        if idx.size == 0:
            break
        xi = x[idx]
        d = np.minimum(xi, H - xi)
        stop = d < EPS
        W[idx[stop]] = np.where(xi[stop] < H / 2, 0.0, H)
        alive[idx[stop]] = False
        go = idx[~stop]
        x[go] += d[~stop] * np.cos(rng.uniform(0, 2 * np.pi, go.size))
    assert not alive.any()
    D = (2 / l) * (-nx) * W
    return D.mean(), D.std() / np.sqrt(n)


def test_offset_below_eps_gives_zero_flux():
    osc = orc.Scene(_strip())
    l = 0.1 * EPS
    c = _cache(l)
    W = 2048
    out = orc.cache_walks(osc, wl.harmonic_2d(1, 1.0, 0.0), None, orc.walk_params(EPS, W, 71), c, records=True)
    assert np.all(out["steps"] == 1)
    assert np.all(out["U"] == 0.0) and np.all(out["D"] == 0.0)
    ex = out["exit"].reshape(-1, W, 2)
    assert np.all(ex[:, :, 0] == 0.0)
    dy = ex[:, :, 1] - c["x"][:, 1:2]
    assert np.all(np.abs(dy) <= l * (1 + 1e-9))
    assert abs(np.mean(dy**2) / (l * l / 2) - 1) < 0.02  # E[nu_y^2] = 1/2
    # tangential variation: the mean of D is 0, not du/dn = -cos y
    out = orc.cache_walks(osc, wl.harmonic_2d(1, 0.0, 1.0), None, orc.walk_params(EPS, W, 73), c)
    D = out["D"]
    assert np.all(out["steps"] == 1)
    assert abs(D.mean()) < 4 * D.std() / np.sqrt(D.size)
    assert np.mean(np.cos(c["x"][:, 1])) > 0.8  # what the flux should have been, in magnitude


def test_offset_ablation_matches_the_scalar_chain():
    osc = orc.Scene(_strip())
    g = wl.harmonic_2d(1, 1.0, 0.0)  # u = x, du/dn = -1 on the wall x = 0
    means = {}
    for lam in (1, 2, 5):
        l = lam * EPS
        W = 8192
        out = orc.cache_walks(osc, g, None, orc.walk_params(EPS, W, 100 + lam), _cache(l))
        D = out["D"]
        m_or, se_or = D.mean(), D.std() / np.sqrt(D.size)
        m_ch, se_ch = _chain_mean(l, 2_000_000, 200 + lam)
        assert abs(m_or - m_ch) < 4 * np.hypot(se_or, se_ch), (lam, m_or, m_ch, se_or, se_ch)
        means[lam] = (m_ch, se_ch)
    # bias shrinks with the offset: l = eps is well off the l = 5 eps value,
    # l = 2 eps much closer
    b1 = means[1][0] - means[5][0]
    b2 = means[2][0] - means[5][0]
    se = means[1][1] + means[5][1]
    assert b1 > 0.05 and b1 > 10 * se
    assert abs(b2) < 0.5 * b1
