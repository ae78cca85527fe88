"""Pins of the oracle's source terms with screening (Eq. 1 with sigma > 0 and
f != 0) and of the first ball's gradient source term in 3D, against closed
forms independent of the oracle's arithmetic:

- the screened ball Green's function: sampling y from the Laplace ball
  density and weighting by orc_screen_source_ratio, R^2/(2 dim) E[ratio]
  equals the value at the centre of the solution of (-Lap + sigma) w = 1
  with w = 0 on the sphere, (1 - P(R))/sigma (P = 1/I0(sR) in 2D, sR/sinh(sR)
  in 3D), by quadrature over t;
- the centre gradient of the in-ball source term: for f(y) = a.y the
  solution w = (a.x)/sigma - (a.x_hat) R I1(sr)/(sigma I1(sR)) (2D) or with
  the spherical i1 (3D) has grad w(c) = (a/sigma)(1 - (sR/2)/I1(sR)) and
  (a/sigma)(1 - sR/(3 i1(sR))); the quadrature of the ratio against the
  gradient sample's density, and a Monte Carlo average of the sampler itself
  (Laplace and screened), reproduce it (the Laplace limits R^2/8 and R^2/10);
- walks: with g = c0 and f = -sigma c0 the solution is u = c0 (grad u = 0) in
  any domain; the screened walks' means of u and grad u (pointwise) and of the
  normal derivative (cache points) match it, in 2D and 3D, while without the
  source term the means of u miss by more than 20 standard errors;
- the Poisson walk in 3D with u = |x|^2 (f = 6) on a box: u and grad u = 2x;
- a source that varies: u = e^(b.x) with |b|^2 != sigma solves the equation
  with f = (|b|^2 - sigma) e^(b.x); Laplace and screened walks, 2D and 3D,
  match u and grad u = b e^(b.x) (the gradient source term's sign and size
  matter here: a constant source's gradient term vanishes in expectation).
"""
import math

import numpy as np
from scipy import integrate, special

import oracle as orc
import workloads as wl

SIG = 9.0


def _sph_i1(z):
    return (z * math.cosh(z) - math.sinh(z)) / (z * z)


def test_screened_source_ratio_integrates_to_the_ball_solution():
    for dim in (2, 3):
        dens = (lambda t: 4 * t * math.log(1 / t)) if dim == 2 else (lambda t: 6 * t * (1 - t))
        for R in (0.05, 0.4, 1.3):
            s = math.sqrt(SIG)
            z = s * R
            P = 1 / special.iv(0, z) if dim == 2 else z / math.sinh(z)
            val, _ = integrate.quad(lambda t: dens(t) * orc.screen_source_ratio(dim, SIG, R, t), 0, 1, limit=200)
            assert abs(R * R / (2 * dim) * val - (1 - P) / SIG) <= 1e-9 * (1 - P) / SIG, (dim, R)
            # sigma -> 0: the Laplace ball, ratio 1
            assert orc.screen_source_ratio(dim, 0.0, R, 0.37) == 1.0
            r = [orc.screen_source_ratio(dim, SIG, R, t) for t in (0.01, 0.3, 0.7, 0.99)]
            assert all(0 < v <= 1 for v in r)


def _grad_closed(dim, R):
    s = math.sqrt(SIG)
    z = s * R
    if dim == 2:
        return (1 - (z / 2) / special.iv(1, z)) / SIG
    return (1 - z / (3 * _sph_i1(z))) / SIG


def test_screened_gradient_source_ratio_against_the_linear_solution():
    for dim in (2, 3):
        q = (lambda t: 1.5 * (1 - t * t) * (2 / 3)) if dim == 2 else (lambda t: 1 - t ** 3)  # density x weight
        for R in (0.05, 0.4, 1.3):
            val, _ = integrate.quad(lambda t: q(t) * t * orc.screen_grad_source_ratio(dim, SIG, R, t), 0, 1,
                                    limit=200)
            got = R * R / dim * val
            want = _grad_closed(dim, R)
            assert abs(got - want) <= 1e-8 * want, (dim, R, got, want)
        # the Laplace limits
        lap, _ = integrate.quad(lambda t: q(t) * t, 0, 1)
        assert abs(lap / dim - (1 / 8 if dim == 2 else 1 / 10)) < 1e-12


def test_gradient_source_sampler_monte_carlo():
    rng = np.random.default_rng(0)
    for dim in (2, 3):
        a = rng.normal(0, 1, dim)
        R = 0.6
        c = np.zeros(dim)
        for sig in (0.0, SIG):
            n = 40000
            acc = np.zeros((n, dim))
            for i in range(n):
                t, yhat, y, m = orc.sample_grad_source(7, i, 0, 2, dim, c, R)
                acc[i] = m * R * orc.screen_grad_source_ratio(dim, sig, R, t) * yhat * (a @ y)
            mean = acc.mean(0)
            se = acc.std(0, ddof=1) / math.sqrt(n)
            want = a * (_grad_closed(dim, R) if sig > 0 else R * R / (8 if dim == 2 else 10))
            assert np.all(np.abs(mean - want) <= 4.5 * se + 1e-12), (dim, sig, mean, want, se)


def _batched(osc, g, f, sigma, pts, W, nb, seed0):
    """Means of u and grad u over nb independent batches of W walks, and the
    standard errors of the means."""
    us, gs = [], []
    for b in range(nb):
        P = orc.walk_params(1e-3, W, seed0 + b, sigma=sigma)
        u, gr, _ = orc.pointwise(osc, g, f, P, pts, with_grad=True)
        us.append(u)
        gs.append(gr)
    us, gs = np.array(us), np.array(gs)
    return us.mean(0), us.std(0, ddof=1) / math.sqrt(nb), gs.mean(0), gs.std(0, ddof=1) / math.sqrt(nb)


def test_screened_walks_with_a_source_reproduce_a_constant():
    c0 = 1.7
    g = wl.Field(wl.FIELD_CONST, [], [c0])
    f = wl.Field(wl.FIELD_CONST, [], [-SIG * c0])
    for dim, scene in ((2, wl.circle_polygon(256)), (3, wl.displaced_icosphere(3, 31, amp=0.1))):
        osc = orc.Scene(scene)
        pts = np.array([[0.1, -0.2, 0.05][:dim], [0.5, 0.3, -0.2][:dim], [-0.6, 0.05, 0.3][:dim]])
        u, su, gr, sg = _batched(osc, g, f, SIG, pts, 400, 16, 91)
        assert np.all(np.abs(u - c0) <= 4.5 * su + 1e-3), (dim, u, su)
        assert np.all(np.abs(gr) <= 4.5 * sg + 1e-3), (dim, gr, sg)
        # without the source term the means are far from c0
        u0, su0, _, _ = _batched(osc, g, None, SIG, pts, 400, 4, 91)
        assert np.all(np.abs(u0 - c0) > 20 * (su + su0)), (dim, u0)
        # cache points: u and the normal derivative (Eq. 7 with the source's
        # gradient term) of every walk, averaged
        c = osc.sample_cache(400, 5e-3, 1, 5)
        m = c["accept"]
        cn = dict(x=c["x"][m], n=c["n"][m], w=c["w"][m], xbar=c["xbar"][m], R0=c["R0"][m])
        ref = orc.cache_walks(osc, g, f, orc.walk_params(1e-3, 64, 93, sigma=SIG), cn)
        U, D = ref["U"], ref["D"]
        assert abs(U.mean() - c0) <= 4.5 * U.std(ddof=1) / math.sqrt(U.size), (dim, U.mean())
        assert abs(D.mean()) <= 4.5 * D.std(ddof=1) / math.sqrt(D.size), (dim, D.mean())


def test_poisson_gradient_source_3d_box():
    full, _, _ = wl.mixed_box((-1, -1, -1), (1, 1, 1), [False] * 6, 4)
    osc = orc.Scene(full)
    g = wl.quadratic(1.0, 0.0)
    f = wl.Field(wl.FIELD_CONST, [], [6.0])
    pts = np.array([[0.3, 0.1, -0.2], [-0.5, 0.6, 0.4], [0.8, -0.7, 0.1]])
    u, su, gr, sg = _batched(osc, g, f, 0.0, pts, 500, 16, 101)
    assert np.all(np.abs(u - (pts ** 2).sum(1)) <= 4.5 * su + 1e-3), (u, su)
    assert np.all(np.abs(gr - 2 * pts) <= 4.5 * sg + 1e-3), (gr, sg)


def test_walks_with_an_exponential_source():
    b3 = np.array([0.9, -0.6, 0.5])
    for dim, scene in ((2, wl.circle_polygon(256)), (3, wl.displaced_icosphere(3, 31, amp=0.1))):
        b = b3[:dim]
        osc = orc.Scene(scene)
        pts = np.array([[0.1, -0.2, 0.05][:dim], [0.5, 0.3, -0.2][:dim], [-0.6, 0.05, 0.3][:dim]])
        for sig in (0.0, SIG):
            g = wl.exp_plane(1.0, b)
            f = wl.exp_plane(float(b @ b) - sig, b)
            u, su, gr, sg = _batched(osc, g, f, sig, pts, 500, 16, 111)
            ue = np.exp(pts @ b)
            assert np.all(np.abs(u - ue) <= 4.5 * su + 1e-3), (dim, sig, u, ue, su)
            assert np.all(np.abs(gr - b[None, :] * ue[:, None]) <= 4.5 * sg + 1e-3), (dim, sig, gr, sg)
