"""Pins of the oracle's random numbers (not gpu).

Philox-4x32-10 is pinned against an independent implementation: rocRAND's
header-only generator, compiled here for the host.  The word -> uniform map and
the samplers are pinned by their defining densities.
"""
import math
import os
import subprocess

import numpy as np
import pytest
from scipy import stats

ROCRAND_HDR = "/opt/rocm/include/rocrand/rocrand_philox4x32_10.h"

KAT_SRC = r"""
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>
int main() {
  unsigned long long seed; unsigned c0, c1, c2, c3;
  while (std::scanf("%llu %u %u %u %u", &seed, &c0, &c1, &c2, &c3) == 5) {
    rocrand_state_philox4x32_10 st;
    unsigned long long offset = 4ull * (c0 | ((unsigned long long)c1 << 32));
    unsigned long long subseq = c2 | ((unsigned long long)c3 << 32);
    rocrand_init(seed, subseq, offset, &st);
    uint4 r = rocrand4(&st);
    std::printf("%u %u %u %u\n", r.x, r.y, r.z, r.w);
  }
}
"""


@pytest.mark.skipif(not os.path.exists(ROCRAND_HDR), reason="rocRAND headers not present")
def test_philox_matches_rocrand(orc, tmp_path):
    src = tmp_path / "kat.cpp"
    src.write_text(KAT_SRC)
    exe = tmp_path / "kat"
    subprocess.run(["g++", "-O1", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include", str(src),
                    "-o", str(exe)], check=True)
    rng = np.random.default_rng(7)
    cases = []
    for i in range(300):
        seed = int(rng.integers(0, 2**63))
        ctr = [int(v) for v in rng.integers(0, 2**32, 4)]
        ctr[1] &= (1 << 29) - 1  # rocRAND takes (ctr0, ctr1) as a 64-bit offset in units of 4
        if i < 20:  # small counters like the ones the walks use
            ctr = [i, 3 * i, 0, i % 7]
        cases.append((seed, ctr))
    inp = "".join(f"{s} {c[0]} {c[1]} {c[2]} {c[3]}\n" for s, c in cases)
    out = subprocess.run([str(exe)], input=inp, capture_output=True, text=True, check=True)
    lines = out.stdout.strip().split("\n")
    assert len(lines) == len(cases)
    for (seed, ctr), line in zip(cases, lines):
        want = [int(v) for v in line.split()]
        got = orc.philox(ctr, [seed & 0xFFFFFFFF, seed >> 32])
        assert got == want, (seed, ctr)


def test_uniform_pair_word_map(orc):
    """The uniform pair uses counter (block, id, batch, tag) and key (seed lo, hi);
    each uniform takes 53 bits from two words."""
    rng = np.random.default_rng(3)
    for _ in range(200):
        seed = int(rng.integers(0, 2**63))
        blk, idx, bat, tag = (int(v) for v in rng.integers(0, 2**31, 4))
        w = orc.philox([blk, idx, bat, tag], [seed & 0xFFFFFFFF, seed >> 32])
        ua, ub = orc.uniform_pair(seed, blk, idx, bat, tag)
        ia = (w[0] << 21) | (w[1] >> 11)
        ib = (w[2] << 21) | (w[3] >> 11)
        assert ua == ia / 2.0**53 and ub == ib / 2.0**53
        assert 0.0 <= ua < 1.0 and 0.0 <= ub < 1.0


def test_uniforms_are_uniform(orc):
    u = np.array([orc.uniform_pair(11, b, i, 0, 1) for b in range(4) for i in range(5000)]).ravel()
    hist, _ = np.histogram(u, bins=40, range=(0, 1))
    chi2 = ((hist - u.size / 40) ** 2 / (u.size / 40)).sum()
    assert stats.chi2.sf(chi2, 39) > 1e-4


def _ks(samples, cdf):
    return stats.kstest(samples, cdf).pvalue


def test_direction_sampler_2d_3d(orc):
    n = 6000
    v2 = np.array([orc.sample_direction(5, 0, i, 0, 1, 2) for i in range(n)])
    assert np.allclose(np.linalg.norm(v2, axis=1), 1, atol=1e-14)
    th = np.mod(np.arctan2(v2[:, 1], v2[:, 0]), 2 * np.pi)
    assert _ks(th, lambda t: t / (2 * np.pi)) > 1e-4
    v3 = np.array([orc.sample_direction(5, 1, i, 0, 1, 3) for i in range(n)])
    assert np.allclose(np.linalg.norm(v3, axis=1), 1, atol=1e-14)
    # uniform on the sphere: z ~ U(-1, 1) (Archimedes) and azimuth uniform
    assert _ks(v3[:, 2], lambda z: (z + 1) / 2) > 1e-4
    ph = np.mod(np.arctan2(v3[:, 1], v3[:, 0]), 2 * np.pi)
    assert _ks(ph, lambda t: t / (2 * np.pi)) > 1e-4


def test_ball_source_radius_densities(orc):
    """Radius of the in-ball source sample follows |G^B| times the shell measure:
    2D 4 s ln(1/s) (CDF s^2 (1 - 2 ln s)), 3D 6 s (1 - s) (CDF 3 s^2 - 2 s^3)."""
    n = 6000
    c2 = np.zeros(2)
    s2 = np.array([np.linalg.norm(orc.sample_ball_source(9, 1, i, 0, 1, 2, c2, 1.0)) for i in range(n)])
    assert _ks(s2, lambda s: np.where(s > 0, s**2 * (1 - 2 * np.log(np.maximum(s, 1e-300))), 0)) > 1e-4
    c3 = np.zeros(3)
    pts = np.array([orc.sample_ball_source(9, 2, i, 0, 1, 3, c3, 2.0) for i in range(n)])
    s3 = np.linalg.norm(pts, axis=1) / 2.0
    assert _ks(s3, lambda s: 3 * s**2 - 2 * s**3) > 1e-4
    # direction of the 3D point is isotropic
    assert _ks(pts[:, 2] / np.linalg.norm(pts, axis=1), lambda z: (z + 1) / 2) > 1e-4


def test_gradient_source_radius_density(orc):
    """2D gradient source radius has density (3/2)(1 - s^2): CDF (3 s - s^3)/2."""
    u = np.random.default_rng(2).random(20000)
    s = np.array([orc.grad_radius(x) for x in u])
    assert _ks(s, lambda t: (3 * t - t**3) / 2) > 1e-4
    # inverse CDF is exact: F(s(u)) = u
    assert np.allclose((3 * s - s**3) / 2, u, atol=1e-14)
