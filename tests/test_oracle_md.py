"""Pins for the binary64 MD oracle (Fig. 7: map over particles of a reduce
over neighbour indices, Lennard-Jones pair force, cutoff).

Nothing re-types the force formula: the pair force is checked against the
numerical derivative of the Lennard-Jones potential, its zero at the
potential minimum 2^(1/6) sigma, Newton's third law on symmetric lists,
invariance under translation and exact rotation, the cutoff, empty slots,
and the order of a neighbour list.
"""
import math

import numpy as np
import pytest

import oracle


def potential(r, eps=1.0, sigma=1.0):
    return 4 * eps * ((sigma / r) ** 12 - (sigma / r) ** 6)


def pair(r, eps=1.0, sigma=1.0, direction=(1.0, 0.0, 0.0)):
    """Force on a particle at the origin from one at r * direction."""
    d = np.array(direction, dtype=np.float64)
    pos = np.zeros((2, 4), np.float32)
    pos[1, :3] = (r * d).astype(np.float32)
    nbr = np.array([[1], [0]], np.int32)
    return oracle.md(pos, nbr, 10.0, eps, sigma), pos


@pytest.mark.parametrize("r", [0.9, 1.0, 1.05, 1.3, 1.7, 2.4])
@pytest.mark.parametrize("eps,sigma", [(1.0, 1.0), (0.5, 1.2)])
def test_force_is_minus_gradient_of_potential(r, eps, sigma):
    f, pos = pair(r, eps, sigma)
    rr = float(pos[1, 0])                   # the stored binary32 distance
    h = 1e-6 * rr
    dudr = (potential(rr + h, eps, sigma) - potential(rr - h, eps, sigma)) / (2 * h)
    # particle 0 at the origin, r = x1 - x0: F_x(p0) = -dU/dx0 = +dU/dr
    assert abs(f[0, 0] - dudr) <= 1e-6 * max(1.0, abs(dudr))
    assert f[0, 1] == 0.0 and f[0, 2] == 0.0
    assert f[1, 0] == -f[0, 0]              # Newton's third law, exactly (same terms)


def test_gradient_all_cases():
    for r in (0.9, 1.0, 1.05, 1.3, 1.7, 2.4):
        for eps, sigma in ((1.0, 1.0), (0.5, 1.2)):
            test_force_is_minus_gradient_of_potential(r, eps, sigma)


def test_zero_force_at_potential_minimum():
    r0 = 2.0 ** (1.0 / 6.0)
    f, pos = pair(r0)
    rr = float(pos[1, 0])
    # the binary32 distance is within 2^-24 relative of r0: |F| <= |dF/dr| * |rr - r0|
    assert abs(f[0, 0]) <= 60.0 * abs(rr - r0) + 1e-12
    assert pair(0.9 * r0)[0][0, 0] < 0 < pair(1.1 * r0)[0][0, 0]   # repulsive inside, attractive outside


def lattice(nside, spacing=1.0, jitter=0.1, seed=0):
    rng = np.random.default_rng(seed)
    g = np.stack(np.meshgrid(*[np.arange(nside)] * 3, indexing="ij"), -1).reshape(-1, 3) * spacing
    g = g + rng.uniform(-jitter, jitter, g.shape)
    pos = np.zeros((len(g), 4), np.float32)
    pos[:, :3] = g
    return pos


def full_lists(pos, rlist):
    p = pos[:, :3].astype(np.float64)
    d2 = ((p[:, None, :] - p[None, :, :]) ** 2).sum(-1)
    n = len(p)
    lists = [[j for j in np.argsort(d2[i]) if j != i and d2[i, j] < rlist * rlist] for i in range(n)]
    k = max(len(l) for l in lists)
    nbr = np.full((n, k), -1, np.int32)
    for i, l in enumerate(lists):
        nbr[i, :len(l)] = l
    return nbr


def test_newton_third_law_on_symmetric_lists():
    pos = lattice(5, seed=1)
    nbr = full_lists(pos, 2.6)
    f, m = oracle.md(pos, nbr, 2.5, 1.0, 1.0, with_mass=True)
    assert np.all(np.abs(f.sum(0)) <= 1e-12 * m.sum(0))
    assert np.any(np.abs(f) > 1.0)                      # not vacuous


def test_translation_and_exact_rotation():
    pos = lattice(4, seed=2)
    pos[:, :3] = np.round(pos[:, :3] * 1024) / 1024     # few mantissa bits: shifts stay exact
    nbr = full_lists(pos, 2.2)
    f = oracle.md(pos, nbr, 2.0, 1.0, 1.0)
    sh = pos.copy()
    sh[:, :3] += np.float32(16.0)
    assert np.allclose(oracle.md(sh, nbr, 2.0, 1.0, 1.0), f, rtol=0, atol=1e-9 * np.abs(f).max())
    rot = pos.copy()                                     # 90 degrees about z: (x, y) -> (-y, x)
    rot[:, 0], rot[:, 1] = -pos[:, 1], pos[:, 0]
    fr = oracle.md(rot, nbr, 2.0, 1.0, 1.0)
    assert np.array_equal(fr[:, 0], -f[:, 1]) and np.array_equal(fr[:, 1], f[:, 0])
    assert np.array_equal(fr[:, 2], f[:, 2])


def test_cutoff_and_empty_slots():
    f_in, _ = pair(1.499)
    pos = np.zeros((2, 4), np.float32)
    pos[1, 0] = 1.501
    nbr = np.array([[1], [0]], np.int32)
    assert np.all(oracle.md(pos, nbr, 1.5, 1.0, 1.0) == 0.0)            # beyond the cutoff
    pos[1, 0] = 1.499
    assert np.all(oracle.md(pos, nbr, 1.5, 1.0, 1.0)[:, 0] != 0.0)      # inside
    padded = np.array([[-1, 1, 2, -7], [0, -1, 99, 2]], np.int32)       # -1, n, 99: empty
    assert np.array_equal(oracle.md(pos, padded, 1.5, 1.0, 1.0), oracle.md(pos, nbr, 1.5, 1.0, 1.0))
    assert oracle.md(np.zeros((0, 4), np.float32), np.zeros((0, 3), np.int32), 1.0, 1.0, 1.0).shape == (0, 3)


def _near_cutoff_pairs(t, count=4, seed=5):
    """Separations q (p at the origin) within a few binary32 ulps of the
    cutoff whose exact squared distance (rationals) is decided differently
    by a binary32 evaluation ((dx dx + dy dy) + dz dz < binary32(t^2)): half
    exactly inside, half exactly outside, each at least 1e-12 relative from
    t^2, so a binary64 evaluation decides them correctly."""
    from fractions import Fraction

    rng = np.random.default_rng(seed)
    t2, t2f = Fraction(t) ** 2, np.float32(t * t)
    got = {True: [], False: []}
    while min(len(v) for v in got.values()) < count:
        d = rng.normal(size=3)
        q = (d / np.linalg.norm(d) * t * (1 + int(rng.integers(-6, 7)) * 2.0 ** -24)).astype(np.float32)
        sq = q * q
        r2f = np.float32(np.float32(sq[0] + sq[1]) + sq[2])
        exact = sum(Fraction(float(v)) ** 2 for v in q)
        inside = exact < t2
        if inside != bool(r2f < t2f) and abs(exact - t2) > Fraction(1, 10 ** 12) * t2 and len(got[inside]) < count:
            got[inside].append(q)
    return got


def test_cutoff_is_the_exact_distance():
    # updateF's test is distance < t: decided on the exact distance of the
    # stored positions, also where a binary32 evaluation of r^2 decides the
    # other way, and strictly (a pair at exactly t is outside)
    t = 2.5
    nbr = np.array([[1], [0]], np.int32)
    for inside, qs in _near_cutoff_pairs(t).items():
        for q in qs:
            pos = np.zeros((2, 4), np.float32)
            pos[1, :3] = q
            f = oracle.md(pos, nbr, t, 1.0, 1.0)
            assert bool(np.any(f != 0.0)) == inside, (q, inside)
    pos = np.zeros((2, 4), np.float32)
    pos[1, 0] = np.float32(t)
    assert np.all(oracle.md(pos, nbr, t, 1.0, 1.0) == 0.0)
    pos[1, 0] = np.nextafter(np.float32(t), np.float32(0))
    assert np.all(oracle.md(pos, nbr, t, 1.0, 1.0)[:, 0] != 0.0)


def test_list_order_changes_only_rounding():
    pos = lattice(4, seed=3)
    nbr = full_lists(pos, 2.4)
    f, m = oracle.md(pos, nbr, 2.3, 1.0, 1.0, with_mass=True)
    rev = np.ascontiguousarray(nbr[:, ::-1])
    fr = oracle.md(pos, rev, 2.3, 1.0, 1.0)
    assert np.all(np.abs(fr - f) <= 1e-13 * m + 1e-300)


@pytest.mark.parametrize("bad", [dict(cutoff=-1.0), dict(sigma=0.0), dict(epsilon=math.nan)])
def test_rejects_bad_parameters(bad):
    args = dict(cutoff=2.0, epsilon=1.0, sigma=1.0)
    args.update(bad)
    with pytest.raises(RuntimeError):
        oracle.md(np.zeros((2, 4), np.float32), np.zeros((2, 1), np.int32), **args)
