"""Pins of the force-bias packing oracle (Sec. 2.4 reading, oracle/packing.py).

* quadrature points: brute-force integer count of the odd grid points in
  the ball, and their volume fraction tends to the ball's;
* overlap volume of two spheres against the closed-form lens volume
  pi (4R + d)(2R - d)^2 / 12, with the error shrinking as the grid refines;
* containment: all of a small sphere's points lie in a large one, and the
  estimate is the small sphere's volume;
* an ellipsoid with three distinct axes contains all of its own points for
  any rotation (a transposed rotation would not), none of a copy beyond its
  tip, and the lens fraction of a copy displaced by an affine image of a
  unit-sphere separation;
* float32 decisions count what float64 ones count (generic placements);
* the pair pushes are equal and opposite: with no clamp the centroid does
  not move; translation of everything in a periodic box changes nothing;
* two overlapping spheres separate along their centre line, symmetrically;
* wall clamping keeps each ellipsoid's extent inside [lo, hi];
* a random dense configuration loses nearly all its overlap.
"""
import numpy as np

from oracle import packing as P


def _rot(rng):
    q, r = np.linalg.qr(rng.standard_normal((3, 3)))
    q = q * np.sign(np.diag(r))
    if np.linalg.det(q) < 0:
        q[:, 0] = -q[:, 0]
    return q


def test_unit_ball_points_brute_force():
    for m in (4, 8, 16):
        n = sum(1 for i in range(m) for j in range(m) for k in range(m)
                if (2 * i + 1 - m) ** 2 + (2 * j + 1 - m) ** 2 + (2 * k + 1 - m) ** 2 <= m * m)
        assert P.unit_ball_points(m).shape == (n, 3)
        assert P.unit_ball_points(m, np.float32).shape == (n, 3)
    frac = [abs(len(P.unit_ball_points(m)) * (2.0 / m) ** 3 / (4 * np.pi / 3) - 1) for m in (8, 16, 32)]
    assert frac[0] > frac[1] > frac[2] and frac[2] < 0.01


def test_sphere_lens_volume():
    R = 5.0
    dom = P.Domain((100.0, 100.0, 100.0), (True, True, True))
    rng = np.random.default_rng(0)
    mean = {}
    for m in (8, 16):
        errs = []
        for d in np.linspace(0.3 * R, 1.7 * R, 8):
            v = rng.standard_normal(3)
            v /= np.linalg.norm(v)
            r = np.array([[50.0, 50.0, 50.0], [50.0, 50.0, 50.0] + d * v])
            pr = P.pair_overlaps(r, np.stack([_rot(rng), _rot(rng)]), np.full((2, 3), R), dom, m)
            exact = np.pi * (4 * R + d) * (2 * R - d) ** 2 / 12
            errs.append(abs(pr[0][4] - exact) / exact)
        mean[m] = np.mean(errs)
        if m == 16:
            assert max(errs) < 0.03
    assert mean[16] < 0.5 * mean[8]


def test_containment():
    rng = np.random.default_rng(1)
    dom = P.Domain((60.0, 60.0, 60.0), (True, True, True))
    r = np.array([[30.0, 30.0, 30.0], [31.0, 29.5, 30.5]])
    s = np.array([[8.0, 8.0, 8.0], [3.0, 3.0, 3.0]])
    (i, j, nij, nji, V), = P.pair_overlaps(r, np.stack([_rot(rng), _rot(rng)]), s, dom, 16)
    Q = len(P.unit_ball_points(16))
    assert nji == Q                      # every point of the small sphere is in the big one
    assert abs(V - P.volume(s[1])) < 0.05 * P.volume(s[1])


def test_own_points_inside_and_disjoint():
    rng = np.random.default_rng(2)
    s = np.array([7.0, 4.0, 2.0])
    U = P.unit_ball_points(8)
    for _ in range(4):
        R = _rot(rng)
        assert P.count_inside(np.zeros(3), R, s, R, s, U) == len(U)
        assert P.count_inside(R[:, 0] * 14.5, R, s, R, s, U) == 0      # touching beyond the tip
        # an affine image of two unit spheres a distance 0.5 apart: the overlap
        # fraction is the lens fraction (4 + 0.5)(2 - 0.5)^2 / 16
        v = rng.standard_normal(3)
        v *= 0.5 / np.linalg.norm(v)
        frac = P.count_inside(R @ (s * v), R, s, R, s, U) / len(U)
        assert abs(frac - 4.5 * 1.5 ** 2 / 16) < 0.04
    # the same body with R transposed is a different ellipsoid: not all points inside
    R = _rot(rng)
    assert P.count_inside(np.zeros(3), R, s, R.T, s, U) < len(U)


def _random_config(rng, n, L, s):
    r = rng.uniform(0, L, (n, 3))
    R = np.stack([_rot(rng) for _ in range(n)])
    return r, R, np.tile(s, (n, 1))


def test_pushes_balance_and_translation_invariance():
    rng = np.random.default_rng(3)
    L = 40.0
    dom = P.Domain((L, L, L), (True, True, True))
    r, R, s = _random_config(rng, 24, L, np.array([6.0, 6.0, 2.5]))
    new, pairs = P.iterate(r, R, s, dom, eta=1e-3, max_move=1e9, m=8)
    assert sum(1 for p in pairs if p[4] > 0) > 10
    disp = P.min_image(new - r, dom)
    assert np.abs(disp.sum(axis=0)).max() < 1e-12 * np.abs(disp).max() * len(r)
    shift = np.array([13.25, -7.5, 21.125])
    new2, _ = P.iterate(np.mod(r + shift, L), R, s, dom, eta=1e-3, max_move=1e9, m=8)
    assert np.abs(P.min_image(new2 - shift - new, dom)).max() < 1e-9


def test_two_spheres_separate_symmetrically():
    dom = P.Domain((50.0, 50.0, 50.0), (True, True, True))
    r = np.array([[20.0, 25.0, 25.0], [27.0, 25.0, 25.0]])
    R = np.stack([np.eye(3), np.eye(3)])
    s = np.full((2, 3), 5.0)
    out = P.run(r, R, s, dom, eta=0.02, max_move=1.0, m=8, n_iter=60)
    assert np.allclose(out[:, 1:], r[:, 1:], atol=1e-12)          # moved along x only
    assert abs(out[:, 0].mean() - r[:, 0].mean()) < 1e-12         # about the midpoint
    d = out[1, 0] - out[0, 0]
    assert P.residual(out, R, s, dom, 8) == (0.0, 0)             # no quadrature point overlaps
    lens = np.pi * (4 * 5.0 + d) * max(10.0 - d, 0.0) ** 2 / 12
    assert lens < 0.01 * P.volume(s[0])                          # nor much true volume


def test_walls_keep_extent_inside():
    rng = np.random.default_rng(4)
    dom = P.Domain((40.0, 30.0, 40.0), (True, False, True), lo=(0, 1.5, 0), hi=(0, 28.5, 0))
    r, R, s = _random_config(rng, 16, 40.0, np.array([6.0, 6.0, 2.5]))
    r[:, 1] = rng.uniform(0, 30, 16)
    out = P.run(r, R, s, dom, eta=2e-3, max_move=1.0, m=8, n_iter=3)
    e = P.extent(R, s)
    assert np.all(out[:, 1] - e[:, 1] >= 1.5 - 1e-12) and np.all(out[:, 1] + e[:, 1] <= 28.5 + 1e-12)
    # the extent is the support of the ellipsoid along y: its points reach it and no further
    U = P.unit_ball_points(32)
    for i in range(3):
        y = (R[i] @ (s[i] * U).T)[1]
        assert y.max() <= e[i, 1] + 1e-12 and y.max() > 0.95 * e[i, 1]


def test_dense_configuration_unpacks():
    rng = np.random.default_rng(5)
    L = 48.0
    dom = P.Domain((L, L, L), (True, True, True))
    s = np.array([6.0, 6.0, 2.2])
    n = int(0.30 * L ** 3 / P.volume(s))
    r, R, sv = _random_config(rng, n, L, s)
    V0, k0 = P.residual(r, R, sv, dom, 8)
    out = P.run(r, R, sv, dom, eta=0.03, max_move=1.0, m=8, n_iter=40)
    V1, k1 = P.residual(out, R, sv, dom, 8)
    print("cells", n, "overlap", V0, "->", V1, "pairs", k0, "->", k1)
    assert V1 < 0.01 * V0 and k1 < 0.2 * k0


def test_float32_decisions_match_float64():
    """The float32 inside tests count what the float64 ones count for a
    generic configuration (no point within rounding of a surface)."""
    rng = np.random.default_rng(6)
    L = 40.0
    dom = P.Domain((L, L, L), (True, True, False), lo=(0, 0, -0.5), hi=(0, 0, 39.5))
    r, R, s = _random_config(rng, 30, L, np.array([6.0, 5.0, 2.5]))
    p64 = P.pair_overlaps(r, R, s, dom, 8, np.float64)
    p32 = P.pair_overlaps(r.astype(np.float32), R.astype(np.float32), s.astype(np.float32), dom, 8,
                          np.float32)
    assert len(p64) > 10
    assert [p[:4] for p in p64] == [p[:4] for p in p32]
