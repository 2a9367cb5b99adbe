"""Pins for the oracle's Radon matrix against things other than the oracle itself.

* hand-derived rows (tests/golden/siddon_hand.json);
* brute force: every ray clipped against every pixel box (Liang-Barsky), with
  the edge rule (half to each pixel sharing an edge) applied explicitly;
* closed forms: chord length through the square and through pixel
  rectangles, disk and ellipse projections in the continuum limit;
* midpoint quadrature of line integrals on 8x8 images;
* invariants: mirror symmetries, the adjoint identity, the nnz estimate.
"""
import json
import math
import os

import numpy as np
import pytest

import oracle
import workloads as W

HERE = os.path.dirname(os.path.abspath(__file__))


def brute_row(n, n_angles, n_bins, k, b):
    """Dense row of R for ray (k, b): clip the ray against each pixel box."""
    h = n / 2.0
    s_b = b - (n_bins - 1) / 2.0
    row = np.zeros(n * n)
    if k == 0 or 2 * k == n_angles:
        vertical = (k == 0)
        pos = s_b + h
        if pos == math.floor(pos):
            e = int(pos)
            for line in (e - 1, e):
                if 0 <= line < n:
                    for r in range(n):
                        j = r * n + line if vertical else line * n + r
                        row[j] += 0.5
        elif 0 < pos < n:
            q = int(math.floor(pos))
            for r in range(n):
                row[r * n + q if vertical else q * n + r] = 1.0
        return row
    th = math.pi * k / n_angles
    c, s = math.cos(th), math.sin(th)
    # p(t) = s_b (c, s) + t (-s, c); clip against [x0,x1] x [y0,y1]
    for iy in range(n):
        for ix in range(n):
            x0, x1 = ix - h, ix - h + 1
            y0, y1 = iy - h, iy - h + 1
            lo, hi = -np.inf, np.inf
            for p0, d, a0, a1 in ((s_b * c, -s, x0, x1), (s_b * s, c, y0, y1)):
                ta, tb = (a0 - p0) / d, (a1 - p0) / d
                lo, hi = max(lo, min(ta, tb)), min(hi, max(ta, tb))
            row[iy * n + ix] = max(0.0, hi - lo)
    return row


def dense_R(n, n_angles, n_bins):
    return oracle.build_R(n, n_angles, n_bins).to_dense()


def test_golden_hand_rows():
    data = json.load(open(os.path.join(HERE, "golden", "siddon_hand.json")))
    for case in data["cases"]:
        cols, vals = oracle.ray(case["n"], case["n_angles"], case["n_bins"], case["k"], case["b"])
        got = {int(c): float(v) for c, v in zip(cols, vals)}
        want = {int(c): float(v) for c, v in case["row"].items()}
        assert set(got) == set(want), (case, got)
        for j in want:
            assert abs(got[j] - want[j]) <= 1e-13, (case, j, got[j], want[j])


@pytest.mark.parametrize("n,n_angles", [(8, 8), (8, 12), (7, 8), (8, 7), (6, 20)])
def test_brute_force_clipping(n, n_angles):
    nb = W.n_bins_for(n)
    # include bins beyond the image and half-integer offsets via an even count too
    for n_bins in (nb, nb + 3):
        R = dense_R(n, n_angles, n_bins)
        for k in range(n_angles):
            for b in range(n_bins):
                want = brute_row(n, n_angles, n_bins, k, b)
                got = R[k * n_bins + b]
                assert np.max(np.abs(got - want)) <= 1e-12, (n, n_angles, n_bins, k, b)


def square_chord(n, c, s, s_b):
    """Length of {p.w = s_b} inside [-n/2, n/2]^2 (trapezoidal projection of a square)."""
    h = n / 2.0
    u, v = abs(c), abs(s)
    if v == 0.0 or u == 0.0:
        return 2 * h if abs(s_b) < h else (h if abs(s_b) == h else 0.0)
    return max(0.0, min(2 * h / u, 2 * h / v, (h * (u + v) - abs(s_b)) / (u * v)))


@pytest.mark.parametrize("n,n_angles", [(16, 15), (32, 24), (33, 10)])
def test_row_sums_are_square_chords(n, n_angles):
    nb = W.n_bins_for(n)
    R = oracle.build_R(n, n_angles, nb)
    rows = np.repeat(np.arange(R.rows), np.diff(R.rp))
    sums = np.bincount(rows, weights=R.v, minlength=R.rows)
    for k in range(n_angles):
        c, s = oracle.trig(k, n_angles)
        for b in range(nb):
            want = square_chord(n, c, s, b - (nb - 1) / 2)
            assert abs(sums[k * nb + b] - want) <= 1e-11 * max(1.0, want), (k, b)


def rect_chord(c, s, s_rel, W_, H_):
    u, v = abs(c), abs(s)
    hw = 0.5 * W_ * u + 0.5 * H_ * v
    if v == 0.0:
        if abs(s_rel) < 0.5 * W_:
            return H_
        return 0.5 * H_ if abs(s_rel) == 0.5 * W_ else 0.0
    if u == 0.0:
        if abs(s_rel) < 0.5 * H_:
            return W_
        return 0.5 * W_ if abs(s_rel) == 0.5 * H_ else 0.0
    return max(0.0, min(W_ / v, H_ / u, (hw - abs(s_rel)) / (u * v)))


def test_pixel_rectangle_phantom_is_exact():
    n, n_angles = 24, 18
    nb = W.n_bins_for(n)
    R = oracle.build_R(n, n_angles, nb)
    ix0, ix1, iy0, iy1 = 5, 14, 8, 20          # pixels ix in [5,14), iy in [8,20)
    mu = np.zeros((n, n))
    mu[iy0:iy1, ix0:ix1] = 1.0
    y = R.matvec(mu.reshape(-1))
    h = n / 2
    W_, H_ = ix1 - ix0, iy1 - iy0
    cx, cy = (ix0 + ix1) / 2 - h, (iy0 + iy1) / 2 - h
    for k in range(n_angles):
        c, s = oracle.trig(k, n_angles)
        for b in range(nb):
            s_rel = (b - (nb - 1) / 2) - (cx * c + cy * s)
            want = rect_chord(c, s, s_rel, W_, H_)
            assert abs(y[k * nb + b] - want) <= 1e-11, (k, b, y[k * nb + b], want)


def test_line_integral_quadrature_8x8():
    n, n_angles = 8, 10
    nb = W.n_bins_for(n)
    R = oracle.build_R(n, n_angles, nb)
    rng = np.random.default_rng(7)
    mu = rng.uniform(0, 1, (n, n))
    y = R.matvec(mu.reshape(-1))
    h = n / 2
    steps = 1_000_000
    checked = 0
    for k in range(1, n_angles):
        if 2 * k == n_angles:
            continue                  # axis-aligned rays on pixel edges: see the edge rule tests
        c, s = oracle.trig(k, n_angles)
        for b in range(0, nb, 2):
            sb = b - (nb - 1) / 2
            L = square_chord(n, c, s, sb)
            if L <= 0:
                continue
            # parametrise across the whole diagonal span and sample midpoints
            T = n * math.sqrt(2) / 2
            t = -T + (np.arange(steps) + 0.5) * (2 * T / steps)
            px, py = sb * c - t * s + h, sb * s + t * c + h
            inside = (px >= 0) & (px < n) & (py >= 0) & (py < n)
            val = mu[np.floor(py[inside]).astype(int), np.floor(px[inside]).astype(int)]
            integral = val.sum() * (2 * T / steps)
            assert abs(integral - y[k * nb + b]) <= 1e-4, (k, b, integral, y[k * nb + b])
            checked += 1
    assert checked > 30


def mirror_x(n):
    j = np.arange(n * n)
    iy, ix = j // n, j % n
    return iy * n + (n - 1 - ix)


def mirror_y(n):
    j = np.arange(n * n)
    iy, ix = j // n, j % n
    return (n - 1 - iy) * n + ix


@pytest.mark.parametrize("n,n_angles", [(16, 12), (15, 9), (20, 16)])
def test_mirror_symmetries_exact(n, n_angles):
    nb = W.n_bins_for(n)
    R = dense_R(n, n_angles, nb)
    mx, my = mirror_x(n), mirror_y(n)
    for k in range(n_angles):
        for b in range(nb):
            row = R[k * nb + b]
            # x -> -x maps angle theta to pi - theta (k -> n_a - k); theta = 0 flips the bin
            kx, bx = (n_angles - k, b) if k else (0, nb - 1 - b)
            np.testing.assert_array_equal(row[mx], R[kx * nb + bx])
            # y -> -y maps (theta, s) to (pi - theta, -s); theta = 0 is unchanged
            ky, by = (n_angles - k, nb - 1 - b) if k else (0, b)
            np.testing.assert_array_equal(row[my], R[ky * nb + by])


@pytest.mark.parametrize("n,n_angles", [(16, 8), (24, 12), (15, 20)])
def test_transpose_symmetries(n, n_angles):
    """The maps behind the layouts stored by symmetry: the transpose of the
    pixel grid carries the ray (theta, s) onto (pi/2 - theta, s), and the
    transpose after x -> -x onto (pi/2 + theta, s), so the ray with bin b at
    pi/2 - theta meets pixel (iy, ix), and the one at pi/2 + theta pixel
    (n-1-iy, ix), with the lengths the ray at theta meets (ix, iy) with."""
    nb = W.n_bins_for(n)
    R = dense_R(n, n_angles, nb)
    j = np.arange(n * n)
    iy, ix = j // n, j % n
    tr = ix * n + iy                  # pixel (iy, ix)
    both = ix * n + (n - 1 - iy)      # pixel (n-1-iy, ix)
    h = n_angles // 2
    for k in range(h + 1):
        for b in range(nb):
            row = R[k * nb + b]
            np.testing.assert_allclose(R[(h - k) * nb + b][tr], row, rtol=0, atol=1e-12)
            if h + k < n_angles:
                np.testing.assert_allclose(R[(h + k) * nb + b][both], row, rtol=0, atol=1e-12)


def test_adjoint_identity_and_transpose():
    w = W.WORKLOADS["small_64_f64"]
    op = oracle.OracleOp(w.n, w.n_angles, w.n_bins, w.mask)
    rng = np.random.default_rng(3)
    x = rng.standard_normal(op.nn)
    y = rng.standard_normal(op.rows)
    lhs, rhs = np.dot(op.fwd(x), y), np.dot(x, op.adj(y))
    assert abs(lhs - rhs) <= 1e-12 * np.linalg.norm(op.fwd(x)) * np.linalg.norm(y)
    # every entry of the transpose is an entry of R at the swapped index
    T = op.MRT
    rows = np.repeat(np.arange(T.rows), np.diff(T.rp))
    for e in rng.integers(0, T.nnz, 200):
        i, j, v = T.ci[e], rows[e], T.v[e]
        c, vv = op.MR.row(i)
        assert vv[np.searchsorted(c, j)] == v


@pytest.mark.parametrize("n,n_angles", [(64, 45), (128, 30), (96, 64)])
def test_nnz_estimate(n, n_angles):
    R = oracle.build_R(n, n_angles, W.n_bins_for(n))
    # a line crosses L(|cos|+|sin|)+1 pixels, which averages to (4/pi)(N^2+N) per angle;
    # for even N the axis-aligned angles put every ray on a pixel edge, which doubles
    # their N^2 entries (half to each neighbour)
    ties = (n % 2 == 0) * (1 + (n_angles % 2 == 0))
    est = 4 / math.pi * n_angles * (n * n + n) + ties * n * n
    assert abs(R.nnz / est - 1) < 0.025


def ellipse_projection(params, n, c, s, s_b):
    """Kak-Slaney analytic projection of additive ellipses (in pixel units)."""
    h = n / 2
    out = 0.0
    for cx, cy, a, b, phi, rho in params:
        cx, cy, a, b = cx * h, cy * h, a * h, b * h
        th = math.atan2(s, c)
        a2 = (a * math.cos(th - phi)) ** 2 + (b * math.sin(th - phi)) ** 2
        sp = s_b - (cx * c + cy * s)
        if sp * sp < a2:
            out += 2 * rho * a * b * math.sqrt(a2 - sp * sp) / a2
    return out


def _projection_error(n, params, n_angles=6):
    nb = W.n_bins_for(n)
    R = oracle.build_R(n, n_angles, nb)
    mu = W.rasterize_ellipses(params, n).reshape(-1)
    y = R.matvec(mu)
    errs, scale = [], 0.0
    for k in range(n_angles):
        c, s = oracle.trig(k, n_angles)
        for b in range(nb):
            want = ellipse_projection(params, n, c, s, b - (nb - 1) / 2)
            errs.append(abs(y[k * nb + b] - want))
            scale = max(scale, want)
    return float(np.mean(errs)) / scale, float(np.max(errs)) / scale


def test_disk_projection_converges():
    params = np.array([[0.1, -0.05, 0.5, 0.5, 0.0, 1.0]])      # disk: a = b
    e1, m1 = _projection_error(64, params)
    e2, m2 = _projection_error(256, params)
    # chord 2 rho sqrt(r^2 - s^2): the pixelisation error of the mean is O(1/N) ...
    assert e2 < e1 / 2.5, (e1, e2)
    assert e2 < 1.0 / 256
    # ... and the worst ray (tangent to a staircase edge) shrinks like N^(-1/2)
    assert m2 < m1 / 1.6, (m1, m2)


def test_ellipse_projection_converges():
    rng = np.random.default_rng(0)
    params = W.ellipse_params(rng, 5)
    e1, _ = _projection_error(64, params)
    e2, _ = _projection_error(256, params)
    assert e2 < e1 / 2.5, (e1, e2)
