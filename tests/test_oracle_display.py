"""Pins for the oracle's display precompute: the view-index map V (section
3.1, Eq. 1-3), the view clusters (appendix B.1) and the remap LUT Psi
(section 4.3, Eq. 8).  CPU only."""
from fractions import Fraction
import math

import numpy as np
import pytest

import oracle
from workloads import DisplayParams, Rational, get_workload


def _fraction_view(x, y, u, N, tan, pitch, off):
    """Eq. 1-3 evaluated with Python's exact rational type."""
    d = 3 * x + u + 3 * y * tan - off
    xo = d - pitch * math.floor(d / pitch)          # mathematical mod, in [0, L_x)
    return math.floor(N * xo / pitch)


# Hand-worked values for the tiny display (W=256, N=16, tan=1/6, L_x=23/5):
#   (x=0,y=0,u=1): d=1,   x_off=1,   j=floor(16*1/4.6)=floor(3.478)=3
#   (x=0,y=0,u=2): d=2,   x_off=2,   j=floor(6.957)=6
#   (x=1,y=0,u=0): d=3,   x_off=3,   j=floor(10.43)=10
#   (x=1,y=0,u=2): d=5,   x_off=0.4, j=floor(1.391)=1
#   (x=0,y=1,u=0): d=0.5, x_off=0.5, j=floor(1.739)=1
#   (x=1,y=1,u=1): d=4.5, x_off=4.5, j=floor(15.65)=15
HAND = [((0, 0, 0), 0), ((0, 0, 1), 3), ((0, 0, 2), 6), ((1, 0, 0), 10), ((1, 0, 2), 1),
        ((0, 1, 0), 1), ((1, 1, 1), 15)]


def test_view_map_hand_worked():
    V = oracle.view_map(get_workload("tiny").display)
    for (x, y, u), j in HAND:
        assert V[y, x, u] == j, (x, y, u)


@pytest.mark.parametrize("name", ["tiny", "display", "outdoor"])
def test_view_map_matches_exact_rationals(name):
    d = get_workload(name).display
    V = oracle.view_map(d)
    assert V.shape == (d.height, d.width, 3)
    assert V.min() >= 0 and V.max() < d.num_views
    rng = np.random.default_rng(7)
    tan, pitch, off = d.tan_slant.fraction(), d.pitch.fraction(), d.offset.fraction()
    xs = rng.integers(0, d.width, 400)
    ys = rng.integers(0, d.height, 400)
    us = rng.integers(0, 3, 400)
    # include the last row/column
    xs[:3], ys[:3] = d.width - 1, d.height - 1
    for x, y, u in zip(xs, ys, us):
        assert V[y, x, u] == _fraction_view(int(x), int(y), int(u), d.num_views, tan, pitch, off)


def test_view_map_negative_offset_and_odd_rationals():
    d = DisplayParams(37, 23, 7, Rational(-3, 11), Rational(17, 3), Rational(-5, 7))
    V = oracle.view_map(d)
    for y in range(d.height):
        for x in range(d.width):
            for u in range(3):
                assert V[y, x, u] == _fraction_view(x, y, u, 7, Fraction(-3, 11), Fraction(17, 3),
                                                    Fraction(-5, 7))


def test_view_map_unslanted_closed_form():
    # tan(alpha) = 0, K = 0, integer pitch: j = floor(N ((3x+u) mod L) / L), same on every row
    d = DisplayParams(40, 5, 9, Rational(0), Rational(6))
    V = oracle.view_map(d)
    s = 3 * np.arange(40)[:, None] + np.arange(3)[None, :]
    want = (9 * (s % 6)) // 6
    for y in range(5):
        np.testing.assert_array_equal(V[y], want)


def test_view_map_fp64_disagrees_but_oracle_is_exact():
    # Evaluating Eq. 1-3 in float64 (the obvious way) puts some subpixels of
    # the 4K display in the wrong view (even j = N); the oracle must not.
    d = get_workload("outdoor").display
    V = oracle.view_map(d)
    y = np.arange(d.height)[:, None, None].astype(np.float64)
    x = np.arange(d.width)[None, :, None].astype(np.float64)
    u = np.arange(3)[None, None, :].astype(np.float64)
    dd = (3 * x + u) + (3 * y) * (1 / 5) - 0.0
    L = 31 / 5
    xo = dd - L * np.floor(dd / L)
    j64 = np.floor(d.num_views * xo / L).astype(np.int64)
    bad = np.argwhere(j64 != V)
    assert len(bad) > 0
    for (yy, xx, uu) in bad[:: max(1, len(bad) // 50)]:
        assert V[yy, xx, uu] == _fraction_view(int(xx), int(yy), int(uu), 100, Fraction(1, 5),
                                                Fraction(31, 5), Fraction(0))


def test_referenced_views():
    V2 = oracle.view_map(get_workload("display").display)
    assert sorted(np.unique(V2).tolist()) == [0, 4, 9, 13, 18, 22, 27, 31, 36, 40]
    V3 = oracle.view_map(get_workload("outdoor").display)
    ref = np.unique(V3)
    assert len(ref) == 31
    assert ref[:5].tolist() == [0, 3, 6, 9, 12]


def test_view_map_rejects_bad_args():
    with pytest.raises(ValueError):
        oracle.view_map(DisplayParams(4, 4, 3, Rational(1, 6), Rational(0)))


@pytest.mark.parametrize("N,S", [(100, 8), (16, 4), (16, 1), (45, 8), (5, 8), (71, 18), (63, 16)])
def test_cluster_table_closed_form(N, S):
    slots, rep = oracle.cluster_table(N, S)
    K = -(-N // S)
    assert slots.shape == (K, S) and rep.shape == (K,)
    flat = slots[:, :].reshape(-1)
    # contiguous, in order, every view once, tail padded with v_{N-1}
    assert flat[:N].tolist() == list(range(N))
    assert (flat[N:] == N - 1).all()
    assert rep.tolist() == [min(k * S + S // 2, N - 1) for k in range(K)]


def test_cluster_table_examples():
    slots, rep = oracle.cluster_table(100, 8)
    assert slots.shape[0] == 13
    assert slots[-1].tolist() == [96, 97, 98, 99, 99, 99, 99, 99]
    assert rep[-1] == 99 and rep[0] == 4
    _, rep1 = oracle.cluster_table(16, 1)
    assert rep1.tolist() == list(range(16))


def _remap_bruteforce(W, H, tw, th, V):
    out = []
    for ty in range(-(-H // th)):
        for tx in range(-(-W // tw)):
            items = []
            for y in range(ty * th, min(H, (ty + 1) * th)):
                for x in range(tx * tw, min(W, (tx + 1) * tw)):
                    for u in range(3):
                        items.append((int(V[y, x, u]), (y * W + x) * 3 + u))
            items.sort(key=lambda t: t[0])        # Python's sort is stable
            out.extend(p for _, p in items)
    return np.array(out, dtype=np.uint32)


@pytest.mark.parametrize("W,H,tw,th", [(37, 23, 8, 8), (50, 20, 16, 16), (33, 17, 32, 8), (16, 16, 16, 16)])
def test_remap_bruteforce(W, H, tw, th):
    d = DisplayParams(W, H, 11, Rational(1, 6), Rational(23, 5), tile_w=tw, tile_h=th)
    V = oracle.view_map(d)
    psi = oracle.remap(d, V)
    np.testing.assert_array_equal(psi, _remap_bruteforce(W, H, tw, th, V))


def test_remap_invariants_tiny():
    d = get_workload("tiny").display
    V = oracle.view_map(d)
    psi = oracle.remap(d, V)
    n = 3 * d.width * d.height
    assert np.array_equal(np.sort(psi), np.arange(n, dtype=np.uint32))     # a permutation
    Vf = V.reshape(-1)
    per_tile = 3 * d.tile_w * d.tile_h
    for t in range(n // per_tile):
        seg = psi[t * per_tile:(t + 1) * per_tile]
        v = Vf[seg]
        assert (np.diff(v) >= 0).all()                                      # Eq. 8
        same = np.diff(v) == 0
        assert (np.diff(seg.astype(np.int64))[same] > 0).all()              # stable
