"""Pin of the oracle's Morton keys (Sec. 5: the double Z-order permutation).

The keys are written out here bit by bit for points whose quantised
coordinates are chosen directly: with the bounding-box corner at 0 and the
largest side 1, the point (q + 1/2) / 2^21 quantises to the integer q on
each axis, and the key puts bit b of x at 3b, of y at 3b + 1, of z at 3b + 2.
A swapped or shifted interleave, a wrong number of bits per axis or a wrong
normalisation changes some of the literal keys below.
"""
import numpy as np

from oracle import solver

S = float(1 << 21)


def _pt(qx, qy, qz):
    return [(qx + 0.5) / S, (qy + 0.5) / S, (qz + 0.5) / S]


CASES = [
    # (qx, qy, qz) -> key, written in binary / powers of two by hand
    ((0, 0, 0), 0),
    ((1, 0, 0), 0b001),
    ((0, 1, 0), 0b010),
    ((0, 0, 1), 0b100),
    ((1, 1, 1), 0b111),
    ((2, 0, 0), 0b001000),
    ((0, 2, 0), 0b010000),
    ((3, 5, 6), 0b110101011),          # x=011, y=101, z=110 -> (z2 y2 x2)(z1 y1 x1)(z0 y0 x0)
    ((1 << 20, 0, 0), 1 << 60),
    ((0, 1 << 20, 0), 1 << 61),
    ((0, 0, 1 << 20), 1 << 62),
    ((1 << 20, 1 << 19, 3 << 19), (1 << 60) + (1 << 58) + (1 << 62) + (1 << 59)),
    (((1 << 21) - 1, (1 << 21) - 1, (1 << 21) - 1), (1 << 63) - 1),
]


def test_morton_keys_written_out():
    pts = np.array([_pt(*q) for q, _ in CASES])
    keys = solver.morton_keys(pts, np.zeros(3), 1.0)
    for (q, ref), k in zip(CASES, keys):
        assert int(k) == ref, (q, int(k), ref)


def test_morton_keys_normalisation():
    # the same lattice points moved and scaled: corner lo, cube side ext
    pts = np.array([_pt(*q) for q, _ in CASES])
    lo, ext = np.array([-3.0, 2.0, 0.5]), 7.5
    keys = solver.morton_keys(lo + ext * pts, lo, ext)
    assert [int(k) for k in keys] == [ref for _, ref in CASES]


def test_morton_order_of_lattice_points():
    # eight cube corners of the first octree level in Z order
    q = [(0, 0, 0), (1, 0, 0), (0, 1, 0), (1, 1, 0), (0, 0, 1), (1, 0, 1), (0, 1, 1), (1, 1, 1)]
    half = 1 << 20
    pts = np.array([_pt(a * half, b * half, c * half) for a, b, c in q])
    perm = np.random.default_rng(5).permutation(8)
    keys = solver.morton_keys(pts[perm], np.zeros(3), 1.0)
    assert list(perm[np.argsort(keys, kind="stable")]) == list(range(8))
