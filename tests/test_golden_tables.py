"""Checks against the tables the paper prints (fixtures under tests/golden/)."""
import math
import os

import numpy as np
import pytest

import workloads as wl
from oracle import asn_oracle as o

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _icosahedron():
    rows = [l for l in open(os.path.join(GOLDEN, "icosahedron_order2.txt"))
            if l.strip() and not l.startswith("#")]
    a = np.array([[float(v) for v in l.split(",")] for l in rows])
    return a[:, :3], a[:, 3]


def test_icosahedron_table_weights_and_symmetry():
    om, w = _icosahedron()
    assert om.shape == (12, 3)
    assert abs(w.sum() - 4 * math.pi) < 1e-14           # Appendix A: weights sum to 4 pi
    assert np.allclose(np.linalg.norm(om, axis=1), 1.0, atol=1e-15)
    for q in range(12):                                  # central symmetry, equal weights
        m = np.where(np.all(np.abs(om + om[q]) < 1e-15, axis=1))[0]
        assert m.size == 1 and w[m[0]] == w[q]
    assert abs(np.dot(w, om[:, 0])) < 1e-14 and abs(np.dot(w, om[:, 2])) < 1e-14


@pytest.mark.parametrize("mode", ["row", "sym"])
def test_kernel_on_icosahedron_table(mode):
    # The oracle's kernel on the paper's own order-2 set (eps = beta / N_q, beta = 4.5).
    om, w = _icosahedron()
    K = o.as_kernel_matrix(om, w, o.kernel_width(12, 4.5), mode)
    assert np.max(np.abs(K.sum(axis=1) - 1)) < 1e-14
    if mode == "sym":
        assert np.max(np.abs(w @ K - w)) < 1e-14


def test_lattice_materials_match_table():
    rows = [l.split(",") for l in open(os.path.join(GOLDEN, "lattice_materials.txt"))
            if l.strip() and not l.startswith("#")]
    table = {r[0].strip(): tuple(float(v) for v in r[1:]) for r in rows}
    p = wl.checkerboard(70, n_polar=2)
    assert (p.x_min, p.x_max, p.y_min, p.y_max, p.t_final) == (0.0, 7.0, 0.0, 7.0, 3.2)
    centre = (35, 35)
    assert (p.sigma_a[centre], p.sigma_s[centre]) == table["orange"][:2]
    assert p.source[centre] * 4 * math.pi == pytest.approx(table["orange"][2], rel=1e-7)
    seen = set()
    for j in range(70):
        for i in range(70):
            key = (float(p.sigma_a[j, i]), float(p.sigma_s[j, i]))
            seen.add(key)
            if p.source[j, i] == 0:
                assert key in {table["white"][:2], table["black"][:2]}
    assert seen == {table["white"][:2], table["black"][:2]}
