"""Pins of the oracle's lattice tables (Sec. II.A, Eq. (1)-(2); Appendix A.1).

The tables are typed from the paper; these tests check them against what the
mathematics fixes: the D3Q19 set, lattice isotropy, and the textbook
d'Humieres polynomial basis written here as polynomials of c.
"""
import itertools

import numpy as np

import oracle as O

CS2 = 1.0 / 3.0


def test_velocity_set_is_d3q19_in_lexicographic_zyx_order():
    t = O.tables()
    c = t["c"]
    expect = [v for v in itertools.product([-1, 0, 1], repeat=3) if sum(abs(a) for a in v) <= 2]
    # (c_z, c_y, c_x) lexicographic order; stored as (c_x, c_y, c_z)
    expect = [(v[2], v[1], v[0]) for v in expect]
    assert [tuple(r) for r in c] == expect
    assert len(c) == 19


def test_opposite_and_mirror_indices():
    t = O.tables()
    c = t["c"]
    assert list(t["opp"]) == [18 - i for i in range(19)]
    for i in range(19):
        j = t["refl"][i]
        assert tuple(c[j]) == (c[i][0], -c[i][1], c[i][2])


def test_weights_lattice_sums_and_isotropy():
    t = O.tables()
    c = t["c"].astype(float)
    w = t["w"]
    assert abs(w.sum() - 1) < 1e-15
    assert np.abs(w @ c).max() < 1e-16
    assert np.allclose(np.einsum("i,ia,ib->ab", w, c, c), CS2 * np.eye(3), atol=1e-16)
    assert np.abs(np.einsum("i,ia,ib,ic->abc", w, c, c, c)).max() < 1e-16
    d = np.eye(3)
    iso = CS2 ** 2 * (np.einsum("ab,cd->abcd", d, d) + np.einsum("ac,bd->abcd", d, d)
                      + np.einsum("ad,bc->abcd", d, d))
    assert np.allclose(np.einsum("i,ia,ib,ic,id->abcd", w, c, c, c, c), iso, atol=1e-16)


def _textbook_rows(c):
    """d'Humieres et al. (2002) D3Q19 moment polynomials, in the paper's row order."""
    cx, cy, cz = c[:, 0], c[:, 1], c[:, 2]
    c2 = cx * cx + cy * cy + cz * cz
    return np.array([
        np.ones_like(cx),
        19 * c2 - 30,
        (21 * c2 * c2 - 53 * c2 + 24) / 2,
        cx, (5 * c2 - 9) * cx,
        cy, (5 * c2 - 9) * cy,
        cz, (5 * c2 - 9) * cz,
        3 * cx * cx - c2,
        (3 * c2 - 5) * (3 * cx * cx - c2),
        cy * cy - cz * cz,
        (3 * c2 - 5) * (cy * cy - cz * cz),
        cx * cy, cy * cz, cx * cz,
        (cy * cy - cz * cz) * cx,
        (cz * cz - cx * cx) * cy,
        (cx * cx - cy * cy) * cz,
    ])


def test_M_rows_equal_textbook_polynomials():
    t = O.tables()
    assert np.array_equal(t["M"], _textbook_rows(t["c"].astype(float)))


def test_M_orthogonal_rows_and_inverse():
    t = O.tables()
    M = t["M"]
    G = M @ M.T
    D = np.array([19, 2394, 252, 10, 40, 10, 40, 10, 40, 36, 72, 12, 24, 4, 4, 4, 8, 8, 8], float)
    assert np.array_equal(G, np.diag(D))
    assert np.abs(M @ t["Minv"] - np.eye(19)).max() < 1e-14
    assert np.abs(t["Minv"] - M.T / D).max() < 1e-15
