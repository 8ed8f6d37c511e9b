"""Pins for the oracle's lattice: the RD3Q41 velocity set and weights
(Sec. IV, Table I) and the seven weight constraints (Sec. III)."""
import itertools
import os

import numpy as np

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _table1():
    rows = []
    with open(os.path.join(GOLDEN, "table1_weights.txt")) as fh:
        for line in fh:
            if line.startswith("#") or not line.strip():
                continue
            parts = line.split()
            rows.append((parts[0], int(parts[-2]), float(parts[-1])))
    return rows


def _shells_by_hand():
    """The five moving shells written out from their definitions."""
    sc1 = [v for v in itertools.product((-1, 0, 1), repeat=3) if sorted(map(abs, v)) == [0, 0, 1]]
    sc2 = [tuple(2 * a for a in v) for v in sc1]
    fcc = [v for v in itertools.product((-1, 0, 1), repeat=3) if sorted(map(abs, v)) == [0, 1, 1]]
    bcc = list(itertools.product((-1, 1), repeat=3))
    half = [tuple(0.5 * a for a in v) for v in bcc]
    return [[(0, 0, 0)], sc1, sc2, fcc, bcc, half]


def test_velocity_set_is_41_in_six_shells(orc):
    c, w, _ = orc.lattice()
    assert c.shape == (41, 3)
    c2 = (c ** 2).sum(1)
    counts = {e: int(np.sum(np.isclose(c2, e))) for e in (0.0, 1.0, 4.0, 2.0, 3.0, 0.75)}
    assert counts == {0.0: 1, 1.0: 6, 4.0: 6, 2.0: 12, 3.0: 8, 0.75: 8}
    # shell order: rest, sc-1, sc-2, fcc-1, bcc-1, bcc-1/2
    expect = [0.0] + [1.0] * 6 + [4.0] * 6 + [2.0] * 12 + [3.0] * 8 + [0.75] * 8
    assert np.array_equal(c2, expect)
    # every velocity distinct, and the set equals the hand-written shells
    hand = sorted(v for sh in _shells_by_hand() for v in sh)
    assert sorted(map(tuple, c.tolist())) == sorted(map(lambda v: tuple(float(a) for a in v), hand))


def test_canonical_order_within_shells(orc):
    c, _, _ = orc.lattice()
    bounds = [(0, 1), (1, 7), (7, 13), (13, 25), (25, 33), (33, 41)]
    for a, b in bounds:
        rows = [tuple(r) for r in c[a:b].tolist()]
        assert rows == sorted(rows, reverse=True)
    assert tuple(c[1]) == (1, 0, 0) and tuple(c[6]) == (-1, 0, 0)
    assert tuple(c[33]) == (0.5, 0.5, 0.5) and tuple(c[40]) == (-0.5, -0.5, -0.5)


def test_weights_are_table_I(orc):
    c, w, _ = orc.lattice()
    c2 = (c ** 2).sum(1)
    for (name, count, weight), e in zip(_table1(), (1.0, 4.0, 2.0, 3.0, 0.75)):
        sel = np.isclose(c2, e)
        assert sel.sum() == count, name
        assert np.all(w[sel] == weight), name
    assert abs(w.sum() - 1.0) < 1e-15
    assert np.all(w > 0)


def test_seven_weight_constraints_hold(orc):
    res = orc.constraint_residuals()
    assert np.max(np.abs(res)) < 1e-14, res


def test_weights_solve_the_seven_constraints_independently(orc):
    """Solve the seven equations of Sec. III for (w0..w5, theta0) by Newton
    in numpy, from shell sums of the hand-written shells, and compare."""
    shells = [np.array(s, dtype=float) for s in _shells_by_hand()]

    def sums(fn):
        return np.array([np.sum([fn(v) for v in sh]) for sh in shells])

    A = np.array([
        sums(lambda v: 1.0),
        sums(lambda v: v[0] ** 2),
        sums(lambda v: v[0] ** 4),
        sums(lambda v: v[0] ** 2 * v[1] ** 2),
        sums(lambda v: v[0] ** 4 * v.dot(v)),
        sums(lambda v: v[0] ** 2 * v.dot(v) ** 2),
        sums(lambda v: v.dot(v) ** 4),
    ])

    def F(x):
        wv, t = x[:6], x[6]
        rhs = np.array([1.0, t, 3 * t ** 2, t ** 2, 21 * t ** 3, 35 * t ** 3, 945 * t ** 4])
        return A @ wv - rhs

    def J(x):
        t = x[6]
        d = -np.array([0.0, 1.0, 6 * t, 2 * t, 63 * t ** 2, 105 * t ** 2, 3780 * t ** 3])
        return np.hstack([A, d[:, None]])

    x = np.array([0.2, 0.05, 0.002, 0.006, 0.005, 0.05, 0.3])
    for _ in range(60):
        x = x - np.linalg.solve(J(x), F(x))
    assert np.max(np.abs(F(x))) < 1e-15
    c, w, theta0 = orc.lattice()
    c2 = (c ** 2).sum(1)
    per_shell = [w[np.isclose(c2, e)][0] for e in (0.0, 1.0, 4.0, 2.0, 3.0, 0.75)]
    assert np.allclose(per_shell, x[:6], rtol=1e-13, atol=0)
    assert abs(theta0 / x[6] - 1.0) < 1e-14
    assert abs(theta0 - 0.2948964908710634) < 2e-16 * 4


def _signed_perms():
    for perm in itertools.permutations(range(3)):
        for signs in itertools.product((-1, 1), repeat=3):
            yield perm, np.array(signs, dtype=float)


def test_closed_under_cubic_group(orc):
    c, w, _ = orc.lattice()
    key = {tuple(v): i for i, v in enumerate(c.tolist())}
    n = 0
    for perm, sg in _signed_perms():
        img = c[:, perm] * sg
        idx = [key[tuple(v)] for v in img.tolist()]
        assert sorted(idx) == list(range(41))
        assert np.array_equal(w[idx], w)
        n += 1
    assert n == 48


def test_isotropic_moments(orc):
    c, w, t = orc.lattice()
    d = np.eye(3)
    # odd moments vanish
    assert np.max(np.abs(w @ c)) < 1e-16
    m3 = np.einsum("q,qa,qb,qc->abc", w, c, c, c)
    assert np.max(np.abs(m3)) < 1e-16
    # second and fourth order are isotropic (Sec. II, the weight conditions)
    m2 = np.einsum("q,qa,qb->ab", w, c, c)
    assert np.allclose(m2, t * d, rtol=0, atol=1e-15)
    m4 = np.einsum("q,qa,qb,qc,qd->abcd", w, c, c, c, c)
    delta4 = (np.einsum("ab,cd->abcd", d, d) + np.einsum("ac,bd->abcd", d, d) + np.einsum("ad,bc->abcd", d, d))
    assert np.allclose(m4, t * t * delta4, rtol=0, atol=1e-15)
    # contracted sixth order: sum w c^2 c_a c_b c_c c_d = 7 theta0^3 Delta
    c2 = (c ** 2).sum(1)
    m6c = np.einsum("q,qa,qb,qc,qd->abcd", w * c2, c, c, c, c)
    assert np.allclose(m6c, 7 * t ** 3 * delta4, rtol=0, atol=1e-15)
    # eighth: sum w c^8 = 945 theta0^4
    assert abs(np.sum(w * c2 ** 4) / (945 * t ** 4) - 1) < 1e-14
