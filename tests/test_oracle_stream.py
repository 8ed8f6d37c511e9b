"""Pins for the oracle's streaming on the two-sublattice bcc grid (Sec. IV)
and for its collision (Sec. II)."""
import numpy as np
import pytest

from paper_1909_08406_amd import workloads as wl


def _brute_force_pull(c, nx, ny, nz):
    """Source of every (q, node) by searching all nodes for the one whose
    position equals (destination position - c_q) modulo the box."""
    x, y, z = wl.positions(nx, ny, nz)
    pos = np.stack([x, y, z], 1)
    box = np.array([nx, ny, nz], dtype=float)
    n = pos.shape[0]
    src = np.zeros((41, n), dtype=np.int64)
    for q in range(41):
        want = np.mod(pos - c[q], box)
        for i in range(n):
            d = np.abs(np.mod(pos - want[i] + 0.5 * box, box) - 0.5 * box).sum(1)
            hit = np.nonzero(d < 1e-9)[0]
            assert hit.size == 1
            src[q, i] = hit[0]
    return src


@pytest.mark.parametrize("dims", [(1, 1, 1), (2, 2, 2), (3, 2, 1), (4, 3, 5), (5, 1, 2)])
def test_pull_map_equals_position_search(orc, dims):
    c, _, _ = orc.lattice()
    assert np.array_equal(orc.pull_map(*dims), _brute_force_pull(c, *dims))


@pytest.mark.parametrize("dims", [(1, 1, 1), (3, 2, 1), (6, 5, 4), (7, 3, 2)])
def test_push_is_inverse_of_pull(orc, dims):
    pull = orc.pull_map(*dims)
    push = orc.push_map(*dims)
    n = pull.shape[1]
    for q in range(41):
        assert np.array_equal(np.sort(pull[q]), np.arange(n))  # a permutation
        assert np.array_equal(push[q][pull[q]], np.arange(n))  # push o pull = id
        assert np.array_equal(pull[q][push[q]], np.arange(n))


def test_pull_map_hand_checked_entries(orc):
    c, _, _ = orc.lattice()
    nx, ny, nz = 4, 4, 4
    pull = orc.pull_map(nx, ny, nz)
    nid = lambda s, x, y, z: ((s * nz + z) * ny + y) * nx + x
    q_half_ppp = 33  # (+1/2, +1/2, +1/2)
    q_half_mmm = 40  # (-1/2, -1/2, -1/2)
    q_sc2_px = 7     # (+2, 0, 0)
    assert tuple(c[q_half_ppp]) == (0.5, 0.5, 0.5)
    assert tuple(c[q_half_mmm]) == (-0.5, -0.5, -0.5)
    assert tuple(c[q_sc2_px]) == (2, 0, 0)
    # corner node (1,1,1) receives +half from the body node of cell (0,0,0)
    assert pull[q_half_ppp, nid(0, 1, 1, 1)] == nid(1, 0, 0, 0)
    # ... and -half from the body node of its own cell
    assert pull[q_half_mmm, nid(0, 1, 1, 1)] == nid(1, 1, 1, 1)
    # body node (3,3,3) (at 3.5) receives -half from corner (0,0,0) (= 4 mod 4)
    assert pull[q_half_mmm, nid(1, 3, 3, 3)] == nid(0, 0, 0, 0)
    # sc-2 wraps by two cells
    assert pull[q_sc2_px, nid(1, 1, 2, 3)] == nid(1, 3, 2, 3)
    assert pull[0, nid(1, 2, 3, 0)] == nid(1, 2, 3, 0)


def test_streaming_only_moves_populations(orc):
    """omega = 0: one step is a pure push along the links."""
    nx, ny, nz = 3, 4, 2
    F = wl.random_state(nx, ny, nz, seed=7)
    _, _, t0 = orc.lattice()
    f = orc.init(nx, ny, nz, *F.absolute(t0))
    g = orc.run(nx, ny, nz, 0.0, f, 1)
    push = orc.push_map(nx, ny, nz)
    ref = np.zeros_like(f)
    for q in range(41):
        ref[q, push[q]] = f[q]
    assert np.array_equal(g, ref)


def test_collision_conserves_per_node(orc):
    nx, ny, nz = 3, 2, 2
    _, _, t0 = orc.lattice()
    F = wl.random_state(nx, ny, nz, seed=8, amp_u=0.15, amp_theta=0.08)
    f = orc.init(nx, ny, nz, *F.absolute(t0))
    # push it off equilibrium by streaming, then collide
    f = orc.run(nx, ny, nz, 0.0, f, 1)
    for omega in (0.6, 1.0, 1.0 / 0.51, 1.95):
        g = orc.collide_field(nx, ny, nz, omega, f)
        mf = orc.moment_fields(f)
        mg = orc.moment_fields(g)
        for k in range(5):
            assert np.max(np.abs(mg[k] - mf[k])) <= 2e-15 * max(1.0, np.max(np.abs(mf[k]))), k
        # and it moved the populations
        assert np.max(np.abs(g - f)) > 1e-6


def test_uniform_equilibrium_is_a_fixed_point(orc):
    nx, ny, nz = 3, 3, 2
    _, _, t0 = orc.lattice()
    n = 2 * nx * ny * nz
    one = np.ones(n)
    f = orc.init(nx, ny, nz, 1.2 * one, 0.05 * one, -0.02 * one, 0.01 * one, 1.03 * t0 * one)
    g = orc.run(nx, ny, nz, 1.0 / 0.6, f, 5)
    assert np.max(np.abs(g - f)) < 4e-15


def test_global_conservation_over_steps(orc):
    nx, ny, nz = 6, 5, 4
    _, _, t0 = orc.lattice()
    F = wl.random_state(nx, ny, nz, seed=9)
    f = orc.init(nx, ny, nz, *F.absolute(t0))
    tot0 = orc.totals(f)
    g = orc.run(nx, ny, nz, 1.0 / 0.55, f, 20)
    tot = orc.totals(g)
    scale = np.array([tot0[0], tot0[0], tot0[0], tot0[0], tot0[4]])
    assert np.max(np.abs(tot - tot0) / scale) < 1e-13
