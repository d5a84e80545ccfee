"""System-level pins for the oracle: Newton's third law and angular momentum
over a whole periodic system, translation and 90-degree rotation
invariance, relabelling, and the lists (all-pairs == cell list, bitwise)."""
import numpy as np
import pytest

import oracle as O
from paper_1607_02427_amd import inputs as I


def _systems():
    return [I.cubes_3d_contact(n_side=4), I.squares_2d_contact(), I.dimer_gas("octahedron", 64),
            I.dimer_gas("tetrahedron", 64), I.dimer_gas("pentagon", 64, dim=2),
            I.dimer_gas("lprism", 32, quad_h=0.05)]


def _axial(W):
    W = W.reshape(3, 3)
    return np.array([W[1, 2] - W[2, 1], W[2, 0] - W[0, 2], W[0, 1] - W[1, 0]])


@pytest.mark.parametrize("k", range(6))
def test_system_newton_and_angular_momentum(k):
    s = _systems()[k]
    r = O.forces(s, mode=1)
    assert r["stats"]["feature_in"] > 0
    Fs = np.abs(r["F"]).max() + 1.0
    assert np.abs(r["F"].sum(axis=0)).max() < 1e-10 * Fs * s.n
    # sum_i tau_i + sum_{i<j} r_ij x F_ij = 0; the second term is the axial part of sum W_i
    L = r["T"].sum(axis=0) + _axial(r["W"].sum(axis=0))
    assert np.abs(L).max() < 1e-10 * Fs * s.n


@pytest.mark.parametrize("k", range(6))
def test_all_pairs_equals_cell_list_forces(k):
    s = _systems()[k]
    a = O.forces(s, mode=0)
    b = O.forces(s, mode=1)
    for key in ("F", "T", "U", "W"):
        assert np.array_equal(a[key], b[key])


@pytest.mark.parametrize("k", [0, 1, 2])
def test_translation_invariance(k):
    s = _systems()[k]
    r0 = O.forces(s)
    t = s.copy()
    shift = np.array([3.3, -1.7, 0.9 if s.dim == 3 else 0.0])
    t.x = (t.x + shift) % t.box
    if s.dim == 2:
        t.x[:, 2] = 0.0
    r1 = O.forces(t)
    Fs = np.abs(r0["F"]).max()
    assert np.abs(r1["F"] - r0["F"]).max() < 1e-9 * Fs
    assert np.abs(r1["T"] - r0["T"]).max() < 1e-9 * Fs
    assert np.abs(r1["U"] - r0["U"]).max() < 1e-9 * np.abs(r0["U"]).max()


def _qmul(a, b):
    w1, x1, y1, z1 = a.T
    w2, x2, y2, z2 = b.T
    return np.stack([w1 * w2 - x1 * x2 - y1 * y2 - z1 * z2, w1 * x2 + x1 * w2 + y1 * z2 - z1 * y2,
                     w1 * y2 - x1 * z2 + y1 * w2 + z1 * x2, w1 * z2 + x1 * y2 - y1 * x2 + z1 * w2], axis=-1)


@pytest.mark.parametrize("k", [0, 1, 2])
def test_quarter_turn_invariance(k):
    """Rotating the whole periodic system by 90 degrees about z (an exact
    permutation of box axes) rotates F, tau and W and leaves U unchanged."""
    s = _systems()[k]
    r0 = O.forces(s)
    t = s.copy()
    Lb = s.box[0]
    x = s.x.copy()
    t.x[:, 0] = (Lb - x[:, 1]) % Lb
    t.x[:, 1] = x[:, 0]
    Rz = np.array([[0.0, -1, 0], [1, 0, 0], [0, 0, 1]])
    qz = np.tile([np.cos(np.pi / 4), 0, 0, np.sin(np.pi / 4)], (s.n, 1))
    t.q = _qmul(qz, s.q)
    r1 = O.forces(t)
    Fs = np.abs(r0["F"]).max()
    assert np.abs(r1["F"] - r0["F"] @ Rz.T).max() < 1e-9 * Fs
    assert np.abs(r1["T"] - r0["T"] @ Rz.T).max() < 1e-9 * Fs
    assert np.abs(r1["U"] - r0["U"]).max() < 1e-9 * np.abs(r0["U"]).max()
    W0 = r0["W"].reshape(-1, 3, 3)
    W1 = r1["W"].reshape(-1, 3, 3)
    assert np.abs(W1 - Rz @ W0 @ Rz.T).max() < 1e-9 * np.abs(W0).max()


def test_relabelling_permutes_outputs():
    s = _systems()[0]
    r0 = O.forces(s)
    perm = np.random.default_rng(9).permutation(s.n)
    t = s.copy()
    t.x, t.q, t.shape_id = s.x[perm], s.q[perm], s.shape_id[perm]
    r1 = O.forces(t)
    for key in ("F", "T", "U", "W"):
        assert np.allclose(r1[key], r0[key][perm], rtol=1e-12, atol=1e-12 * np.abs(r0[key]).max())


@pytest.mark.parametrize("k", range(6))
def test_lists_all_pairs_equals_cells(k):
    s = _systems()[k]
    osys = O.OracleSystem.of(s)
    rl = osys.r_list(0.3)
    a, na, ma = O.nbr_list(s, rl, cap=96, mode=0)
    b, nb, mb = O.nbr_list(s, rl, cap=96, mode=1)
    assert ma == mb and ma <= 96
    assert np.array_equal(na, nb)
    for i in range(s.n):
        assert np.array_equal(a[: na[i], i], b[: nb[i], i])
        assert np.all(np.diff(a[: na[i], i]) > 0)
    # symmetric: j in row i  <=>  i in row j
    pairs = {(i, int(j)) for i in range(s.n) for j in a[: na[i], i]}
    assert all((j, i) in pairs for i, j in pairs)


def test_cell_list_definition():
    s = I.cubes_3d(n_side=6)
    osys = O.OracleSystem.of(s)
    rl = osys.r_list(0.3)
    nc, cs, cp = O.cell_list(s, rl)
    assert np.array_equal(nc, np.floor(s.box / rl).astype(int))
    w = s.box / nc
    c = np.minimum(np.floor(s.x / w).astype(int), nc - 1)
    lin = c[:, 0] + nc[0] * (c[:, 1] + nc[1] * c[:, 2])
    for cell in range(int(np.prod(nc))):
        members = cp[cs[cell]:cs[cell + 1]]
        assert np.array_equal(members, np.flatnonzero(lin == cell))


def test_list_radius_definition():
    """r_list = 2 R_max + 2^(1/6) (2 r_max) + skin."""
    s = I.cubes_3d(n_side=4)
    rl = O.OracleSystem.of(s).r_list(0.3)
    assert rl == pytest.approx(2 * np.sqrt(0.75) + 1.122462048309373 * 0.3 + 0.3, rel=1e-15)


def test_nbr_list_capacity_reports_overflow():
    s = I.cubes_3d_contact(n_side=4)
    rl = O.OracleSystem.of(s).r_list(0.3)
    _, n_nbr, maxrow = O.nbr_list(s, rl, cap=4, mode=1)
    assert maxrow > 4 and n_nbr.max() == 4
