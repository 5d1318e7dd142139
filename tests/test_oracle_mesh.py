"""Pins of the oracle's mesh, node numbering and tagger (CPU)."""
import os

import numpy as np
import pytest

from oracle import mesh, fem

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.mark.parametrize("n", [1, 2, 3])
def test_entity_counts_brute_force(n):
    coords, tets = mesh.kuhn_mesh(n)
    V, E, F, T = mesh.entity_counts(n)
    e, f = mesh.count_entities(tets)
    assert (len(coords), e, f, len(tets)) == (V, E, F, T)
    assert V - E + F - T == 1          # Euler characteristic of a ball


@pytest.mark.parametrize("n", [1, 2, 4])
def test_volumes(n):
    coords, tets = mesh.kuhn_mesh(n)
    v = mesh.tet_volumes(coords, tets)
    assert np.allclose(np.abs(v), 1.0 / (6 * n ** 3), rtol=0, atol=1e-15)
    assert abs(np.abs(v).sum() - 1.0) < 1e-13
    # vertex order is increasing global id, so the sign follows the permutation parity
    assert np.all(np.diff(tets, axis=1) > 0)


@pytest.mark.parametrize("p", [1, 2, 3, 4])
@pytest.mark.parametrize("n", [1, 2, 3])
def test_node_counts(n, p):
    if p == 4 and n == 3:
        pytest.skip("covered by smaller cases")
    coords, tets = mesh.kuhn_mesh(n)
    d = fem.Discretisation(coords, tets, p)
    V, E, F, T = mesh.entity_counts(n)
    hier = [V, V + E, V + 2 * E + F, V + 3 * E + 3 * F + T][p - 1]
    assert d.n_nodes == (p * n + 1) ** 3 == hier


def _read_golden(name):
    rows = {}
    with open(os.path.join(GOLDEN, name)) as fh:
        for line in fh:
            line = line.split("#")[0].split()
            if line:
                rows[tuple(line[:-1])] = float(line[-1])
    return rows


def test_paper_dof_counts_are_hierarchic():
    """Sec. 7 DOF counts: V, V+E, V+2E+F with the printed tet count give chi = 1."""
    g = _read_golden("dof_counts.txt")
    T = int(g[("tets",)])
    s1, s2, s3 = (int(g[("scalar", str(p))]) for p in (1, 2, 3))
    V = s1
    E = s2 - s1
    F = s3 - s1 - 2 * E
    assert V - E + F - T == 1
    for p in (1, 2, 3):
        assert int(g[("mech", str(p))]) == 3 * int(g[("scalar", str(p))])


def test_tagger_volume_fraction_converges():
    """Yarn volume fraction tends to 4 * pi * 0.2 * 0.06 (four elliptical sections)."""
    target = 4 * np.pi * 0.2 * 0.06
    errs = []
    for n in (16, 32, 64):
        coords, tets = mesh.kuhn_mesh(n)
        c = mesh.centroids(coords, tets)
        phase, axis = mesh.yarn_test(c[:, 0], c[:, 1], c[:, 2])
        frac = np.mean(phase > 0)
        errs.append(abs(frac - target))
        for y in range(1, 5):      # the four yarns are congruent
            assert abs(np.mean(phase == y) - target / 4) < 0.25 * target / 4
    assert errs[-1] < 0.01 * target
    assert errs[2] < errs[0]


def test_tagger_axes_and_no_overlap():
    n = 24
    coords, tets = mesh.kuhn_mesh(n)
    c = mesh.centroids(coords, tets)
    phase, axis = mesh.yarn_test(c[:, 0], c[:, 1], c[:, 2])
    yarn = phase > 0
    assert np.allclose(np.linalg.norm(axis[yarn], axis=1), 1.0)
    assert np.all(axis[~yarn] == 0.0)
    warp = (phase == 1) | (phase == 2)
    weft = (phase == 3) | (phase == 4)
    assert np.all(axis[warp, 1] == 0.0) and np.all(axis[warp, 0] > 0)
    assert np.all(axis[weft, 0] == 0.0) and np.all(axis[weft, 1] > 0)
    # count centroids that lie in more than one ellipse: the geometry has none
    hits = 0
    for y_idx in range(4):
        one = mesh.YARNS[y_idx:y_idx + 1]
        saved = mesh.YARNS
        try:
            mesh.YARNS = one
            ph, _ = mesh.yarn_test(c[:, 0], c[:, 1], c[:, 2])
        finally:
            mesh.YARNS = saved
        hits = hits + (ph > 0)
    assert hits.max() <= 1
    # centreline points are inside their yarn, a point 0.07 above is not
    for kind, off, phs in mesh.YARNS:
        x = np.linspace(0.0, 1.0, 17)
        zc = 0.5 + (1 if kind == 0 else -1) * 0.12 * np.sin(2 * np.pi * x + phs)
        if kind == 0:
            ph, _ = mesh.yarn_test(x, np.full_like(x, off), zc)
            ph2, _ = mesh.yarn_test(x, np.full_like(x, off), zc + 0.07)
        else:
            ph, _ = mesh.yarn_test(np.full_like(x, off), x, zc)
            ph2, _ = mesh.yarn_test(np.full_like(x, off), x, zc + 0.07)
        assert np.all(ph > 0) and np.all(ph2 == 0)


def test_yarn_test_values_and_tangents_agree_with_the_tagger():
    """The per-yarn ellipse values and tangents (used to judge exact-tie tags) give
    the tagger's phase (first yarn with f <= 1) and axis on every tet."""
    for n in (3, 8):
        c, t, ph, ax = mesh.plain_weave(n)
        cen = mesh.centroids(c, t)
        f = mesh.yarn_test_values(cen[:, 0], cen[:, 1], cen[:, 2])
        tang = mesh.yarn_tangents(cen[:, 0], cen[:, 1], cen[:, 2])
        inside = f <= 1.0
        first = np.where(inside.any(axis=1), inside.argmax(axis=1) + 1, 0)
        assert np.array_equal(first, ph)
        yarn = ph > 0
        assert np.allclose(tang[yarn, ph[yarn] - 1], ax[yarn], rtol=0, atol=1e-15)
        assert np.allclose(np.linalg.norm(tang, axis=-1), 1.0)
