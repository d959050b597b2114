"""Input generators: the slab-streamed extraction equals the whole-grid one,
and the strut lattices are closed surfaces of the genus their graph fixes
(struts - nodes + 1)."""
import numpy as np
import pytest

import meshgen as mg


def test_slab_extraction_equals_whole_grid():
    f = mg.pretzel_sdf()
    glo, ghi = mg._fitted_grid((-2.95, -1.35, -0.35), (2.95, 1.35, 0.35), (36, 30, 20), 2)
    a = mg.marching_tets(f, glo, ghi, (36, 30, 20))
    for slab in (1, 5, 64):
        b = mg.marching_tets_slabs(lambda x, Y, Z: f(np.full_like(Y, x), Y, Z), glo, ghi, (36, 30, 20), slab=slab)
        assert np.array_equal(a.xyz, b.xyz)
        ta = np.sort(np.sort(a.tri, axis=1), axis=0)
        tb = np.sort(np.sort(b.tri, axis=1), axis=0)
        assert np.array_equal(np.unique(ta, axis=0), np.unique(tb, axis=0)) and a.nf == b.nf


@pytest.mark.parametrize("n,grid", [(1, 20), (2, 36), (3, 52), (10, 128)])
def test_lattice_genus(n, grid):
    m = mg.lattice(n, grid, rng_seed=0)
    chi = mg.euler_characteristic(m.tri, m.nv)
    assert (2 - chi) // 2 == mg.lattice_genus(n)
    # closed: every directed edge appears once and its reverse once
    t = m.tri.astype(np.int64)
    e = np.concatenate([t[:, [0, 1]], t[:, [1, 2]], t[:, [2, 0]]])
    k = e[:, 0] * m.nv + e[:, 1]
    kr = e[:, 1] * m.nv + e[:, 0]
    assert np.unique(k).size == k.size
    assert np.array_equal(np.sort(k), np.sort(kr))
    assert 0 <= m.seed < m.nv


def test_lattice_genus_formula():
    # the config's 10^3-cell lattice: 3630 struts on 1331 nodes
    assert mg.lattice_genus(10) == 3630 - 1331 + 1 == 2300


def test_uv_sphere_is_closed_outward_with_wide_poles():
    m = mg.uv_sphere(30, 40, rng_seed=0)
    assert mg.euler_characteristic(m.tri, m.nv) == 2
    t = m.tri.astype(np.int64)
    e = np.concatenate([t[:, [0, 1]], t[:, [1, 2]], t[:, [2, 0]]])
    k = e[:, 0] * m.nv + e[:, 1]
    assert np.unique(k).size == k.size
    assert np.array_equal(np.sort(k), np.sort(e[:, 1] * m.nv + e[:, 0]))
    deg = np.bincount(e[:, 0], minlength=m.nv)
    assert deg[0] == 40 and deg[-1] == 40 and set(deg[1:-1].tolist()) == {5, 6}
    p = m.xyz[t]
    n = np.cross(p[:, 1] - p[:, 0], p[:, 2] - p[:, 0])
    assert (np.einsum("ij,ij->i", n, p.mean(axis=1)) > 0).all()
