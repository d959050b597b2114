"""Pins of the oracle's Reeb junction refinement (Section "Reeb Graph
Extraction": the second pass improves where the junctions sit; Section
"Introduction": a Reeb graph from a diffusion initiated at a detected
handle loop).  The reading: the initial pass again, started from the
vertices within the seed radius of the first kept handle loop's inside
vertices, ranked by hop distance from the smallest of them.  Pinned by
facts outside the oracle's arithmetic:

* a seed set of one vertex is the hop ball around it: every result equals
  the ordinary run from that vertex;
* on a torus of revolution the diffusion from a meridian handle loop runs
  around the tube both ways and the two fronts meet on the far side: the
  merge junction sits on the tube's core circle, opposite the handle loop;
* from a handle loop the pass still finds genus-many handle loops;
* a seed set that names no vertex of the mesh is refused.
"""
import math

import numpy as np
import pytest

import meshgen as mg


def test_single_vertex_set_is_the_ball(oracle_mod):
    for m in (mg.torus_grid(rng_seed=0), mg.multi_torus(2, 28, rng_seed=3)):
        a = oracle_mod.run(m.xyz, m.tri, seed_vertex=m.seed)
        b = oracle_mod.run(m.xyz, m.tri, seed_vertex=m.seed, seed_set=[m.seed])
        assert a.status == b.status == 0
        assert a.steps == b.steps
        assert np.array_equal(a.T, b.T) and np.array_equal(a.rnd, b.rnd)
        assert np.array_equal(a.parent, b.parent) and np.array_equal(a.events, b.events)
        assert np.array_equal(a.loop_he, b.loop_he)


def test_torus_merge_junction_on_the_core_opposite_the_loop(oracle_mod):
    R, r = 1.0, 0.4           # torus_grid's radii, axis z
    m = mg.torus_grid(rng_seed=0)
    first, second = oracle_mod.reeb_refined(m.xyz, m.tri, seed_vertex=m.seed)
    assert first.n_handles == 1 and second is not None
    assert second.status == 0 and second.n_handles == 1
    ss = oracle_mod.refinement_seed_set(first)
    # the seed region is an annulus: two initial fronts
    nodes, edges = second.reeb()
    assert sum(1 for e in edges if e[0] == 0) == 2
    merges = [n for n in nodes[1:] if n[0] == 2]
    assert merges
    p = np.array(merges[0][6:9])
    assert math.hypot(math.hypot(p[0], p[1]) - R, p[2]) < 0.1 * r
    c = m.xyz[ss].mean(axis=0)
    d = abs((math.degrees(math.atan2(p[1], p[0]) - math.atan2(c[1], c[0])) + 180.0) % 360.0 - 180.0)
    assert abs(d - 180.0) < 15.0, d


@pytest.mark.parametrize("make,g", [
    (lambda: mg.multi_torus(2, 28, rng_seed=3), 2),
    (lambda: mg.pretzel(40, rng_seed=5), 3),
    (lambda: mg.multi_torus(4, 40, rng_seed=4), 4),
])
def test_refinement_pass_finds_the_genus(oracle_mod, make, g):
    m = make()
    first, second = oracle_mod.reeb_refined(m.xyz, m.tri, seed_vertex=m.seed)
    assert first.n_handles == g
    assert second is not None and second.status == 0
    assert second.n_handles == g
    assert len(second.tunnel_loops()) == g


def test_seed_set_out_of_range_is_refused(oracle_mod):
    m = mg.torus_grid(rng_seed=0)
    r = oracle_mod.run(m.xyz, m.tri, seed_vertex=0, seed_set=[0, m.nv])
    assert r.status == -1
