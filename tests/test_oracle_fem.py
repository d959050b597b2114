"""Pins of the oracle's cotangent finite-element operator (Section
"Mathematical representation and data structure", "Implementation details":
the standard linear finite-element discretisation of the Laplacian), from
facts outside the oracle:

* the stiffness entries equal an independent P1 assembly from the gradients
  of the hat functions over each triangle, and the lumped masses equal the
  row sums of the consistent P1 mass matrix;
* on a mesh whose faces are all equilateral with one valence (octahedron,
  icosahedron) the scaled operator is the uniform graph Laplacian: every
  coefficient is 1;
* on a fine sphere of radius r the unscaled operator maps the height z to
  about -2 z / r^2 (z is an eigenfunction of the Laplace-Beltrami operator
  with eigenvalue -2/r^2);
* the explicit step size is 50 over the largest absolute row sum of the
  scaled operator (the uniform case: 50 / max degree);
* a run with the operator on surfaces of known genus finds that many handle
  and tunnel loops, and on the octahedron it matches the uniform run.
"""
import math

import numpy as np
import pytest

import meshgen as mg


def _p1_assembly(xyz, tri):
    """Stiffness K (dict of edge -> -K_uv = cot weight) and lumped mass from
    hat-function gradients and the consistent mass matrix (per triangle
    area/12 * (1 + delta_ij)), assembled triangle by triangle."""
    nv = xyz.shape[0]
    W = {}
    mass = np.zeros(nv)
    for t in np.asarray(tri, dtype=np.int64):
        P = xyz[t]
        n = np.cross(P[1] - P[0], P[2] - P[0])
        A2 = np.linalg.norm(n)
        nh = n / A2
        # gradient of the hat of vertex i: (nh x e_i) / A2, e_i the edge
        # opposite i, oriented counter-clockwise
        G = np.array([np.cross(nh, P[(i + 2) % 3] - P[(i + 1) % 3]) / A2 for i in range(3)])
        area = 0.5 * A2
        for i in range(3):
            for j in range(i + 1, 3):
                key = (min(t[i], t[j]), max(t[i], t[j]))
                W[key] = W.get(key, 0.0) - area * float(G[i] @ G[j])
        Mc = area / 12.0 * (np.ones((3, 3)) + np.eye(3))
        mass[t] += Mc.sum(axis=1)
    return W, mass


def _oracle_pairs(xyz, tri):
    from oracle import fem_operator
    rp, adj, g, mass, sigma, dmax = fem_operator(xyz, tri)
    src = np.repeat(np.arange(xyz.shape[0]), np.diff(rp))
    return src, adj.astype(np.int64), g, mass, sigma, dmax


def _meshes():
    pz = mg.pretzel(32, rng_seed=2)
    return [mg.torus_grid(rng_seed=0), mg.relaxed(pz, mg.pretzel_sdf(), 10), mg.icosphere(2)]


@pytest.mark.parametrize("i", range(3))
def test_fem_matches_p1_assembly(i):
    m = _meshes()[i]
    src, adj, g, mass, sigma, dmax = _oracle_pairs(m.xyz, m.tri)
    W, M = _p1_assembly(m.xyz, m.tri)
    assert np.allclose(mass, M, rtol=1e-12, atol=0)
    # the same coefficient from both ends of every edge, equal to the
    # assembled stiffness
    k = g * mass[src] / sigma
    ref = np.array([W[(min(a, b), max(a, b))] for a, b in zip(src.tolist(), adj.tolist())])
    assert np.allclose(k, ref, rtol=1e-10, atol=1e-13 * np.abs(ref).max())
    # lumped masses sum to the surface area; sigma is sqrt(3) x mean mass
    area = sum(0.5 * np.linalg.norm(np.cross(m.xyz[b] - m.xyz[a], m.xyz[c] - m.xyz[a])) for a, b, c in m.tri)
    assert math.isclose(mass.sum(), area, rel_tol=1e-12)
    assert math.isclose(sigma, math.sqrt(3.0) * area / m.nv, rel_tol=1e-12)
    # step rule: largest absolute row sum
    rows = np.zeros(m.nv)
    np.add.at(rows, src, np.abs(g))
    assert math.isclose(dmax, rows.max(), rel_tol=1e-13)


@pytest.mark.parametrize("mesh,val", [(mg.octahedron(), 4), (mg.icosphere(0), 5)])
def test_fem_is_the_graph_laplacian_on_equilateral_meshes(mesh, val):
    src, adj, g, mass, sigma, dmax = _oracle_pairs(mesh.xyz, mesh.tri)
    assert np.abs(g - 1.0).max() < 1e-14
    assert np.bincount(src).tolist() == [val] * mesh.nv
    assert abs(dmax - val) < 1e-13


def test_fem_sphere_height_is_an_eigenfunction():
    errs = []
    for sd in (2, 3, 4):
        m = mg.icosphere(sd)
        src, adj, g, mass, sigma, dmax = _oracle_pairs(m.xyz, m.tri)
        k = g * mass[src] / sigma
        z = m.xyz[:, 2]
        Lz = np.zeros(m.nv)
        np.add.at(Lz, src, k * (z[adj] - z[src]))
        Lz /= mass
        errs.append(np.mean(np.abs(Lz + 2.0 * z)))
        # Rayleigh quotient of the stiffness over the lumped mass: the
        # eigenvalue 2 / r^2 of the height function
        rq = 0.5 * np.sum(k * (z[adj] - z[src]) ** 2) / np.sum(mass * z * z)
        assert abs(rq - 2.0) < 1e-2
    assert errs[0] > errs[1] > errs[2] and errs[2] < 3e-3


def test_fem_first_step_matches_p1_step(oracle_mod):
    """One field step of a run with the finite-element operator equals an
    explicit Euler step built from the independent P1 assembly (step 50 over
    the largest absolute row sum, operator sqrt(3) x mean mass x M^-1 K)."""
    from _topo import hop_ball
    m = mg.relaxed(mg.pretzel(32, rng_seed=2), mg.pretzel_sdf(), 10)
    r = oracle_mod.run(m.xyz, m.tri, seed_vertex=m.seed, fem=1, max_steps=3, ckpt_steps=[1, 2])
    W, M = _p1_assembly(m.xyz, m.tri)
    sigma = math.sqrt(3.0) * M.sum() / m.nv
    keys = np.array(list(W.keys()), dtype=np.int64)
    w = np.array(list(W.values()))
    D = np.zeros(m.nv)
    np.add.at(D, keys[:, 0], np.abs(w))
    np.add.at(D, keys[:, 1], np.abs(w))
    D = sigma * D / M
    c = (50.0 / D.max()) * (0.25 / 2.0)
    a, wp, e = 1.0 / 25.0, (1.0 / 25.0) / 5.0, 1.0 / 30.0
    rho = (hop_ball(m.tri, m.nv, m.seed, 2) >= 0).astype(np.float64)
    for step in (1, 2):
        lap = np.zeros(m.nv)
        np.add.at(lap, keys[:, 0], w * (rho[keys[:, 1]] - rho[keys[:, 0]]))
        np.add.at(lap, keys[:, 1], w * (rho[keys[:, 0]] - rho[keys[:, 1]]))
        lap = sigma * lap / M
        x = rho + c * ((a * lap + wp * (2.0 * rho - 1.0)) + e * np.sqrt(np.clip(rho * (1.0 - rho), 0, None)))
        rho = np.clip(x, 0.0, 1.0)
        assert np.allclose(r.ckpt[step], rho, rtol=0, atol=1e-12), step


@pytest.mark.parametrize("case", ["sphere", "torus", "double_torus", "pretzel"])
def test_fem_run_finds_genus_many_loops(oracle_mod, case):
    if case == "sphere":
        m, g = mg.icosphere(3), 0
    elif case == "torus":
        m, g = mg.torus_grid(rng_seed=1), 1
    elif case == "double_torus":
        m, g = mg.relaxed(mg.multi_torus(2, 28, rng_seed=3), mg.sdf_union_tori([(-0.8, 0, 0), (0.8, 0, 0)]), 10), 2
    else:
        m, g = mg.relaxed(mg.pretzel(32, rng_seed=2), mg.pretzel_sdf(), 10), 3
    r = oracle_mod.run(m.xyz, m.tri, seed_vertex=m.seed, fem=1)
    assert r.status == 0
    assert r.genus == g
    assert r.n_handles == g and len(r.tunnel_loops()) == g
    assert r.n_inside == m.nv
