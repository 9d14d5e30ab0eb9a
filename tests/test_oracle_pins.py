"""Pins of three oracle rules that the solver tests alone would not catch.

* overlap growth (oracle.ddm.overlap_tets): one vertex-adjacency layer around one interior
  cube of the Kuhn lattice holds exactly 120 tets, counted by hand below; a second layer is
  checked against a plain set-based growth written here;
* partition-of-unity owner (oracle.ddm.owners): a dof shared by several subdomains belongs to
  the lowest subdomain id, checked on a two-cube mesh whose interface dofs are counted by hand,
  under two labellings;
* attenuation (oracle.fem.wavenumber, Q branch): the complex velocity c = v (1 + i / (2 Q)) of
  viscous media (paper: section "Tetrahedral finite element method") with the exp(+i omega t)
  convention gives k with Re k / (2 |Im k|) = Q (the usual definition of the quality factor
  for a plane wave), a hand value, decay of exp(-i k x), the lossless limit, and a positive
  imaginary part of x^H A x for fields that vanish on the boundary.

Hand count of one layer around cube c (tet = c' + {0, e_p0, e_p0 + e_p1, (1,1,1)} for the
six axis permutations p).  A tet of cube c' = c + d touches a corner c + b (b in {0,1}^3) iff
one of its reference vertices u has u_a = 0 where d_a = +1 and u_a = 1 where d_a = -1:
* d in {0,1}^3 (8 cubes): u = 0 works, all 6 tets: 48;
* d in {0,-1}^3 minus d = 0 (7 cubes): u = (1,1,1) works, all 6 tets: 42;
* mixed signs: only u = e_p0 (needs exactly one -1 axis, p0 = it) or u = e_p0 + e_p1 (needs
  exactly one +1 axis, p2 = it):
  - one +1, one -1, one 0 (6 cubes): 2 + 2 - 1 = 3 tets each: 18;
  - one +1, two -1 (3 cubes): p2 fixed, 2 tets each: 6;
  - two +1, one -1 (3 cubes): p0 fixed, 2 tets each: 6.
Total 48 + 42 + 18 + 6 + 6 = 120 (27 cubes visited).  Growing across faces instead would
give 6 + 12 = 18, no growth 6.
"""
import numpy as np

import workloads as w
from oracle import ddm, fem


def _lattice(n):
    xs = np.arange(n + 1, dtype=np.float64)
    return w.kuhn_mesh(xs, xs, xs)


def _grow_sets(tets, seed_tets, delta):
    """Plain growth: each layer adds every tet sharing a vertex with the current set."""
    cur = set(int(t) for t in seed_tets)
    for _ in range(delta):
        verts = set(int(v) for t in cur for v in tets[t])
        cur = cur | {t for t in range(tets.shape[0]) if verts.intersection(int(v) for v in tets[t])}
    return np.array(sorted(cur))


def test_kuhn_cube_corner_incidence():
    """The fixture: corners c and c + (1,1,1) lie in all six tets of a cube, the other six
    corners in two each."""
    tets, coords = _lattice(1)
    cnt = np.bincount(tets.ravel(), minlength=8)
    diag = [0, 7]  # vertex ids of (0,0,0) and (1,1,1)
    assert list(cnt[diag]) == [6, 6]
    assert sorted(np.delete(cnt, diag)) == [2] * 6


def test_overlap_one_layer_hand_count():
    n = 5
    tets, coords = _lattice(n)
    cube = np.arange(tets.shape[0]) // 6
    c0 = 2 + n * (2 + n * 2)  # interior cube (2, 2, 2)
    part = np.where(cube == c0, 0, 1).astype(np.int32)
    nv = coords.shape[0]
    assert ddm.overlap_tets(tets, nv, part, 0, 0).size == 6
    one = ddm.overlap_tets(tets, nv, part, 0, 1)
    assert one.size == 120
    # every added tet lies in one of the 27 cubes around c0
    ci, cj, ck = cube[one] % n, (cube[one] // n) % n, cube[one] // (n * n)
    assert np.all(np.abs(ci - 2) <= 1) and np.all(np.abs(cj - 2) <= 1) and np.all(np.abs(ck - 2) <= 1)
    assert np.unique(cube[one]).size == 27
    np.testing.assert_array_equal(one, _grow_sets(tets, np.nonzero(part == 0)[0], 1))


def test_overlap_two_layers_contains_one():
    n = 6
    tets, coords = _lattice(n)
    rng = np.random.default_rng(3)
    part = rng.integers(0, 4, tets.shape[0] // 6).repeat(6).astype(np.int32)
    nv = coords.shape[0]
    for i in range(4):
        one = ddm.overlap_tets(tets, nv, part, i, 1)
        two = ddm.overlap_tets(tets, nv, part, i, 2)
        assert np.all(np.isin(one, two)) and two.size > one.size
        np.testing.assert_array_equal(two, _grow_sets(tets, np.nonzero(part == i)[0], 2))


def _two_cubes():
    tets, coords = w.kuhn_mesh([0.0, 1.0, 2.0], [0.0, 1.0], [0.0, 1.0])
    return fem.Mesh(tets, coords)


def test_owner_is_lowest_subdomain_id():
    """Cube 0 (x < 1) and cube 1 (x > 1): 4^3 dofs each, 16 shared on the plane x = 1."""
    mesh = _two_cubes()
    assert mesh.n == 7 * 4 * 4
    d0, d1 = set(mesh.tet_dofs[:6].ravel().tolist()), set(mesh.tet_dofs[6:].ravel().tolist())
    shared = np.array(sorted(d0 & d1))
    only0, only1 = np.array(sorted(d0 - d1)), np.array(sorted(d1 - d0))
    assert len(d0) == len(d1) == 64 and shared.size == 16
    for lab0, lab1 in ((0, 1), (1, 0), (2, 5), (5, 2)):
        part = np.repeat([lab0, lab1], 6).astype(np.int32)
        own = ddm.owners(mesh, part, 6)
        assert np.all(own[shared] == min(lab0, lab1))
        assert np.all(own[only0] == lab0) and np.all(own[only1] == lab1)


def test_wavenumber_quality_factor():
    om = 2 * np.pi
    # hand value: v = 2, Q = 50, f = 1 -> c = 2 + 0.02 i, k = 2 pi / c = pi (1 - 0.01 i) / 1.0001
    k = fem.wavenumber(np.array([2.0]), 1.0, np.array([50.0]))[0]
    assert abs(k - np.pi * (1 - 0.01j) / 1.0001) <= 1e-15 * abs(k)
    for Q in (5.0, 80.0, 200.0, 1e4):
        k = fem.wavenumber(np.array([3.0]), 2.0, np.array([Q]))[0]
        assert k.imag < 0 and k.real > 0
        np.testing.assert_allclose(k.real / (2 * abs(k.imag)), Q, rtol=1e-12)
        assert abs(np.exp(-1j * k * 1.0)) < 1.0  # an outgoing wave decays with distance
    k = fem.wavenumber(np.array([3.0]), 2.0, np.array([1e300]))[0]
    assert abs(k - om * 2.0 / 3.0) <= 1e-15 * abs(k)
    np.testing.assert_array_equal(fem.wavenumber(np.array([3.0]), 2.0), [om * 2.0 / 3.0 + 0j])


def test_attenuating_operator_absorbs_inside():
    """For x vanishing on the boundary, Im(x^H A x) = -Im(k^2) x^H M x > 0 with attenuation
    (no boundary term), and 0 without it."""
    p = w.unit_cube_problem(3, freq=1.5)
    mesh = fem.Mesh(p.tets, p.coords, p.face_bc)
    xyz = fem.dof_coordinates(mesh.tets, mesh.coords, mesh.tet_dofs, mesh.n)
    inner = np.all((xyz > 1e-9) & (xyz < 1 - 1e-9), axis=1)
    rng = np.random.default_rng(11)
    x = (rng.standard_normal(mesh.n) + 1j * rng.standard_normal(mesh.n)) * inner
    _, M, _ = fem.assemble_parts(mesh)
    mass = np.vdot(x, M @ x).real
    A0 = fem.assemble_operator(mesh, p.velocity, p.freq)
    assert abs(np.vdot(x, A0 @ x).imag) <= 1e-12 * abs(np.vdot(x, A0 @ x))
    for Q in (20.0, 100.0):
        A = fem.assemble_operator(mesh, p.velocity, p.freq, np.full(mesh.tets.shape[0], Q))
        k = 2 * np.pi * p.freq / p.velocity[0] / (1 + 0.5j / Q)
        im = np.vdot(x, A @ x).imag
        assert im > 0
        np.testing.assert_allclose(im, -(k * k).imag * mass, rtol=1e-10)


def test_smooth_pou_hand_values_and_unity():
    """Smooth partition of unity on two cubes.  Overlap 0: the 16 interface dofs get 1/2 in
    each subdomain, the others 1.  Overlap 1: every tet of one cube touches the interface
    vertex shared with the other, so each subdomain holds both cubes; a dof of cube 0 off the
    interface has layer 0 in subdomain 0 and 1 in subdomain 1: raw weights 1 and 1/2,
    normalised 2/3 and 1/3.  The weights sum to 1 at every dof."""
    mesh = _two_cubes()
    part = np.repeat([0, 1], 6).astype(np.int32)
    d0, d1 = set(mesh.tet_dofs[:6].ravel().tolist()), set(mesh.tet_dofs[6:].ravel().tolist())
    shared = np.array(sorted(d0 & d1))
    only0 = np.array(sorted(d0 - d1))
    for delta in (0, 1):
        subs, own = ddm.build_subdomains(mesh, np.ones(12), 0.3, None, part, 2, delta)
        wts = ddm.smooth_pou(mesh, part, 2, delta, subs)
        acc = np.zeros(mesh.n)
        for sd, wi in zip(subs, wts):
            acc[sd.gdofs] += wi
            assert np.all(wi > 0) and np.all(wi <= 1)
        np.testing.assert_allclose(acc, 1.0, rtol=0, atol=1e-15)
        full0 = np.zeros(mesh.n)
        full0[subs[0].gdofs] = wts[0]
        np.testing.assert_allclose(full0[shared], 0.5, rtol=0, atol=1e-15)
        np.testing.assert_allclose(full0[only0], 1.0 if delta == 0 else 2.0 / 3.0, rtol=0, atol=1e-15)
    # a larger cut with two overlap layers: weights still sum to 1 everywhere
    tets, coords = _lattice(6)
    m6 = fem.Mesh(tets, coords)
    part6 = w.box_partition(6, 6, 6, 3, 2, 1)
    subs, own = ddm.build_subdomains(m6, np.ones(tets.shape[0]), 0.3, None, part6, 6, 2)
    acc = np.zeros(m6.n)
    for sd, wi in zip(subs, ddm.smooth_pou(m6, part6, 6, 2, subs)):
        acc[sd.gdofs] += wi
    np.testing.assert_allclose(acc, 1.0, rtol=0, atol=1e-15)
