"""Oracle: P3 degrees of freedom, element matrices and global assembly (CPU, FP64).

TEST INFRASTRUCTURE ONLY: imported by tests/, the graft smoke check and bench.py's CPU
baseline leg; the product path never imports it.

Follows the paper's section "Tetrahedral finite element method": the Helmholtz equation
(eq. 1, (Delta + k^2) u = b with k = omega / c, c complex in viscous media) discretised with
continuous P3 Lagrange elements on tetrahedra into A u = b (eq. 2), with first-order
absorbing conditions on the vertical and bottom faces and a homogeneous Dirichlet
condition on the top face.

Readings where the paper is silent (listed in the design doc):
* time convention exp(+i w t): c = v (1 + i/(2Q)), outgoing waves exp(-i k r), absorbing
  condition d_n u + i k u = g, weak form A = K - k^2 M + i k M_G (complex symmetric);
* v and Q are constant per tet (the caller samples them), so all integrals are exact;
* Dirichlet dofs keep their row/column in the pattern with zero off-diagonals and a unit
  diagonal;
* global dof numbering = rank of an integer key per node (see dof_keys).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from . import p3

BC_NONE, BC_IMPEDANCE, BC_DIRICHLET = 0, 1, 2


# ----------------------------------------------------------------------------- dofs


def dof_keys(tets):
    """Integer key (v0, v1, v2, sub) of each of the 20 local nodes of each tet, (T,20,4).

    vertex g             -> (g, -1, -1, 0)
    edge lo<hi           -> (lo, hi, -1, 0) for the node at 2/3 lo + 1/3 hi,
                            (lo, hi, -1, 1) for the node at 1/3 lo + 2/3 hi
    face a<b<c           -> (a, b, c, 0)
    """
    tets = np.asarray(tets, np.int64)
    T = tets.shape[0]
    keys = np.full((T, 20, 4), -1, np.int64)
    keys[:, :, 3] = 0
    for v in range(4):
        keys[:, v, 0] = tets[:, v]
    for e, (a, b) in enumerate(p3.EDGES):
        ga, gb = tets[:, a], tets[:, b]
        lo, hi = np.minimum(ga, gb), np.maximum(ga, gb)
        a_is_lo = ga < gb
        for node, near_a in ((4 + 2 * e, True), (5 + 2 * e, False)):
            keys[:, node, 0] = lo
            keys[:, node, 1] = hi
            near_lo = a_is_lo if near_a else ~a_is_lo
            keys[:, node, 3] = np.where(near_lo, 0, 1)
    for f in range(4):
        tri = np.sort(tets[:, list(p3.FACES[f])], axis=1)
        keys[:, 16 + f, 0:3] = tri
    return keys


def dof_numbering(tets):
    """Global dof id of each local node (T,20) int32 and the dof count.

    Id = rank of the node's key in ascending lexicographic order (-1 sorts first)."""
    keys = dof_keys(tets).reshape(-1, 4)
    uniq, inv = np.unique(keys, axis=0, return_inverse=True)
    return inv.reshape(-1, 20).astype(np.int32), int(uniq.shape[0])


def dof_coordinates(tets, coords, tet_dofs, n):
    """Physical position of every dof (n,3)."""
    lam = np.array([[float(x) for x in pt] for pt in p3.node_barycentrics()])  # (20,4)
    pos = np.einsum("lv,tvd->tld", lam, coords[tets])
    out = np.empty((n, 3))
    out[tet_dofs.ravel()] = pos.reshape(-1, 3)
    return out


def face_neighbours(tets):
    """For every (tet, local face) the neighbouring tet across it, or -1 on the boundary."""
    tets = np.asarray(tets, np.int64)
    T = tets.shape[0]
    tri = np.concatenate([np.sort(tets[:, list(p3.FACES[f])], axis=1) for f in range(4)])  # (4T,3)
    owner = np.concatenate([np.arange(T)] * 4)
    lf = np.repeat(np.arange(4), T)
    order = np.lexsort((tri[:, 2], tri[:, 1], tri[:, 0]))
    st = tri[order]
    same = np.all(st[1:] == st[:-1], axis=1)
    nb = np.full((T, 4), -1, np.int64)
    idx = np.nonzero(same)[0]
    a, b = order[idx], order[idx + 1]
    nb[owner[a], lf[a]] = owner[b]
    nb[owner[b], lf[b]] = owner[a]
    return nb


def boundary_tags(tets, face_bc):
    """Tag per (tet, face): BC_NONE on interior faces, the caller's tag on boundary faces."""
    nb = face_neighbours(tets)
    tags = np.where(nb < 0, np.asarray(face_bc, np.int64), BC_NONE)
    return tags, nb


def dirichlet_dofs(tet_dofs, tags, n):
    mask = np.zeros(n, bool)
    for f in range(4):
        sel = tags[:, f] == BC_DIRICHLET
        if sel.any():
            nodes = p3.face_nodes(f)
            mask[tet_dofs[sel][:, nodes].ravel()] = True
    return mask


# ------------------------------------------------------------------- element matrices


def geometry(tets, coords):
    """|T| (T,), grad lambda (T,4,3), face areas (T,4)."""
    P = coords[np.asarray(tets, np.int64)]  # (T,4,3)
    J = np.stack([P[:, 1] - P[:, 0], P[:, 2] - P[:, 0], P[:, 3] - P[:, 0]], axis=2)  # columns
    det = np.linalg.det(J)
    vol = np.abs(det) / 6.0
    Jinv = np.linalg.inv(J)
    grads = np.empty((P.shape[0], 4, 3))
    grads[:, 1:] = Jinv
    grads[:, 0] = -Jinv.sum(axis=1)
    area = np.empty((P.shape[0], 4))
    for f in range(4):
        a, b, c = p3.FACES[f]
        area[:, f] = 0.5 * np.linalg.norm(np.cross(P[:, b] - P[:, a], P[:, c] - P[:, a]), axis=1)
    return vol, grads, area


def wavenumber(velocity, freq, Q=None):
    """k_e = omega / c_e with c_e = v_e (1 + i / (2 Q_e)) (c_e = v_e without Q)."""
    c = np.asarray(velocity, np.complex128)
    if Q is not None:
        c = c * (1.0 + 1j / (2.0 * np.asarray(Q, np.float64)))
    return 2.0 * np.pi * freq / c


def element_parts(tets, coords, sel=None):
    """Per-tet stiffness K_e (T,20,20), mass M_e (T,20,20) and face masses |f| Fhat_f (T,4,20,20)."""
    Mh, Sh, Fh = p3.reference_matrices()
    if sel is not None:
        tets = np.asarray(tets)[sel]
    vol, grads, area = geometry(tets, coords)
    G = np.einsum("tad,tbd->tab", grads, grads)
    K = vol[:, None, None] * np.einsum("tab,abij->tij", G, Sh)
    M = vol[:, None, None] * Mh[None]
    F = area[:, :, None, None] * Fh[None]
    return K, M, F


def element_matrices(tets, coords, velocity, freq, Q, robin_faces, sel=None):
    """A_e = K_e - k_e^2 M_e + i k_e sum_{f in robin_faces[e]} |f| Fhat_f  (T,20,20) complex."""
    K, M, F = element_parts(tets, coords, sel)
    k = wavenumber(velocity, freq, Q)
    rf = np.asarray(robin_faces, bool)
    if sel is not None:
        k, rf = k[sel], rf[sel]
    Fs = np.einsum("tf,tfij->tij", rf.astype(np.float64), F)
    return K - (k**2)[:, None, None] * M + (1j * k)[:, None, None] * Fs


# ------------------------------------------------------------------------- assembly


def assemble(tet_dofs, Ae, n, dirichlet=None, rows_of=None):
    """Sum element matrices into CSR (columns ascending, duplicates summed).

    The pattern is every (i, j) pair that shares an element; explicit zeros are kept.
    Dirichlet dofs: row and column zeroed, unit diagonal (pattern unchanged)."""
    td = np.asarray(tet_dofs, np.int64)
    T = td.shape[0]
    rows = np.repeat(td, 20, axis=1).ravel()
    cols = np.tile(td, (1, 20)).ravel()
    vals = np.asarray(Ae).reshape(T, 400).ravel()
    A = sp.coo_matrix((vals, (rows, cols)), shape=(n, n)).tocsr()
    A.sum_duplicates()
    A.sort_indices()
    if dirichlet is not None and dirichlet.any():
        A = A.tocoo()
        r, c, v = A.row, A.col, A.data.copy()
        kill = dirichlet[r] | dirichlet[c]
        v[kill] = 0.0
        v[kill & (r == c)] = 1.0
        A = sp.csr_matrix((v, (r, c)), shape=(n, n))
        A.sort_indices()
    return A


def pattern(tet_dofs, n):
    """CSR pattern (indptr int64, indices int32) of the global operator."""
    td = np.asarray(tet_dofs, np.int64)
    rows = np.repeat(td, 20, axis=1).ravel()
    cols = np.tile(td, (1, 20)).ravel()
    key = np.unique(rows * n + cols)
    r, c = key // n, key % n
    indptr = np.zeros(n + 1, np.int64)
    np.add.at(indptr, r + 1, 1)
    return np.cumsum(indptr), c.astype(np.int32)


class Mesh:
    """Mesh with its P3 dof map, face neighbours and boundary tags."""

    def __init__(self, tets, coords, face_bc=None):
        self.tets = np.asarray(tets, np.int32)
        self.coords = np.asarray(coords, np.float64)
        T = self.tets.shape[0]
        if face_bc is None:
            face_bc = np.full((T, 4), BC_IMPEDANCE, np.int8)
        self.tet_dofs, self.n = dof_numbering(self.tets)
        self.tags, self.nb = boundary_tags(self.tets, face_bc)
        self.dirichlet = dirichlet_dofs(self.tet_dofs, self.tags, self.n)
        self.impedance = self.tags == BC_IMPEDANCE


def assemble_operator(mesh: Mesh, velocity, freq, Q=None):
    """Global A = K - k^2 M + i k M_G with Dirichlet rows as identity."""
    Ae = element_matrices(mesh.tets, mesh.coords, velocity, freq, Q, mesh.impedance)
    return assemble(mesh.tet_dofs, Ae, mesh.n, mesh.dirichlet)


def assemble_parts(mesh: Mesh):
    """Global K, M and M_G (impedance faces) without Dirichlet treatment (for invariants)."""
    K, M, F = element_parts(mesh.tets, mesh.coords)
    MG = np.einsum("tf,tfij->tij", mesh.impedance.astype(np.float64), F)
    return tuple(assemble(mesh.tet_dofs, X, mesh.n) for X in (K, M, MG))


def assemble_rows(mesh: Mesh, velocity, freq, Q, rows):
    """Rows `rows` of the global operator, computed from the tets touching them only.

    Returns a dict row -> (cols ascending, values)."""
    rows = np.asarray(rows, np.int64)
    want = np.zeros(mesh.n, bool)
    want[rows] = True
    sel = np.nonzero(want[mesh.tet_dofs].any(axis=1))[0]
    Ae = element_matrices(mesh.tets, mesh.coords, velocity, freq, Q, mesh.impedance, sel=sel)
    td = mesh.tet_dofs[sel].astype(np.int64)
    out = {}
    for r in rows:
        acc = {}
        for t in range(td.shape[0]):
            hit = np.nonzero(td[t] == r)[0]
            for i in hit:
                for j in range(20):
                    c = int(td[t, j])
                    acc[c] = acc.get(c, 0) + Ae[t, i, j]
        cols = np.array(sorted(acc), np.int64)
        vals = np.array([acc[c] for c in cols], np.complex128)
        if mesh.dirichlet[r]:
            vals[:] = 0
            vals[cols == r] = 1
        else:
            vals[mesh.dirichlet[cols]] = 0
        out[int(r)] = (cols, vals)
    return out
