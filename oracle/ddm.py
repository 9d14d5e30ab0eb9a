"""Oracle: overlapping decomposition, partition of unity, local ORAS operators, coarse space.

TEST INFRASTRUCTURE ONLY (tests/, graft smoke check, bench.py CPU baseline).

Follows the paper's section "Domain decomposition preconditioner":
* eq. (oras): M1^{-1} = sum_i R_i^T D_i A_i^{-1} R_i, with Boolean restrictions R_i, a
  diagonal partition of unity D_i and local operators A_i carrying absorbing
  (transmission) conditions on the subdomain interfaces;
* eq. (2lvl): M^{-1} = M1^{-1} (I - A Q) + Q, Q = Z E^{-1} Z^T, E = Z^T A Z, with Z the
  interpolation between the fine space and a finite element space on a coarse mesh.

Readings (the abstract gives no construction details; listed in the design doc):
* overlap: delta layers of tets, each layer adds every tet sharing a vertex;
* partition of unity: Boolean, a dof belongs to the lowest subdomain id whose
  non-overlapping part touches it; or (variant) smooth: a dof's raw weight in subdomain i is
  1 - l/(delta + 1), l its overlap layer in i (0 on the tets of the non-overlapping part, k on
  those the k-th growth step added), normalised over the subdomains that hold the dof;
* transmission condition: the same first-order Robin term i k |f| Fhat_f as the
  absorbing boundary, on every face of the overlapped subdomain whose neighbour tet lies
  outside it; Dirichlet dofs of the global problem stay identity rows locally;
* coarse space: P1 on a coarse tet mesh, Z[j, c] = barycentric c of fine node j in the
  lowest-id coarse tet containing it, |Z| <= 1e-12 dropped, rows of Dirichlet dofs zero;
* coarse solve: dense LU with partial pivoting; or (InexactCoarse) the paper's iterative one,
  10 GMRES iterations on E preconditioned by one-level ORAS on the coarse level, read as: the
  coarse subdomain i holds the coarse dofs whose basis functions are nonzero on its overlapped
  fine dofs, its local operator is the Galerkin projection Z_i^T A_i Z_i of the fine local
  operator onto them (Z_i: the rows of Z on those fine dofs), and a coarse dof belongs to the
  subdomain that owns the fine dof at its vertex (Boolean partition of unity).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import krylov
from .fem import BC_IMPEDANCE, Mesh, assemble, dof_coordinates, element_matrices


def vertex_to_tets(tets, n_verts):
    t = np.asarray(tets, np.int64)
    rows = t.ravel()
    cols = np.repeat(np.arange(t.shape[0]), 4)
    return sp.csr_matrix((np.ones(rows.size, np.int8), (rows, cols)), shape=(n_verts, t.shape[0]))


def tet_layers(tets, n_verts, partition, i, delta, v2t=None):
    """Layer of every tet in subdomain i grown by delta vertex-adjacency layers: 0 for the
    tets of the non-overlapping part, k for those the k-th growth step added, -1 outside."""
    if v2t is None:
        v2t = vertex_to_tets(tets, n_verts)
    t = np.asarray(tets, np.int64)
    lay = np.where(np.asarray(partition) == i, 0, -1)
    for k in range(1, delta + 1):
        verts = np.zeros(n_verts, bool)
        verts[t[lay >= 0].ravel()] = True
        touched = np.asarray(v2t[verts].sum(axis=0)).ravel() > 0
        lay = np.where((lay < 0) & touched, k, lay)
    return lay


def smooth_pou(mesh: Mesh, partition, n_sub, delta, subs):
    """Weights D_i of the smooth partition of unity, aligned with each subdomain's sorted dofs:
    raw weight 1 - l/(delta + 1) with l the smallest layer of the subdomain's tets holding
    the dof, divided by the sum of the raw weights of all subdomains holding it (summed in
    subdomain order)."""
    nverts = mesh.coords.shape[0]
    v2t = vertex_to_tets(mesh.tets, nverts)
    raw = []
    for i, sd in enumerate(subs):
        lay = tet_layers(mesh.tets, nverts, partition, i, delta, v2t)
        sel = np.nonzero(lay >= 0)[0]
        dl = np.full(mesh.n, delta + 1, np.int64)
        np.minimum.at(dl, mesh.tet_dofs[sel].ravel().astype(np.int64), np.repeat(lay[sel], 20))
        raw.append(1.0 - dl[sd.gdofs] / (delta + 1.0))
    tot = np.zeros(mesh.n)
    for sd, r in zip(subs, raw):
        tot[sd.gdofs] += r
    return [r / tot[sd.gdofs] for sd, r in zip(subs, raw)]


def overlap_tets(tets, n_verts, partition, i, delta, v2t=None):
    """Sorted tet ids of subdomain i grown by delta vertex-adjacency layers."""
    if v2t is None:
        v2t = vertex_to_tets(tets, n_verts)
    cur = np.asarray(partition) == i
    t = np.asarray(tets, np.int64)
    for _ in range(delta):
        verts = np.zeros(n_verts, bool)
        verts[t[cur].ravel()] = True
        touched = np.asarray(v2t[verts].sum(axis=0)).ravel() > 0
        cur = cur | touched
    return np.nonzero(cur)[0]


class Subdomain:
    """R_i (sorted global dofs), D_i (Boolean owner flags) and the local operator A_i."""

    def __init__(self, gdofs, owned, tets_local, robin_faces, A_local):
        self.gdofs = gdofs
        self.owned = owned
        self.tets = tets_local
        self.robin_faces = robin_faces
        self.A = A_local
        self.lu = None


def owners(mesh: Mesh, partition, n_sub):
    """Owner subdomain of each dof: the minimum i whose non-overlapping tets contain it."""
    own = np.full(mesh.n, n_sub, np.int64)
    part = np.asarray(partition, np.int64)
    np.minimum.at(own, mesh.tet_dofs.ravel().astype(np.int64), np.repeat(part, 20))
    return own


def build_subdomains(mesh: Mesh, velocity, freq, Q, partition, n_sub, delta):
    nverts = mesh.coords.shape[0]
    v2t = vertex_to_tets(mesh.tets, nverts)
    own = owners(mesh, partition, n_sub)
    subs = []
    for i in range(n_sub):
        tl = overlap_tets(mesh.tets, nverts, partition, i, delta, v2t)
        inside = np.zeros(mesh.tets.shape[0], bool)
        inside[tl] = True
        nb = mesh.nb[tl]
        cut = (nb >= 0) & ~inside[np.maximum(nb, 0)]
        robin = mesh.impedance[tl] | cut
        gd = np.unique(mesh.tet_dofs[tl].ravel())
        loc = np.full(mesh.n, -1, np.int64)
        loc[gd] = np.arange(gd.size)
        td_local = loc[mesh.tet_dofs[tl]]
        robin_full = np.zeros((mesh.tets.shape[0], 4), bool)
        robin_full[tl] = robin
        Ae = element_matrices(mesh.tets, mesh.coords, velocity, freq, Q, robin_full, sel=tl)
        Ai = assemble(td_local, Ae, gd.size, mesh.dirichlet[gd])
        subs.append(Subdomain(gd, own[gd] == i, tl, robin, Ai))
    return subs, own


def factor_subdomains(subs, dtype=np.complex128):
    for s in subs:
        s.lu = spla.splu(s.A.astype(dtype).tocsc(), permc_spec="MMD_AT_PLUS_A")
    return subs


# ---------------------------------------------------------------------------- coarse


def coarse_interpolation(mesh: Mesh, coarse_tets, coarse_coords, eps=1e-12):
    """Z (n x n_c, CSR, real): P1 barycentrics of each fine dof in the lowest-id coarse tet
    containing it; entries with |lambda| <= eps dropped; Dirichlet rows zero."""
    xyz = dof_coordinates(mesh.tets, mesh.coords, mesh.tet_dofs, mesh.n)
    ct = np.asarray(coarse_tets, np.int64)
    P = np.asarray(coarse_coords, np.float64)[ct]
    J = np.stack([P[:, 1] - P[:, 0], P[:, 2] - P[:, 0], P[:, 3] - P[:, 0]], axis=2)
    Jinv = np.linalg.inv(J)
    lo, hi = P.min(axis=1), P.max(axis=1)
    # bucket the coarse tets on a uniform grid of their bounding boxes
    gmin, gmax = P.reshape(-1, 3).min(axis=0), P.reshape(-1, 3).max(axis=0)
    nb = max(1, int(round(ct.shape[0] ** (1 / 3))))
    cell = (gmax - gmin) / nb + 1e-300
    def cidx(x):
        return np.clip(((x - gmin) / cell).astype(np.int64), 0, nb - 1)
    clo, chi = cidx(lo - 1e-9 * (gmax - gmin)), cidx(hi + 1e-9 * (gmax - gmin))
    buckets = {}
    for t in range(ct.shape[0]):
        for a in range(clo[t, 0], chi[t, 0] + 1):
            for b in range(clo[t, 1], chi[t, 1] + 1):
                for c in range(clo[t, 2], chi[t, 2] + 1):
                    buckets.setdefault((a, b, c), []).append(t)
    rows, cols, vals = [], [], []
    cell_of = cidx(xyz)
    for j in range(mesh.n):
        if mesh.dirichlet[j]:
            continue
        cand = buckets.get(tuple(cell_of[j]), [])
        found = None
        for t in cand:  # ascending tet ids
            l123 = Jinv[t] @ (xyz[j] - P[t, 0])
            lam = np.array([1.0 - l123.sum(), l123[0], l123[1], l123[2]])
            if np.all(lam >= -eps):
                found = (t, lam)
                break
        if found is None:
            raise ValueError(f"fine dof {j} is outside the coarse mesh")
        t, lam = found
        for v in range(4):
            if abs(lam[v]) > eps:
                rows.append(j)
                cols.append(int(ct[t, v]))
                vals.append(lam[v])
    nc = int(np.asarray(coarse_coords).shape[0])
    Z = sp.csr_matrix((np.array(vals), (np.array(rows), np.array(cols))), shape=(mesh.n, nc))
    Z.sum_duplicates()
    Z.sort_indices()
    return Z


class Coarse:
    def __init__(self, Z, A, dtype=np.complex128):
        self.Z = Z
        AZ = A @ Z.astype(np.complex128)
        self.E = (Z.T.astype(np.complex128) @ AZ).toarray()
        self.lu = sla.lu_factor(self.E.astype(dtype))
        self.dtype = dtype

    def solve(self, v):
        """q = Z E^{-1} Z^T v for a block v (n, s)."""
        y = self.Z.T @ v
        return self.Z @ sla.lu_solve(self.lu, y.astype(self.dtype)).astype(np.complex128)


def coarse_owners(mesh: Mesh, coarse_coords, own):
    """Owner subdomain of each coarse dof: the owner of the fine dof at its vertex (the
    coarse vertices are fine vertices: the coarse mesh takes every k-th vertex plane)."""
    xyz = dof_coordinates(mesh.tets, mesh.coords, mesh.tet_dofs, mesh.n)
    cc = np.asarray(coarse_coords, np.float64)
    scale = max(1.0, float(np.abs(xyz).max()))
    key = lambda x: tuple(np.round(x / scale * 1e9).astype(np.int64))
    at = {key(xyz[j]): j for j in range(mesh.n)}
    return np.array([own[at[key(c)]] for c in cc], np.int64)


class InexactCoarse:
    """The paper's coarse solve (section "Domain decomposition preconditioner", after eq.
    oras): E y = Z^T v solved by `iters` block GMRES iterations from y = 0, right-
    preconditioned by one-level ORAS on the coarse level, M_c^{-1} = sum_i Rc_i^T Dc_i
    E_i^{-1} Rc_i with E_i = Z_i^T A_i Z_i (dense LU per coarse subdomain)."""

    def __init__(self, Z, A, subs, cown, iters=10):
        self.Z = Z
        self.iters = iters
        self.E = (Z.T.astype(np.complex128) @ (A @ Z.astype(np.complex128))).tocsr()  # sparse
        self.loc = []
        for i, s in enumerate(subs):
            Zi = Z[s.gdofs].tocsr()
            J = np.unique(Zi.indices)
            Zi = Zi[:, J].astype(np.complex128)
            Ei = (Zi.T @ (s.A @ Zi)).toarray()
            self.loc.append((J, sla.lu_factor(Ei), cown[J] == i))

    def precond(self, r):
        z = np.zeros_like(r)
        for J, lu, own in self.loc:
            z[J[own]] += sla.lu_solve(lu, r[J])[own]
        return z

    def solve(self, v):
        """q = Z y with y the GMRES iterate for E y = Z^T v, for a block v (n, s)."""
        y0 = self.Z.T @ v
        y, _ = krylov.block_fgmres(lambda x: self.E @ x, y0, self.precond, fixed_iters=self.iters, m=self.iters)
        return self.Z @ y


# ------------------------------------------------------------------------ preconditioner


class ORAS:
    """Two-level ORAS preconditioner, eqs. (2lvl) and (oras)."""

    def __init__(self, A, subs, coarse=None, dtype=np.complex128, weights=None):
        self.A = A
        self.subs = subs
        self.coarse = coarse
        self.dtype = dtype
        self.weights = weights  # None: Boolean partition of unity; else smooth_pou's weights

    def one_level(self, t):
        """sum_i R_i^T D_i A_i^{-1} R_i t for a block t (n, s)."""
        z = np.zeros_like(t, dtype=np.complex128)
        for k, s in enumerate(self.subs):
            ti = t[s.gdofs].astype(self.dtype)
            yi = s.lu.solve(ti).astype(np.complex128)
            if self.weights is None:
                z[s.gdofs[s.owned]] += yi[s.owned]
            else:
                z[s.gdofs] += self.weights[k][:, None] * yi if yi.ndim == 2 else self.weights[k] * yi
        return z

    def apply(self, v):
        v = np.asarray(v, np.complex128)
        squeeze = v.ndim == 1
        if squeeze:
            v = v[:, None]
        if self.coarse is None:
            z = self.one_level(v)
        else:
            q = self.coarse.solve(v)
            t = v - self.A @ q
            z = self.one_level(t) + q
        return z[:, 0] if squeeze else z


def build_preconditioner(mesh: Mesh, A, velocity, freq, Q, partition, n_sub, delta,
                         coarse_tets=None, coarse_coords=None, dtype=np.complex128, pou="boolean"):
    subs, own = build_subdomains(mesh, velocity, freq, Q, partition, n_sub, delta)
    factor_subdomains(subs, dtype)
    coarse = None
    if coarse_tets is not None:
        Z = coarse_interpolation(mesh, coarse_tets, coarse_coords)
        coarse = Coarse(Z, A, dtype)
    weights = smooth_pou(mesh, partition, n_sub, delta, subs) if pou == "smooth" else None
    return ORAS(A, subs, coarse, dtype, weights)
