"""Oracle: right-hand sides (point sources, plane-wave impedance data).

TEST INFRASTRUCTURE ONLY (tests/, graft smoke check, bench.py CPU baseline).

Point sources follow the paper's experiment set-up (section "Numerical results": a point
source in the Overthrust box); the load is amp * phi_j(x_s), i.e. the discrete form of
-(Delta + k^2) u = amp * delta(x - x_s) under the sign reading of eq. (1) used here.
The plane-wave load is the impedance datum g = i k (1 + d.n) exp(i k d.x) of the exact
solution u = exp(i k d.x), used as a manufactured solution.
"""
from __future__ import annotations

import numpy as np

from . import p3
from .fem import Mesh, wavenumber


def barycentrics(tets, coords, x):
    """Barycentric coordinates (T,4) of point x in every tet."""
    P = coords[np.asarray(tets, np.int64)]
    J = np.stack([P[:, 1] - P[:, 0], P[:, 2] - P[:, 0], P[:, 3] - P[:, 0]], axis=2)
    lam = np.empty((P.shape[0], 4))
    lam[:, 1:] = np.linalg.solve(J, (np.asarray(x, np.float64)[None, :] - P[:, 0])[:, :, None])[:, :, 0]
    lam[:, 0] = 1.0 - lam[:, 1:].sum(axis=1)
    return lam


def locate(tets, coords, x, eps=1e-12):
    """Lowest tet id whose barycentrics of x are all >= -eps; -1 if none."""
    lam = barycentrics(tets, coords, x)
    inside = np.nonzero(np.all(lam >= -eps, axis=1))[0]
    if inside.size == 0:
        return -1, None
    t = int(inside[0])
    return t, lam[t]


def point_sources(mesh: Mesh, xyz, amp=None):
    """Loads f[s, j] = amp_s * phi_j(x_s), zero on Dirichlet dofs.  Returns (ns, n) complex."""
    xyz = np.atleast_2d(np.asarray(xyz, np.float64))
    ns = xyz.shape[0]
    out = np.zeros((ns, mesh.n), np.complex128)
    for s in range(ns):
        t, lam = locate(mesh.tets, mesh.coords, xyz[s])
        if t < 0:
            raise ValueError(f"source {s} outside the mesh")
        phi = p3.eval_basis_float(lam[None])[0]
        a = 1.0 if amp is None else amp[s]
        out[s, mesh.tet_dofs[t]] += a * phi
    out[:, mesh.dirichlet] = 0.0
    return out


def triangle_rule(n=8):
    """Collapsed (Duffy) Gauss-Legendre rule on the reference triangle {u,v>=0, u+v<=1}.

    Points (m,2) and weights (m,) summing to 1/2; exact for polynomials of degree 2n-2."""
    g, w = np.polynomial.legendre.leggauss(n)
    g = 0.5 * (g + 1.0)
    w = 0.5 * w
    U, V = np.meshgrid(g, g, indexing="ij")
    WU, WV = np.meshgrid(w, w, indexing="ij")
    u = U.ravel()
    v = (V * (1.0 - U)).ravel()
    wt = (WU * WV * (1.0 - U)).ravel()
    return np.stack([u, v], axis=1), wt


def plane_wave_load(mesh: Mesh, velocity, freq, direction, n_quad=8):
    """f_j = sum over impedance faces of int_f g phi_j dS, g = i k (1 + d.n) e^{i k d.x}."""
    d = np.asarray(direction, np.float64)
    k = wavenumber(velocity, freq)
    pts, wts = triangle_rule(n_quad)
    f = np.zeros(mesh.n, np.complex128)
    coords = mesh.coords
    for face in range(4):
        sel = np.nonzero(mesh.impedance[:, face])[0]
        if sel.size == 0:
            continue
        a, b, c = p3.FACES[face]
        P = coords[mesh.tets[sel].astype(np.int64)]  # (m,4,3)
        e1, e2 = P[:, b] - P[:, a], P[:, c] - P[:, a]
        cr = np.cross(e1, e2)
        area2 = np.linalg.norm(cr, axis=1)
        nrm = cr / area2[:, None]
        flip = np.einsum("md,md->m", nrm, P[:, a] - P[:, face]) < 0
        nrm[flip] *= -1
        # barycentric coords of the quadrature points in the tet
        lam = np.zeros((pts.shape[0], 4))
        lam[:, a] = 1.0 - pts[:, 0] - pts[:, 1]
        lam[:, b] = pts[:, 0]
        lam[:, c] = pts[:, 1]
        phi = p3.eval_basis_float(lam)  # (q,20)
        X = np.einsum("qv,mvd->mqd", lam, P)  # (m,q,3)
        km = k[sel][:, None]
        g = 1j * km * (1.0 + (nrm @ d))[:, None] * np.exp(1j * km * (X @ d))  # (m,q)
        contrib = np.einsum("mq,q,qj->mj", g, wts, phi) * area2[:, None]  # |f| = area2/2, weights sum 1/2
        np.add.at(f, mesh.tet_dofs[sel].ravel(), contrib.ravel())
    f[mesh.dirichlet] = 0.0
    return f


def plane_wave_nodal(mesh: Mesh, velocity, freq, direction, dof_xyz):
    k = wavenumber(velocity, freq)
    if not np.allclose(k, k[0]):
        raise ValueError("plane wave needs a constant wavenumber")
    return np.exp(1j * k[0] * (dof_xyz @ np.asarray(direction, np.float64)))
