"""Independent reference assemblies used to pin the oracle.

Everything here is built from the weak forms by Gauss quadrature (Q1 on
boxes, Sec. 3.2 of the paper) or from textbook closed forms, never from the
oracle's own formulas, so that a dropped term, a wrong sign or a transposed
index in the oracle shows up as a mismatch."""
from __future__ import annotations

import itertools

import numpy as np
import scipy.sparse as sp

GAUSS2 = (np.array([0.5 - 0.5 / np.sqrt(3.0), 0.5 + 0.5 / np.sqrt(3.0)]),
          np.array([0.5, 0.5]))


def q1_shape(xi):
    """Values and reference gradients of the 8 trilinear shape functions at a
    point of the unit cube; local node a = bx | by<<1 | bz<<2."""
    x, y, z = xi
    vals = np.zeros(8)
    grads = np.zeros((8, 3))
    for a in range(8):
        bx, by, bz = a & 1, (a >> 1) & 1, (a >> 2) & 1
        fx = x if bx else 1 - x
        fy = y if by else 1 - y
        fz = z if bz else 1 - z
        dx = 1.0 if bx else -1.0
        dy = 1.0 if by else -1.0
        dz = 1.0 if bz else -1.0
        vals[a] = fx * fy * fz
        grads[a] = (dx * fy * fz, fx * dy * fz, fx * fy * dz)
    return vals, grads


def element_matrices(size=(1.0, 1.0, 1.0)):
    """Stiffness and mass of one box element of the given edge lengths, by
    2x2x2 Gauss quadrature (exact for these polynomial integrands)."""
    pts, wts = GAUSS2
    ax, ay, az = size
    K = np.zeros((8, 8))
    M = np.zeros((8, 8))
    vol = ax * ay * az
    for (ix, iy, iz) in itertools.product(range(2), repeat=3):
        v, g = q1_shape((pts[ix], pts[iy], pts[iz]))
        w = wts[ix] * wts[iy] * wts[iz] * vol
        gp = g / np.array([ax, ay, az])
        K += w * gp @ gp.T
        M += w * np.outer(v, v)
    return K, M


def assemble_box(nx, ny, nz, coefK, coefM=None, xs=None, ys=None, zs=None):
    """Sparse Q1 matrix  sum_e coefK_e K_e + coefM_e M_e  on a node box.

    ``coefK``/``coefM`` are per element (x fastest); ``xs, ys, zs`` are node
    coordinates (default unit spacing)."""
    xs = np.arange(nx, dtype=float) if xs is None else np.asarray(xs, float)
    ys = np.arange(ny, dtype=float) if ys is None else np.asarray(ys, float)
    zs = np.arange(nz, dtype=float) if zs is None else np.asarray(zs, float)
    rows, cols, vals = [], [], []
    e = 0
    cache = {}
    for k in range(nz - 1):
        for j in range(ny - 1):
            for i in range(nx - 1):
                size = (xs[i + 1] - xs[i], ys[j + 1] - ys[j], zs[k + 1] - zs[k])
                key = tuple(np.round(size, 14))
                if key not in cache:
                    cache[key] = element_matrices(size)
                Ke, Me = cache[key]
                Ae = coefK[e] * Ke
                if coefM is not None:
                    Ae = Ae + coefM[e] * Me
                ids = [(i + (a & 1)) + nx * ((j + ((a >> 1) & 1)) + ny * (k + ((a >> 2) & 1)))
                       for a in range(8)]
                for a in range(8):
                    for b in range(8):
                        if Ae[a, b] != 0.0:
                            rows.append(ids[a]); cols.append(ids[b]); vals.append(Ae[a, b])
                e += 1
    n = nx * ny * nz
    return sp.csr_matrix((vals, (rows, cols)), shape=(n, n))


def stencil_to_dense(dims, S):
    nx, ny, nz = dims
    n = nx * ny * nz
    A = np.zeros((n, n))
    S = np.asarray(S).reshape(n, 27)
    for k in range(nz):
        for j in range(ny):
            for i in range(nx):
                r = i + nx * (j + ny * k)
                for o in range(27):
                    dx, dy, dz = o % 3 - 1, (o // 3) % 3 - 1, o // 9 - 1
                    ii, jj, kk = i + dx, j + dy, k + dz
                    if 0 <= ii < nx and 0 <= jj < ny and 0 <= kk < nz:
                        A[r, ii + nx * (jj + ny * kk)] += S[r, o]
                    else:
                        assert S[r, o] == 0.0
    return A


def dense_to_stencil(dims, A):
    nx, ny, nz = dims
    n = nx * ny * nz
    A = A.toarray() if sp.issparse(A) else np.asarray(A)
    S = np.zeros((n, 27))
    for k in range(nz):
        for j in range(ny):
            for i in range(nx):
                r = i + nx * (j + ny * k)
                for o in range(27):
                    dx, dy, dz = o % 3 - 1, (o // 3) % 3 - 1, o // 9 - 1
                    ii, jj, kk = i + dx, j + dy, k + dz
                    if 0 <= ii < nx and 0 <= jj < ny and 0 <= kk < nz:
                        S[r, o] = A[r, ii + nx * (jj + ny * kk)]
    return S


def coarse_coords(x):
    """Coordinates kept by 'even indices plus the last' coarsening."""
    n = len(x)
    if n <= 2:
        return np.asarray(x, float)
    idx = list(range(0, n, 2))
    if idx[-1] != n - 1:
        idx.append(n - 1)
    return np.asarray(x, float)[idx]


def galerkin_by_quadrature(fine_x, fine_y, fine_z, coefK):
    """Coarse stiffness  int sigma grad(Phi_I).grad(Phi_J)  with sigma
    piecewise constant on the FINE elements and Phi the Q1 basis of the coarse
    grid, integrated by Gauss quadrature on every fine element."""
    cx, cy, cz = coarse_coords(fine_x), coarse_coords(fine_y), coarse_coords(fine_z)
    ncx, ncy, ncz = len(cx), len(cy), len(cz)
    nc = ncx * ncy * ncz
    A = np.zeros((nc, nc))
    pts, wts = GAUSS2

    def locate(c, t):
        I = np.searchsorted(c, t, side="right") - 1
        I = min(max(I, 0), len(c) - 2)
        return I, (t - c[I]) / (c[I + 1] - c[I]), c[I + 1] - c[I]

    nfx, nfy, nfz = len(fine_x), len(fine_y), len(fine_z)
    e = 0
    for k in range(nfz - 1):
        for j in range(nfy - 1):
            for i in range(nfx - 1):
                x0, x1 = fine_x[i], fine_x[i + 1]
                y0, y1 = fine_y[j], fine_y[j + 1]
                z0, z1 = fine_z[k], fine_z[k + 1]
                vol = (x1 - x0) * (y1 - y0) * (z1 - z0)
                for (ix, iy, iz) in itertools.product(range(2), repeat=3):
                    X = x0 + pts[ix] * (x1 - x0)
                    Y = y0 + pts[iy] * (y1 - y0)
                    Z = z0 + pts[iz] * (z1 - z0)
                    w = wts[ix] * wts[iy] * wts[iz] * vol * coefK[e]
                    I, tx, ax = locate(cx, (x0 + x1) / 2)
                    J, ty, ay = locate(cy, (y0 + y1) / 2)
                    K, tz, az = locate(cz, (z0 + z1) / 2)
                    _, gx = None, None
                    v, g = q1_shape(((X - cx[I]) / ax, (Y - cy[J]) / ay, (Z - cz[K]) / az))
                    g = g / np.array([ax, ay, az])
                    ids = [(I + (a & 1)) + ncx * ((J + ((a >> 1) & 1)) + ncy * (K + ((a >> 2) & 1)))
                           for a in range(8)]
                    for a in range(8):
                        for b in range(8):
                            A[ids[a], ids[b]] += w * g[a] @ g[b]
                e += 1
    return A, (ncx, ncy, ncz)
