"""Helpers shared by the GPU tests (test code only)."""
import numpy as np
import scipy.sparse as sp


def stencil_to_sparse(coef, nx, ny, nz):
    """Assemble the N x N matrix of a (ndir, N) stencil in the library's
    direction order (centre, -x, +x, -y, +y, -z, +z)."""
    coef = np.asarray(coef)
    ndir, N = coef.shape
    idx = np.arange(N).reshape(nz, ny, nx)
    x = np.broadcast_to(np.arange(nx)[None, None, :], (nz, ny, nx)).ravel()
    y = np.broadcast_to(np.arange(ny)[None, :, None], (nz, ny, nx)).ravel()
    z = np.broadcast_to(np.arange(nz)[:, None, None], (nz, ny, nx)).ravel()
    i = idx.ravel()
    rows, cols, vals = [i], [i], [coef[0]]
    nbrs = [(x > 0, -1), (x < nx - 1, 1), (y > 0, -nx), (y < ny - 1, nx),
            (z > 0, -nx * ny), (z < nz - 1, nx * ny)]
    for k in range(1, ndir):
        ok, off = nbrs[k - 1]
        rows.append(i[ok])
        cols.append(i[ok] + off)
        vals.append(coef[k][ok])
        assert np.all(coef[k][~ok] == 0.0), "coefficient toward a missing neighbour"
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=(N, N))


def sparse_to_stencil(M, nx, ny, nz):
    """Inverse of stencil_to_sparse for a matrix with the 5/7-point pattern."""
    M = sp.csr_matrix(M)
    N = nx * ny * nz
    ndir = 7 if nz > 1 else 5
    coef = np.zeros((ndir, N))
    idx = np.arange(N)
    x = idx % nx
    y = (idx // nx) % ny
    z = idx // (nx * ny)
    coef[0] = M.diagonal()
    nbrs = [(x > 0, -1), (x < nx - 1, 1), (y > 0, -nx), (y < ny - 1, nx),
            (z > 0, -nx * ny), (z < nz - 1, nx * ny)]
    for k in range(1, ndir):
        ok, off = nbrs[k - 1]
        coef[k][ok] = np.asarray(M[idx[ok], idx[ok] + off]).ravel()
    return coef


def rel_inf(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))
