"""ORACLE (test infrastructure only): pupil, guide-star projection and
Shack-Hartmann geometry in plain FP64 NumPy.

Layered atmosphere and projections (Sec. 2.1, eq. (2) for natural guide
stars; the cone-effect version for laser guide stars that follows it):
a layer at altitude h is sampled at s * r + theta * h, with s = 1 - h/H for a
laser guide star at altitude H and s = 1 for a natural guide star.

Readings where the paper is silent:
* layer pixel p of an N x N layer with spacing d sits at (p - N/2) d;
* pupil node i of an n_sub x n_sub Fried sensor of diameter D sits at
  (i - n_sub/2) D/n_sub, i = 0..n_sub;
* layers are sampled by bilinear interpolation; i0 = floor(u) clamped to
  [0, N-2], and a node whose u falls outside [0, N-1] is an error;
* a subaperture is active iff its centre lies in the closed annulus of outer
  diameter D and inner diameter eps*D.
"""
import numpy as np


def layer_coords(N, d):
    return (np.arange(N) - N / 2.0) * d


def node_coords(n_sub, D):
    return (np.arange(n_sub + 1) - n_sub / 2.0) * (D / n_sub)


def subaperture_mask(n_sub, D, eps):
    """Active subapertures [i][j] (i along x)."""
    c = (np.arange(n_sub) + 0.5 - n_sub / 2.0) * (D / n_sub)
    r2 = c[:, None] ** 2 + c[None, :] ** 2
    return (r2 <= (D / 2.0) ** 2) & (r2 >= (eps * D / 2.0) ** 2)


class FootprintError(ValueError):
    pass


def bilinear_axis(x_nodes, scale, shift, N, d):
    """Per node: (i0, t) with the sample at (1-t) f[i0] + t f[i0+1]."""
    u = (scale * x_nodes + shift) / d + N / 2.0
    if np.any(u < 0.0) or np.any(u > N - 1):
        raise FootprintError("projection footprint leaves the layer grid")
    i0 = np.clip(np.floor(u).astype(np.int64), 0, N - 2)
    return i0, u - i0


def bilinear_matrix(x_nodes, scale, shift, N, d):
    """The same interpolation as a dense (n_nodes x N) matrix (for tests and
    the separable preconditioner)."""
    i0, t = bilinear_axis(x_nodes, scale, shift, N, d)
    B = np.zeros((len(x_nodes), N))
    r = np.arange(len(x_nodes))
    B[r, i0] += 1.0 - t
    B[r, i0 + 1] += t
    return B


def project_layer(phi, ix0, tx, jy0, ty):
    """Bilinear samples of one layer at the node grid (ix0, tx) x (jy0, ty)."""
    a = (1 - tx)[:, None] * (1 - ty)[None, :] * phi[np.ix_(ix0, jy0)]
    b = tx[:, None] * (1 - ty)[None, :] * phi[np.ix_(ix0 + 1, jy0)]
    c = (1 - tx)[:, None] * ty[None, :] * phi[np.ix_(ix0, jy0 + 1)]
    e = tx[:, None] * ty[None, :] * phi[np.ix_(ix0 + 1, jy0 + 1)]
    return a + b + c + e


def project_layer_adjoint(v, ix0, tx, jy0, ty, N):
    """Transpose of ``project_layer``: scatter node values into the layer."""
    out = np.zeros((N, N))
    I0, J0 = np.meshgrid(ix0, jy0, indexing="ij")
    TX, TY = np.meshgrid(tx, ty, indexing="ij")
    np.add.at(out, (I0, J0), (1 - TX) * (1 - TY) * v)
    np.add.at(out, (I0 + 1, J0), TX * (1 - TY) * v)
    np.add.at(out, (I0, J0 + 1), (1 - TX) * TY * v)
    np.add.at(out, (I0 + 1, J0 + 1), TX * TY * v)
    return out


def fried_slopes(u, mask):
    """Fried-geometry Shack-Hartmann slopes (eq. (3) with the constant taken as
    1/d_sub and the integral by the trapezoid rule): returns the x-slopes of
    the active subapertures in row-major order, then the y-slopes."""
    sx = 0.5 * ((u[1:, :-1] - u[:-1, :-1]) + (u[1:, 1:] - u[:-1, 1:]))
    sy = 0.5 * ((u[:-1, 1:] - u[:-1, :-1]) + (u[1:, 1:] - u[1:, :-1]))
    return np.concatenate([sx[mask], sy[mask]])


def fried_adjoint(w, mask):
    """Transpose of ``fried_slopes``: slopes -> node field."""
    n = mask.shape[0]
    S = int(mask.sum())
    wx = np.zeros((n, n))
    wy = np.zeros((n, n))
    wx[mask] = w[:S]
    wy[mask] = w[S:]
    v = np.zeros((n + 1, n + 1))
    v[1:, :-1] += 0.5 * wx
    v[:-1, :-1] -= 0.5 * wx
    v[1:, 1:] += 0.5 * wx
    v[:-1, 1:] -= 0.5 * wx
    v[:-1, 1:] += 0.5 * wy
    v[:-1, :-1] -= 0.5 * wy
    v[1:, 1:] += 0.5 * wy
    v[1:, :-1] -= 0.5 * wy
    return v


def aggregation_cells(mask, k):
    """Low-order sensor of k x k subapertures built from the fine grid: cell
    (ci, cj) holds fine subapertures i in [ci n/k, (ci+1) n/k).  Returns the
    list of active cells (row-major) and, for each, the boolean fine mask."""
    n = mask.shape[0]
    assert n % k == 0
    b = n // k
    cells = []
    for ci in range(k):
        for cj in range(k):
            m = np.zeros_like(mask)
            m[ci * b:(ci + 1) * b, cj * b:(cj + 1) * b] = True
            m &= mask
            if m.any():
                cells.append(m)
    return cells
