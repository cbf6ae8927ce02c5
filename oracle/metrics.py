"""Grid metrics of a structured block: face area vectors and cell volumes.

The paper stores per-face normals and per-cell volumes (the grid variables
used by the boundary and flux kernels of Sec. 7.2, V2-V4) but does not print
how they are formed.  Reading used here (finite-volume form of eq. (1)):

* 2D: the area vector of the face joining nodes a -> b is (y_b - y_a, -(x_b - x_a))
  for i-faces (a = (i, j), b = (i, j+1)) and (-(y_b - y_a), x_b - x_a) for
  j-faces (a = (i, j), b = (i+1, j)); both point toward increasing index.
  Cell area = half the cross product of the two cell diagonals.
* 3D: the area vector of a quadrilateral face a, b, c, d is
  1/2 (c - a) x (d - b), with the node order chosen so that it points toward
  increasing index.  Cell volume = 1/3 sum over the six faces of
  (mean of the face's four nodes) . (outward area vector).

Returned shapes (nodes are (dim, [nk+1,] nj+1, ni+1)):
  S[0] i-faces (dim, [nk,] nj, ni+1); S[1] j-faces (dim, [nk,] nj+1, ni);
  S[2] k-faces (3, nk+1, nj, ni); vol (., nj, ni).
"""
import torch


def _cross(a, b):
    return torch.stack([a[1] * b[2] - a[2] * b[1],
                        a[2] * b[0] - a[0] * b[2],
                        a[0] * b[1] - a[1] * b[0]])


def metrics_2d(nodes):
    x, y = nodes[0], nodes[1]  # (nj+1, ni+1)
    # i-faces: from node (i, j) to node (i, j+1)
    dxi = x[1:, :] - x[:-1, :]
    dyi = y[1:, :] - y[:-1, :]
    Si = torch.stack([dyi, -dxi])  # (2, nj, ni+1)
    # j-faces: from node (i, j) to node (i+1, j)
    dxj = x[:, 1:] - x[:, :-1]
    dyj = y[:, 1:] - y[:, :-1]
    Sj = torch.stack([-dyj, dxj])  # (2, nj+1, ni)
    # cell area from the diagonals (i,j)->(i+1,j+1) and (i+1,j)->(i,j+1)
    d1x = x[1:, 1:] - x[:-1, :-1]
    d1y = y[1:, 1:] - y[:-1, :-1]
    d2x = x[1:, :-1] - x[:-1, 1:]
    d2y = y[1:, :-1] - y[:-1, 1:]
    vol = 0.5 * (d1x * d2y - d1y * d2x)
    return [Si, Sj], vol


def _quad_area(a, b, c, d):
    return 0.5 * _cross(c - a, d - b)


def metrics_3d(nodes):
    P = nodes  # (3, nk+1, nj+1, ni+1), index [c, k, j, i]
    # i-face at (i, j, k): a=(i,j,k) b=(i,j+1,k) c=(i,j+1,k+1) d=(i,j,k+1)
    a = P[:, :-1, :-1, :]
    b = P[:, :-1, 1:, :]
    c = P[:, 1:, 1:, :]
    d = P[:, 1:, :-1, :]
    Si = _quad_area(a, b, c, d)
    ci = 0.25 * (a + b + c + d)
    # j-face at (i, j, k): a=(i,j,k) b=(i,j,k+1) c=(i+1,j,k+1) d=(i+1,j,k)
    a = P[:, :-1, :, :-1]
    b = P[:, 1:, :, :-1]
    c = P[:, 1:, :, 1:]
    d = P[:, :-1, :, 1:]
    Sj = _quad_area(a, b, c, d)
    cj = 0.25 * (a + b + c + d)
    # k-face at (i, j, k): a=(i,j,k) b=(i+1,j,k) c=(i+1,j+1,k) d=(i,j+1,k)
    a = P[:, :, :-1, :-1]
    b = P[:, :, :-1, 1:]
    c = P[:, :, 1:, 1:]
    d = P[:, :, 1:, :-1]
    Sk = _quad_area(a, b, c, d)
    ck = 0.25 * (a + b + c + d)
    # volume: 1/3 sum_f xbar_f . S_f(outward); high faces outward = +S, low = -S
    fi = (ci * Si).sum(0)  # (nk, nj, ni+1)
    fj = (cj * Sj).sum(0)  # (nk, nj+1, ni)
    fk = (ck * Sk).sum(0)  # (nk+1, nj, ni)
    vol = ((fi[:, :, 1:] - fi[:, :, :-1]) + (fj[:, 1:, :] - fj[:, :-1, :])
           + (fk[1:] - fk[:-1])) / 3.0
    return [Si, Sj, Sk], vol


def metrics(nodes):
    nodes = torch.as_tensor(nodes, dtype=torch.float64)
    if nodes.shape[0] == 2:
        return metrics_2d(nodes)
    return metrics_3d(nodes)
