"""Transducer and reconstruction-grid geometry (float32 arrays, metres).

Element and voxel coordinates are float32 ``[N, 3]`` arrays as in the paper's
memory table (Table 4): receive-element coordinates and output-grid
coordinates are both float32 triplets.  The grid is an arbitrary point list;
the helpers below emit regular grids with depth (z) varying fastest.
"""

import numpy as np


def linear_array(n_elem, pitch):
    """Linear array along x, centred on the origin, in the z = 0 plane."""
    x = (np.arange(n_elem, dtype=np.float64) - (n_elem - 1) / 2.0) * pitch
    xyz = np.zeros((n_elem, 3), dtype=np.float64)
    xyz[:, 0] = x
    return xyz.astype(np.float32)


def matrix_array(nx, ny, pitch):
    """nx-by-ny matrix array in the z = 0 plane, element e = iy * nx + ix."""
    ix = np.arange(nx, dtype=np.float64)
    iy = np.arange(ny, dtype=np.float64)
    gx, gy = np.meshgrid((ix - (nx - 1) / 2.0) * pitch, (iy - (ny - 1) / 2.0) * pitch, indexing="xy")
    xyz = np.zeros((nx * ny, 3), dtype=np.float64)
    xyz[:, 0] = gx.ravel()
    xyz[:, 1] = gy.ravel()
    return xyz.astype(np.float32)


def grid_2d(xs, zs):
    """2D grid in the x-z plane; voxel v = ix * len(zs) + iz (depth fastest)."""
    xs = np.asarray(xs, dtype=np.float64)
    zs = np.asarray(zs, dtype=np.float64)
    gx, gz = np.meshgrid(xs, zs, indexing="ij")
    xyz = np.zeros((gx.size, 3), dtype=np.float64)
    xyz[:, 0] = gx.ravel()
    xyz[:, 2] = gz.ravel()
    return xyz.astype(np.float32)


def grid_3d(xs, ys, zs):
    """3D grid; voxel v = (ix * len(ys) + iy) * len(zs) + iz (depth fastest)."""
    xs = np.asarray(xs, dtype=np.float64)
    ys = np.asarray(ys, dtype=np.float64)
    zs = np.asarray(zs, dtype=np.float64)
    gx, gy, gz = np.meshgrid(xs, ys, zs, indexing="ij")
    return np.stack([gx.ravel(), gy.ravel(), gz.ravel()], axis=1).astype(np.float32)
