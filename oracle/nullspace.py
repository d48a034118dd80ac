"""Rigid body modes from node coordinates (oracle side; test infrastructure only).

Section 2: for 3D elasticity the near-nullspace is the six rigid body modes,
computed from the grid coordinates and given as an n x 6 matrix B.  Reading
(the paper gives no formula): with d = x - centroid of all nodes, the columns
are the three unit translations and the three infinitesimal rotations
r_x = (0, -d_z, d_y), r_y = (d_z, 0, -d_x), r_z = (-d_y, d_x, 0), stored
node-major to match the unknown numbering.

Pinned: K B = 0 for the stiffness of an unconstrained mesh (rigid motions cost
no strain energy).
"""
import numpy as np


def rigid_body_modes(coords):
    coords = np.asarray(coords, dtype=np.float64)
    nb = coords.shape[0]
    d = coords - coords.mean(axis=0)
    B = np.zeros((nb, 3, 6))
    B[:, 0, 0] = 1.0
    B[:, 1, 1] = 1.0
    B[:, 2, 2] = 1.0
    # rotation about x: (0, -dz, dy)
    B[:, 1, 3] = -d[:, 2]
    B[:, 2, 3] = d[:, 1]
    # rotation about y: (dz, 0, -dx)
    B[:, 0, 4] = d[:, 2]
    B[:, 2, 4] = -d[:, 0]
    # rotation about z: (-dy, dx, 0)
    B[:, 0, 5] = -d[:, 1]
    B[:, 1, 5] = d[:, 0]
    return B.reshape(3 * nb, 6)
