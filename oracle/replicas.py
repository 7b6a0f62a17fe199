"""Light-cone replicas with per-replica transforms, FP64 (test infrastructure only).

The paper tiles the light cone by replicating the periodic box along the line of sight and
transforms each replica at random (Sec. 6.2). Reading used here: replica k holds the
line-of-sight planes j with k n <= j < (k + 1) n (plane j at z_j = j * cell) and is the
box seen through a symmetry of the cubic lattice plus an integer translation, so mesh
nodes land on mesh nodes:

    replica axis a (0 = x, 1 = y, 2 = z = line of sight) runs along box axis perm[a] with
    orientation sign[a] = +-1, and replica node u sits on box node
        x[perm[a]] = sign[a] * u[a] + shift[perm[a]]   (mod n).

The transforms are inputs (one row (perm0, perm1, perm2, sign0, sign1, sign2, shift0,
shift1, shift2) per replica, replica k using row k mod rows); the identity table gives the
plain periodic replication. A field f of the box reads f(x(u)) in replica coordinates, so
its gradient along replica axis a is sign[a] times the box gradient along perm[a]; with
the antisymmetric fourth-order difference this holds exactly on the mesh.
"""
import numpy as np

IDENTITY = (0, 1, 2, 1, 1, 1, 0, 0, 0)


def split(row):
    row = [int(v) for v in row]
    return row[0:3], row[3:6], row[6:9]


def box_nodes(row, u, n):
    """Box node indices (..., 3) in (x, y, z) order of replica node indices u (..., 3)."""
    perm, sign, shift = split(row)
    u = np.asarray(u)
    xb = np.empty_like(u)
    for a in range(3):
        xb[..., perm[a]] = sign[a] * u[..., a] + shift[perm[a]]
    return np.mod(xb, n)


def lens_plane(fields, j, n, table, grad=True):
    """Line-of-sight plane j in its replica's frame, as 2D arrays [v, u].

    fields: (G_x, G_y, G_z) box meshes [z, y, x] when grad, else one scalar box mesh.
    Returns (G_u, G_v) (the transverse gradient in the replica frame) or the scalar plane."""
    row = table[(j // n) % len(table)]
    perm, sign, _ = split(row)
    uy, ux = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    u = np.stack([ux, uy, np.full_like(ux, j % n)], axis=-1)
    xb = box_nodes(row, u, n)
    at = lambda f: f[xb[..., 2], xb[..., 1], xb[..., 0]]
    if not grad:
        return at(fields)
    return sign[0] * at(fields[perm[0]]), sign[1] * at(fields[perm[1]])


def validate(table, n):
    for row in table:
        perm, sign, shift = split(row)
        if sorted(perm) != [0, 1, 2] or any(s not in (-1, 1) for s in sign) or \
                any(not 0 <= t < n for t in shift):
            raise ValueError(f"bad replica transform {row}")
