"""Crystal geometry for the synthetic bcc-W workloads.

Pure geometry (lattice points, rotations, wrapping into an orthorhombic box).
Nothing here evaluates a potential, a region weight or any other step of the
mixed force evaluation; both the oracle and the HIP path consume its output.
"""
import numpy as np

A_W = 3.165  # bcc W lattice constant in Angstrom (the value the workloads use)


def bcc_cubic(nx, ny, nz, a=A_W):
    """Conventional cubic bcc supercell, atoms ordered cell by cell (x fastest
    in the innermost loop is irrelevant; the order is fixed and documented):
    for i in x, for j in y, for k in z: corner atom then body-centre atom."""
    basis = np.array([[0.0, 0.0, 0.0], [0.5, 0.5, 0.5]])
    ii, jj, kk = np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij")
    cells = np.stack([ii.ravel(), jj.ravel(), kk.ravel()], axis=1).astype(np.float64)
    pos = (cells[:, None, :] + basis[None, :, :]).reshape(-1, 3) * a
    return pos


def screw_cell(a=A_W):
    """The 6-atom orthorhombic bcc cell with x=[1 0 -1], y=[-1 2 -1], z=[111]
    (edge lengths sqrt(2)a, sqrt(6)a, sqrt(3)a/2). Returns (positions, edges)."""
    e1 = np.array([1.0, 0.0, -1.0]) / np.sqrt(2.0)
    e2 = np.array([-1.0, 2.0, -1.0]) / np.sqrt(6.0)
    e3 = np.array([1.0, 1.0, 1.0]) / np.sqrt(3.0)
    R = np.stack([e1, e2, e3])  # rows: new axes in cubic coordinates
    edges = np.array([np.sqrt(2.0) * a, np.sqrt(6.0) * a, np.sqrt(3.0) * a / 2.0])
    rng = np.arange(-4, 5)
    pts = []
    for i in rng:
        for j in rng:
            for k in rng:
                for b in ((0.0, 0.0, 0.0), (0.5, 0.5, 0.5)):
                    pts.append((i + b[0], j + b[1], k + b[2]))
    pts = np.array(pts) * a
    rot = pts @ R.T
    frac = rot / edges
    keep = np.all((frac > -1e-9) & (frac < 1.0 - 1e-9), axis=1)
    cell = rot[keep]
    cell = np.where(np.abs(cell) < 1e-9, 0.0, cell)
    # canonical order: sort by (z, y, x) rounded
    key = np.lexsort((np.round(cell[:, 0], 6), np.round(cell[:, 1], 6), np.round(cell[:, 2], 6)))
    cell = cell[key]
    assert cell.shape[0] == 6, cell.shape
    return cell, edges


def replicate(cell, edges, nx, ny, nz):
    ii, jj, kk = np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij")
    shifts = np.stack([ii.ravel(), jj.ravel(), kk.ravel()], axis=1) * edges
    return (shifts[:, None, :] + cell[None, :, :]).reshape(-1, 3)


def wrap(pos, L, periodic):
    """Wrap periodic coordinates into [0, L); x -= L*floor(x/L)."""
    out = pos.copy()
    for d in range(3):
        if periodic[d]:
            out[:, d] = out[:, d] - L[d] * np.floor(out[:, d] / L[d])
            # floor can leave exactly L after rounding; fold it back to 0
            out[:, d] = np.where(out[:, d] >= L[d], out[:, d] - L[d], out[:, d])
    return out


def oriented_bcc(x_dir, y_dir, z_dir, periods, a=A_W):
    """Orthorhombic periodic bcc cell whose edges run along the given cubic
    directions (mutually orthogonal Miller vectors) with the given edge
    lengths in units of a (each a lattice period along its direction).
    Atoms sorted by (z, y, x)."""
    R = np.stack([np.asarray(d, np.float64) / np.linalg.norm(d) for d in (x_dir, y_dir, z_dir)])
    assert np.allclose(R @ R.T, np.eye(3))
    edges = np.asarray(periods, np.float64) * a
    m = int(np.ceil(np.linalg.norm(edges) / a)) + 1
    rng = np.arange(-m, m + 1)
    ii, jj, kk = np.meshgrid(rng, rng, rng, indexing="ij")
    corners = np.stack([ii.ravel(), jj.ravel(), kk.ravel()], axis=1).astype(np.float64)
    pts = np.concatenate([corners, corners + 0.5]) * a
    rot = pts @ R.T
    frac = rot / edges
    keep = np.all((frac > -1e-9) & (frac < 1.0 - 1e-9), axis=1)
    cell = np.where(np.abs(rot[keep]) < 1e-9, 0.0, rot[keep])
    key = np.lexsort((np.round(cell[:, 0], 6), np.round(cell[:, 1], 6), np.round(cell[:, 2], 6)))
    cell = cell[key]
    assert len(cell) == int(round(2.0 * np.prod(edges) / a ** 3)), len(cell)
    return cell, edges
