"""Regular Kuhn-split tetrahedral grids (the synthetic stand-in for the
paper's regular embedding meshes, Sec. 5).

Node id = i + (nx+1) * (j + (ny+1) * k) for lattice point (i, j, k); rest
position h * (i, j, k).  Every cube is split into the 6 tetrahedra that share
its main diagonal (one per ordering of the three axes), which gives a
conforming mesh.  Each tet is stored with positive orientation.
"""
import itertools
import numpy as np

_PERMS = list(itertools.permutations(range(3)))


def _perm_sign(p):
    s = 1
    p = list(p)
    for i in range(len(p)):
        for j in range(i + 1, len(p)):
            if p[i] > p[j]:
                s = -s
    return s


def grid_node_id(i, j, k, nx, ny):
    return i + (nx + 1) * (j + (ny + 1) * k)


def kuhn_grid(nx, ny, nz, h=1.0):
    """Return (rest[3][n] float64, tets[4][T] int32) for an nx*ny*nz cell grid."""
    ii, jj, kk = np.meshgrid(np.arange(nx + 1), np.arange(ny + 1), np.arange(nz + 1),
                             indexing="ij")
    n = (nx + 1) * (ny + 1) * (nz + 1)
    rest = np.empty((3, n), dtype=np.float64)
    ids = grid_node_id(ii, jj, kk, nx, ny).ravel()
    rest[0, ids] = h * ii.ravel()
    rest[1, ids] = h * jj.ravel()
    rest[2, ids] = h * kk.ravel()

    # cells ordered k (slowest), j, i (fastest); 6 tets per cell
    ck, cj, ci = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    ci, cj, ck = ci.ravel(), cj.ravel(), ck.ravel()
    ncell = ci.size
    tets = np.empty((4, ncell, 6), dtype=np.int64)
    for t, p in enumerate(_PERMS):
        off = np.zeros(3, dtype=np.int64)
        verts = [grid_node_id(ci, cj, ck, nx, ny)]
        for ax in p:
            off[ax] += 1
            verts.append(grid_node_id(ci + off[0], cj + off[1], ck + off[2], nx, ny))
        if _perm_sign(p) < 0:          # keep det(D_m) > 0
            verts[1], verts[2] = verts[2], verts[1]
        for a in range(4):
            tets[a, :, t] = verts[a]
    return rest, tets.reshape(4, ncell * 6).astype(np.int32)


def layer_mask(nx, ny, nz, ks):
    """Boolean node mask selecting the lattice layers k in `ks`."""
    kk = np.broadcast_to(np.arange(nz + 1)[:, None, None], (nz + 1, ny + 1, nx + 1))
    return np.isin(kk, np.asarray(list(ks))).ravel()


def kuhn_grid_slit(nx, ny, nz, h, zs, ys_end):
    """Kuhn grid with a zero-thickness slit on the plane k = zs over
    j < ys_end: those nodes get a twin (appended ids) used by the tets above
    the plane, so the two lips can separate and collide.  The line j = ys_end
    stays shared.  Returns (rest, tets, twins) with twins (2, n_twins) =
    (lower-lip id, upper-lip id)."""
    rest, tets = kuhn_grid(nx, ny, nz, h)
    n0 = rest.shape[1]
    ii, jj = np.meshgrid(np.arange(nx + 1), np.arange(ys_end), indexing="ij")
    lower = grid_node_id(ii.ravel(), jj.ravel(), zs, nx, ny)
    upper = n0 + np.arange(lower.size)
    twin_of = np.full(n0, -1, dtype=np.int64)
    twin_of[lower] = upper
    rest = np.concatenate([rest, rest[:, lower]], axis=1)
    # cells are ordered k, j, i with 6 tets each: tets of cells with k >= zs
    ncell_layer = nx * ny * 6
    above = np.arange(tets.shape[1]) >= zs * ncell_layer
    t = tets.astype(np.int64)
    sub = t[:, above]
    tw = twin_of[sub]
    sub = np.where(tw >= 0, tw, sub)
    t[:, above] = sub
    return rest, t.astype(np.int32), np.vstack([lower, upper]).astype(np.int64)
