"""Penalty collision terms (paper Sec. 3.3 and Sec. 4.1).

Proxies p_j = sum_i w_(j,i) x_i (eq. p_j_v).  A proxy found inside an
obstacle is projected to the obstacle surface t_j and a zero-rest-length
spring of stiffness c_j joins them, giving
E_col = sum_j c_j/2 ||p_j - t_j||^2 delta_j, which separates by coordinate
(eq. e_col_j) into 1/2 (W x^(v) - t^(v))^T C (W x^(v) - t^(v)) (eq. E_col_C).
With t and C frozen its Hessian is W^T C W and its force -W^T C (W x - t)
(Sec. 4.1; the '+t' printed there is read as '-t', consistent with eq.
E_col_C).

Penalties are given as fixed-width lists: idx (P, 8) region-local node ids
(-1 = unused slot), w (P, 8) weights, c (P,), t (3, P).
"""
import numpy as np

SLOTS = 8


def detect_spheres(p, centers, radii, k):
    """Collision detection against rigid spheres for proxy positions p (3, np).

    A proxy is in collision iff ||p - c_s|| < r_s (strict).  Its target is the
    closest surface point t = c_s + r_s (p - c_s)/||p - c_s|| (direction +z
    when p sits exactly at the centre).  With several spheres the deepest
    penetration r_s - ||p - c_s|| wins; ties go to the lowest sphere index.
    Returns (c (np,), t (3, np)); inactive proxies get c = 0 and t = p.
    """
    npx = p.shape[1]
    c = np.zeros(npx)
    t = p.copy()
    best = np.full(npx, -np.inf)
    for s in range(centers.shape[1]):
        d = p - centers[:, s:s + 1]
        dist = np.sqrt(np.sum(d * d, axis=0))
        depth = radii[s] - dist
        hit = (dist < radii[s]) & (depth > best)
        if not np.any(hit):
            continue
        dirn = np.zeros_like(d)
        nz = dist > 0
        dirn[:, nz] = d[:, nz] / dist[nz]
        dirn[2, ~nz] = 1.0
        tgt = centers[:, s:s + 1] + radii[s] * dirn
        t[:, hit] = tgt[:, hit]
        c[hit] = k
        best[hit] = depth[hit]
    return c, t


def conforming_penalties(proxy_local, c, t):
    """Penalty lists for proxies that are region nodes themselves (W rows are
    unit selections, Sec. 3.3)."""
    P = proxy_local.size
    idx = np.full((P, SLOTS), -1, dtype=np.int32)
    w = np.zeros((P, SLOTS))
    idx[:, 0] = proxy_local
    w[:, 0] = 1.0
    return idx, w, np.asarray(c, dtype=np.float64), np.asarray(t, dtype=np.float64)


def penalty_matrix(m, idx, w, c):
    """Dense m x m C_22 = W^T C W (eq. E_col_C Hessian; the additive term of eq. k22)."""
    Pm = np.zeros((m, m))
    for j in range(idx.shape[0]):
        if c[j] == 0.0:
            continue
        for a in range(idx.shape[1]):
            ia = idx[j, a]
            if ia < 0:
                continue
            for b in range(idx.shape[1]):
                ib = idx[j, b]
                if ib < 0:
                    continue
                Pm[ia, ib] += c[j] * w[j, a] * w[j, b]
    return Pm


def penalty_force(m, idx, w, c, t, x2):
    """f_col = -W^T C (W x2 - t) per coordinate (Sec. 4.1, sign read from eq. E_col_C).
    x2: (3, m) region positions; returns (3, m)."""
    f = np.zeros((3, m))
    for j in range(idx.shape[0]):
        if c[j] == 0.0:
            continue
        sl = idx[j] >= 0
        ids = idx[j][sl]
        ws = w[j][sl]
        r = x2[:, ids] @ ws - t[:, j]          # (3,) = W x - t for this proxy
        for a, wa in zip(ids, ws):
            f[:, a] -= c[j] * wa * r
    return f


def penalty_energy(idx, w, c, t, x2):
    """E_col = sum_j c_j / 2 ||W_j x - t_j||^2 over active penalties (Sec. 3.3)."""
    e = 0.0
    for j in range(idx.shape[0]):
        if c[j] == 0.0:
            continue
        sl = idx[j] >= 0
        r = x2[:, idx[j][sl]] @ w[j][sl] - t[:, j]
        e += 0.5 * c[j] * float(r @ r)
    return e


def detect_pairs(x2, pairs_local, k):
    """Two-sided contact of paired lip nodes (self-collision of a slit): pair
    (a, b) = (lower-lip node, upper-lip node) is in collision iff the upper
    node lies strictly below the lower one, z_b < z_a.  An active pair is a
    zero-rest-length spring between the two nodes: W row [1, -1] on (a, b),
    target t = 0 (Sec. 3.3 with the proxy and the surface point both on the
    mesh).  Returns penalty lists (idx, w, c, t) with one entry per pair."""
    P = pairs_local.shape[1]
    idx = np.full((P, SLOTS), -1, dtype=np.int32)
    w = np.zeros((P, SLOTS))
    idx[:, 0] = pairs_local[0]
    idx[:, 1] = pairs_local[1]
    w[:, 0] = 1.0
    w[:, 1] = -1.0
    active = x2[2, pairs_local[1]] < x2[2, pairs_local[0]]
    c = np.where(active, float(k), 0.0)
    return idx, w, c, np.zeros((3, P))


# ---- embedded proxies and rest-pose level sets ----------------------------
# A proxy embedded in the mesh (Sec. 3.3, eq. p_j_v) moves with the
# tetrahedron that contains it in the rest pose: p_j = sum_k w_k x_k over that
# tet's four nodes, with w the barycentric coordinates of its rest position.
# Self-collision (Sec. 5.1, rest-pose level sets): a proxy that has entered
# another part of the body is located in that part's deformed tets, taken
# back to the rest pose with the same barycentric coordinates, and tested
# against a signed distance phi of that part's rest shape (phi < 0 inside);
# inside, its target is the rest-pose closest surface point carried forward to
# the deformed configuration by the tet that contains it.

BARY_TOL = 1e-12


def barycentric(pt, corners):
    """Barycentric coordinates (4,) of point pt (3,) in the tet with corner
    positions corners (3, 4): solve [x1-x0, x2-x0, x3-x0] l = pt - x0."""
    D = corners[:, 1:] - corners[:, :1]
    l = np.linalg.solve(D, pt - corners[:, 0])
    return np.concatenate([[1.0 - l.sum()], l])


def locate(pt, tets, pos, tol=BARY_TOL, exclude=()):
    """Lowest index e of a tet (tets (4, T) node ids into pos (3, *)) that
    contains pt, i.e. whose barycentric coordinates are all >= -tol, skipping
    tets that share a node with `exclude`; (-1, None) if there is none."""
    ex = set(int(v) for v in exclude)
    for e in range(tets.shape[1]):
        nodes = tets[:, e]
        if ex and any(int(v) in ex for v in nodes):
            continue
        b = barycentric(pt, pos[:, nodes])
        if np.all(b >= -tol):
            return e, b
    return -1, None


def embed_points(P_rest, tets, rest, tol=BARY_TOL):
    """Embedding of proxy rest positions P_rest (3, n) in the tets (4, T) (node
    ids into rest (3, *)): per proxy the containing tet (lowest index), its
    four node ids and barycentric weights.  Returns (tet (n,), idx (n, 4),
    w (n, 4)); a proxy outside every tet gets tet -1, idx -1, w 0."""
    n = P_rest.shape[1]
    tet = np.full(n, -1, dtype=np.int64)
    idx = np.full((n, 4), -1, dtype=np.int32)
    w = np.zeros((n, 4))
    for j in range(n):
        e, b = locate(P_rest[:, j], tets, rest, tol)
        if e >= 0:
            tet[j] = e
            idx[j] = tets[:, e]
            w[j] = b
    return tet, idx, w


def embedded_positions(x2, eidx, ew):
    """p_j = sum_k w_jk x_(idx_jk) (eq. p_j_v), (3, n)."""
    return np.einsum("vjk,jk->vj", x2[:, eidx], ew)


def embedded_sphere_penalties(x2, eidx, ew, centers, radii, k):
    """Sphere detection for embedded proxies: the sphere rule of detect_spheres
    applied to p_j, one penalty per proxy whose W row is the proxy's four
    barycentric weights."""
    p = embedded_positions(x2, eidx, ew)
    c, t = detect_spheres(p, centers, radii, k)
    P = eidx.shape[0]
    idx = np.full((P, SLOTS), -1, dtype=np.int32)
    w = np.zeros((P, SLOTS))
    idx[:, :4] = eidx
    w[:, :4] = ew
    return idx, w, c, t


def levelset_gradient(corners_rest, phi4):
    """Gradient of the linear interpolant of the nodal values phi4 (4,) over a
    tet with rest corner positions (3, 4): D^T g = phi_k - phi_0."""
    D = corners_rest[:, 1:] - corners_rest[:, :1]
    return np.linalg.solve(D.T, phi4[1:] - phi4[0])


def levelset_penalties(x2, rest2, eidx, ew, prox_body, cand, cand_phi, cand_body, k,
                       tol=BARY_TOL):
    """Rest-pose level-set self-collision of embedded proxies.  The bodies are
    given by candidate tets cand (4, nc) (region-local node ids), the signed
    distance of their body's rest shape at their four corners cand_phi (4, nc)
    (phi < 0 inside; linear over the tet) and a body id cand_body (nc,); proxy
    j belongs to body prox_body[j] and is tested against the other bodies.

    Per proxy j: p = sum w x2 over its embedding tet; the lowest candidate tet
    e of another body that contains p in the deformed configuration x2 (tets
    sharing a node with the proxy's own tet are skipped too); X = its rest
    point with the same barycentric coordinates b, phi(X) = sum b phi_e; if
    phi(X) < 0, the rest-pose surface point X_s = X - phi(X) g / |g|^2 (g =
    grad phi on e), located in the rest candidate tets of the same body (lowest
    index, same skip rule) with coordinates b'.  The penalty is a
    zero-rest-length spring between the proxy and that surface point: W row =
    [w over the proxy's nodes, -b' over the surface tet's nodes] (a node
    present twice carries the sum of its weights, in its first slot), target
    0, stiffness k.  Otherwise c = 0.  Returns penalty lists (idx, w, c, t),
    one entry per proxy."""
    P = eidx.shape[0]
    idx = np.full((P, SLOTS), -1, dtype=np.int32)
    w = np.zeros((P, SLOTS))
    c = np.zeros(P)
    t = np.zeros((3, P))
    p_all = embedded_positions(x2, eidx, ew)
    for j in range(P):
        idx[j, :4] = eidx[j]
        w[j, :4] = ew[j]
        other = np.nonzero(cand_body != prox_body[j])[0]
        e, b = locate(p_all[:, j], cand[:, other], x2, tol, exclude=eidx[j])
        if e < 0:
            continue
        body = cand_body[other[e]]
        nodes = cand[:, other[e]]
        phi4 = cand_phi[:, other[e]]
        X = rest2[:, nodes] @ b
        ph = float(phi4 @ b)
        if not ph < 0.0:
            continue
        g = levelset_gradient(rest2[:, nodes], phi4)
        gg = float(g @ g)
        if gg == 0.0:
            continue
        Xs = X - ph * g / gg
        same = np.nonzero(cand_body == body)[0]
        e2, b2 = locate(Xs, cand[:, same], rest2, tol, exclude=eidx[j])
        if e2 < 0:
            continue
        row_i = [int(v) for v in eidx[j]]
        row_w = list(ew[j])
        for v, bv in zip(cand[:, same[e2]], b2):
            if int(v) in row_i:
                row_w[row_i.index(int(v))] -= bv
            else:
                row_i.append(int(v))
                row_w.append(-bv)
        idx[j, :len(row_i)] = row_i
        w[j, :len(row_w)] = row_w
        c[j] = k
    return idx, w, c, t
