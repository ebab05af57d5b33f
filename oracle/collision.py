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
