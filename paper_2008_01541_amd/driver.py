"""Algorithm 1 of the paper driven through the C ABI, on one HIP stream.

Only buffers and call order live here; every step of an iteration is one of
the library's entry points (the zero fill of the accumulated region
correction at the start of an outer iteration is buffer initialisation)."""
import numpy as np

from ._lib import PDContext, PD_FP64


class Alg1Runner:
    """Buffers and call sequence for outer/inner iterations with sphere
    obstacles and conforming proxies."""

    def __init__(self, rest, tets, region, dirichlet, mu, proxies_global, k_pen, device="cuda"):
        import torch
        self.torch = torch
        self.ctx = PDContext(rest, tets, region, dirichlet, mu)
        c = self.ctx
        dev = torch.device(device)
        f64 = dict(dtype=torch.float64, device=dev)
        self.rest_np = np.ascontiguousarray(rest, dtype=np.float64)
        self.x = torch.tensor(self.rest_np, **f64).reshape(-1)
        self.f = torch.zeros(3 * c.n, **f64)
        m = c.m
        self.x2, self.ft, self.fb, self.fcol, self.g, self.u, self.delta2 = \
            (torch.zeros(3 * m, **f64) for _ in range(7))
        pos = np.full(c.n, -1, dtype=np.int64)
        pos[c.region_ids] = np.arange(m)
        loc = pos[np.asarray(proxies_global)]
        if loc.size and (loc < 0).any():
            raise ValueError("every proxy must be a free region node")
        self.n_prox = loc.size
        self.prox = torch.tensor(loc.astype(np.int32), device=dev)
        self.idx = torch.empty(8 * self.n_prox, dtype=torch.int32, device=dev)
        self.w = torch.empty(8 * self.n_prox, **f64)
        self.c = torch.empty(self.n_prox, **f64)
        self.t = torch.empty(3 * self.n_prox, **f64)
        self.k_pen = float(k_pen)
        self.spheres = None
        self.pairs = None

    def set_spheres(self, centers, radii):
        sph = np.vstack([np.asarray(centers, dtype=np.float64),
                         np.asarray(radii, dtype=np.float64)[None, :]])
        self.spheres = self.torch.tensor(np.ascontiguousarray(sph), dtype=self.torch.float64,
                                         device=self.x.device).reshape(-1)

    def set_positions(self, x):
        self.x.copy_(self.torch.as_tensor(np.ascontiguousarray(x, dtype=np.float64)).reshape(-1))

    def use_pairs(self, pairs_global):
        """Switch detection to paired region nodes (self-contact of a slit)."""
        import torch
        c = self.ctx
        pos = np.full(c.n, -1, dtype=np.int64)
        pos[c.region_ids] = np.arange(c.m)
        loc = pos[np.asarray(pairs_global)]
        if (loc < 0).any():
            raise ValueError("every paired node must be a free region node")
        npr = loc.shape[1]
        dev = self.x.device
        self.pairs = torch.tensor(np.ascontiguousarray(loc, dtype=np.int32), device=dev).reshape(-1)
        self.n_prox = npr
        self.idx = torch.empty(8 * npr, dtype=torch.int32, device=dev)
        self.w = torch.empty(8 * npr, dtype=torch.float64, device=dev)
        self.c = torch.empty(npr, dtype=torch.float64, device=dev)
        self.t = torch.empty(3 * npr, dtype=torch.float64, device=dev)

    def detect(self):
        c = self.ctx
        if self.pairs is not None:
            c.detect_pairs(self.pairs, self.k_pen, self.x2, self.idx, self.w, self.c, self.t)
        else:
            c.detect_spheres(self.prox, self.spheres, self.k_pen, self.x2, self.idx, self.w,
                             self.c, self.t)

    def inner_iteration(self, prec=PD_FP64, rot_fp32=False, want_info=False):
        c = self.ctx
        self.detect()
        c.collision_update(self.idx, self.w, self.c, self.t, self.x2, self.fcol)
        c.local_step_region(self.x2, self.fb, rot_fp32=rot_fp32)
        c.assemble_rhs(self.ft, self.fb, self.fcol, self.g)
        info = c.global_solve(self.g, self.u, prec, want_info=want_info)
        c.inner_update(self.u, self.x2, self.delta2, self.ft)
        return info

    def outer_iteration(self, n_inner=1, prec=PD_FP64, rot_fp32=False, want_info=False):
        c = self.ctx
        c.local_step_full(self.x, self.f)
        c.condense_rhs(self.f, self.ft)
        c.region_gather(self.x, self.x2)
        self.delta2.zero_()
        infos = [self.inner_iteration(prec, rot_fp32, want_info) for _ in range(n_inner)]
        c.backsub(self.delta2, self.x)
        return infos

    def positions(self):
        return self.x.reshape(3, -1).cpu().numpy()
