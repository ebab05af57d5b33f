"""Algorithm 1 of the paper driven through the C ABI.

Only buffers and call order live here; every step of an iteration is one of
the library's entry points (the zero fill of the accumulated region
correction at the start of an outer iteration is buffer initialisation).
outer_iteration runs one iteration on the context stream; run_pipelined
overlaps consecutive iterations on two streams."""
import numpy as np

from ._lib import PDContext, PD_FP64


class Alg1Runner:
    """Buffers and call sequence for outer/inner iterations with sphere
    obstacles and conforming proxies."""

    def __init__(self, rest, tets, region, dirichlet, mu, proxies_global, k_pen, device="cuda",
                 density=0.0, dt=0.0, mu_prime=0.0, sigma_min=0.0, sigma_max=0.0,
                 interior="levels", nd_leaf=0):
        import torch
        self.torch = torch
        self.ctx = PDContext(rest, tets, region, dirichlet, mu, density=density, dt=dt,
                             mu_prime=mu_prime, sigma_min=sigma_min, sigma_max=sigma_max,
                             interior=interior, nd_leaf=nd_leaf)
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
        self.mode = "nodes"
        self.dt = float(dt)
        if self.dt > 0.0:
            # backward Euler: inertial target y = x_n + dt v_n (from rest at rest)
            self.y = self.x.clone()
            self.x_prev = self.x.clone()
            self.v = torch.zeros_like(self.x)
            c.set_inertia_target(self.y)

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
        self.mode = "pairs"
        self.n_prox = npr
        self.idx = torch.empty(8 * npr, dtype=torch.int32, device=dev)
        self.w = torch.empty(8 * npr, dtype=torch.float64, device=dev)
        self.c = torch.empty(npr, dtype=torch.float64, device=dev)
        self.t = torch.empty(3 * npr, dtype=torch.float64, device=dev)

    def _penalty_buffers(self, n):
        import torch
        dev = self.x.device
        self.n_prox = n
        self.idx = torch.empty(8 * n, dtype=torch.int32, device=dev)
        self.w = torch.empty(8 * n, dtype=torch.float64, device=dev)
        self.c = torch.empty(n, dtype=torch.float64, device=dev)
        self.t = torch.empty(3 * n, dtype=torch.float64, device=dev)

    def embed(self, pts, cand_local, pos=None):
        """Embedding of rest points pts (3, n) in the region tets cand_local
        (4, nc) (pd_embed_points, at the region's rest positions unless pos
        is given).  Returns device tensors (tet, eidx [n][4], ew [n][4])."""
        import torch
        c = self.ctx
        dev = self.x.device
        n = np.asarray(pts).shape[1]
        if pos is None:
            pos = torch.empty(3 * c.m, dtype=torch.float64, device=dev)
            c.region_gather(torch.tensor(self.rest_np, device=dev).reshape(-1), pos)
        tet = torch.empty(n, dtype=torch.int32, device=dev)
        eidx = torch.empty(4 * n, dtype=torch.int32, device=dev)
        ew = torch.empty(4 * n, dtype=torch.float64, device=dev)
        c.embed_points(torch.tensor(np.ascontiguousarray(pts, dtype=np.float64), device=dev).reshape(-1),
                       torch.tensor(np.ascontiguousarray(cand_local, dtype=np.int32), device=dev).reshape(-1),
                       pos, tet, eidx, ew)
        return tet, eidx, ew

    def use_embedded(self, eidx, ew):
        """Switch detection to sphere contact of embedded proxies (device eidx
        int32 [n][4], ew [n][4] from embed())."""
        self.mode = "embedded"
        self.eidx, self.ew = eidx, ew
        self.pairs = None
        self._penalty_buffers(eidx.numel() // 4)

    def use_levelset(self, eidx, ew, prox_body, cand_local, cand_phi, cand_body):
        """Switch detection to rest-pose level-set self-collision of embedded
        proxies (pd_detect_levelset): proxies eidx/ew with body ids prox_body,
        bodies given by candidate region tets cand_local (4, nc), their corner
        signed distances cand_phi (4, nc) and body ids cand_body (nc,)."""
        import torch
        c = self.ctx
        dev = self.x.device
        self.mode = "levelset"
        self.pairs = None
        self.eidx, self.ew = eidx, ew
        self.ls_body = torch.tensor(np.ascontiguousarray(prox_body, dtype=np.int32), device=dev)
        self.ls_cand = torch.tensor(np.ascontiguousarray(cand_local, dtype=np.int32), device=dev).reshape(-1)
        self.ls_phi = torch.tensor(np.ascontiguousarray(cand_phi, dtype=np.float64), device=dev).reshape(-1)
        self.ls_cbody = torch.tensor(np.ascontiguousarray(cand_body, dtype=np.int32), device=dev)
        self.rest2 = torch.empty(3 * c.m, dtype=torch.float64, device=dev)
        c.region_gather(torch.tensor(self.rest_np, device=dev).reshape(-1), self.rest2)
        self._penalty_buffers(eidx.numel() // 4)

    def detect(self):
        c = self.ctx
        if self.mode == "embedded":
            c.detect_embedded_spheres(self.eidx, self.ew, self.spheres, self.k_pen, self.x2,
                                      self.idx, self.w, self.c, self.t)
        elif self.mode == "levelset":
            c.detect_levelset(self.eidx, self.ew, self.ls_body, self.ls_cand, self.ls_phi,
                              self.ls_cbody, self.rest2, self.k_pen, self.x2, self.idx, self.w,
                              self.c, self.t)
        elif self.pairs is not None:
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
        c.local_step_full(self.x, self.f, rot_fp32=rot_fp32)
        c.condense_rhs(self.f, self.ft)
        c.region_gather(self.x, self.x2)
        self.delta2.zero_()
        infos = [self.inner_iteration(prec, rot_fp32, want_info) for _ in range(n_inner)]
        c.backsub(self.delta2, self.x)
        return infos

    def run_pipelined(self, n_iters, spheres_of=None, n_workgroups=0, factor_stream=None,
                      overlap_forward=True, before_local=None):
        """n_iters outer iterations with one inner iteration each, pipelined
        over two streams.  The factorization side of iteration k (detection,
        penalties, region local step, H = S + W^T C W and its Cholesky factor)
        needs only the region positions after the inner update of iteration
        k - 1, so it runs on a second stream while the back substitution of
        k - 1, the full local step and the condensation of k run on the context
        stream.  With overlap_forward (the default) the forward solve is
        enqueued on the context stream without waiting for the factorization
        and follows its tile flags, and the backward solve waits for its end;
        otherwise both triangular solves follow the factorization.  The solves
        and the inner update join both streams.  The arithmetic is that of
        outer_iteration(n_inner=1), except that the region positions are
        carried over from the inner update instead of being gathered from x
        after the back substitution (the same values: delta2 holds the single
        update).  spheres_of(k) gives the obstacle spheres of iteration k
        (None keeps the current ones); before_local(k), if given, runs on the
        context stream between the back substitution of k - 1 and the full
        local step of k (e.g. to move prescribed Dirichlet nodes in x, as a
        caller of outer_iteration would before each call)."""
        torch = self.torch
        c = self.ctx
        s_main = c.stream
        s_fac = factor_stream if factor_stream is not None else torch.cuda.Stream(device=self.x.device)
        c.region_gather(self.x, self.x2)
        ev_upd = torch.cuda.Event()
        ev_upd.record(s_main)
        for k in range(n_iters):
            if spheres_of is not None:
                self.spheres = spheres_of(k)
            # factorization side of iteration k
            s_fac.wait_event(ev_upd)
            c.use_stream(s_fac)
            self.detect()
            c.collision_update(self.idx, self.w, self.c, self.t, self.x2, self.fcol)
            c.local_step_region(self.x2, self.fb)
            ev_pen = torch.cuda.Event()          # penalties and f_beta ready
            ev_pen.record(s_fac)
            c.factor(n_workgroups, overlap_forward=overlap_forward)
            ev_fac = torch.cuda.Event()
            ev_fac.record(s_fac)
            # sweep side: finish iteration k - 1, start iteration k
            c.use_stream(s_main)
            if k > 0:
                c.backsub(self.delta2, self.x)
            if before_local is not None:
                with torch.cuda.stream(s_main):
                    before_local(k)
            c.local_step_full(self.x, self.f)
            c.condense_rhs(self.f, self.ft)
            with torch.cuda.stream(s_main):
                self.delta2.zero_()
            s_main.wait_event(ev_pen)
            c.assemble_rhs(self.ft, self.fb, self.fcol, self.g)
            if not overlap_forward:
                s_main.wait_event(ev_fac)
            c.global_solve(self.g, self.u)
            c.inner_update(self.u, self.x2, self.delta2, self.ft)
            ev_upd = torch.cuda.Event()
            ev_upd.record(s_main)
        c.backsub(self.delta2, self.x)

    def set_state(self, x, v):
        """Backward Euler: positions x_n and velocities v_n at the start of a
        step (host (3, n) arrays); sets x, x_prev = x_n and y = x_n + dt v_n
        through pd_time_step_advance from x_n - dt v_n."""
        torch = self.torch
        x = np.ascontiguousarray(x, dtype=np.float64)
        v = np.ascontiguousarray(v, dtype=np.float64)
        self.set_positions(x)
        self.x_prev.copy_(torch.as_tensor(x - self.dt * v).reshape(-1))
        self.ctx.time_step_advance(self.x, self.x_prev, self.v, self.y)

    def advance_time_step(self):
        """Backward Euler, after the step's iterations: v = (x - x_prev) / dt,
        x_prev = x, y = x + dt v for the next step."""
        self.ctx.time_step_advance(self.x, self.x_prev, self.v, self.y)

    def positions(self):
        return self.x.reshape(3, -1).cpu().numpy()

    def close(self):
        """Frees the library context (waits for its stream)."""
        self.ctx.close()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
        return False
